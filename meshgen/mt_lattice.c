/*
 * mt_lattice.c -- compiled twin of meshgen.lattice (input generation only:
 * no arithmetic of the loop-shrinking method lives here).
 *
 * Level-0 surface of the strut-lattice signed distance function extracted
 * by marching tetrahedra, exactly as meshgen.marching_tets_slabs does it:
 * six tetrahedra per grid cell (the tet and case tables come from the
 * Python module, so both generators use one definition), a sample below 0
 * is inside, vertices on crossed tet edges at t = fa / (fa - fb), welded by
 * their global grid-edge key (smaller grid id * npts + larger grid id) and
 * numbered in ascending key order.  Every floating-point expression is the
 * one numpy evaluates, in the same order (built with -ffp-contract=off), so
 * the vertex positions are bit-identical; triangles come out in another
 * order, which no consumer depends on.  Cell layers are processed in
 * parallel (OpenMP).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double n, radius;
    double lo[3], h[3];
    int64_t nx, ny, nz;
} grid_t;

/* signed distance to the struts of the n^3-cell lattice, as
   meshgen.lattice_plane_sdf evaluates it */
static double sdf(const grid_t *g, double x, double Y, double Z) {
    const double n = g->n;
    double jj = fmin(fmax(rint(Y), 0.0), n);
    double kk = fmin(fmax(rint(Z), 0.0), n);
    double ii = fmin(fmax(rint(x), 0.0), n);
    double ex = 0.0;
    if (-x > ex) ex = -x;
    if (x - n > ex) ex = x - n;
    double ey = fmax(0.0, fmax(-Y, Y - n));
    double ez = fmax(0.0, fmax(-Z, Z - n));
    double dyj = Y - jj, dzk = Z - kk, dxi = x - ii;
    double d1 = sqrt(dyj * dyj + dzk * dzk + ex * ex);
    double d2 = sqrt(dxi * dxi + dzk * dzk + ey * ey);
    double d3 = sqrt(dxi * dxi + dyj * dyj + ez * ez);
    return fmin(fmin(d1, d2), d3) - g->radius;
}

static double coord(const grid_t *g, int ax, int64_t i) { return g->lo[ax] + g->h[ax] * (double)i; }

static double sdf_at(const grid_t *g, int64_t gid) {
    int64_t i = gid / (g->ny * g->nz), r = gid % (g->ny * g->nz);
    int64_t j = r / g->nz, k = r % g->nz;
    return sdf(g, coord(g, 0, i), coord(g, 1, j), coord(g, 2, k));
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    int64_t *tri;    /* [nt][3] edge keys */
    int64_t nt, cap;
    int64_t *uk;     /* sorted unique corner keys */
    int64_t nu;
    int64_t split;   /* uk[0..split) have their smaller grid id in the layer's lower plane */
} layer_t;

static int push_tri(layer_t *L, int64_t a, int64_t b, int64_t c) {
    if (L->nt == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 4096;
        int64_t *p = (int64_t *)realloc(L->tri, (size_t)nc * 3 * sizeof(int64_t));
        if (!p) return -1;
        L->tri = p;
        L->cap = nc;
    }
    L->tri[3 * L->nt] = a;
    L->tri[3 * L->nt + 1] = b;
    L->tri[3 * L->nt + 2] = c;
    L->nt++;
    return 0;
}

/* binary search of key in a[0..n) (present) */
static int64_t find(const int64_t *a, int64_t n, int64_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

void mt_free(void *p) { free(p); }

/* tets: [6][4] local corner indices (dx + 2 dy + 4 dz); cases: [16][2][3][2]
   tet-local vertex pairs; ntri: [16].  Returns 0 on success, -1 when out of
   memory; *xyz_out [nv][3] and *tri_out [nf][3] are freed with mt_free. */
int mt_lattice(int32_t n_cells, double radius, int64_t nx, int64_t ny, int64_t nz, const double *lo,
               const double *hi, const int64_t *tets, const int64_t *cases, const int64_t *ntri,
               int64_t *nv_out, int64_t *nf_out, double **xyz_out, int32_t **tri_out) {
    grid_t g;
    g.n = (double)n_cells;
    g.radius = radius;
    g.nx = nx; g.ny = ny; g.nz = nz;
    const int64_t dims[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = lo[a];
        g.h[a] = (hi[a] - lo[a]) / ((double)dims[a] - 1.0);
    }
    const int64_t npts = nx * ny * nz, pl = ny * nz, nl = nx - 1;
    int64_t coff[8];
    for (int c = 0; c < 8; ++c) coff[c] = (int64_t)(c & 1) * pl + (int64_t)((c >> 1) & 1) * nz + ((c >> 2) & 1);
    layer_t *L = (layer_t *)calloc((size_t)nl, sizeof(layer_t));
    if (!L) return -1;
    int fail = 0;
    /* contiguous chunks of layers per task, so a task reuses its upper plane */
    const int64_t chunk = 8;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (int64_t c0 = 0; c0 < nl; c0 += chunk) {
        double *F0 = (double *)malloc((size_t)pl * sizeof(double));
        double *F1 = (double *)malloc((size_t)pl * sizeof(double));
        if (!F0 || !F1) { free(F0); free(F1); fail |= 1; continue; }
        for (int64_t q = 0; q < pl; ++q) F0[q] = sdf(&g, coord(&g, 0, c0), coord(&g, 1, q / nz), coord(&g, 2, q % nz));
        const int64_t c1 = c0 + chunk < nl ? c0 + chunk : nl;
        for (int64_t i = c0; i < c1 && !fail; ++i) {
            for (int64_t q = 0; q < pl; ++q)
                F1[q] = sdf(&g, coord(&g, 0, i + 1), coord(&g, 1, q / nz), coord(&g, 2, q % nz));
            layer_t *Li = &L[i];
            for (int64_t j = 0; j + 1 < ny && !fail; ++j)
                for (int64_t k = 0; k + 1 < nz; ++k) {
                    int bits = 0;
                    for (int c = 0; c < 8; ++c) {
                        const int64_t q = ((c >> 1) & 1 ? j + 1 : j) * nz + ((c >> 2) & 1 ? k + 1 : k);
                        const double f = (c & 1) ? F1[q] : F0[q];
                        bits |= (f < 0.0) << c;
                    }
                    if (bits == 0 || bits == 255) continue;
                    const int64_t base = i * pl + j * nz + k;
                    for (int t = 0; t < 6; ++t) {
                        int64_t gid[4];
                        int cs = 0;
                        for (int q = 0; q < 4; ++q) {
                            const int c = (int)tets[4 * t + q];
                            gid[q] = base + coff[c];
                            cs |= ((bits >> c) & 1) << q;
                        }
                        for (int kk = 0; kk < ntri[cs]; ++kk) {
                            int64_t key[3];
                            for (int e = 0; e < 3; ++e) {
                                const int64_t a = cases[((cs * 2 + kk) * 3 + e) * 2];
                                const int64_t b = cases[((cs * 2 + kk) * 3 + e) * 2 + 1];
                                const int64_t ga = gid[a], gb = gid[b];
                                key[e] = (ga < gb ? ga : gb) * npts + (ga < gb ? gb : ga);
                            }
                            if (push_tri(Li, key[0], key[1], key[2])) { fail |= 1; break; }
                        }
                    }
                }
            double *sw = F0; F0 = F1; F1 = sw;
            /* unique corner keys of the layer, split by the plane of their
               smaller grid id (the layer's lower plane i or upper plane i+1) */
            if (!fail && Li->nt) {
                Li->uk = (int64_t *)malloc((size_t)Li->nt * 3 * sizeof(int64_t));
                if (!Li->uk) { fail |= 1; break; }
                memcpy(Li->uk, Li->tri, (size_t)Li->nt * 3 * sizeof(int64_t));
                qsort(Li->uk, (size_t)(Li->nt * 3), sizeof(int64_t), cmp_i64);
                int64_t u = 0;
                for (int64_t q = 0; q < Li->nt * 3; ++q)
                    if (q == 0 || Li->uk[q] != Li->uk[q - 1]) Li->uk[u++] = Li->uk[q];
                Li->nu = u;
                const int64_t bound = (i + 1) * pl * npts;     /* first key whose smaller id is in plane i+1 */
                Li->split = find(Li->uk, u, bound);
            }
        }
        free(F0); free(F1);
    }
    if (fail) {
        for (int64_t i = 0; i < nl; ++i) { free(L[i].tri); free(L[i].uk); }
        free(L);
        return -1;
    }
    /* keys whose smaller grid id lies in plane p come from layer p-1 (upper
       part) and layer p (lower part): merge the two sorted lists per plane */
    int64_t *pcount = (int64_t *)calloc((size_t)nx + 1, sizeof(int64_t));
    int64_t **pkeys = (int64_t **)calloc((size_t)nx, sizeof(int64_t *));
    if (!pcount || !pkeys) { free(pcount); free(pkeys); return -1; }
#pragma omp parallel for schedule(dynamic, 4) reduction(| : fail)
    for (int64_t p = 0; p < nx; ++p) {
        const int64_t *A = p > 0 ? L[p - 1].uk + L[p - 1].split : NULL;
        const int64_t na = p > 0 ? L[p - 1].nu - L[p - 1].split : 0;
        const int64_t *B = p < nl ? L[p].uk : NULL;
        const int64_t nb = p < nl ? L[p].split : 0;
        int64_t *out = (int64_t *)malloc((size_t)(na + nb + 1) * sizeof(int64_t));
        if (!out) { fail |= 1; continue; }
        int64_t ia = 0, ib = 0, n = 0;
        while (ia < na || ib < nb) {
            int64_t x;
            if (ib >= nb || (ia < na && A[ia] <= B[ib])) x = A[ia++];
            else x = B[ib++];
            if (n == 0 || out[n - 1] != x) out[n++] = x;
        }
        pkeys[p] = out;
        pcount[p + 1] = n;
    }
    if (fail) return -1;
    for (int64_t p = 0; p < nx; ++p) pcount[p + 1] += pcount[p];
    const int64_t nv = pcount[nx];
    int64_t nf = 0;
    int64_t *toff = (int64_t *)malloc((size_t)(nl + 1) * sizeof(int64_t));
    double *xyz = (double *)malloc((size_t)nv * 3 * sizeof(double) + 8);
    if (!toff || !xyz) return -1;
    for (int64_t i = 0; i < nl; ++i) { toff[i] = nf; nf += L[i].nt; }
    toff[nl] = nf;
    int32_t *tri = (int32_t *)malloc((size_t)nf * 3 * sizeof(int32_t) + 8);
    if (!tri) return -1;
    /* positions of the welded vertices */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < nx; ++p) {
        const int64_t n = pcount[p + 1] - pcount[p];
        for (int64_t q = 0; q < n; ++q) {
            const int64_t key = pkeys[p][q], ga = key / npts, gb = key % npts;
            const double fa = sdf_at(&g, ga), fb = sdf_at(&g, gb);
            const double tt = fa / (fa - fb);
            const int64_t ia = ga / pl, ja = (ga % pl) / nz, ka = ga % nz;
            const int64_t ib = gb / pl, jb = (gb % pl) / nz, kb = gb % nz;
            const double pa[3] = {coord(&g, 0, ia), coord(&g, 1, ja), coord(&g, 2, ka)};
            const double pb[3] = {coord(&g, 0, ib), coord(&g, 1, jb), coord(&g, 2, kb)};
            double *o = xyz + 3 * (pcount[p] + q);
            for (int a = 0; a < 3; ++a) o[a] = pa[a] + tt * (pb[a] - pa[a]);
        }
    }
    /* triangles: corner keys to vertex ids */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nl; ++i) {
        for (int64_t q = 0; q < L[i].nt * 3; ++q) {
            const int64_t key = L[i].tri[q];
            const int64_t p = (key / npts) / pl;
            const int64_t n = pcount[p + 1] - pcount[p];
            tri[3 * toff[i] + q] = (int32_t)(pcount[p] + find(pkeys[p], n, key));
        }
        free(L[i].tri);
        free(L[i].uk);
    }
    for (int64_t p = 0; p < nx; ++p) free(pkeys[p]);
    free(pkeys); free(pcount); free(toff); free(L);
    *nv_out = nv;
    *nf_out = nf;
    *xyz_out = xyz;
    *tri_out = tri;
    return 0;
}
