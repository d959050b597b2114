/*
 * vls_oracle.c -- plain, slow, sequential CPU oracle of the initial pass of
 * the variational loop-shrinking method (Weinrauch et al., "A Variational
 * Loop Shrinking Analogy for Handle and Tunnel Detection and Reeb Graph
 * Construction on Surfaces", ACM TOG).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (one function per stage, each citing the passage it
 * follows):
 *   - field step: explicit Euler step of the two-phase specialisation of the
 *     diffuse-interface evolution equation (Section "Mathematical
 *     representation and data structure", evolution equation and its
 *     specialised form with the sqrt contact term; explicit Euler with a
 *     constant step; coefficients mu=1/4, e=1/30, a=1/25, w=a/5 from
 *     "Implementation details"), followed by the column normalisation, which
 *     for one region plus the base layer is a clip to [0,1];
 *   - optionally (fem) the Laplacian of linear finite elements (cotangent
 *     weights, lumped mass) in place of the uniform graph Laplacian, scaled
 *     to equal it on equilateral meshes ("Implementation details");
 *   - thresholding into an inside set and the front = triangles with one or
 *     two inside vertices (Section "Performance Considerations");
 *   - front labelling by connected components of front triangles joined
 *     through crossed edges (same section);
 *   - branching / collision events, handle count "layers involved minus
 *     one", handle loops from the involved fronts before the merge with the
 *     longest ignored (Section "Initial Pass");
 *   - tunnel candidate by backtracing against the diffusion gradient
 *     (Introduction; Section "Tunnel loop pass", first paragraph);
 *   - Reeb graph nodes at front events with the node at the mean of the
 *     involved band (Section "Reeb Graph Extraction").
 *
 * Readings of points the paper leaves open (uniform graph Laplacian,
 * unsquared gradient coefficient, antisymmetric contact coefficient, n = 2,
 * clip, dt = 50/dmax, seed hop ball of radius 2, tau = 0.5, monotone inside
 * set grown by closure rounds, canonical rank order, lower-link event
 * classification, handle count h = (k-1-(m-s))/2) are implemented exactly as
 * listed in the design notes of the repository.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * Floating point: every expression is evaluated left to right as written, no
 * contraction, IEEE sqrt; the neighbour sum runs over ascending neighbour ids.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID_ARG (-1)
#define ORC_E_NOT_MANIFOLD (-2)
#define ORC_E_HAS_BOUNDARY (-3)
#define ORC_E_NOT_CONNECTED (-4)
#define ORC_E_NOT_ORIENTABLE (-5)
#define ORC_E_SEED_INVALID (-6)
#define ORC_E_STALLED (-7)
#define ORC_E_OUT_OF_MEMORY (-8)
#define ORC_E_INVARIANT (-13)

#define T_OUT INT64_MAX

enum { NODE_SEED = 0, NODE_SPLIT = 1, NODE_MERGE = 2, NODE_VANISH = 3, NODE_DEGENERATE = 4 };

typedef struct {
    double tau, mu, a, w, e;
    int32_t dt_mode;      /* 0: dt = 50/dmax, 1: dt = 0.25/dmax            */
    int32_t seed_radius;  /* hop radius of the initial region              */
    int64_t seed_vertex;
    int64_t max_steps;
    int64_t stall_steps;
    int32_t dense;        /* 1: update every vertex every step             */
    int32_t n_ckpt;
    const int64_t *ckpt_steps;
    int32_t fem;          /* 1: cotangent finite-element operator           */
    int64_t n_seed_set;   /* > 0: the initial region grows from this set    */
    const int32_t *seed_set;
} orc_params;

/* growable arrays */
typedef struct { int64_t *p; int64_t n, cap; } vec64;
typedef struct { double *p; int64_t n, cap; } vecd;

static int v64_push(vec64 *v, int64_t x) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 64;
        int64_t *np = (int64_t *)realloc(v->p, (size_t)nc * sizeof(int64_t));
        if (!np) return -1;
        v->p = np; v->cap = nc;
    }
    v->p[v->n++] = x;
    return 0;
}
static int vd_push(vecd *v, double x) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 64;
        double *np = (double *)realloc(v->p, (size_t)nc * sizeof(double));
        if (!np) return -1;
        v->p = np; v->cap = nc;
    }
    v->p[v->n++] = x;
    return 0;
}

typedef struct {
    int32_t status;
    int64_t nv, nf, nnz;
    int32_t dmax;
    int64_t chi_mesh;
    /* mesh */
    const double *xyz;
    int64_t *rp;      /* [nv+1] */
    int32_t *adj;     /* [nnz] neighbours ascending by id                   */
    int32_t *cyc;     /* [nnz] neighbours in counter-clockwise link order   */
    int32_t *src;     /* [nnz] owner vertex of each half-edge (cyc layout)  */
    /* state */
    double *rho;
    int64_t *T;       /* insertion step, T_OUT if outside                   */
    int32_t *rnd;     /* closure round (hop for the seed ball)              */
    int32_t *parent;
    int32_t *depth;
    int64_t *lid;     /* [nnz] front id of crossed half-edge u->x (cyc idx)  */
    int64_t *hstamp;  /* [nnz] walk marks                                   */
    int64_t stampc;
    /* results */
    int64_t steps, n_inside, next_front;
    int64_t chi, b;
    int64_t active_updates;
    vec64 steplog;    /* per step: chi_t, b_t, |N_t|                        */
    vec64 ev;         /* per event: 14 fields, see orc_events              */
    vec64 ev_ids;     /* concatenated in-ids then out-ids per event         */
    vecd ev_pos;      /* per event 3 doubles: Reeb node position            */
    vec64 fr_birth, fr_death;
    /* loops: the involved pre-event loops of every event with s >= 2       */
    vec64 lp;         /* per loop: 6 fields: event, front id, kept(handle), offset, count, a-vertex */
    vecd lp_len;
    vec64 lp_he;      /* concatenated (u, x) pairs                          */
    vecd lp_pts;      /* concatenated points xyz                            */
    /* tunnels: per handle loop: offset, count into tn_v                    */
    vec64 tn, tn_v;
    /* checkpoints */
    int32_t n_ckpt;
    int64_t *ckpt_steps;
    double *ckpt;     /* [n_ckpt][nv]                                       */
    int32_t *ckpt_done;
    int64_t gsum_h;   /* handle loops emitted                               */
    int64_t gsum_x;   /* extra cycles of degenerate events                  */
    /* finite-element operator (fem runs only)                              */
    double *fem_g;    /* [nnz] coefficient of half-edge v->adj[i]           */
    double *fem_mass; /* [nv] lumped mass                                   */
    double fem_sigma, fem_dmax;
} orc;

/* ------------------------------------------------------------------------ */
/* mesh: validation, ascending adjacency, counter-clockwise links            */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int build_mesh(orc *o, int64_t nv, const double *xyz, int64_t nf, const int32_t *tri) {
    o->nv = nv; o->nf = nf; o->xyz = xyz;
    if (nv < 4 || nf < 4 || !xyz || !tri) return ORC_E_INVALID_ARG;
    for (int64_t f = 0; f < 3 * nf; ++f)
        if (tri[f] < 0 || tri[f] >= nv) return ORC_E_INVALID_ARG;
    for (int64_t f = 0; f < nf; ++f) {
        int32_t a = tri[3 * f], b = tri[3 * f + 1], c = tri[3 * f + 2];
        if (a == b || b == c || a == c) return ORC_E_NOT_MANIFOLD;
    }
    /* every directed edge once, and its twin present */
    int64_t nd = 3 * nf;
    int64_t *dk = (int64_t *)malloc((size_t)nd * sizeof(int64_t));
    if (!dk) return ORC_E_OUT_OF_MEMORY;
    for (int64_t f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            int64_t u = tri[3 * f + k], x = tri[3 * f + (k + 1) % 3];
            dk[3 * f + k] = u * nv + x;
        }
    qsort(dk, (size_t)nd, sizeof(int64_t), cmp_i64);
    for (int64_t i = 1; i < nd; ++i)
        if (dk[i] == dk[i - 1]) { free(dk); return ORC_E_NOT_ORIENTABLE; }
    for (int64_t i = 0; i < nd; ++i) {
        int64_t u = dk[i] / nv, x = dk[i] % nv, key = x * nv + u;
        if (!bsearch(&key, dk, (size_t)nd, sizeof(int64_t), cmp_i64)) { free(dk); return ORC_E_HAS_BOUNDARY; }
    }
    free(dk);
    /* link pairs per vertex: triangle (v,a,b) gives link edge a->b */
    int64_t *cnt = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    if (!cnt) return ORC_E_OUT_OF_MEMORY;
    for (int64_t f = 0; f < 3 * nf; ++f) cnt[tri[f] + 1]++;
    for (int64_t v = 0; v < nv; ++v) {
        if (cnt[v + 1] == 0) { free(cnt); return ORC_E_NOT_CONNECTED; }
        cnt[v + 1] += cnt[v];
    }
    int64_t nnz = cnt[nv];
    o->nnz = nnz;
    o->rp = (int64_t *)malloc((size_t)(nv + 1) * sizeof(int64_t));
    int32_t *la = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    int32_t *lb = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    o->adj = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    o->cyc = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    o->src = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    if (!o->rp || !la || !lb || !fill || !o->adj || !o->cyc || !o->src) {
        free(cnt); free(la); free(lb); free(fill); return ORC_E_OUT_OF_MEMORY;
    }
    memcpy(o->rp, cnt, (size_t)(nv + 1) * sizeof(int64_t));
    free(cnt);
    for (int64_t v = 0; v < nv; ++v) fill[v] = o->rp[v];
    for (int64_t f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            int32_t v = tri[3 * f + k], a = tri[3 * f + (k + 1) % 3], b = tri[3 * f + (k + 2) % 3];
            la[fill[v]] = a; lb[fill[v]] = b; fill[v]++;
        }
    free(fill);
    int32_t dmax = 0;
    for (int64_t v = 0; v < nv; ++v) {
        int64_t b0 = o->rp[v], d = o->rp[v + 1] - b0;
        if (d < 3) { free(la); free(lb); return ORC_E_NOT_MANIFOLD; }
        if (d > dmax) dmax = (int32_t)d;
        /* start at the smallest neighbour id, follow a -> b */
        int32_t start = la[b0];
        for (int64_t i = 1; i < d; ++i) if (la[b0 + i] < start) start = la[b0 + i];
        int32_t cur = start;
        for (int64_t i = 0; i < d; ++i) {
            o->cyc[b0 + i] = cur;
            o->src[b0 + i] = (int32_t)v;
            int64_t hit = -1;
            for (int64_t j = 0; j < d; ++j) if (la[b0 + j] == cur) { if (hit >= 0) { free(la); free(lb); return ORC_E_NOT_MANIFOLD; } hit = j; }
            if (hit < 0) { free(la); free(lb); return ORC_E_NOT_MANIFOLD; }
            cur = lb[b0 + hit];
        }
        if (cur != start) { free(la); free(lb); return ORC_E_NOT_MANIFOLD; }
        /* the cycle must visit d distinct neighbours */
        memcpy(o->adj + b0, o->cyc + b0, (size_t)d * sizeof(int32_t));
        qsort(o->adj + b0, (size_t)d, sizeof(int32_t), cmp_i32);
        for (int64_t i = 1; i < d; ++i)
            if (o->adj[b0 + i] == o->adj[b0 + i - 1]) { free(la); free(lb); return ORC_E_NOT_MANIFOLD; }
    }
    free(la); free(lb);
    o->dmax = dmax;
    /* connected */
    int32_t *q = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
    char *seen = (char *)calloc((size_t)nv, 1);
    if (!q || !seen) { free(q); free(seen); return ORC_E_OUT_OF_MEMORY; }
    int64_t qh = 0, qt = 0;
    q[qt++] = 0; seen[0] = 1;
    while (qh < qt) {
        int32_t v = q[qh++];
        for (int64_t i = o->rp[v]; i < o->rp[v + 1]; ++i)
            if (!seen[o->adj[i]]) { seen[o->adj[i]] = 1; q[qt++] = o->adj[i]; }
    }
    free(q); free(seen);
    if (qt != nv) return ORC_E_NOT_CONNECTED;
    o->chi_mesh = nv - nnz / 2 + nf;
    return ORC_OK;
}

/* index of half-edge u->x in the counter-clockwise layout, -1 if none */
static int64_t he_find(const orc *o, int64_t u, int64_t x) {
    for (int64_t i = o->rp[u]; i < o->rp[u + 1]; ++i)
        if (o->cyc[i] == x) return i;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* field step (evolution equation, two-phase form, explicit Euler, clip)     */
/* ------------------------------------------------------------------------ */
static double field_value(const orc *o, const double *rho, int64_t v, double c,
                          double a, double w, double e) {
    int64_t b0 = o->rp[v], b1 = o->rp[v + 1];
    double s = rho[o->adj[b0]];
    for (int64_t i = b0 + 1; i < b1; ++i) s = s + rho[o->adj[i]];
    double r = rho[v];
    double lap;
    if (o->fem_g) {
        lap = o->fem_g[b0] * (rho[o->adj[b0]] - r);
        for (int64_t i = b0 + 1; i < b1; ++i) lap = lap + o->fem_g[i] * (rho[o->adj[i]] - r);
    } else {
        lap = s - (double)(b1 - b0) * r;
    }
    double d = (a * lap + w * (2.0 * r - 1.0)) + e * sqrt(r * (1.0 - r));
    double x = r + c * d;
    if (x < 0.0) x = 0.0;
    if (x > 1.0) x = 1.0;
    return x;
}

/* ------------------------------------------------------------------------ */
/* cotangent finite-element operator (Section "Mathematical representation   */
/* and data structure", "Implementation details": the Laplacian of linear    */
/* finite elements on the surface mesh)                                      */
/* ------------------------------------------------------------------------ */
/* For a vertex v with counter-clockwise link c_0..c_{d-1}:
     mass m_v  = (sum_k area(v, c_k, c_{k+1})) / 3         (lumped P1 mass)
     k_vu      = (cot of the angle opposite vu in (v,u,a) +
                  cot of the angle opposite vu in (v,b,u)) / 2
                 with a, b the link successor and predecessor of u
     (L rho)(v) = sigma / m_v * sum_u k_vu (rho_u - rho_v)
   sigma = sqrt(3) times the mean lumped mass: on a mesh of equilateral
   triangles with one valence every coefficient sigma k_vu / m_v is 1, so
   the operator is the uniform graph Laplacian there and the coefficients
   a, w, e and the step rule keep their meaning.  The explicit step uses the
   largest absolute row sum in place of the maximum degree. */
static double tri_area(const double *x, int64_t v, int64_t p, int64_t q) {
    const double e0 = x[3 * p] - x[3 * v], e1 = x[3 * p + 1] - x[3 * v + 1], e2 = x[3 * p + 2] - x[3 * v + 2];
    const double f0 = x[3 * q] - x[3 * v], f1 = x[3 * q + 1] - x[3 * v + 1], f2 = x[3 * q + 2] - x[3 * v + 2];
    const double c0 = e1 * f2 - e2 * f1, c1 = e2 * f0 - e0 * f2, c2 = e0 * f1 - e1 * f0;
    return 0.5 * sqrt((c0 * c0 + c1 * c1) + c2 * c2);
}

/* cotangent of the angle at apex between the edges to v and to u */
static double cot_at(const double *x, int64_t apex, int64_t v, int64_t u) {
    const double p0 = x[3 * v] - x[3 * apex], p1 = x[3 * v + 1] - x[3 * apex + 1], p2 = x[3 * v + 2] - x[3 * apex + 2];
    const double q0 = x[3 * u] - x[3 * apex], q1 = x[3 * u + 1] - x[3 * apex + 1], q2 = x[3 * u + 2] - x[3 * apex + 2];
    const double dot = (p0 * q0 + p1 * q1) + p2 * q2;
    const double c0 = p1 * q2 - p2 * q1, c1 = p2 * q0 - p0 * q2, c2 = p0 * q1 - p1 * q0;
    return dot / sqrt((c0 * c0 + c1 * c1) + c2 * c2);
}

static int fem_operator(orc *o) {
    const int64_t nv = o->nv;
    const double *x = o->xyz;
    o->fem_g = (double *)malloc((size_t)o->nnz * sizeof(double));
    o->fem_mass = (double *)malloc((size_t)nv * sizeof(double));
    if (!o->fem_g || !o->fem_mass) return ORC_E_OUT_OF_MEMORY;
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t b0 = o->rp[v], d = o->rp[v + 1] - b0;
        double S = 0.0;
        for (int64_t k = 0; k < d; ++k) S = S + tri_area(x, v, o->cyc[b0 + k], o->cyc[b0 + (k + 1) % d]);
        o->fem_mass[v] = S / 3.0;
    }
    double T = 0.0;
    for (int64_t v = 0; v < nv; ++v) T = T + o->fem_mass[v];
    o->fem_sigma = (sqrt(3.0) * T) / (double)nv;
    o->fem_dmax = 0.0;
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t b0 = o->rp[v], d = o->rp[v + 1] - b0;
        double D = 0.0;
        for (int64_t i = b0; i < b0 + d; ++i) {
            const int64_t u = o->adj[i];
            int64_t k = 0;
            while (o->cyc[b0 + k] != u) ++k;
            const int64_t a = o->cyc[b0 + (k + 1) % d], b = o->cyc[b0 + (k + d - 1) % d];
            const double kvu = 0.5 * (cot_at(x, a, v, u) + cot_at(x, b, v, u));
            o->fem_g[i] = (o->fem_sigma * kvu) / o->fem_mass[v];
            D = D + fabs(o->fem_g[i]);
        }
        if (D > o->fem_dmax) o->fem_dmax = D;
    }
    return ORC_OK;
}

/* a vertex whose value is 0 or 1 and whose neighbours all share it is a
   fixed point of the step (its Laplacian is 0 and the clip restores it) */
static int quiescent(const orc *o, const double *rho, int64_t v) {
    double r = rho[v];
    if (!(r == 0.0 || r == 1.0)) return 0;
    for (int64_t i = o->rp[v]; i < o->rp[v + 1]; ++i)
        if (rho[o->adj[i]] != r) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* rank order and the inside predicate                                       */
/* ------------------------------------------------------------------------ */
static int lower(const orc *o, int64_t u, int64_t v) {
    if (o->T[u] != o->T[v]) return o->T[u] < o->T[v];
    if (o->rnd[u] != o->rnd[v]) return o->rnd[u] < o->rnd[v];
    return u < v;
}

/* inside test during a walk: mode 0 = state before inserting cur,
   mode 1 = state after inserting cur, mode 2 = plain T[] <= tcut */
typedef struct { int64_t cur; int mode; int64_t tcut; } inside_ctx;
static int is_in(const orc *o, const inside_ctx *c, int64_t y) {
    if (c->mode == 2) return o->T[y] <= c->tcut;
    if (y == c->cur) return c->mode == 1;
    if (o->T[y] == T_OUT) return 0;
    return lower(o, y, c->cur);
}

/* successor of crossed half-edge e=(u->x) along its loop: the triangle
   (u, x, y) containing directed edge u->x has exactly one other crossed
   edge: (y,x) if y is inside, else (u,y). */
static int64_t he_next(const orc *o, const inside_ctx *c, int64_t e) {
    int64_t u = o->src[e];
    int64_t j = e + 1;
    if (j == o->rp[u + 1]) j = o->rp[u];
    int64_t y = o->cyc[j];
    if (is_in(o, c, y)) return he_find(o, y, o->cyc[e]);
    return j;
}

/* walk the loop through crossed half-edge e0; returns the half-edges in
   loop order starting at the minimum key (u*nv + x); marks them with
   stamp; the vec is overwritten */
static int walk_loop(orc *o, const inside_ctx *c, int64_t e0, int64_t stamp, vec64 *out) {
    out->n = 0;
    int64_t e = e0, guard = 0, best = -1, bestkey = INT64_MAX;
    do {
        if (v64_push(out, e)) return ORC_E_OUT_OF_MEMORY;
        o->hstamp[e] = stamp;
        int64_t key = (int64_t)o->src[e] * o->nv + o->cyc[e];
        if (key < bestkey) { bestkey = key; best = out->n - 1; }
        e = he_next(o, c, e);
        if (e < 0 || ++guard > o->nnz) return ORC_E_INVARIANT;
    } while (e != e0);
    /* rotate to start at the minimum key */
    int64_t n = out->n;
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!tmp) return ORC_E_OUT_OF_MEMORY;
    for (int64_t i = 0; i < n; ++i) tmp[i] = out->p[(best + i) % n];
    memcpy(out->p, tmp, (size_t)n * sizeof(int64_t));
    free(tmp);
    return ORC_OK;
}

static int64_t loop_minkey(const orc *o, const vec64 *l) {
    return (int64_t)o->src[l->p[0]] * o->nv + o->cyc[l->p[0]];
}

/* crossing point on crossed edge (u inside, x outside) at the threshold */
static void crossing_point(const orc *o, int64_t u, int64_t x, double tau, double *p) {
    double ru = o->rho[u], rx = o->rho[x];
    double den = ru - rx;
    double t;
    if (den <= 0.0) t = 0.5;
    else {
        t = (ru - tau) / den;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    const double *pu = o->xyz + 3 * u, *px = o->xyz + 3 * x;
    p[0] = pu[0] + t * (px[0] - pu[0]);
    p[1] = pu[1] + t * (px[1] - pu[1]);
    p[2] = pu[2] + t * (px[2] - pu[2]);
}

static double polyline_length(const double *pts, int64_t n) {
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *p = pts + 3 * i, *q = pts + 3 * ((i + 1) % n);
        double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
        L = L + sqrt((dx * dx + dy * dy) + dz * dz);
    }
    return L;
}

/* Reeb node position: mean of the distinct vertices of the front triangles
   of the given loops, summed in ascending vertex id */
static int band_mean(orc *o, vec64 *loops, int nloops, double *pos) {
    int64_t tot = 0;
    for (int i = 0; i < nloops; ++i) tot += loops[i].n;
    int64_t *ids = (int64_t *)malloc((size_t)(3 * tot + 1) * sizeof(int64_t));
    if (!ids) return ORC_E_OUT_OF_MEMORY;
    int64_t n = 0;
    for (int i = 0; i < nloops; ++i)
        for (int64_t k = 0; k < loops[i].n; ++k) {
            int64_t e = loops[i].p[k], u = o->src[e];
            int64_t j = e + 1;
            if (j == o->rp[u + 1]) j = o->rp[u];
            ids[n++] = u; ids[n++] = o->cyc[e]; ids[n++] = o->cyc[j];
        }
    qsort(ids, (size_t)n, sizeof(int64_t), cmp_i64);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0 && ids[i] == ids[i - 1]) continue;
        sx = sx + o->xyz[3 * ids[i]];
        sy = sy + o->xyz[3 * ids[i] + 1];
        sz = sz + o->xyz[3 * ids[i] + 2];
        cnt++;
    }
    free(ids);
    pos[0] = sx / (double)cnt; pos[1] = sy / (double)cnt; pos[2] = sz / (double)cnt;
    return ORC_OK;
}

/* record one involved pre-event loop (handle candidate) */
static int record_loop(orc *o, int64_t event, int64_t fid, int kept, int64_t avert,
                       const vec64 *l, double tau, double *len_out) {
    int64_t off = o->lp_he.n / 2;
    double *pts = (double *)malloc((size_t)(3 * l->n) * sizeof(double));
    if (!pts) return ORC_E_OUT_OF_MEMORY;
    for (int64_t k = 0; k < l->n; ++k) {
        int64_t e = l->p[k], u = o->src[e], x = o->cyc[e];
        crossing_point(o, u, x, tau, pts + 3 * k);
        if (v64_push(&o->lp_he, u) || v64_push(&o->lp_he, x)) { free(pts); return ORC_E_OUT_OF_MEMORY; }
        for (int q = 0; q < 3; ++q) if (vd_push(&o->lp_pts, pts[3 * k + q])) { free(pts); return ORC_E_OUT_OF_MEMORY; }
    }
    double L = polyline_length(pts, l->n);
    free(pts);
    if (v64_push(&o->lp, event) || v64_push(&o->lp, fid) || v64_push(&o->lp, kept) ||
        v64_push(&o->lp, off) || v64_push(&o->lp, l->n) || v64_push(&o->lp, avert) ||
        vd_push(&o->lp_len, L)) return ORC_E_OUT_OF_MEMORY;
    *len_out = L;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* event resolution for a saddle or vanish insertion of v                     */
/* (Section "Initial Pass": branching and collision of advancing fronts)     */
/* ------------------------------------------------------------------------ */
static int resolve_event(orc *o, int64_t v, int64_t t, int full, int64_t k,
                         const char *lowflag, double tau) {
    int64_t b0 = o->rp[v], d = o->rp[v + 1] - b0;
    int rc;
    /* distinct front ids on the lower segments; a-vertex per id */
    int64_t *sid = (int64_t *)malloc((size_t)d * sizeof(int64_t));
    int64_t *sa = (int64_t *)malloc((size_t)d * sizeof(int64_t));
    int64_t *se = (int64_t *)malloc((size_t)d * sizeof(int64_t));
    if (!sid || !sa || !se) { free(sid); free(sa); free(se); return ORC_E_OUT_OF_MEMORY; }
    int64_t s = 0;
    for (int64_t i = 0; i < d; ++i) {
        if (!lowflag[i]) continue;
        int64_t u = o->cyc[b0 + i];
        int64_t eu = he_find(o, u, v);
        int64_t id = o->lid[eu];
        int64_t j;
        for (j = 0; j < s; ++j) if (sid[j] == id) break;
        if (j == s) { sid[s] = id; sa[s] = u; se[s] = eu; s++; }
        else if (lower(o, u, sa[j])) { sa[j] = u; }
    }
    /* sort ids ascending (insertion sort; s is tiny) */
    for (int64_t i = 1; i < s; ++i)
        for (int64_t j = i; j > 0 && sid[j] < sid[j - 1]; --j) {
            int64_t t1 = sid[j]; sid[j] = sid[j - 1]; sid[j - 1] = t1;
            t1 = sa[j]; sa[j] = sa[j - 1]; sa[j - 1] = t1;
            t1 = se[j]; se[j] = se[j - 1]; se[j - 1] = t1;
        }
    /* the pre-event loops */
    vec64 *pre = (vec64 *)calloc((size_t)s, sizeof(vec64));
    if (!pre) { free(sid); free(sa); free(se); return ORC_E_OUT_OF_MEMORY; }
    inside_ctx cpre = { v, 0, 0 };
    for (int64_t j = 0; j < s; ++j) {
        rc = walk_loop(o, &cpre, se[j], ++o->stampc, &pre[j]);
        if (rc) goto fail;
    }
    /* the post-event loops through v's new crossed half-edges */
    inside_ctx cpost = { v, 1, 0 };
    int64_t m = 0, mcap = d;
    vec64 *post = (vec64 *)calloc((size_t)mcap, sizeof(vec64));
    if (!post) { rc = ORC_E_OUT_OF_MEMORY; goto fail; }
    int64_t pstamp = ++o->stampc;
    for (int64_t i = 0; i < d; ++i) {
        if (lowflag[i]) continue;
        int64_t e = b0 + i;
        if (o->hstamp[e] == pstamp) continue;
        rc = walk_loop(o, &cpost, e, pstamp, &post[m]);
        if (rc) { for (int64_t q = 0; q <= m; ++q) free(post[q].p); free(post); goto fail; }
        m++;
    }
    /* the new loops were found in counter-clockwise order of their first
       new half-edge around v (v's link starts at its smallest neighbour id);
       fresh front ids follow that order */
    /* Euler bookkeeping: dchi = 1-k (saddle) or +1 (vanish); db = m-s */
    int64_t h = 0, x = 0;
    if (full) {
        if (m != 0 || s != 1) { rc = ORC_E_INVARIANT; goto failpost; }
    } else {
        int64_t num = k - 1 - (m - s);
        if (num < 0 || (num & 1)) { rc = ORC_E_INVARIANT; goto failpost; }
        h = num / 2;
        x = h - (s - 1);
        if (x < 0) { rc = ORC_E_INVARIANT; goto failpost; }
    }
    int64_t type;
    if (full) type = NODE_VANISH;
    else if (x > 0) type = NODE_DEGENERATE;
    else if (s >= 2) type = NODE_MERGE;
    else type = NODE_SPLIT;
    int64_t event = o->ev.n / 14;
    int64_t node = event + 1;              /* node 0 is the seed            */
    /* handle loops: drop the longest involved loop (ties: larger id)      */
    double *len = (double *)malloc((size_t)s * sizeof(double));
    if (!len) { rc = ORC_E_OUT_OF_MEMORY; goto failpost; }
    int64_t drop = -1;
    int64_t first_loop = o->lp.n / 6;
    if (s >= 2) {
        for (int64_t j = 0; j < s; ++j) {
            rc = record_loop(o, event, sid[j], 0, sa[j], &pre[j], tau, &len[j]);
            if (rc) { free(len); goto failpost; }
        }
        drop = 0;
        for (int64_t j = 1; j < s; ++j)
            if (len[j] >= len[drop]) drop = j;   /* ascending ids: ties -> larger id */
        for (int64_t j = 0; j < s; ++j) {
            if (j == drop) continue;
            o->lp.p[6 * (first_loop + j) + 2] = 1;   /* kept = handle loop */
            o->gsum_h += 1;
            /* tunnel candidate: a_j -> ... -> LCA <- ... <- a_drop, closed via v */
            int64_t aj = sa[j], a0 = sa[drop];
            int64_t off = o->tn_v.n;
            if (v64_push(&o->tn_v, v)) { free(len); rc = ORC_E_OUT_OF_MEMORY; goto failpost; }
            int64_t p1 = aj, p2 = a0;
            vec64 down = {0};
            while (o->depth[p1] > o->depth[p2]) { v64_push(&o->tn_v, p1); p1 = o->parent[p1]; }
            while (o->depth[p2] > o->depth[p1]) { v64_push(&down, p2); p2 = o->parent[p2]; }
            while (p1 != p2) {
                v64_push(&o->tn_v, p1); p1 = o->parent[p1];
                v64_push(&down, p2); p2 = o->parent[p2];
            }
            v64_push(&o->tn_v, p1);                    /* the common ancestor */
            for (int64_t q = down.n - 1; q >= 0; --q) v64_push(&o->tn_v, down.p[q]);
            free(down.p);
            v64_push(&o->tn, first_loop + j);           /* loop index          */
            v64_push(&o->tn, off);
            v64_push(&o->tn, o->tn_v.n - off);
        }
    }
    free(len);
    /* Reeb node position: mean of the involved band */
    double pos[3];
    if ((rc = band_mean(o, pre, (int)s, pos))) goto failpost;
    /* front ids */
    for (int64_t j = 0; j < s; ++j) {
        if (v64_push(&o->ev_ids, sid[j])) { rc = ORC_E_OUT_OF_MEMORY; goto failpost; }
        o->fr_death.p[sid[j]] = node;
    }
    for (int64_t i = 0; i < m; ++i) {
        int64_t nid = o->next_front++;
        if (v64_push(&o->fr_birth, node) || v64_push(&o->fr_death, -1) ||
            v64_push(&o->ev_ids, nid)) { rc = ORC_E_OUT_OF_MEMORY; goto failpost; }
        for (int64_t q = 0; q < post[i].n; ++q) o->lid[post[i].p[q]] = nid;
    }
    int64_t rec[14] = { t, v, type, full ? 0 : k, s, m, h, x, node,
                        o->rnd[v], full ? 1 : 0, 0, 0, 0 };
    for (int q = 0; q < 14; ++q) v64_push(&o->ev, rec[q]);
    vd_push(&o->ev_pos, pos[0]); vd_push(&o->ev_pos, pos[1]); vd_push(&o->ev_pos, pos[2]);
    o->chi += full ? 1 : 1 - k;
    o->b += m - s;
    o->gsum_x += x;
    rc = ORC_OK;
failpost:
    for (int64_t q = 0; q < mcap; ++q) free(post[q].p);
    free(post);
fail:
    for (int64_t j = 0; j < s; ++j) free(pre[j].p);
    free(pre); free(sid); free(sa); free(se);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* insertion of one vertex in rank order: lower-link classification         */
/* ------------------------------------------------------------------------ */
static int insert_vertex(orc *o, int64_t v, int64_t t, double tau) {
    int64_t b0 = o->rp[v], d = o->rp[v + 1] - b0;
    char lowflag[4096];
    char *lf = d <= 4096 ? lowflag : (char *)malloc((size_t)d);
    if (!lf) return ORC_E_OUT_OF_MEMORY;
    int64_t nlow = 0;
    int64_t par = -1;
    for (int64_t i = 0; i < d; ++i) {
        int64_t u = o->cyc[b0 + i];
        lf[i] = (char)(o->T[u] != T_OUT && lower(o, u, v));
        if (lf[i]) {
            nlow++;
            if (par < 0 || lower(o, u, par)) par = u;
        }
    }
    int rc = ORC_OK;
    if (nlow == 0) { rc = ORC_E_INVARIANT; goto done; }
    o->parent[v] = (int32_t)par;
    o->depth[v] = o->depth[par] + 1;
    int full = nlow == d;
    int64_t k = 0;
    if (!full)
        for (int64_t i = 0; i < d; ++i)
            if (lf[i] && !lf[(i + d - 1) % d]) k++;
    if (!full && k == 1) {
        /* regular: the single segment keeps its front id */
        int64_t id = -1;
        for (int64_t i = 0; i < d; ++i)
            if (lf[i]) {
                int64_t e = he_find(o, o->cyc[b0 + i], v);
                if (id < 0) id = o->lid[e];
                else if (o->lid[e] != id) { rc = ORC_E_INVARIANT; goto done; }
            }
        for (int64_t i = 0; i < d; ++i)
            if (!lf[i]) o->lid[b0 + i] = id;
    } else {
        rc = resolve_event(o, v, t, full, k, lf, tau);
    }
    o->n_inside++;
done:
    if (lf != lowflag) free(lf);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* seed: hop ball of radius r0 around the seed vertex; or, from a seed set   */
/* S (the Reeb refinement's second pass starts at a handle loop), the        */
/* vertices within r0 hops of S, ranked by their hop distance inside that    */
/* region from s = min S.  S = {s} gives the ball.                           */
/* ------------------------------------------------------------------------ */
static int seed_init(orc *o, int64_t s, int32_t r0, const int32_t *set, int64_t nset) {
    int64_t nv = o->nv;
    int32_t *hop = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
    int32_t *q = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
    if (!hop || !q) { free(hop); free(q); return ORC_E_OUT_OF_MEMORY; }
    for (int64_t v = 0; v < nv; ++v) hop[v] = -1;
    int64_t qh = 0, qt = 0;
    if (nset > 0) {
        for (int64_t i = 0; i < nset; ++i)
            if (hop[set[i]] < 0) { hop[set[i]] = 0; q[qt++] = set[i]; }
    } else {
        q[qt++] = (int32_t)s; hop[s] = 0;
    }
    while (qh < qt) {
        int32_t v = q[qh++];
        if (hop[v] >= r0) continue;
        for (int64_t i = o->rp[v]; i < o->rp[v + 1]; ++i) {
            int32_t u = o->adj[i];
            if (hop[u] < 0) { hop[u] = hop[v] + 1; q[qt++] = u; }
        }
    }
    if (nset > 0) {
        /* re-rank the region by hop distance from s inside it: q becomes
           that breadth-first order, hop that distance */
        int32_t *d = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
        if (!d) { free(hop); free(q); return ORC_E_OUT_OF_MEMORY; }
        for (int64_t v = 0; v < nv; ++v) d[v] = hop[v] >= 0 ? -1 : -2;
        int64_t n_region = qt;
        qh = 0; qt = 0;
        q[qt++] = (int32_t)s; d[s] = 0;
        while (qh < qt) {
            int32_t v = q[qh++];
            for (int64_t i = o->rp[v]; i < o->rp[v + 1]; ++i) {
                int32_t u = o->adj[i];
                if (d[u] == -1) { d[u] = d[v] + 1; q[qt++] = u; }
            }
        }
        for (int64_t v = 0; v < nv; ++v) hop[v] = d[v];
        free(d);
        if (qt != n_region) { free(hop); free(q); return ORC_E_SEED_INVALID; }
    }
    for (int64_t i = 0; i < qt; ++i) {
        int32_t v = q[i];
        o->T[v] = 0; o->rnd[v] = hop[v]; o->rho[v] = 1.0;
    }
    o->n_inside = qt;
    /* parent = minimum-rank lower neighbour, in rank order */
    for (int64_t i = 0; i < qt; ++i) {
        int32_t v = q[i];
        if (v == s) { o->parent[v] = -1; o->depth[v] = 0; continue; }
        int64_t par = -1;
        for (int64_t j = o->rp[v]; j < o->rp[v + 1]; ++j) {
            int64_t u = o->adj[j];
            if (o->T[u] == 0 && lower(o, u, v) && (par < 0 || lower(o, u, par))) par = u;
        }
        o->parent[v] = (int32_t)par;
    }
    /* BFS order is non-decreasing in hop, so depth can be filled in order */
    for (int64_t i = 0; i < qt; ++i) {
        int32_t v = q[i];
        if (v != s) o->depth[v] = o->depth[o->parent[v]] + 1;
    }
    /* Euler characteristic of the full subcomplex on the ball */
    int64_t ne = 0, nfb = 0;
    for (int64_t i = 0; i < qt; ++i) {
        int32_t v = q[i];
        for (int64_t j = o->rp[v]; j < o->rp[v + 1]; ++j) {
            int32_t u = o->cyc[j];
            int64_t jn = j + 1 == o->rp[v + 1] ? o->rp[v] : j + 1;
            int32_t y = o->cyc[jn];
            if (o->T[u] == 0 && u > v) ne++;
            if (o->T[u] == 0 && o->T[y] == 0 && v < u && v < y) nfb++;
        }
    }
    o->chi = qt - ne + nfb;
    /* initial loops */
    inside_ctx c0 = { -1, 2, 0 };
    int64_t cap = 8, nl = 0;
    vec64 *loops = (vec64 *)calloc((size_t)cap, sizeof(vec64));
    int64_t stamp = ++o->stampc;
    int rc = ORC_OK;
    for (int64_t i = 0; i < qt && rc == ORC_OK; ++i) {
        int32_t v = q[i];
        for (int64_t j = o->rp[v]; j < o->rp[v + 1]; ++j) {
            if (o->T[o->cyc[j]] == 0 || o->hstamp[j] == stamp) continue;
            if (nl == cap) {
                vec64 *nl2 = (vec64 *)realloc(loops, (size_t)(2 * cap) * sizeof(vec64));
                if (!nl2) { rc = ORC_E_OUT_OF_MEMORY; break; }
                memset(nl2 + cap, 0, (size_t)cap * sizeof(vec64));
                loops = nl2; cap *= 2;
            }
            rc = walk_loop(o, &c0, j, stamp, &loops[nl]);
            if (rc) break;
            nl++;
        }
    }
    if (rc == ORC_OK) {
        for (int64_t i = 1; i < nl; ++i)
            for (int64_t j = i; j > 0 && loop_minkey(o, &loops[j]) < loop_minkey(o, &loops[j - 1]); --j) {
                vec64 t1 = loops[j]; loops[j] = loops[j - 1]; loops[j - 1] = t1;
            }
        for (int64_t i = 0; i < nl; ++i) {
            int64_t id = o->next_front++;
            v64_push(&o->fr_birth, 0); v64_push(&o->fr_death, -1);
            for (int64_t k = 0; k < loops[i].n; ++k) o->lid[loops[i].p[k]] = id;
        }
        o->b = nl;
        if (nl < 1 || 2 - o->chi - nl != 0) rc = ORC_E_SEED_INVALID;
    }
    for (int64_t i = 0; i < cap; ++i) free(loops[i].p);
    free(loops); free(hop); free(q);
    return rc;
}

/* rank order inside one step: (round, id) pairs */
static int cmp_pair(const void *a, const void *b) {
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    if (x[0] != y[0]) return (x[0] > y[0]) - (x[0] < y[0]);
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/* ------------------------------------------------------------------------ */
/* the initial pass                                                          */
/* ------------------------------------------------------------------------ */
static int run(orc *o, const orc_params *p) {
    int64_t nv = o->nv;
    const double a = p->a, w = p->w, e = p->e, tau = p->tau;
    if (p->fem) {
        int fr = fem_operator(o);
        if (fr) return fr;
    }
    const double dmx = p->fem ? o->fem_dmax : (double)o->dmax;
    double dt = p->dt_mode == 1 ? 0.25 / dmx : 50.0 / dmx;
    double c = dt * (p->mu / 2.0);
    o->rho = (double *)calloc((size_t)nv, sizeof(double));
    o->T = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    o->rnd = (int32_t *)calloc((size_t)nv, sizeof(int32_t));
    o->parent = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
    o->depth = (int32_t *)calloc((size_t)nv, sizeof(int32_t));
    o->lid = (int64_t *)malloc((size_t)o->nnz * sizeof(int64_t));
    o->hstamp = (int64_t *)calloc((size_t)o->nnz, sizeof(int64_t));
    double *tmp = (double *)malloc((size_t)nv * sizeof(double));
    int64_t *cur = (int64_t *)malloc((size_t)nv * sizeof(int64_t));   /* vertices updated this step */
    int64_t *nxt = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    int64_t *mark = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    int64_t *cand = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    int64_t *pend = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    int64_t *cmark = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    int64_t *nt = (int64_t *)malloc((size_t)2 * nv * sizeof(int64_t));
    if (!o->rho || !o->T || !o->rnd || !o->parent || !o->depth || !o->lid || !o->hstamp ||
        !tmp || !cur || !nxt || !mark || !cand || !pend || !cmark || !nt) {
        free(tmp); free(cur); free(nxt); free(mark); free(cand); free(pend); free(cmark); free(nt);
        return ORC_E_OUT_OF_MEMORY;
    }
    for (int64_t v = 0; v < nv; ++v) { o->T[v] = T_OUT; o->parent[v] = -1; mark[v] = -1; cmark[v] = -1; }
    for (int64_t i = 0; i < o->nnz; ++i) o->lid[i] = -1;
    int rc;
    if (p->seed_vertex < 0 || p->seed_vertex >= nv || p->seed_radius < 0 || p->n_seed_set < 0) {
        rc = ORC_E_INVALID_ARG; goto out;
    }
    if (p->n_seed_set > 0) {
        /* the region's root is the smallest vertex of the set */
        int64_t mn = nv;
        for (int64_t i = 0; i < p->n_seed_set; ++i) {
            if (p->seed_set[i] < 0 || p->seed_set[i] >= nv) { rc = ORC_E_INVALID_ARG; goto out; }
            if (p->seed_set[i] < mn) mn = p->seed_set[i];
        }
        rc = seed_init(o, mn, p->seed_radius, p->seed_set, p->n_seed_set);
    } else {
        rc = seed_init(o, p->seed_vertex, p->seed_radius, NULL, 0);
    }
    if (rc) goto out;
    if (o->n_inside == nv) { o->steps = 0; goto out; }
    /* initial update set: everything within one hop of a non-quiescent vertex */
    int64_t ncur = 0;
    for (int64_t v = 0; v < nv; ++v)
        if (!quiescent(o, o->rho, v)) {
            if (mark[v] != 0) { mark[v] = 0; cur[ncur++] = v; }
            for (int64_t i = o->rp[v]; i < o->rp[v + 1]; ++i) {
                int64_t u = o->adj[i];
                if (mark[u] != 0) { mark[u] = 0; cur[ncur++] = u; }
            }
        }
    int64_t npend = 0, last_insert = 0;
    for (int64_t t = 1;; ++t) {
        if (t > p->max_steps) { rc = ORC_E_STALLED; o->steps = t - 1; break; }
        /* (i) field, Jacobi: every value of step t from step t-1 */
        int64_t nupd = p->dense ? nv : ncur;
        int64_t nnext = 0;
        for (int64_t i = 0; i < nupd; ++i) {
            int64_t v = p->dense ? i : cur[i];
            tmp[i] = field_value(o, o->rho, v, c, a, w, e);
            if (!p->dense && !quiescent(o, o->rho, v)) {
                if (mark[v] != t) { mark[v] = t; nxt[nnext++] = v; }
                for (int64_t j = o->rp[v]; j < o->rp[v + 1]; ++j) {
                    int64_t u = o->adj[j];
                    if (mark[u] != t) { mark[u] = t; nxt[nnext++] = u; }
                }
            }
        }
        for (int64_t i = 0; i < nupd; ++i) o->rho[p->dense ? i : cur[i]] = tmp[i];
        o->active_updates += nupd;
        /* (ii) crossers: outside vertices above the threshold */
        int64_t ncand = 0;
        for (int64_t i = 0; i < npend; ++i) {
            int64_t v = pend[i];
            if (cmark[v] != t) { cmark[v] = t; cand[ncand++] = v; }
        }
        for (int64_t i = 0; i < nupd; ++i) {
            int64_t v = p->dense ? i : cur[i];
            if (cmark[v] != t) { cmark[v] = t; cand[ncand++] = v; }
        }
        int64_t nx = 0;
        for (int64_t i = 0; i < ncand; ++i) {
            int64_t v = cand[i];
            if (o->T[v] == T_OUT && o->rho[v] > tau) cand[nx++] = v;
        }
        /* closure rounds: round 0 touches the inside set of step t-1,
           round j touches round j-1 */
        int64_t nn = 0;
        int32_t round = 0;
        for (;;) {
            int64_t added = 0;
            for (int64_t i = 0; i < nx; ++i) {
                int64_t v = cand[i];
                if (o->T[v] != T_OUT) continue;
                int hit = 0;
                for (int64_t j = o->rp[v]; j < o->rp[v + 1] && !hit; ++j) {
                    int64_t u = o->adj[j];
                    if (round == 0) hit = o->T[u] < t;
                    else hit = o->T[u] == t && o->rnd[u] == round - 1;
                }
                if (hit) { nt[2 * (nn + added)] = round; nt[2 * (nn + added) + 1] = v; added++; }
            }
            if (!added) break;
            for (int64_t i = nn; i < nn + added; ++i) { o->T[nt[2 * i + 1]] = t; o->rnd[nt[2 * i + 1]] = round; }
            nn += added;
            round++;
        }
        npend = 0;
        for (int64_t i = 0; i < nx; ++i) if (o->T[cand[i]] == T_OUT) pend[npend++] = cand[i];
        /* (iii) insert in rank order (round, id) */
        qsort(nt, (size_t)nn, 2 * sizeof(int64_t), cmp_pair);
        for (int64_t i = 0; i < nn; ++i) {
            rc = insert_vertex(o, nt[2 * i + 1], t, tau);
            if (rc) goto out;
        }
        /* (iv) Euler identity: genus swept so far */
        /* the swept genus (2 - chi_t - b_t)/2 equals the handle loops
           counted so far plus the extra cycles of degenerate events */
        int64_t twog = 2 - o->chi - o->b;
        if (twog < 0 || (twog & 1) || twog / 2 != o->gsum_h + o->gsum_x) { rc = ORC_E_INVARIANT; goto out; }
        v64_push(&o->steplog, o->chi); v64_push(&o->steplog, o->b); v64_push(&o->steplog, nn);
        for (int32_t q = 0; q < o->n_ckpt; ++q)
            if (o->ckpt_steps[q] == t) { memcpy(o->ckpt + (size_t)q * nv, o->rho, (size_t)nv * sizeof(double)); o->ckpt_done[q] = 1; }
        if (nn) last_insert = t;
        if (o->n_inside == nv) { o->steps = t; rc = ORC_OK; break; }
        if (t - last_insert >= p->stall_steps) { o->steps = t; rc = ORC_E_STALLED; break; }
        if (!p->dense) { int64_t *sw = cur; cur = nxt; nxt = sw; ncur = nnext; }
    }
out:
    free(tmp); free(cur); free(nxt); free(mark); free(cand); free(pend); free(cmark); free(nt);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* exported interface (ctypes)                                               */
/* ------------------------------------------------------------------------ */
void orc_free(void *h);

void *orc_run(int64_t nv, const double *xyz, int64_t nf, const int32_t *tri, const orc_params *p) {
    orc *o = (orc *)calloc(1, sizeof(orc));
    if (!o) return NULL;
    o->status = build_mesh(o, nv, xyz, nf, tri);
    if (o->status) return o;
    o->n_ckpt = p->n_ckpt;
    if (p->n_ckpt > 0) {
        o->ckpt_steps = (int64_t *)malloc((size_t)p->n_ckpt * sizeof(int64_t));
        o->ckpt = (double *)calloc((size_t)p->n_ckpt * (size_t)nv, sizeof(double));
        o->ckpt_done = (int32_t *)calloc((size_t)p->n_ckpt, sizeof(int32_t));
        if (!o->ckpt_steps || !o->ckpt || !o->ckpt_done) { o->status = ORC_E_OUT_OF_MEMORY; return o; }
        memcpy(o->ckpt_steps, p->ckpt_steps, (size_t)p->n_ckpt * sizeof(int64_t));
    }
    o->status = run(o, p);
    o->xyz = NULL;   /* borrowed */
    return o;
}

int32_t orc_status(void *h) { return ((orc *)h)->status; }

/* summary: status, steps, n_events, n_handle_loops, chi_mesh, chi_final,
   b_final, n_inside, dmax, n_fronts, active_updates, nnz, n_loops, n_tunnels */
void orc_summary(void *h, int64_t *out) {
    orc *o = (orc *)h;
    out[0] = o->status; out[1] = o->steps; out[2] = o->ev.n / 14; out[3] = o->gsum_h;
    out[4] = o->chi_mesh; out[5] = o->chi; out[6] = o->b; out[7] = o->n_inside;
    out[8] = o->dmax; out[9] = o->next_front; out[10] = o->active_updates; out[11] = o->nnz;
    out[12] = o->lp.n / 6; out[13] = o->tn.n / 3;
}
const int64_t *orc_T(void *h) { return ((orc *)h)->T; }
const int32_t *orc_rnd(void *h) { return ((orc *)h)->rnd; }
const int32_t *orc_parent(void *h) { return ((orc *)h)->parent; }
const double *orc_rho(void *h) { return ((orc *)h)->rho; }
const int32_t *orc_cyc(void *h) { return ((orc *)h)->cyc; }
const int64_t *orc_rp(void *h) { return ((orc *)h)->rp; }
const double *orc_ckpt(void *h, int32_t i) { orc *o = (orc *)h; return o->ckpt_done[i] ? o->ckpt + (size_t)i * o->nv : NULL; }
const int64_t *orc_steplog(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->steplog.n / 3; return o->steplog.p; }
const int64_t *orc_events(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->ev.n / 14; return o->ev.p; }
const int64_t *orc_event_ids(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->ev_ids.n; return o->ev_ids.p; }
const double *orc_event_pos(void *h) { return ((orc *)h)->ev_pos.p; }
const int64_t *orc_front_birth(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->fr_birth.n; return o->fr_birth.p; }
const int64_t *orc_front_death(void *h) { return ((orc *)h)->fr_death.p; }
const int64_t *orc_loops(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->lp.n / 6; return o->lp.p; }
const double *orc_loop_len(void *h) { return ((orc *)h)->lp_len.p; }
const int64_t *orc_loop_he(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->lp_he.n / 2; return o->lp_he.p; }
const double *orc_loop_pts(void *h) { return ((orc *)h)->lp_pts.p; }
const int64_t *orc_tunnels(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->tn.n / 3; return o->tn.p; }
const int64_t *orc_tunnel_v(void *h, int64_t *n) { orc *o = (orc *)h; *n = o->tn_v.n; return o->tn_v.p; }

void orc_free(void *h) {
    orc *o = (orc *)h;
    if (!o) return;
    free(o->rp); free(o->adj); free(o->cyc); free(o->src);
    free(o->rho); free(o->T); free(o->rnd); free(o->parent); free(o->depth);
    free(o->lid); free(o->hstamp);
    free(o->steplog.p); free(o->ev.p); free(o->ev_ids.p); free(o->ev_pos.p);
    free(o->fr_birth.p); free(o->fr_death.p);
    free(o->lp.p); free(o->lp_len.p); free(o->lp_he.p); free(o->lp_pts.p);
    free(o->tn.p); free(o->tn_v.p);
    free(o->ckpt_steps); free(o->ckpt); free(o->ckpt_done);
    free(o->fem_g); free(o->fem_mass);
    free(o);
}

/* the finite-element operator alone: rp [nv+1] and adj [nnz] (ascending
   neighbours), coefficients g [nnz] (sigma k_vu / m_v), masses [nv],
   scal = {sigma, largest absolute row sum}; nnz = 3 nf on a closed mesh.
   Returns 0 or a mesh error. */
int32_t orc_fem_operator(int64_t nv, const double *xyz, int64_t nf, const int32_t *tri, int64_t *rp,
                         int32_t *adj, double *g, double *mass, double *scal) {
    orc *o = (orc *)calloc(1, sizeof(orc));
    if (!o) return ORC_E_OUT_OF_MEMORY;
    int32_t rc = build_mesh(o, nv, xyz, nf, tri);
    if (!rc) rc = fem_operator(o);
    if (!rc) {
        memcpy(rp, o->rp, (size_t)(nv + 1) * sizeof(int64_t));
        memcpy(adj, o->adj, (size_t)o->nnz * sizeof(int32_t));
        memcpy(g, o->fem_g, (size_t)o->nnz * sizeof(double));
        memcpy(mass, o->fem_mass, (size_t)nv * sizeof(double));
        scal[0] = o->fem_sigma;
        scal[1] = o->fem_dmax;
    }
    o->xyz = NULL;
    orc_free(o);
    return rc;
}
