/*
 * vls_passes.c -- plain, slow, sequential CPU oracle of the tunnel-loop and
 * handle-refinement passes of the variational loop-shrinking method
 * (Weinrauch et al., ACM TOG; Section "Tunnel loop pass", Section "Handle
 * refinement pass", Section "Performance Considerations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * One pass is a diffusion of a single region whose base layer is implicit
 * (one minus the region's value), on a restricted operator:
 *   - only domain vertices carry a field; the others stay 0 and are not
 *     neighbours of anything (the diffusion is restricted to an area);
 *   - the cut edges (the edges a loop crosses) are not edges of the operator
 *     (the loop is a border the diffusion cannot pass);
 *   - the start vertices (one side of the loop) begin at 1 and form the
 *     inside set of step 0, every other vertex begins at 0.
 * Each step is the field step of the initial pass (same two-phase equation,
 * coefficients, time step, clip, evaluation order) with the neighbour sum
 * over the operator's neighbours in ascending id; then the threshold and
 * closure rounds of the initial pass over the operator's edges.  Each
 * inserted vertex gets an arrival time within its step, where its value
 * crossed the threshold by linear interpolation between the fields of the
 * two steps, (t - 1) + clamp((tau - rho_{t-1}) / (rho_t - rho_{t-1}), 0, 1)
 * (0 if the value did not grow; start vertices arrive at 0).  A vertex's
 * parent is the lower operator neighbour (rank (step, round, id) below its
 * own) over which the arrival time falls fastest per unit length,
 * (arrival(v) - arrival(u)) / |x_v - x_u|, ties to the smaller rank: one
 * step of steepest descent of the arrival time, the discrete streamline
 * against the diffusion.
 * The pass ends at the first step in which a target vertex (the other side
 * of the loop) joins; the vertex reached is the target of smallest rank in
 * that step.  The streamline traced back from it is its parent chain, which
 * ends at a start vertex.
 *
 * A pass whose field no longer changes (every domain vertex a fixed point of
 * the step) and has no crosser waiting ends as stalled, as does one that
 * reaches max_steps or goes stall_steps steps without an insertion.
 *
 * Build: with vls_oracle.c, gcc -O2 -ffp-contract=off -fno-fast-math
 * Floating point: every expression is evaluated left to right as written, no
 * contraction, IEEE sqrt; the neighbour sum runs over ascending neighbour ids.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PASS_OK 0
#define PASS_E_INVALID_ARG (-1)
#define PASS_E_STALLED (-7)
#define PASS_E_OUT_OF_MEMORY (-8)
#define PASS_T_OUT INT64_MAX

typedef struct {
    double tau, mu, a, w, e;
    int32_t dt_mode;       /* 0: dt = 50/dmax, 1: dt = 0.25/dmax (dmax of the whole mesh) */
    int32_t n_ckpt;
    int64_t max_steps, stall_steps;
    const int64_t *ckpt_steps;
} orc_pass_params;

/* ascending adjacency of the mesh, as the initial pass's oracle builds it */
typedef struct {
    int64_t nv;
    int32_t dmax;
    const int64_t *rp;
    const int32_t *adj;
    const uint8_t *cutv;  /* vertices with a cut edge (only their edges are looked up) */
} pass_mesh;

static int pass_cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* is {v, u} an edge of the restricted operator? */
static int op_edge(const pass_mesh *g, const uint8_t *dom, const int64_t *cut, int64_t ncut, int64_t v, int64_t u) {
    if (!dom[u] || !dom[v]) return 0;
    if (ncut == 0 || !g->cutv[v] || !g->cutv[u]) return 1;
    int64_t lo = v < u ? v : u, hi = v < u ? u : v;
    int64_t key = lo * g->nv + hi;
    return bsearch(&key, cut, (size_t)ncut, sizeof(int64_t), pass_cmp_i64) == NULL;
}

/* field step of vertex v on the restricted operator */
static double pass_value(const pass_mesh *g, const uint8_t *dom, const int64_t *cut, int64_t ncut,
                         const double *rho, int64_t v, double c, double a, double w, double e) {
    double s = 0.0;
    int64_t deg = 0;
    for (int64_t i = g->rp[v]; i < g->rp[v + 1]; ++i) {
        int64_t u = g->adj[i];
        if (!op_edge(g, dom, cut, ncut, v, u)) continue;
        s = s + rho[u];
        deg++;
    }
    double r = rho[v];
    double lap = s - (double)deg * r;
    double d = (a * lap + w * (2.0 * r - 1.0)) + e * sqrt(r * (1.0 - r));
    double x = r + c * d;
    if (x < 0.0) x = 0.0;
    if (x > 1.0) x = 1.0;
    return x;
}

/* a fixed point of the step: value 0 or 1 and every operator neighbour equal */
static int pass_fixed(const pass_mesh *g, const uint8_t *dom, const int64_t *cut, int64_t ncut,
                      const double *rho, int64_t v) {
    double r = rho[v];
    if (!(r == 0.0 || r == 1.0)) return 0;
    for (int64_t i = g->rp[v]; i < g->rp[v + 1]; ++i) {
        int64_t u = g->adj[i];
        if (op_edge(g, dom, cut, ncut, v, u) && rho[u] != r) return 0;
    }
    return 1;
}

static int rank_lower(const int64_t *T, const int32_t *rnd, int64_t u, int64_t v) {
    if (T[u] != T[v]) return T[u] < T[v];
    if (rnd[u] != rnd[v]) return rnd[u] < rnd[v];
    return u < v;
}

static int pass_cmp_pair(const void *a, const void *b) {
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    if (x[0] != y[0]) return (x[0] > y[0]) - (x[0] < y[0]);
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/*
 * One pass.  dom, target: uint8[nv]; cut: sorted keys lo*nv+hi of the cut
 * edges; start: the start vertices (in the domain).  Outputs (caller
 * arrays of nv): T (insertion step, INT64_MAX outside), rnd, parent, rho
 * (field at the last step), ckpt ([n_ckpt][nv] fields at ckpt_steps).
 * res[0] = status, res[1] = steps, res[2] = vertex reached (-1 if none),
 * res[3] = vertex updates (domain size per step).
 */
int orc_pass_run(int64_t nv, int32_t dmax, const int64_t *rp, const int32_t *adj, const double *xyz, const uint8_t *dom,
                 const int64_t *cut, int64_t ncut, const int32_t *start, int64_t nstart, const uint8_t *target,
                 const orc_pass_params *p, int64_t *T, int32_t *rnd, int32_t *parent, double *rho, double *ta,
                 double *ckpt, int64_t *res) {
    res[0] = PASS_E_INVALID_ARG; res[1] = 0; res[2] = -1; res[3] = 0;
    for (int64_t i = 1; i < ncut; ++i)
        if (cut[i] <= cut[i - 1]) return PASS_E_INVALID_ARG;
    uint8_t *cutv = (uint8_t *)calloc((size_t)nv, 1);
    if (!cutv) { res[0] = PASS_E_OUT_OF_MEMORY; return PASS_E_OUT_OF_MEMORY; }
    for (int64_t i = 0; i < ncut; ++i) {
        int64_t lo = cut[i] / nv, hi = cut[i] % nv;
        if (lo < 0 || hi >= nv || lo >= hi) { free(cutv); return PASS_E_INVALID_ARG; }
        cutv[lo] = 1;
        cutv[hi] = 1;
    }
    pass_mesh g = {nv, dmax, rp, adj, cutv};
    for (int64_t v = 0; v < nv; ++v) { rho[v] = 0.0; T[v] = PASS_T_OUT; rnd[v] = 0; parent[v] = -1; ta[v] = 0.0; }
    if (nstart < 1) { free(cutv); return PASS_E_INVALID_ARG; }
    for (int64_t i = 0; i < nstart; ++i) {
        int64_t s = start[i];
        if (s < 0 || s >= nv || !dom[s]) { free(cutv); return PASS_E_INVALID_ARG; }
        rho[s] = 1.0;
        T[s] = 0;
    }
    const double a = p->a, w = p->w, e = p->e, tau = p->tau;
    const double dt = p->dt_mode == 1 ? 0.25 / (double)dmax : 50.0 / (double)dmax;
    const double c = dt * (p->mu / 2.0);
    double *tmp = (double *)malloc((size_t)nv * sizeof(double));
    double *prev = (double *)malloc((size_t)nv * sizeof(double));
    int64_t *nt = (int64_t *)malloc((size_t)2 * nv * sizeof(int64_t));
    int64_t *cand = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    if (!tmp || !prev || !nt || !cand) {
        free(tmp); free(prev); free(nt); free(cand); free(cutv);
        res[0] = PASS_E_OUT_OF_MEMORY;
        return PASS_E_OUT_OF_MEMORY;
    }
    int64_t last_insert = 0, nonfixed_prev = -1, npend = 0;
    int rc = PASS_OK;
    for (int64_t t = 1;; ++t) {
        if (t > p->max_steps) { rc = PASS_E_STALLED; res[1] = t - 1; break; }
        /* the field stopped changing: every domain vertex was a fixed point
           at the field of step t-2, so the fields of t-1 and later equal it */
        if (nonfixed_prev == 0 && npend == 0) { rc = PASS_E_STALLED; res[1] = t - 1; break; }
        /* field, Jacobi over the domain; count the vertices that are not
           fixed points at the field of step t-1 */
        int64_t nonfixed = 0, ndom = 0;
        for (int64_t v = 0; v < nv; ++v) {
            if (!dom[v]) continue;
            ndom++;
            if (!pass_fixed(&g, dom, cut, ncut, rho, v)) nonfixed++;
            tmp[v] = pass_value(&g, dom, cut, ncut, rho, v, c, a, w, e);
        }
        for (int64_t v = 0; v < nv; ++v) if (dom[v]) { prev[v] = rho[v]; rho[v] = tmp[v]; }
        res[3] += ndom;
        nonfixed_prev = nonfixed;
        /* crossers: outside domain vertices above the threshold */
        int64_t nx = 0;
        for (int64_t v = 0; v < nv; ++v)
            if (dom[v] && T[v] == PASS_T_OUT && rho[v] > tau) cand[nx++] = v;
        /* closure rounds over the operator's edges */
        int64_t nn = 0;
        for (int32_t round = 0;; ++round) {
            int64_t added = 0;
            for (int64_t i = 0; i < nx; ++i) {
                int64_t v = cand[i];
                if (T[v] != PASS_T_OUT) continue;
                int hit = 0;
                for (int64_t j = rp[v]; j < rp[v + 1] && !hit; ++j) {
                    int64_t u = adj[j];
                    if (!op_edge(&g, dom, cut, ncut, v, u)) continue;
                    if (round == 0) hit = T[u] < t;
                    else hit = T[u] == t && rnd[u] == round - 1;
                }
                if (hit) { nt[2 * (nn + added)] = round; nt[2 * (nn + added) + 1] = v; added++; }
            }
            if (!added) break;
            for (int64_t i = nn; i < nn + added; ++i) { T[nt[2 * i + 1]] = t; rnd[nt[2 * i + 1]] = round; }
            nn += added;
        }
        npend = nx - nn;
        /* arrival times, parents, and the first target in rank order */
        qsort(nt, (size_t)nn, 2 * sizeof(int64_t), pass_cmp_pair);
        for (int64_t i = 0; i < nn; ++i) {
            int64_t v = nt[2 * i + 1];
            double d = rho[v] - prev[v];
            double f = d > 0.0 ? (tau - prev[v]) / d : 0.0;
            if (f < 0.0) f = 0.0;
            if (f > 1.0) f = 1.0;
            ta[v] = (double)(t - 1) + f;
        }
        int64_t reached = -1;
        for (int64_t i = 0; i < nn; ++i) {
            int64_t v = nt[2 * i + 1], best = -1;
            double best_slope = 0.0;
            for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
                int64_t u = adj[j];
                if (!op_edge(&g, dom, cut, ncut, v, u) || !rank_lower(T, rnd, u, v)) continue;
                double dx = xyz[3 * u] - xyz[3 * v], dy = xyz[3 * u + 1] - xyz[3 * v + 1];
                double dz = xyz[3 * u + 2] - xyz[3 * v + 2];
                double slope = (ta[v] - ta[u]) / sqrt((dx * dx + dy * dy) + dz * dz);
                if (best < 0 || slope > best_slope || (slope == best_slope && rank_lower(T, rnd, u, best))) {
                    best = u;
                    best_slope = slope;
                }
            }
            parent[v] = (int32_t)best;
            if (reached < 0 && target[v]) reached = v;
        }
        for (int32_t q = 0; q < p->n_ckpt; ++q)
            if (p->ckpt_steps[q] == t) memcpy(ckpt + (size_t)q * nv, rho, (size_t)nv * sizeof(double));
        if (nn) last_insert = t;
        if (reached >= 0) { res[1] = t; res[2] = reached; rc = PASS_OK; break; }
        if (t - last_insert >= p->stall_steps) { rc = PASS_E_STALLED; res[1] = t; break; }
    }
    free(tmp); free(prev); free(nt); free(cand); free(cutv);
    res[0] = rc;
    return rc;
}
