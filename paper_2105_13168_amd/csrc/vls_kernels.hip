// vls_kernels.hip -- HIP kernels (gfx950) for the initial pass of the
// variational loop-shrinking method.
//
// One persistent cooperative kernel advances the diffusion front step by
// step with a single grid barrier per step:
//   * workgroups 1..G-1 run the field phase of step t+1 over the update list
//     (explicit Euler step of the two-phase diffuse-interface equation with
//     the clip that the column normalisation reduces to; Section
//     "Mathematical representation and data structure"), grow the next
//     update list and collect threshold-crossing candidates;
//   * workgroup 0 runs the topology phase of step t: closure rounds that
//     grow the inside set through adjacency, lower-link classification of
//     each inserted vertex, the front-tag update of regular insertions, and
//     for saddle / vanish insertions the event resolution (branching and
//     collision, Section "Initial Pass"; front labelling over crossed edges,
//     Section "Performance Considerations").
// The field never depends on the fronts (one dense field plus integer front
// bookkeeping), so step t's topology and step t+1's field run concurrently.
//
// Post-passes compute Reeb node positions (mean of the involved band,
// Section "Reeb Graph Extraction") and tunnel candidates (streamline traced
// back against the diffusion, Introduction).
//
// Floating point: FP64, evaluated exactly as written (built with
// -ffp-contract=off), neighbour sums in ascending neighbour id.
#include <climits>
#include <mutex>
#include <unordered_map>

#include "vls_internal.h"

namespace vls {

#define NT 256               // threads per workgroup (4 wave64)
#define WAVE 64
#define MAXDEG 64            // vertex degree bound of the event path (one lane per link position)
#define WCK 64               // walk checkpoints per involved loop
#define MAXBP 256            // rank-order breakpoints per event step kept in LDS
#define GLOBAL_AS __attribute__((address_space(1)))   // global memory (avoids flat accesses)
// Sub-phase clocks of the topology and event paths (diagnostics in the run
// summary); each read waits for the scalar memory counter, so they can be
// compiled out with -DVLS_DETAIL_CLOCKS=0.
#ifndef VLS_DETAIL_CLOCKS
#define VLS_DETAIL_CLOCKS 1
#endif
#define DCLK() (VLS_DETAIL_CLOCKS ? __builtin_amdgcn_s_memrealtime() : 0ull)
typedef int32_t v4i __attribute__((ext_vector_type(4)));

enum { NODE_SEED = 0, NODE_SPLIT = 1, NODE_MERGE = 2, NODE_VANISH = 3, NODE_DEGENERATE = 4 };
enum { ST_OK = 0, ST_SEED_INVALID = -6, ST_STALLED = -7, ST_INVARIANT = -13, ST_CAPACITY = -14 };

__device__ __forceinline__ bool rank_lt(uint64_t ka, int32_t a, uint64_t kb, int32_t b) {
    return ka < kb || (ka == kb && a < b);
}

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads on the dependent-latency chains of the step kernel (adjacency,
// keys, tags, loop walks).  An agent-scope relaxed atomic load returns a
// dependent scattered access in about a quarter of the latency of a plain
// cached load on MI355X (measured), and it is always coherent.
template <typename T> __device__ __forceinline__ T ldg(const T *p) {
    return __hip_atomic_load((const GLOBAL_AS T *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Data written by one workgroup and read by another inside the step kernel
// (field buffers, update / candidate lists, the key hint) go through these
// accessors.  CM = 1: agent-scope relaxed atomics, coherent across the XCDs'
// separate L2 caches by themselves, so the grid barrier needs no acquire-side
// cache invalidation and read-only mesh data stays cached between steps.
// CM = 0: plain accesses, made coherent by full agent-scope fences at the
// barrier.
template <int CM> __device__ __forceinline__ double ldx(const double *p) {
    if constexpr (CM) return __hip_atomic_load((const GLOBAL_AS double *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *(const GLOBAL_AS double *)p;
}
template <int CM> __device__ __forceinline__ void stx(double *p, double v) {
    if constexpr (CM) __hip_atomic_store((GLOBAL_AS double *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *(GLOBAL_AS double *)p = v;
}
template <int CM> __device__ __forceinline__ int32_t ldx(const int32_t *p) {
    if constexpr (CM) return __hip_atomic_load((const GLOBAL_AS int32_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *(const GLOBAL_AS int32_t *)p;
}
template <int CM> __device__ __forceinline__ void stx(int32_t *p, int32_t v) {
    if constexpr (CM) __hip_atomic_store((GLOBAL_AS int32_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *(GLOBAL_AS int32_t *)p = v;
}
template <int CM> __device__ __forceinline__ uint64_t ldx(const uint64_t *p) {
    if constexpr (CM) return __hip_atomic_load((const GLOBAL_AS uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *(const GLOBAL_AS uint64_t *)p;
}

// Grid barrier over all co-resident workgroups: monotonic arrival counter.
// Release side: every wave's stores complete (__syncthreads), then an
// agent-scope release by the arriving thread.  Acquire side: CM = 0 a full
// agent-scope fence; CM = 1 only an ordering point (shared data is read
// with coherent loads).
template <int CM>
__device__ __forceinline__ void grid_sync(Ctl *ctl, unsigned long long G, unsigned long long &epoch) {
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += 1;
        const unsigned long long target = epoch * G;
        if constexpr (CM) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        else __threadfence();
        atomicAdd(&ctl->bar, 1ull);
        while (__hip_atomic_load(&ctl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
            __builtin_amdgcn_s_sleep(1);
        if constexpr (CM) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        else __threadfence();
    }
    __syncthreads();
}

__device__ __forceinline__ void fail(const DState &s, int code, int detail) {
    if (atomicCAS(&s.ctl->status, 0, code) == 0) s.ctl->err_code = detail;
    __hip_atomic_store(&s.ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Walks along a loop of crossed half-edges, in the state where the inside
// set is {y : rank(y) < rank(v)} (plus v itself when post): the triangle
// (u, x, y) holding directed edge e = u->x has one more crossed edge, (y,x)
// (= nin[e]) if y is inside, else (u,y) (= succ[e]).  One 16 B record per
// half-edge gives succ[e], nin[e], y and x.
// A walk along a loop with its next step's loads issued together: the state
// holds the current half-edge, its owner and its record, and a step loads
// the key of y and both candidate successors' records at once (which one
// follows depends on that key), so a step costs one round trip instead of
// two.  The owner of the successor needs no load: y for nin[e], the same
// owner for succ[e].
struct Walk {
    int32_t e, src;
    v4i r;
};
__device__ __forceinline__ Walk walk_at(const DMesh &m, int32_t e) {
    Walk w;
    w.e = e;
    w.src = ldg(m.src + e);
    w.r = *(const GLOBAL_AS v4i *)(m.hrec + 4 * (int64_t)e);
    return w;
}
__device__ __forceinline__ void walk_step(const DMesh &m, const uint64_t *__restrict__ key, Walk &w, uint64_t kv,
                                          int32_t v, bool post) {
    const int32_t y = w.r.z;
    const uint64_t ky = ldg(key + y);
    const v4i ra = *(const GLOBAL_AS v4i *)(m.hrec + 4 * (int64_t)w.r.y);
    const v4i rb = *(const GLOBAL_AS v4i *)(m.hrec + 4 * (int64_t)w.r.x);
    const bool in = rank_lt(ky, y, kv, v) || (post && y == v);
    w.e = in ? w.r.y : w.r.x;
    w.src = in ? y : w.src;
    w.r = in ? ra : rb;
}

// ---------------------------------------------------------------------------
// initialisation of a run
// ---------------------------------------------------------------------------
__global__ void k_init(DState s, int32_t nv, int64_t nnz) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the control block starts at zero (a kernel rather than a memset node,
    // so the run sequence holds no memset)
    if (blockIdx.x == 0) {
        unsigned long long *c = (unsigned long long *)s.ctl;
        for (size_t i = threadIdx.x; i < sizeof(Ctl) / 8; i += blockDim.x) c[i] = 0ull;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
        s.lid[i] = -1;
        if (i < nv) {
            s.rho0[i] = 0.0;
            s.rho1[i] = 0.0;
            s.key[i] = KEY_OUT;
            s.parent[i] = -1;
            s.depth[i] = 0;
            s.stamp[i] = 0;
            s.mark[0][i] = 0;
            s.mark[1][i] = 0;
            s.cstamp[i] = -1;
        }
        // +0.0 at index nv of both field buffers (inside their tail
        // padding): the dense step's padding slots gather it
        if (i == nv) {
            s.rho0[i] = 0.0;
            s.rho1[i] = 0.0;
        }
    }
}

hipError_t launch_init(const DMesh &m, const DState &s, int64_t nnz, hipStream_t st) {
    int blocks = (int)((nnz + NT - 1) / NT);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(NT), 0, st, s, m.nv, nnz);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// seed: hop ball B(s, r0) inside, field 1 on B; the update list of step 1 is
// every vertex within r0+2 hops; initial loops numbered by their smallest
// crossed half-edge key (inside*nv + outside).  With a seed set S (the Reeb
// refinement's pass from a handle loop) the region is every vertex within r0
// hops of S, its vertices ranked by hop distance inside the region from
// s = min S; S = {s} gives the ball.
// ---------------------------------------------------------------------------
struct SeedSh {
    int n;           // vertices listed so far
    int layer_beg, layer_end;
    int add;
    int nball;
    unsigned long long ne, nf;
    int nloops;
    int bad;
    int nregion;     // seed-set mode: region size
};

__global__ void __launch_bounds__(NT) k_seed(DMesh m, DState s, DParams p) {
    __shared__ SeedSh sh;
    __shared__ long long loopkey[64];
    __shared__ int loopstart[64];
    const int tid = threadIdx.x;
    int32_t *list = s.L;       // BFS order, hop in Lrnd
    const int nset = p.n_seed_set;
    if (tid == 0) {
        const int n0 = nset > 0 ? nset : 1;
        sh.n = n0; sh.layer_beg = 0; sh.layer_end = n0; sh.nball = 0; sh.ne = 0; sh.nf = 0;
        sh.nloops = 0; sh.bad = 0; sh.add = 0; sh.nregion = 0;
        if (nset <= 0) {
            list[0] = (int32_t)p.seed;
            s.Lrnd[0] = 0;
            s.cstamp[p.seed] = -2;
        }
    }
    for (int i = tid; i < nset; i += NT) {
        const int32_t v = p.seed_set[i];
        list[i] = v;
        s.Lrnd[i] = 0;
        s.cstamp[v] = -2;
    }
    __syncthreads();
    for (int h = 1; h <= p.r0 + 2; ++h) {
        const int beg = sh.layer_beg, end = sh.layer_end;
        for (int i = beg + tid; i < end; i += NT) {
            const int32_t v = list[i];
            for (int32_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
                const int32_t u = m.adj[j];
                if (atomicCAS(&s.cstamp[u], -1, -2) == -1) {
                    const int slot = atomicAdd(&sh.n, 1);
                    list[slot] = u;
                    s.Lrnd[slot] = h;
                }
            }
        }
        __syncthreads();
        if (tid == 0) { sh.layer_beg = end; sh.layer_end = sh.n; }
        __syncthreads();
    }
    const int ntot = sh.n;
    if (nset > 0) {
        // hop distance from s inside the region (depth, -1 until reached),
        // breadth first with the queue in cand[0]
        int myreg = 0;
        for (int i = tid; i < ntot; i += NT)
            if (s.Lrnd[i] <= p.r0) { s.depth[list[i]] = -1; myreg++; }
        atomicAdd(&sh.nregion, myreg);
        __syncthreads();
        int32_t *q = s.cand[0];
        if (tid == 0) {
            q[0] = (int32_t)p.seed;
            s.depth[p.seed] = 0;
            sh.add = 1; sh.layer_beg = 0; sh.layer_end = 1;
        }
        __syncthreads();
        for (int h = 1;; ++h) {
            const int beg = sh.layer_beg, end = sh.layer_end;
            if (beg == end) break;
            for (int i = beg + tid; i < end; i += NT) {
                const int32_t v = q[i];
                for (int32_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
                    const int32_t u = m.adj[j];
                    if (s.depth[u] == -1 && atomicCAS(&s.depth[u], -1, h) == -1) q[atomicAdd(&sh.add, 1)] = u;
                }
            }
            __syncthreads();
            if (tid == 0) { sh.layer_beg = end; sh.layer_end = sh.add; }
            __syncthreads();
        }
        if (tid == 0 && sh.add != sh.nregion) sh.bad = 4;
        __syncthreads();
    }
    // ball membership, field, update list of step 1 (stamp 1)
    int myball = 0;
    for (int i = tid; i < ntot; i += NT) {
        const int32_t v = list[i];
        const int h = s.Lrnd[i];
        if (h <= p.r0) {
            // step 0, round = hop (from s inside the region with a seed set)
            s.key[v] = nset > 0 ? (uint64_t)(s.depth[v] < 0 ? 0 : s.depth[v]) : (uint64_t)h;
            s.rho0[v] = 1.0;
            s.rho1[v] = 1.0;
            myball++;
        }
        s.act[1][i] = v;
        s.mark[1][v] = 1;
    }
    atomicAdd(&sh.nball, myball);
    __syncthreads();
    // parent = minimum-rank lower neighbour; depth = hop (the parent is one hop closer)
    long long my_ne = 0, my_nf = 0;
    for (int i = tid; i < ntot; i += NT) {
        const int32_t v = list[i];
        const int h = s.Lrnd[i];
        if (h > p.r0) continue;
        const uint64_t kv = s.key[v];
        int32_t par = -1;
        uint64_t kp = KEY_OUT;
        for (int32_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
            const int32_t u = m.cyc[j];
            const uint64_t ku = s.key[u];
            const int32_t y = m.cyc[m.succ[j]];
            const uint64_t ky = s.key[y];
            if (ku != KEY_OUT && rank_lt(ku, u, kv, v) && (par < 0 || rank_lt(ku, u, kp, par))) { par = u; kp = ku; }
            if (ku != KEY_OUT && u > v) my_ne++;
            if (ku != KEY_OUT && ky != KEY_OUT && v < u && v < y) my_nf++;
        }
        s.parent[v] = par;
        s.depth[v] = nset > 0 ? (int32_t)kv : h;
    }
    atomicAdd(&sh.ne, (unsigned long long)my_ne);
    atomicAdd(&sh.nf, (unsigned long long)my_nf);
    __syncthreads();
    // initial loops: walked by thread 0 (the ball boundary is short)
    if (tid == 0) {
        const int64_t nvv = m.nv;
        int nl = 0;
        for (int i = 0; i < ntot && !sh.bad; ++i) {
            const int32_t v = list[i];
            if (s.Lrnd[i] > p.r0) continue;
            for (int32_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
                if (s.key[m.cyc[j]] != KEY_OUT || s.lid[j] >= 0) continue;
                if (nl == 64) { sh.bad = 2; break; }
                int32_t e = j;
                long long best = LLONG_MAX;
                int64_t guard = 0;
                do {
                    s.lid[e] = nl;
                    const long long k = (long long)m.src[e] * nvv + m.cyc[e];
                    if (k < best) best = k;
                    // inside = step-0 key (not KEY_OUT); v = -1 never matches
                    const int32_t jj = m.succ[e];
                    const int32_t y = m.cyc[jj];
                    e = s.key[y] != KEY_OUT ? m.nin[e] : jj;
                    if (++guard > m.nnz) { sh.bad = 3; break; }
                } while (e != j);
                loopkey[nl] = best;
                loopstart[nl] = j;
                nl++;
            }
        }
        // order loops by their smallest key; rank[i] = front id of walk i
        int rank[64];
        for (int i = 0; i < nl; ++i) {
            int r = 0;
            for (int q = 0; q < nl; ++q) if (loopkey[q] < loopkey[i]) r++;
            rank[i] = r;
        }
        for (int i = 0; i < nl && !sh.bad; ++i) {
            int32_t e = loopstart[i];
            do {
                s.lid[e] = rank[i];
                const int32_t jj = m.succ[e];
                e = s.key[m.cyc[jj]] != KEY_OUT ? m.nin[e] : jj;
            } while (e != loopstart[i]);
            s.tag_parent[i] = i;
            s.tag_fid[i] = i;
            s.front_birth[i] = 0;
            s.front_death[i] = -1;
        }
        sh.nloops = nl;
        Ctl *c = s.ctl;
        c->stop_step = LLONG_MAX;
        const long long chi = (long long)sh.nball - (long long)sh.ne + (long long)sh.nf;
        c->chi = chi;
        c->b = nl;
        c->n_inside = sh.nball;
        c->next_front = nl;
        c->n_tags = nl;
        c->cnt_act[1] = ntot;
        c->last_insert = 0;
        if (sh.bad == 2) { c->status = ST_CAPACITY; c->err_code = 1; c->done = 1; }
        else if (sh.bad == 4) { c->status = ST_SEED_INVALID; c->done = 1; }
        else if (sh.bad) { c->status = ST_INVARIANT; c->err_code = 2; c->done = 1; }
        else if (nl < 1 || 2 - chi - nl != 0) { c->status = ST_SEED_INVALID; c->done = 1; }
        else if (sh.nball == nvv) { c->done = 1; }
    }
}

hipError_t launch_seed(const DMesh &m, const DState &s, const DParams &p, hipStream_t st) {
    hipLaunchKernelGGL(k_seed, dim3(1), dim3(NT), 0, st, m, s, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// field phase of step t: rho_t from rho_{t-1} over the update list C_t
// ---------------------------------------------------------------------------
#define GB ELL_W   // neighbours gathered per vertex in registers (one padded row)

// Field phase of step t: rho_t from rho_{t-1} over the update set C_t.
//
// C_t = A_{t-2} u N(A_{t-2}), A_s = vertices that are not fixed points of
// the step at rho_s (a value 0 or 1 with every neighbour equal is rewritten
// unchanged).  Every vertex that can change at step t is in C_t, so the
// double buffer stays exact for the others.  Membership is kept in a mark
// array per step parity: while computing step t, a vertex of A_{t-1} writes
// mark[t+1] on itself and its ring (plain stores, all writers store the same
// value); C_{t+1} = {mark == t+1}.  The list L_t handed to step t+1 holds
// C_t (each member appends itself) plus the neighbours of A_{t-1} outside
// C_t (claimed once through an exchange on a step stamp); a listed vertex
// whose mark says it is not in C_{t+1} is dropped by step t+1.
//
// The work is one chain of dependent memory round trips per list entry:
// entry -> (padded neighbour row, own value, mark, key) -> (neighbour
// values, marks, stamps) -> (stores, claim exchanges) -> (one list and one
// candidate reservation per wave) -> list stores.  Each thread runs FK
// entries through every stage together so that their round trips overlap.
//
// FE: the finite-element operator, sum_j g_j (rho_j - rho_v) over the
// ascending neighbours with the coefficients of half-edges rp[v] + j, in
// place of sum_j rho_j - deg rho_v; the fixed-point test is unchanged (a
// value 0 or 1 with every neighbour equal has a zero sum either way).
template <int CM, int FK = 2, bool FE = false>
__device__ __forceinline__ void phase_field(const DMesh &m, const DState &s, const DParams &p, int64_t t,
                            int worker, int nworkers) {
    Ctl *ctl = s.ctl;
    const int n = ld_relaxed(&ctl->cnt_act[t & 3]);
    const int32_t *__restrict__ list = s.act[t & 1];
    int32_t *__restrict__ out = s.act[(t + 1) & 1];
    int *outcnt = &ctl->cnt_act[(t + 1) & 3];
    const double *__restrict__ rin = ((t - 1) & 1) ? s.rho1 : s.rho0;
    double *__restrict__ rout = (t & 1) ? s.rho1 : s.rho0;
    const int32_t *__restrict__ mk_cur = s.mark[t & 1];
    int32_t *__restrict__ mk_next = s.mark[(t + 1) & 1];
    int32_t *__restrict__ cl = s.cand[t & 1];
    int *clc = &ctl->cnt_cand[t & 3];
    const int32_t cur = (int32_t)t, next = (int32_t)(t + 1);
    const int lane = __lane_id();
    const int per = (n + nworkers - 1) / nworkers;
    const int beg = worker * per;
    const int end = min(n, beg + per);
    long long upd = 0, degsum = 0;
    for (int base = beg; base < end; base += FK * NT) {
        int32_t v[FK], d[FK];
        bool keep[FK], cand[FK], big[FK];
        uint32_t cmask[FK];          // bit j: neighbour nb[k][j] claimed as new
        int32_t nb[FK][GB];
        double r[FK];
        uint64_t kv[FK];
        int nbig = 0;                // claims of a wide vertex, appended one by one
        // entries
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            const int i = base + k * NT + threadIdx.x;
            v[k] = i < end ? ldx<CM>(list + i) : -1;
        }
        // padded neighbour row, own value, own mark, own key (and the row
        // offset of the operator's coefficients)
        int32_t mv[FK];
        int32_t rb[FK];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            keep[k] = false; cand[k] = false; big[k] = false; cmask[k] = 0; d[k] = 0;
            if (v[k] >= 0) {
                const GLOBAL_AS v4i *row = (const GLOBAL_AS v4i *)(m.ell + (int64_t)v[k] * GB);
#pragma unroll
                for (int q = 0; q < GB / 4; ++q) {
                    const v4i w = row[q];
                    nb[k][4 * q] = w.x; nb[k][4 * q + 1] = w.y; nb[k][4 * q + 2] = w.z; nb[k][4 * q + 3] = w.w;
                }
                r[k] = ldx<CM>(rin + v[k]);
                mv[k] = ldx<CM>(mk_cur + v[k]);
                kv[k] = ldx<CM>(s.key + v[k]);
                rb[k] = FE ? ldg(m.rp + v[k]) : 0;
            } else {
#pragma unroll
                for (int j = 0; j < GB; ++j) nb[k][j] = 0;
                r[k] = 0.0; mv[k] = 0; kv[k] = 0; rb[k] = 0;
            }
        }
        // neighbour values, marks and stamps; sum, fixed-point test, marks,
        // claims, new value
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            keep[k] = v[k] >= 0 && mv[k] == cur;
            big[k] = keep[k] && nb[k][0] < 0;
        }
        double xs[FK][GB];
        int32_t mu[FK][GB], st[FK][GB];
        double gw[FE ? FK : 1][FE ? GB : 1];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            if (keep[k] && !big[k]) {
                // padding slots (the vertex itself) read index nv instead, in
                // the buffers' tail padding: the same address on every lane,
                // so a padded slot costs one request rather than one per
                // lane; those slots are never used
                int32_t g[GB];
#pragma unroll
                for (int j = 0; j < GB; ++j) g[j] = nb[k][j] != v[k] ? nb[k][j] : (int32_t)m.nv;
#pragma unroll
                for (int j = 0; j < GB; ++j) xs[k][j] = ldx<CM>(rin + g[j]);
#pragma unroll
                for (int j = 0; j < GB; ++j) mu[k][j] = ldx<CM>(mk_cur + g[j]);
#pragma unroll
                for (int j = 0; j < GB; ++j) st[k][j] = *(const GLOBAL_AS int32_t *)(s.stamp + g[j]);
                if constexpr (FE) {
#pragma unroll
                    for (int j = 0; j < GB; ++j) gw[k][j] = nb[k][j] != v[k] ? ldg(m.fem_g + rb[k] + j) : 0.0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            if (!keep[k]) continue;
            const int32_t vk = v[k];
            const double rk = r[k];
            bool quiet = (rk == 0.0 || rk == 1.0);
            double sum;
            int dk;
            if (!big[k]) {
                // row padded with the vertex itself after its d neighbours
                dk = 0;
#pragma unroll
                for (int j = 0; j < GB; ++j) dk += nb[k][j] != vk;
                if constexpr (FE) sum = gw[k][0] * (xs[k][0] - rk);
                else sum = xs[k][0];
                quiet = quiet && xs[k][0] == rk;
#pragma unroll
                for (int j = 1; j < GB; ++j)
                    if (j < dk) {
                        if constexpr (FE) sum = sum + gw[k][j] * (xs[k][j] - rk);
                        else sum = sum + xs[k][j];
                        quiet = quiet && xs[k][j] == rk;
                    }
                if (!quiet) {
                    stx<CM>(mk_next + vk, next);
#pragma unroll
                    for (int j = 0; j < GB; ++j)
                        if (j < dk) {
                            stx<CM>(mk_next + nb[k][j], next);
                            // outside C_t: not listed by itself, claim it once
                            if (mu[k][j] != cur && st[k][j] != next && atomicExch(&s.stamp[nb[k][j]], next) != next)
                                cmask[k] |= 1u << j;
                        }
                }
            } else {
                // degree above the row width: row offsets and the ascending list
                const int32_t b = ldg(m.rp + vk), e = ldg(m.rp + vk + 1);
                dk = e - b;
                const double x0 = ldx<CM>(rin + m.adj[b]);
                if constexpr (FE) sum = ldg(m.fem_g + b) * (x0 - rk);
                else sum = x0;
                quiet = quiet && x0 == rk;
                for (int32_t j = b + 1; j < e; ++j) {
                    const double xn = ldx<CM>(rin + m.adj[j]);
                    if constexpr (FE) sum = sum + ldg(m.fem_g + j) * (xn - rk);
                    else sum = sum + xn;
                    quiet = quiet && xn == rk;
                }
                if (!quiet) {
                    stx<CM>(mk_next + vk, next);
                    for (int32_t j = b; j < e; ++j) {
                        const int32_t u = m.adj[j];
                        stx<CM>(mk_next + u, next);
                        if (ldx<CM>(mk_cur + u) != cur && s.stamp[u] != next && atomicExch(&s.stamp[u], next) != next) {
                            stx<CM>(out + atomicAdd(outcnt, 1), u);
                            ++nbig;
                        }
                    }
                }
            }
            d[k] = dk;
            const double lap = FE ? sum : sum - (double)dk * rk;
            const double dd = (p.a * lap + p.w * (2.0 * rk - 1.0)) + p.e * sqrt(rk * (1.0 - rk));
            double x = rk + p.c * dd;
            if (x < 0.0) x = 0.0;
            if (x > 1.0) x = 1.0;
            stx<CM>(rout + vk, x);
            upd += 1;
            degsum += dk;
            // new crossers only: a vertex above tau at step t-1 and still
            // outside was a candidate then and waits on the pending list
            cand[k] = rk <= p.tau && x > p.tau && kv[k] == KEY_OUT;
        }
        (void)nbig;
        // appends: members of C_t and claimed vertices to the next list,
        // crossers to the candidate list; one wave-wide prefix sum (both
        // counts packed in one word) and one reservation per list per wave
        int nl = 0, nc = 0;
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            nl += (int)keep[k] + __popc(cmask[k]);
            nc += (int)cand[k];
        }
        const int own = nl | (nc << 16);
        int inc = own;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const int y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        const int tot = __shfl(inc, WAVE - 1);
        if (tot == 0) continue;
        int lb = 0, cb = 0;
        if (lane == WAVE - 1) {
            if (tot & 0xffff) lb = atomicAdd(outcnt, tot & 0xffff);
            if (tot >> 16) cb = atomicAdd(clc, tot >> 16);
        }
        lb = __shfl(lb, WAVE - 1);
        cb = __shfl(cb, WAVE - 1);
        int lo = lb + ((inc - own) & 0xffff);
        int co = cb + ((inc - own) >> 16);
#pragma unroll
        for (int k = 0; k < FK; ++k) {
            if (keep[k]) stx<CM>(out + lo++, v[k]);
#pragma unroll
            for (int j = 0; j < GB; ++j)
                if ((cmask[k] >> j) & 1u) stx<CM>(out + lo++, nb[k][j]);
            if (cand[k]) stx<CM>(cl + co++, v[k]);
        }
    }
    // wave reduction of the counters, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        upd += __shfl_down(upd, off);
        degsum += __shfl_down(degsum, off);
    }
    if (lane == 0 && upd) {
        atomicAdd((unsigned long long *)&ctl->active_updates, (unsigned long long)upd);
        atomicAdd((unsigned long long *)&ctl->active_deg, (unsigned long long)degsum);
    }
}

// Dense field step t: every vertex each step.  The update set is not used;
// the vertices it would skip are exact fixed points of the step, so the
// field is bit-identical to the update-set step's.  Crossers (value above
// tau for the first time, key hint outside) go to the candidate list as
// there.
//
// The step is a stream over the compressed rows: per vertex its value (8 B
// read, 8 B written), its row offset (4 B) and its neighbour ids (4 B
// each), plus gathers of neighbour values that mostly hit the caches.  Work
// is cut into tiles of DT consecutive vertices, four consecutive vertices
// per lane, so a lane's ids are one contiguous run of the row array.  Tile
// q belongs to wave q mod (all field waves): at any moment the waves work
// on one window of ids and the gathers hit L2.  A wave stages its tile's id
// segment in its own LDS slice.  Per tile it issues the gathers first and
// then the loads of the next tile (its id segment in 16-byte chunks, its
// values, and the row offsets of the tile after it); memory counters
// retire in order, so consuming the gathers leaves the next tile's loads
// in flight under this tile's arithmetic.  Every streamed load is issued
// unconditionally at a clamped in-bounds address (the mesh and field
// buffers carry tail padding), so no loaded register outlives its tile.
#define DT 256                 // vertices per wave tile (4 per lane)
#define DACAP 2048             // ids of one tile that fit the wave's LDS slice
#define DSL (DACAP + 16)       // slice length: reads up to DW - 1 past a segment stay inside
#define DCH (DACAP / 4 / WAVE) // 16-byte id chunks per lane
#define LDS_AS __attribute__((address_space(3)))

typedef double dbl2 __attribute__((ext_vector_type(2)));

struct DRows {
    int32_t r[5];    // row offsets of the lane's vertices 4 lane + 0..4 (nnz past nv)
};

// row offsets of the tile at base, as loaded (read-only mesh data; the row
// array has 16 bytes of tail padding, so a 16-byte load at an index <= nv
// stays inside); dense_rows_fix clamps them once they have arrived
__device__ __forceinline__ void dense_load_rp(const DMesh &m, int64_t base, int lane, DRows &t) {
    const int64_t nv = m.nv;
    const GLOBAL_AS int32_t *rp = (const GLOBAL_AS int32_t *)m.rp;
    const int64_t i0 = base + 4 * lane;
    const int64_t ic = i0 <= nv ? i0 : (nv & ~3ll);
    const v4i w = *(const GLOBAL_AS v4i *)(rp + ic);
    t.r[0] = w.x; t.r[1] = w.y; t.r[2] = w.z; t.r[3] = w.w;
    t.r[4] = rp[ic + 4 <= nv ? ic + 4 : nv];
}
__device__ __forceinline__ void dense_rows_fix(const DMesh &m, int64_t base, int lane, DRows &t) {
    const int64_t nv = m.nv;
    const int64_t i0 = base + 4 * lane;
    const int32_t nnz = (int32_t)m.nnz;
#pragma unroll
    for (int k = 0; k < 5; ++k) t.r[k] = i0 + k <= nv ? t.r[k] : nnz;
}

// own values of the lane's four vertices (field buffers have 64 bytes of
// tail padding; values past nv are not used); coherent loads one by one
// when the field is shared that way
template <int CM>
__device__ __forceinline__ void dense_load_own(const double *rin, int64_t base, int64_t nv, int lane, dbl2 (&x)[2]) {
    int64_t i0 = base + 4 * lane;
    i0 = i0 < nv ? i0 : 0;
    if constexpr (CM == 0) {
        x[0] = *(const GLOBAL_AS dbl2 *)(rin + i0);
        x[1] = *(const GLOBAL_AS dbl2 *)(rin + i0 + 2);
    } else {
        x[0].x = ldx<CM>(rin + i0);
        x[0].y = ldx<CM>(rin + i0 + 1);
        x[1].x = ldx<CM>(rin + i0 + 2);
        x[1].y = ldx<CM>(rin + i0 + 3);
    }
}

// id chunks of a segment [lo, hi) (lo < hi <= lo + DACAP - 3): chunk c
// covers ids from (lo & ~3) + 4c; chunks past the segment reload its last
// one
__device__ __forceinline__ void dense_load_ids(const DMesh &m, int32_t lo, int32_t hi, int lane, v4i (&a)[DCH]) {
    const int32_t a0 = lo & ~3;
    const int n4 = (hi - a0 + 3) >> 2;
    const GLOBAL_AS v4i *src = (const GLOBAL_AS v4i *)(m.adj + a0);
#pragma unroll
    for (int j = 0; j < DCH; ++j) {
        const int c = lane + WAVE * j;
        a[j] = src[c < n4 ? c : n4 - 1];
    }
}

// field value at a vertex id through a 32-bit byte offset from the buffer
// (scalar base + vector offset addressing; the dense step requires
// nv < 2^29)
template <int CM> __device__ __forceinline__ double ld_field(const double *base, int32_t i) {
    const GLOBAL_AS double *a = (const GLOBAL_AS double *)((const GLOBAL_AS char *)base + ((uint32_t)i << 3));
    if constexpr (CM) return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *a;
}

__device__ __forceinline__ void dense_store_ids(LDS_AS int32_t *ids, int lane, const v4i (&a)[DCH]) {
#pragma unroll
    for (int j = 0; j < DCH; ++j) *(LDS_AS v4i *)(ids + 4 * (lane + WAVE * j)) = a[j];
}

// One tile of the dense step with its ids from the wave's LDS slice
// (IDS_LDS) or from the row array (a segment too long for the slice).
// Straight-line code: each of the lane's four vertices gathers DW slots,
// issued unconditionally, and sums them in slot (ascending id) order; slots
// past its degree gather the +0.0 kept at index nv of the field buffers,
// which leaves a sum of non-negative values unchanged.  Degrees above DW (none on
// marching-tetrahedra surfaces, whose degrees are 4..9) add their further
// neighbours one by one.  Between the gathers and their use it issues the
// next tile's loads.
#define DW 9
struct DCoef {
    double a, w, e, c, tau;
};
template <int CM, bool IDS_LDS>
__device__ __forceinline__ void dense_tile(const DMesh &m, const DState &s, const DCoef &cf, const double *rin,
                                           double *rout, const LDS_AS int32_t *ids, const DRows &rc, int32_t a0,
                                           const dbl2 (&own)[2], int64_t base, int lane, int32_t plo,
                                           int32_t phi, int64_t pq, int64_t pqq, v4i (&ac)[DCH],
                                           dbl2 (&ownn)[2], DRows &rnn, bool (&cand)[4], long long &upd,
                                           long long &degsum) {
    const int64_t nv = m.nv;
    const GLOBAL_AS int32_t *adj = (const GLOBAL_AS int32_t *)m.adj;
    const int64_t v0 = base + 4 * lane;
    const int32_t zero_slot = (int32_t)nv;
    int32_t u[4][DW];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t dk = rc.r[k + 1] - rc.r[k];
#pragma unroll
        for (int j = 0; j < DW; ++j) {
            int32_t w;
            if constexpr (IDS_LDS) {
                w = ids[rc.r[k] - a0 + j];
            } else {
                int64_t ix = (int64_t)rc.r[k] + j;
                ix = ix < m.nnz ? ix : m.nnz - 1;
                w = adj[ix];
            }
            u[k][j] = j < dk ? w : zero_slot;
        }
    }
    double xs[4][DW];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < DW; ++j) xs[k][j] = ld_field<CM>(rin, u[k][j]);
    __builtin_amdgcn_sched_barrier(0);
    // the next tile's loads: ids of segment [plo, phi), values of tile pq,
    // row offsets of tile pqq (in-bounds stand-ins when there is none)
    dense_load_ids(m, plo, phi, lane, ac);
    dense_load_own<CM>(rin, pq * DT, nv, lane, ownn);
    dense_load_rp(m, pqq * DT, lane, rnn);
    __builtin_amdgcn_sched_barrier(0);
    const double xr[4] = {own[0].x, own[0].y, own[1].x, own[1].y};
    double xo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t dk = rc.r[k + 1] - rc.r[k];
        double sum = xs[k][0];
#pragma unroll
        for (int j = 1; j < DW; ++j) sum = sum + xs[k][j];
        for (int32_t j = DW; j < dk; ++j) {
            const int32_t w = IDS_LDS ? ids[rc.r[k] - a0 + j] : adj[rc.r[k] + j];
            sum = sum + ldx<CM>(rin + w);
        }
        const double rk = xr[k];
        const double lap = sum - (double)dk * rk;
        const double dd = (cf.a * lap + cf.w * (2.0 * rk - 1.0)) + cf.e * sqrt(rk * (1.0 - rk));
        double x = rk + cf.c * dd;
        if (x < 0.0) x = 0.0;
        if (x > 1.0) x = 1.0;
        xo[k] = x;
        cand[k] = v0 + k < nv && rk <= cf.tau && x > cf.tau;
        if (v0 + k < nv) {
            upd += 1;
            degsum += dk;
        }
    }
    if (CM == 0 && v0 + 4 <= nv) {
        dbl2 a, b;
        a.x = xo[0]; a.y = xo[1]; b.x = xo[2]; b.y = xo[3];
        *(GLOBAL_AS dbl2 *)(rout + v0) = a;
        *(GLOBAL_AS dbl2 *)(rout + v0 + 2) = b;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (v0 + k < nv) stx<CM>(rout + v0 + k, xo[k]);
    }
    // new crossers only: a vertex above tau at step t-1 and still outside
    // was a candidate then and is pending; the key is read for crossers only
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (cand[k]) cand[k] = ldx<CM>(s.key + v0 + k) == KEY_OUT;
}

// Position of field workgroup `worker` (block worker + 1; block 0 runs the
// topology) in XCD-major order.  Workgroups are dispatched to the NXCD
// XCDs round-robin by block index, so in this order consecutive positions
// share an XCD: the tiles of one round that an XCD works on are then one
// contiguous range, and its L2 holds their neighbourhoods instead of every
// XCD touching the whole round.  Any other dispatch only changes speed.
#define NXCD 8
__device__ __forceinline__ int dense_worker_pos(int worker, int nworkers) {
    const int b = worker + 1, x = b % NXCD;
    int pos = 0;
    for (int y = 0; y < x; ++y) pos += y == 0 ? nworkers / NXCD : (y <= nworkers ? (nworkers - y) / NXCD + 1 : 0);
    return pos + (x == 0 ? b / NXCD - 1 : (b - x) / NXCD);
}

template <int CM>
__device__ __forceinline__ void phase_field_dense(const DMesh &m, const DState &s, const DParams &p, int64_t t,
                                                  int worker, int nworkers, LDS_AS int32_t *lds_all) {
    Ctl *ctl = s.ctl;
    const double *__restrict__ rin = ((t - 1) & 1) ? s.rho1 : s.rho0;
    double *__restrict__ rout = (t & 1) ? s.rho1 : s.rho0;
    int32_t *__restrict__ cl = s.cand[t & 1];
    int *clc = &ctl->cnt_cand[t & 3];
    const int lane = __lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    LDS_AS int32_t *ids = lds_all + wv * DSL;
    const DCoef cf = {p.a, p.w, p.e, p.c, p.tau};
    const int64_t nv = m.nv;
    const int64_t nw = (int64_t)nworkers * (NT / WAVE);
    const int64_t ntiles = (nv + DT - 1) / DT;
    long long upd = 0, degsum = 0;
    int64_t q = (int64_t)dense_worker_pos(worker, nworkers) * (NT / WAVE) + wv;
    if (q < ntiles) {
        // prologue: tile q staged, row offsets of tile q+nw loading
        DRows rc, rn;
        dbl2 own[2], ownn[2];
        v4i ac[DCH];
        dense_load_rp(m, q * DT, lane, rc);
        dense_load_rp(m, (q + nw < ntiles ? q + nw : q) * DT, lane, rn);
        dense_rows_fix(m, q * DT, lane, rc);
        int32_t lo = __builtin_amdgcn_readfirstlane(rc.r[0]);
        int32_t hi = __builtin_amdgcn_readlane(rc.r[4], WAVE - 1);
        bool fits = hi - (lo & ~3) <= DACAP;
        // a vertex has at least three neighbours, so [lo, lo + 1) is a
        // valid stand-in segment
        dense_load_ids(m, lo, fits ? hi : lo + 1, lane, ac);
        dense_load_own<CM>(rin, q * DT, nv, lane, own);
        if (fits) dense_store_ids(ids, lane, ac);
        for (;;) {
            const int64_t base = q * DT;
            const int64_t qn = q + nw, qnn = qn + nw;
            const bool hn = qn < ntiles, hnn = qnn < ntiles;
            int32_t lon = lo, hin = lo + 1;
            bool fitn = false;
            if (hn) {
                dense_rows_fix(m, qn * DT, lane, rn);
                lon = __builtin_amdgcn_readfirstlane(rn.r[0]);
                hin = __builtin_amdgcn_readlane(rn.r[4], WAVE - 1);
                fitn = hin - (lon & ~3) <= DACAP;
            }
            const int32_t plo = fitn ? lon : lo, phi = fitn ? hin : lo + 1;
            const int64_t pq = hn ? qn : q, pqq = hnn ? qnn : q;
            bool cand[4];
            DRows rnn;
            if (fits)
                dense_tile<CM, true>(m, s, cf, rin, rout, ids, rc, lo & ~3, own, base, lane, plo, phi, pq, pqq, ac,
                                     ownn, rnn, cand, upd, degsum);
            else
                dense_tile<CM, false>(m, s, cf, rin, rout, ids, rc, lo & ~3, own, base, lane, plo, phi, pq, pqq, ac,
                                      ownn, rnn, cand, upd, degsum);
            const int nc = (int)cand[0] + (int)cand[1] + (int)cand[2] + (int)cand[3];
            int inc = nc;
#pragma unroll
            for (int off = 1; off < WAVE; off <<= 1) {
                const int y = __shfl_up(inc, off);
                if (lane >= off) inc += y;
            }
            const int tot = __builtin_amdgcn_readlane(inc, WAVE - 1);
            if (tot) {
                int cb = 0;
                if (lane == WAVE - 1) cb = atomicAdd(clc, tot);
                cb = __shfl(cb, WAVE - 1);
                int co = cb + inc - nc;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (cand[k]) stx<CM>(cl + co++, (int32_t)(base + 4 * lane + k));
            }
            if (!hn) break;
            // the next tile's ids into the slice (every read of this tile's
            // ids is above, in program order)
            if (fitn) dense_store_ids(ids, lane, ac);
            q = qn;
            rc = rn;
            rn = rnn;
            lo = lon;
            fits = fitn;
            own[0] = ownn[0];
            own[1] = ownn[1];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        upd += __shfl_down(upd, off);
        degsum += __shfl_down(degsum, off);
    }
    if (lane == 0 && upd) {
        atomicAdd((unsigned long long *)&ctl->active_updates, (unsigned long long)upd);
        atomicAdd((unsigned long long *)&ctl->active_deg, (unsigned long long)degsum);
    }
}

// ---------------------------------------------------------------------------
// topology phase of step t (one workgroup)
// ---------------------------------------------------------------------------
struct KSh {
    int nL, nN, nnew, event, maxround, npend, flag;
    int nev_step;
    // event-path tables (wave 0)
    int runid[MAXDEG];
    int ostart[MAXDEG / 2 + 1], oend[MAXDEG / 2 + 1];
    int sig[MAXDEG / 2 + 1];
    int fin[MAXDEG / 2 + 1];
    int steps_w[MAXDEG / 2 + 1];
    int cyc_of[MAXDEG / 2 + 1];
    int newtag[MAXDEG / 2 + 1];
    int newid[MAXDEG / 2 + 1];
    int root_run[MAXDEG / 2 + 1];      // root per lower run
    int lrstart[MAXDEG / 2 + 1];       // start position per lower run
    int sroot[MAXDEG / 2 + 1];         // distinct roots (ascending front id)
    int sfid[MAXDEG / 2 + 1];
    int srep[MAXDEG / 2 + 1];
    int sa[MAXDEG / 2 + 1];
    long long lplen[MAXDEG / 2 + 1];
    long long lpoff[MAXDEG / 2 + 1];
    long long lpmin[MAXDEG / 2 + 1];
    double lplength[MAXDEG / 2 + 1];
    long long lpk[MAXDEG / 2 + 1];      // checkpoint stride of each involved loop's walk
    int lpnck[MAXDEG / 2 + 1];          // checkpoints kept
    // rank-order breakpoints of an event step (events, round starts)
    int nbp;
    int bpu[MAXBP];
    int bps[MAXBP];
};

// root of a front tag; -1 when the tag is not a valid one (a broken
// invariant, reported by the caller)
__device__ __forceinline__ int32_t tag_find(int32_t *tp, int32_t ntags, int32_t x) {
    if (x < 0 || x >= ntags) return -1;
    int32_t r = x;
    for (int32_t g = 0; tp[r] != r; ++g) {
        if (g > ntags) return -1;
        r = tp[r];
    }
    while (tp[x] != r) { const int32_t n = tp[x]; tp[x] = r; x = n; }
    return r;
}

// block-wide bitonic sort of n keys (ascending); a holds a power-of-two
// padded array of size np (padding = UINT64_MAX)
__device__ void block_bitonic(uint64_t *a, int np) {
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += NT) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t x = a[i], y = a[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) { a[i] = y; a[ixj] = x; }
                }
            }
            __syncthreads();
        }
    }
}

// regular insertion of v (one lower arc): its new crossed half-edges carry
// the tag of the arc, read from the half-edge (parent -> v)
__device__ __forceinline__ bool load_lrow(const DMesh &m, int32_t x, int32_t *nb, int32_t &b, int &d);

// insertion of a regular vertex v (parent and key already set): its new
// crossed half-edges (towards neighbours ranked after it) take the tag of
// the half-edge (parent -> v); depth = depth(parent) + 1
__device__ __forceinline__ void regular_insert(const DMesh &m, const DState &s, int32_t v) {
    const int32_t par = ldg(s.parent + v);
    const uint64_t kv = ldg(s.key + v);
    int32_t nb[GB];
    int32_t b;
    int d;
    if (load_lrow(m, v, nb, b, d)) {
        uint64_t kn[GB];
#pragma unroll
        for (int j = 0; j < GB; ++j) kn[j] = nb[j] >= 0 ? ldg(s.key + nb[j]) : KEY_OUT;
        int ppos = -1;
#pragma unroll
        for (int j = 0; j < GB; ++j)
            if (nb[j] == par && par >= 0) ppos = j;
        const int32_t tag = ppos >= 0 ? ldg(s.lid + ldg(m.rev + b + ppos)) : -1;
        s.depth[v] = par >= 0 ? ldg(s.depth + par) + 1 : 0;
#pragma unroll
        for (int j = 0; j < GB; ++j)
            if (j < d && !rank_lt(kn[j], nb[j], kv, v)) s.lid[b + j] = tag;
        return;
    }
    const int32_t e = ldg(m.rp + v + 1);
    int32_t tag = -1;
    for (int32_t j = b; j < e; ++j)
        if (ldg(m.cyc + j) == par) tag = ldg(s.lid + ldg(m.rev + j));
    s.depth[v] = par >= 0 ? ldg(s.depth + par) + 1 : 0;
    for (int32_t j = b; j < e; ++j) {
        const int32_t u = ldg(m.cyc + j);
        if (!rank_lt(ldg(s.key + u), u, kv, v)) s.lid[j] = tag;
    }
}

// crossing point of edge (u inside, x outside) at the threshold
template <int CM>
__device__ __forceinline__ void crossing_point(const DMesh &m, const double *rho, int32_t u,
                                               int32_t x, double tau, double *pt) {
    const double ru = ldx<CM>(rho + u), rx = ldx<CM>(rho + x);
    const double den = ru - rx;
    double t;
    if (den <= 0.0) {
        t = 0.5;
    } else {
        t = (ru - tau) / den;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    const double *pu = m.xyz + 3 * (int64_t)u, *px = m.xyz + 3 * (int64_t)x;
    pt[0] = pu[0] + t * (px[0] - pu[0]);
    pt[1] = pu[1] + t * (px[1] - pu[1]);
    pt[2] = pu[2] + t * (px[2] - pu[2]);
}

// Saddle or vanish insertion of v at step t, resolved by wave 0 (all 64
// lanes call it with the same v).
template <int CM>
__device__ __forceinline__ void resolve_event(const DMesh &m, const DState &s, const DParams &p, int64_t t,
                              int32_t v, KSh *sh, const double *rho) {
    Ctl *ctl = s.ctl;
    const int lane = __lane_id();
    if (lane == 0) ctl->clk_ev0 = DCLK();
    const int32_t b = m.rp[v];
    const int d = m.rp[v + 1] - b;
    const uint64_t kv = s.key[v];
    const unsigned long long full_mask = d == 64 ? ~0ull : ((1ull << d) - 1ull);
    int32_t u = -1;
    uint64_t ku = KEY_OUT;
    bool low = false;
    if (lane < d) {
        u = m.cyc[b + lane];
        ku = s.key[u];
        low = rank_lt(ku, u, kv, v);
    }
    const unsigned long long lm = __ballot(low) & full_mask;
    const bool full = lm == full_mask;
    // prev[j] = low[j-1], nxt[j] = low[j+1] (cyclic within d)
    const unsigned long long prevm = ((lm << 1) | (lm >> (d - 1))) & full_mask;
    const unsigned long long nextm = ((lm >> 1) | (lm << (d - 1))) & full_mask;
    const unsigned long long lstart = lm & ~prevm;           // first positions of lower runs
    const unsigned long long ostartm = ~lm & full_mask & prevm;
    const unsigned long long oendm = ~lm & full_mask & nextm;
    const int k = full ? 0 : __popcll(lstart);
    // parent / depth
    const int32_t par = s.parent[v];
    if (lane == 0) s.depth[v] = s.depth[par] + 1;
    // roots of the lower runs (vanish: the whole link is one run, position 0)
    const int nruns = full ? 1 : k;
    if (lane == 0) {
        unsigned long long mm = full ? 1ull : lstart;
        for (int r = 0; r < nruns; ++r) {
            const int pos = __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            sh->lrstart[r] = pos;
            sh->root_run[r] = tag_find(s.tag_parent, ctl->n_tags, s.lid[m.rev[b + pos]]);
            if (sh->root_run[r] < 0) fail(s, ST_INVARIANT, 13);
        }
        // distinct roots, ascending front id
        int ns = 0;
        for (int r = 0; r < nruns; ++r) {
            const int rt = sh->root_run[r];
            int q = 0;
            while (q < ns && sh->sroot[q] != rt) q++;
            if (q == ns) { sh->sroot[ns] = rt; sh->sfid[ns] = s.tag_fid[rt]; sh->srep[ns] = sh->lrstart[r]; ns++; }
        }
        for (int i = 1; i < ns; ++i)
            for (int j = i; j > 0 && sh->sfid[j] < sh->sfid[j - 1]; --j) {
                int t1 = sh->sfid[j]; sh->sfid[j] = sh->sfid[j - 1]; sh->sfid[j - 1] = t1;
                t1 = sh->sroot[j]; sh->sroot[j] = sh->sroot[j - 1]; sh->sroot[j - 1] = t1;
                t1 = sh->srep[j]; sh->srep[j] = sh->srep[j - 1]; sh->srep[j - 1] = t1;
            }
        sh->flag = ns;
    }
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    if (__shfl(ld_relaxed(&ctl->status), 0) != 0) return;
    const int sN = __shfl(sh->flag, 0);
    // minimum-rank lower neighbour per involved front (tunnel end points)
    {
        int myroot = -1;
        if (low) myroot = tag_find(s.tag_parent, ctl->n_tags, s.lid[m.rev[b + lane]]);
        for (int q = 0; q < sN; ++q) {
            const int rt = sh->sroot[q];
            const bool mine = low && myroot == rt;
            // reduction for the minimum rank among lanes with mine
            uint64_t bk = mine ? ku : KEY_OUT;
            int32_t bu = mine ? u : 0x7fffffff;
            for (int off = 32; off > 0; off >>= 1) {
                const uint64_t ok = __shfl_xor(bk, off);
                const int32_t ou = __shfl_xor(bu, off);
                if (rank_lt(ok, ou, bk, bu)) { bk = ok; bu = ou; }
            }
            if (lane == 0) sh->sa[q] = bu;
        }
    }
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    // ---- merge: the involved loops before v joins (handle loops) ----------
    int keep_loop0 = 0;
    const unsigned long long q0 = DCLK();
    if (!full && sN >= 2) {
        if (sN > MAXDEG / 2) { if (lane == 0) fail(s, ST_CAPACITY, 3); return; }
        long long n = 0, best = LLONG_MAX, bestidx = 0;
        int32_t e0 = -1;
        // one walk per involved loop (one lane per loop); it keeps at most
        // WCK checkpoints, evenly spaced at a power-of-two stride K (halved
        // into every other one and K doubled when full), so the output pass
        // below re-walks only K-step segments, one lane per segment
        int32_t *ck = s.wck + (int64_t)lane * WCK;
        long long K = 1;
        int nck = 0;
        if (lane < sN) {
            e0 = m.rev[b + sh->srep[lane]];
            Walk w = walk_at(m, e0);
            do {
                if ((n & (K - 1)) == 0) {
                    if (nck == WCK) {
                        for (int c = 0; c < WCK / 2; ++c) ck[c] = ck[2 * c];
                        nck = WCK / 2;
                        K *= 2;
                    }
                    if ((n & (K - 1)) == 0) ck[nck++] = w.e;
                }
                const long long key = (long long)w.src * m.nv + w.r.w;
                if (key < best) { best = key; bestidx = n; }
                n++;
                walk_step(m, s.key, w, kv, v, false);
            } while (w.e != e0 && n <= m.nnz);
            if (n > m.nnz) fail(s, ST_INVARIANT, 4);
            sh->lplen[lane] = n;
            sh->lpmin[lane] = bestidx;
            sh->lpk[lane] = K;
            sh->lpnck[lane] = nck;
        }
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        if (__shfl(ld_relaxed(&ctl->status), 0) != 0) return;
        if (lane == 0) {
            long long tot = 0;
            for (int q = 0; q < sN; ++q) tot += sh->lplen[q];
            const long long base = ctl->lp_he_used;
            const int nl0 = ctl->n_loops;
            if (base + tot > s.lp_he_cap || nl0 + sN > s.lp_cap) {
                fail(s, ST_CAPACITY, 5);
                sh->flag = -1;
            } else {
                long long o = base;
                for (int q = 0; q < sN; ++q) { sh->lpoff[q] = o; o += sh->lplen[q]; }
                ctl->lp_he_used = o;
                ctl->n_loops = nl0 + sN;
                sh->flag = nl0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        const int nl0 = __shfl(sh->flag, 0);
        if (nl0 < 0) return;
        keep_loop0 = nl0;
        // output, loop by loop: crossed edges from the minimum key on, their
        // crossing points, then the segment lengths; the length is summed in
        // that order by one lane
        for (int q = 0; q < sN; ++q) {
            const long long nq = sh->lplen[q], bq = sh->lpmin[q], Kq = sh->lpk[q], off = sh->lpoff[q];
            const int ncq = sh->lpnck[q];
            const int32_t *ckq = s.wck + (int64_t)q * WCK;
            for (int c = lane; c < ncq; c += WAVE) {
                Walk w = walk_at(m, ckq[c]);
                const long long i0 = (long long)c * Kq;
                const long long i1 = i0 + Kq < nq ? i0 + Kq : nq;
                for (long long i = i0; i < i1; ++i) {
                    const long long rel = i - bq;
                    const long long pos = off + (rel < 0 ? rel + nq : rel);
                    const int32_t uu = w.src, xx = w.r.w;
                    s.lp_he[2 * pos] = uu;
                    s.lp_he[2 * pos + 1] = xx;
                    crossing_point<CM>(m, rho, uu, xx, p.tau, s.lp_pts + 3 * pos);
                    walk_step(m, s.key, w, kv, v, false);
                }
            }
            __builtin_amdgcn_wave_barrier();
            __threadfence_block();
            for (long long i = lane; i < nq; i += WAVE) {
                const double *pa = s.lp_pts + 3 * (off + i);
                const double *pb = s.lp_pts + 3 * (off + (i + 1 == nq ? 0 : i + 1));
                const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
                s.wseg[i] = sqrt((dx * dx + dy * dy) + dz * dz);
            }
            __builtin_amdgcn_wave_barrier();
            __threadfence_block();
            if (lane == 0) {
                double L = 0.0;
                for (long long i = 0; i < nq; ++i) L = L + s.wseg[i];
                sh->lplength[q] = L;
            }
            __builtin_amdgcn_wave_barrier();
            __threadfence_block();
        }
    }
    const unsigned long long q1 = DCLK();
    unsigned long long q2 = q1, q3 = q1;
    // ---- the loops after v joins: walkers from the end of each new arc ----
    int mN = 0;
    if (!full) {
        if (k > MAXDEG / 2) { if (lane == 0) fail(s, ST_CAPACITY, 6); return; }
        // run id of every outside position: index of the end position that
        // closes its arc (ends in ascending order)
        if (lane < d && !low) {
            const unsigned long long ge = oendm >> lane;
            int endpos;
            if (ge) endpos = lane + __ffsll((long long)ge) - 1;
            else endpos = __ffsll((long long)oendm) - 1;
            sh->runid[lane] = __popcll(oendm & ((endpos == 0) ? 0ull : ((1ull << endpos) - 1ull)));
        }
        if (lane < k) {
            // lane-th end / start positions (ascending)
            unsigned long long mm = oendm;
            for (int q = 0; q < lane; ++q) mm &= mm - 1;
            sh->oend[lane] = __ffsll((long long)mm) - 1;
        }
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        if (lane < d && !low && (ostartm >> lane & 1ull)) sh->ostart[sh->runid[lane]] = lane;
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        Walk w;
        w.e = -1;
        w.src = -1;
        if (lane < k) w = walk_at(m, b + sh->oend[lane]);
        bool done = lane >= k;
        int steps = 0, tgt = -1;
        // checkpoints of each walker's arc (same scheme as the merge walks),
        // for the relabel below
        int32_t *ckw = s.wck + (int64_t)lane * WCK;
        long long K = 1;
        int nck = 0;
        if (lane < k) ckw[nck++] = w.e;
        for (;;) {
            const unsigned long long act = __ballot(!done) & ((k == 64) ? ~0ull : ((1ull << k) - 1ull));
            if (__popcll(act) <= 1) break;
            if (!done) {
                walk_step(m, s.key, w, kv, v, true);
                steps++;
                if ((steps & (K - 1)) == 0) {
                    if (nck == WCK) {
                        for (int c = 0; c < WCK / 2; ++c) ckw[c] = ckw[2 * c];
                        nck = WCK / 2;
                        K *= 2;
                    }
                    if ((steps & (K - 1)) == 0) ckw[nck++] = w.e;
                }
                if (w.src == v) { done = true; tgt = sh->runid[w.e - b]; }
                if (steps > m.nnz) { fail(s, ST_INVARIANT, 7); done = true; tgt = 0; }
            }
        }
        if (lane < k) {
            sh->fin[lane] = done ? 1 : 0;
            sh->sig[lane] = tgt;
            sh->steps_w[lane] = steps;
            sh->lpk[lane] = K;
            sh->lpnck[lane] = nck;
        }
        q2 = DCLK();
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        if (__shfl(ld_relaxed(&ctl->status), 0) != 0) return;
        if (lane == 0) {
            // the unfinished walker (if any) closes onto the one arc nobody reached
            unsigned long long hit = 0;
            int unf = -1;
            for (int o = 0; o < k; ++o) { if (sh->fin[o]) hit |= 1ull << sh->sig[o]; else unf = o; }
            if (unf >= 0) {
                const unsigned long long rem = ~hit & ((k == 64) ? ~0ull : ((1ull << k) - 1ull));
                sh->sig[unf] = __ffsll((long long)rem) - 1;
            }
            // cycles of the arc permutation = the loops after the insertion
            for (int o = 0; o < k; ++o) sh->cyc_of[o] = -1;
            int nc = 0;
            int minpos[MAXDEG / 2 + 1];
            long long wlen[MAXDEG / 2 + 1];
            for (int o = 0; o < k; ++o) {
                if (sh->cyc_of[o] >= 0) continue;
                int q = o, mp = 1 << 30;
                long long wl = 0;
                int guard = 0;
                while (sh->cyc_of[q] < 0 && guard++ <= k) {
                    sh->cyc_of[q] = nc;
                    const int st = sh->ostart[q], en = sh->oend[q];
                    const int mpos = st <= en ? st : 0;
                    if (mpos < mp) mp = mpos;
                    wl += sh->steps_w[q];
                    q = sh->sig[q];
                }
                minpos[nc] = mp;
                wlen[nc] = wl;
                nc++;
            }
            // the loop holding the unfinished walker keeps the old tags
            int big = 0;
            if (unf >= 0) big = sh->cyc_of[unf];
            else for (int c = 1; c < nc; ++c) if (wlen[c] > wlen[big]) big = c;
            // new front ids in counter-clockwise order of the first new half-edge
            int order[MAXDEG / 2 + 1];
            for (int c = 0; c < nc; ++c) {
                int r = 0;
                for (int q = 0; q < nc; ++q) if (minpos[q] < minpos[c]) r++;
                order[c] = r;
            }
            const int fid0 = ctl->next_front;
            if (fid0 + nc > s.front_cap || ctl->n_tags + nc > s.tag_cap) {
                fail(s, ST_CAPACITY, 8);
                sh->flag = -1;
            } else {
                ctl->next_front = fid0 + nc;
                const int R0 = sh->sroot[0];
                for (int q = 1; q < sN; ++q) s.tag_parent[sh->sroot[q]] = R0;
                for (int c = 0; c < nc; ++c) {
                    sh->newid[c] = fid0 + order[c];
                    if (c == big) {
                        sh->newtag[c] = R0;
                        s.tag_fid[R0] = fid0 + order[c];
                    } else {
                        const int tg = ctl->n_tags++;
                        s.tag_parent[tg] = tg;
                        s.tag_fid[tg] = fid0 + order[c];
                        sh->newtag[c] = tg;
                    }
                }
                sh->flag = nc;
                sh->maxround = big;   // reuse: index of the big loop
            }
        }
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        mN = __shfl(sh->flag, 0);
        if (mN < 0) return;
        const int big = __shfl(sh->maxround, 0);
        // tags of the new arcs, and relabel of every loop but the big one
        q3 = DCLK();
        if (lane < d && !low) s.lid[b + lane] = sh->newtag[sh->cyc_of[sh->runid[lane]]];
        // the arcs walked to completion: edges 1 .. steps-1 of each walk,
        // replayed in K-step segments from its checkpoints, one lane each
        for (int o = 0; o < k; ++o) {
            if (sh->cyc_of[o] == big) continue;
            const int32_t tg = sh->newtag[sh->cyc_of[o]];
            const long long so = sh->steps_w[o], Ko = sh->lpk[o];
            const int nco = sh->lpnck[o];
            const int32_t *cko = s.wck + (int64_t)o * WCK;
            for (int c = lane; c < nco; c += WAVE) {
                Walk w = walk_at(m, cko[c]);
                const long long i0 = (long long)c * Ko;
                const long long i1 = i0 + Ko < so ? i0 + Ko : so;
                for (long long i = i0; i < i1; ++i) {
                    if (i >= 1) s.lid[w.e] = tg;
                    walk_step(m, s.key, w, kv, v, true);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
    }
    // ---- bookkeeping: h, x, node, records ----------------------------------
    if (lane == 0) {
        const unsigned long long q4 = DCLK();
        ctl->clk_evp[0] += q1 - q0;          // merge walks and loop output
        ctl->clk_evp[1] += q2 - q1;          // split walkers
        ctl->clk_evp[2] += q4 - q3;          // relabel walks
        ctl->clk_evp[3] += q0 - ctl->clk_ev0 + (q3 - q2);   // the rest
        long long h = 0, xx = 0;
        bool ok = true;
        if (full) {
            ok = (sN == 1);
        } else {
            const long long num = (long long)k - 1 - ((long long)mN - sN);
            if (num < 0 || (num & 1)) ok = false;
            h = num / 2;
            xx = h - (sN - 1);
            if (xx < 0) ok = false;
        }
        const int ev = ctl->n_events;
        const long long idoff = ctl->ev_ids_used;
        if (!ok) {
            fail(s, ST_INVARIANT, 9);
        } else if (ev >= s.ev_cap || idoff + sN + mN > s.ev_ids_cap || sN > 16) {
            fail(s, ST_CAPACITY, 10);
        } else {
            const int type = full ? NODE_VANISH : (xx > 0 ? NODE_DEGENERATE : (sN >= 2 ? NODE_MERGE : NODE_SPLIT));
            const int node = ev + 1;
            int64_t *rec = s.ev + 16 * (int64_t)ev;
            rec[0] = t; rec[1] = v; rec[2] = type; rec[3] = full ? 0 : k; rec[4] = sN; rec[5] = mN;
            rec[6] = h; rec[7] = xx; rec[8] = node; rec[9] = (int64_t)(kv & 0xffffffffull);
            rec[10] = full ? 1 : 0; rec[11] = idoff; rec[12] = 0; rec[13] = 0; rec[14] = 0; rec[15] = 0;
            for (int q = 0; q < sN; ++q) {
                s.ev_ids[idoff + q] = sh->sfid[q];
                s.ev_rep[16 * (int64_t)ev + q] = sh->srep[q];
                s.front_death[sh->sfid[q]] = node;
            }
            if (!full) {
                for (int c = 0; c < mN; ++c) {
                    // out ids listed in ascending (counter-clockwise) order
                    s.ev_ids[idoff + sN + (sh->newid[c] - ctl->next_front + mN)] = sh->newid[c];
                    s.front_birth[sh->newid[c]] = node;
                    s.front_death[sh->newid[c]] = -1;
                }
            }
            ctl->ev_ids_used = idoff + sN + mN;
            ctl->n_events = ev + 1;
            if (type == NODE_DEGENERATE) ctl->n_degenerate += 1;
            ctl->chi += full ? 1 : 1 - k;
            ctl->b += (long long)mN - sN;
            ctl->gsum_x += xx;
            // handle loops: every involved loop but the longest (ties: larger id)
            if (!full && sN >= 2) {
                int drop = 0;
                for (int q = 1; q < sN; ++q) if (sh->lplength[q] >= sh->lplength[drop]) drop = q;
                for (int q = 0; q < sN; ++q) {
                    int64_t *lr = s.lp + 8 * (int64_t)(keep_loop0 + q);
                    lr[0] = ev; lr[1] = sh->sfid[q]; lr[2] = q != drop; lr[3] = sh->lpoff[q];
                    lr[4] = sh->lplen[q]; lr[5] = sh->sa[q];
                    lr[6] = __double_as_longlong(sh->lplength[q]); lr[7] = 0;
                    if (q != drop) {
                        const int tnn = ctl->n_tunnels++;
                        int32_t *tr = s.tn + 4 * (int64_t)tnn;
                        tr[0] = keep_loop0 + q; tr[1] = v; tr[2] = sh->sa[q]; tr[3] = sh->sa[drop];
                        ctl->gsum_h += 1;
                    }
                }
            }
            const long long twog = 2 - ctl->chi - ctl->b;
            if (twog != 2 * (ctl->gsum_h + ctl->gsum_x)) fail(s, ST_INVARIANT, 11);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
}

template <int CM, int CAP>
__device__ __forceinline__ void phase_topo_global(const DMesh &m, const DState &s, const DParams &p, int64_t t,
                                  KSh *sh, uint64_t *lsort, int sort_cap) {
    Ctl *ctl = s.ctl;
    const double *__restrict__ rho = (t & 1) ? s.rho1 : s.rho0;
    const int tid = threadIdx.x;
    const unsigned long long g0 = DCLK();
    unsigned long long g1 = g0, g2 = g0, g3 = g0;
    if (tid == 0) { sh->nL = 0; sh->nN = 0; sh->nnew = 0; sh->event = 0; sh->npend = 0; }
    __syncthreads();
    // 1. candidates: this step's crossers plus the pending ones, de-duplicated
    const int nc = ld_relaxed(&ctl->cnt_cand[t & 3]);
    const int np = ctl->cnt_pend[(t - 1) & 1];
    const int32_t *cl = s.cand[t & 1];
    const int32_t *pl = s.pend[(t - 1) & 1];
    for (int i = tid; i < nc + np; i += NT) {
        const int32_t x = i < nc ? ldx<CM>(cl + i) : pl[i - nc];
        if (s.key[x] == KEY_OUT && ldx<CM>(rho + x) > p.tau) {
            if (atomicExch(&s.cstamp[x], (int32_t)t) != (int32_t)t) {
                const int slot = atomicAdd(&sh->nL, 1);
                s.L[slot] = x;
                s.Lrnd[slot] = -1;
            }
        }
    }
    __syncthreads();
    const int nL = sh->nL;
    const uint64_t tk = (uint64_t)t << 32;
    int round = 0;
    g1 = g2 = g3 = DCLK();
    if (nL > 0) {
        // 2. closure rounds: round 0 touches the inside set of step t-1,
        //    round j touches round j-1
        for (;;) {
            const uint64_t want = tk | (uint64_t)(round - 1);
            for (int i = tid; i < nL; i += NT) {
                int flag = 0;
                if (s.Lrnd[i] == -1) {
                    const int32_t x = s.L[i];
                    int32_t nb[GB];
                    int32_t b;
                    int d;
                    if (load_lrow(m, x, nb, b, d)) {
                        uint64_t kn[GB];
#pragma unroll
                        for (int j = 0; j < GB; ++j) kn[j] = nb[j] >= 0 ? ldg(s.key + nb[j]) : KEY_OUT;
#pragma unroll
                        for (int j = 0; j < GB; ++j)
                            flag |= nb[j] >= 0 && (round == 0 ? (kn[j] < tk) : (kn[j] == want));
                    } else {
                        for (int32_t j = b; j < ldg(m.rp + x + 1); ++j) {
                            const uint64_t kk = s.key[m.adj[j]];
                            if (round == 0 ? (kk < tk) : (kk == want)) { flag = 1; break; }
                        }
                    }
                }
                s.Lcls[i] = flag;
            }
            __syncthreads();
            int mine = 0;
            for (int i = tid; i < nL; i += NT)
                if (s.Lcls[i]) { s.Lrnd[i] = round; s.key[s.L[i]] = tk | (uint64_t)round; mine++; }
            if (mine) atomicAdd(&sh->nnew, mine);
            __syncthreads();
            const int nnew = sh->nnew;
            __syncthreads();
            if (tid == 0) { sh->nN += nnew; sh->nnew = 0; }
            __syncthreads();
            if (nnew == 0) break;
            if (sh->nN == nL) { round++; break; }
            round++;
        }
        // rounds used: 0 .. round-1
        const int nrounds = round;
        g2 = DCLK();
        // 3. lower-link classification of every inserted vertex
        for (int i = tid; i < nL; i += NT) {
            if (s.Lrnd[i] < 0) continue;
            const int32_t v = s.L[i];
            const uint64_t kv = s.key[v];
            int32_t nb[GB];
            int32_t b;
            int d;
            int nlow = 0, runs = 0;
            int32_t par = -1;
            uint64_t kp = KEY_OUT;
            if (load_lrow(m, v, nb, b, d)) {
                uint64_t kn[GB];
#pragma unroll
                for (int j = 0; j < GB; ++j) kn[j] = nb[j] >= 0 ? ldg(s.key + nb[j]) : KEY_OUT;
                bool prev = false;
#pragma unroll
                for (int j = 0; j < GB; ++j)
                    if (j == d - 1) prev = rank_lt(kn[j], nb[j], kv, v);
#pragma unroll
                for (int j = 0; j < GB; ++j) {
                    if (j >= d) continue;
                    const bool low = rank_lt(kn[j], nb[j], kv, v);
                    if (low) {
                        nlow++;
                        if (!prev) runs++;
                        if (par < 0 || rank_lt(kn[j], nb[j], kp, par)) { par = nb[j]; kp = kn[j]; }
                    }
                    prev = low;
                }
            } else {
                d = ldg(m.rp + v + 1) - b;
                int32_t ulast = m.cyc[b + d - 1];
                bool prev = rank_lt(s.key[ulast], ulast, kv, v);
                for (int j = 0; j < d; ++j) {
                    const int32_t u = m.cyc[b + j];
                    const uint64_t ku = s.key[u];
                    const bool low = rank_lt(ku, u, kv, v);
                    if (low) {
                        nlow++;
                        if (!prev) runs++;
                        if (par < 0 || rank_lt(ku, u, kp, par)) { par = u; kp = ku; }
                    }
                    prev = low;
                }
            }
            const int cls = nlow == d ? -1 : runs;
            s.Lcls[i] = cls;
            s.parent[v] = par;
            if (cls != 1) atomicOr(&sh->event, 1);
            if (nlow == 0 || d > MAXDEG) atomicOr(&sh->event, 2);
        }
        __syncthreads();
        g3 = DCLK();
        if (sh->event & 2) {
            if (tid == 0) fail(s, ST_INVARIANT, 12);
        } else if (!sh->event) {
            // 4a. all insertions regular: tags follow the parent edge, by round
            for (int r = 0; r < nrounds; ++r) {
                for (int i = tid; i < nL; i += NT)
                    if (s.Lrnd[i] == r) regular_insert(m, s, s.L[i]);
                __syncthreads();
            }
        } else {
            // 4b. events: rank order (round, id); regular runs between events in
            //     parallel by round, each event by wave 0.  The order is sorted
            //     in LDS (the candidate tables are unused on this path) up to
            //     sort_cap entries, else in global memory; its breakpoints
            //     (events, first entries of a round) are found in parallel.
            const int nN = sh->nN;
            int npow = 1;
            while (npow < nN) npow <<= 1;
            uint64_t *arr = npow <= sort_cap ? lsort : s.ord;
            for (int i = tid; i < npow; i += NT) arr[i] = ~0ull;
            __syncthreads();
            if (tid == 0) { sh->nnew = 0; sh->nbp = 0; }
            __syncthreads();
            for (int i = tid; i < nL; i += NT) {
                if (s.Lrnd[i] < 0) continue;
                const int slot = atomicAdd(&sh->nnew, 1);
                arr[slot] = ((uint64_t)s.Lrnd[i] << 33) | ((uint64_t)s.L[i] << 1) | (uint64_t)(s.Lcls[i] != 1);
            }
            __syncthreads();
            block_bitonic(arr, npow);
            for (int i = tid; i < nN; i += NT)
                if ((arr[i] & 1ull) || (i > 0 && (arr[i] >> 33) != (arr[i - 1] >> 33))) {
                    const int k = atomicAdd(&sh->nbp, 1);
                    if (k < MAXBP) sh->bpu[k] = i;
                }
            __syncthreads();
            const int nbp = sh->nbp < MAXBP ? sh->nbp : MAXBP;
            const bool bp_ok = sh->nbp <= MAXBP;
            for (int i = tid; i < nbp; i += NT) {
                const int x = sh->bpu[i];
                int r = 0;
                for (int j = 0; j < nbp; ++j) r += sh->bpu[j] < x;
                sh->bps[r] = x;
            }
            __syncthreads();
            int pos = 0, kb = 0;
            while (pos < nN) {
                // the regular segment [pos, q) ends at the next event q; with
                // the breakpoints known, a round change inside it is a
                // breakpoint too, so each run [a0, a1) is one round
                int q, qr;
                if (bp_ok) {
                    while (kb < nbp && sh->bps[kb] < pos) kb++;
                    qr = kb < nbp ? sh->bps[kb] : nN;
                    if (qr == pos && !(arr[pos] & 1ull)) {
                        kb++;
                        qr = kb < nbp ? sh->bps[kb] : nN;
                    }
                    q = (qr < nN && (arr[qr] & 1ull)) ? qr : nN;
                    if (qr < nN && !(arr[qr] & 1ull)) q = -1;     // round change, no event yet
                } else {
                    q = pos;
                    while (q < nN && !(arr[q] & 1ull)) q++;
                    qr = q;
                }
                const int stop = q < 0 ? qr : q;
                int a0 = pos;
                while (a0 < stop) {
                    int a1 = stop;
                    if (!bp_ok) {
                        const int r = (int)(arr[a0] >> 33);
                        a1 = a0;
                        while (a1 < stop && (int)(arr[a1] >> 33) == r) a1++;
                    }
                    for (int i = a0 + tid; i < a1; i += NT)
                        regular_insert(m, s, (int32_t)((arr[i] >> 1) & 0xffffffffull));
                    __syncthreads();
                    a0 = a1;
                }
                if (q < 0) {
                    pos = qr;              // continue with the next round
                    continue;
                }
                if (q < nN) {
                    if (tid < WAVE)
                        resolve_event<CM>(m, s, p, t, (int32_t)((arr[q] >> 1) & 0xffffffffull), sh, rho);
                    __syncthreads();
                    if (ld_relaxed(&ctl->status) != 0) break;
                }
                pos = q + 1;
            }
            if (tid == 0) ctl->event_steps += 1;
        }
    }
    // 5. crossers not connected this step wait for the next
    for (int i = tid; i < nL; i += NT)
        if (s.Lrnd[i] < 0) s.pend[t & 1][atomicAdd(&sh->npend, 1)] = s.L[i];
    __syncthreads();
    if (tid == 0) {
        const unsigned long long g4 = DCLK();
        ctl->clk_g[0] += g1 - g0;
        ctl->clk_g[1] += g2 - g1;
        ctl->clk_g[2] += g3 - g2;
        ctl->clk_g[3] += g4 - g3;
        ctl->cnt_pend[t & 1] = sh->npend;
        const int nN = sh->nN;
        ctl->n_inside += nN;
        if (nN) ctl->last_insert = t;
        ctl->steps = t;
        if (ctl->status != 0) {
            ctl->done = 1;
        } else if (ctl->n_inside == m.nv) {
            ctl->done = 1;
        } else if (t - ctl->last_insert >= p.stall_steps || t >= p.max_steps) {
            ctl->status = ST_STALLED;
            ctl->done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// topology phase, small steps: the step's candidates, their closure rounds,
// classes and parents live in LDS; an LDS hash maps a vertex to its entry so
// that same-step neighbours are recognised without re-reading global keys
// ---------------------------------------------------------------------------
#define LCAP 2048            // candidates of the solo kernel's LDS topology path
#define LCAP_BATCH 1024      // the batched kernel's (two workgroups per CU)

template <int CAP>
struct KL {
    static constexpr int HCAP = 2 * CAP;      // hash slots (load factor <= 1/2)
    int32_t Lv[CAP];        // candidate vertex
    int32_t Lr[CAP];        // closure round (-1: not connected)
    int32_t Lc[CAP];        // lower arcs (-1: full link)
    int32_t Lp[CAP];        // parent vertex
    int32_t Lq[CAP];        // link position of the parent
    int32_t Lt[CAP];        // round 0: tag of the half-edge (parent -> v)
    int32_t Ld[CAP];        // round 0: depth of v
    uint64_t Lm[CAP];       // lower-neighbour mask (link positions < 64)
    int32_t Lb[CAP];        // first half-edge of v
    int32_t Lg[CAP];        // degree of v
    int32_t hk[HCAP];       // hash: vertex id (-1 empty)
    int32_t hv[HCAP];       // hash: entry index
};

// the dense field step borrows the LDS of the topology's sort buffer and
// tables (contiguous) for its wave slices
static_assert(LCAP_BATCH * sizeof(uint64_t) + sizeof(KL<LCAP_BATCH>) >= (NT / WAVE) * DSL * sizeof(int32_t),
              "dense field LDS slices");
static_assert((DSL * sizeof(int32_t)) % 16 == 0, "dense slices stay 16-byte aligned");

__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

template <int CAP>
__device__ __forceinline__ uint32_t hslot(int32_t x) {
    return ((uint32_t)x * 2654435761u) >> (32 - ilog2(KL<CAP>::HCAP));
}

template <int CAP>
__device__ __forceinline__ int hfind(const KL<CAP> *kl, int32_t x) {
    constexpr int HCAP = KL<CAP>::HCAP;
    uint32_t h = hslot<CAP>(x);
    for (int g = 0; g < HCAP; ++g) {
        const int32_t k = kl->hk[h];
        if (k == x) return kl->hv[h];
        if (k < 0) return -1;
        h = (h + 1) & (HCAP - 1);
    }
    return -1;
}

// gathers link positions [c0, c0+GB) of vertex x (counter-clockwise order)
// and the keys of those neighbours, as one batch each
__device__ __forceinline__ void gather_link(const DMesh &m, const uint64_t *key, int32_t b, int d, int c0,
                                            int32_t *nb, uint64_t *kn) {
#pragma unroll
    for (int j = 0; j < GB; ++j) nb[j] = c0 + j < d ? ldg(m.cyc + b + c0 + j) : -1;
#pragma unroll
    for (int j = 0; j < GB; ++j) kn[j] = nb[j] >= 0 ? ldg(key + nb[j]) : KEY_OUT;
}

// link row of x in one 64 B load: counter-clockwise neighbours from the
// smallest id (then -1) and the first half-edge of x in the last slot;
// false for a vertex wider than the row (its link is read through rp/cyc)
__device__ __forceinline__ bool load_lrow(const DMesh &m, int32_t x, int32_t *nb, int32_t &b, int &d) {
    const GLOBAL_AS v4i *row = (const GLOBAL_AS v4i *)(m.lrow + (int64_t)x * ELL_W);
    int32_t r[ELL_W];
#pragma unroll
    for (int q = 0; q < ELL_W / 4; ++q) {
        const v4i w = row[q];
        r[4 * q] = w.x; r[4 * q + 1] = w.y; r[4 * q + 2] = w.z; r[4 * q + 3] = w.w;
    }
    b = r[ELL_W - 1];
    if (r[0] < -1) return false;
    int n = 0;
#pragma unroll
    for (int j = 0; j < ELL_W - 1; ++j) {
        nb[j] = r[j];
        n += r[j] >= 0;
    }
    nb[ELL_W - 1] = -1;
    d = n;
    return true;
}

// the link of x (ids, then their keys) from its 64 B link row, for a vertex
// of at most ELL_W - 1 neighbours: four 16 B loads for the ids instead of
// one load per id (the topology workgroup's gathers are bound by the number
// of memory instructions its CU issues more than by their latency)
__device__ __forceinline__ void gather_link_row(const DMesh &m, const uint64_t *key, int32_t x, int32_t *nb,
                                                uint64_t *kn) {
    const GLOBAL_AS v4i *row = (const GLOBAL_AS v4i *)(m.lrow + (int64_t)x * ELL_W);
#pragma unroll
    for (int q = 0; q < ELL_W / 4; ++q) {
        const v4i w = row[q];
        nb[4 * q] = w.x; nb[4 * q + 1] = w.y; nb[4 * q + 2] = w.z; nb[4 * q + 3] = w.w;
    }
    nb[ELL_W - 1] = -1;   // that slot holds the first half-edge index
#pragma unroll
    for (int j = 0; j < GB; ++j) kn[j] = nb[j] >= 0 ? ldg(key + nb[j]) : KEY_OUT;
}

template <int CM, int CAP>
__device__ __forceinline__ void phase_topo_lds(const DMesh &m, const DState &s, const DParams &p, int64_t t,
                               KSh *sh, KL<CAP> *kl, uint64_t *lsort, int nc, int np) {
    constexpr int HCAP = KL<CAP>::HCAP;
    Ctl *ctl = s.ctl;
    const double *__restrict__ rho = (t & 1) ? s.rho1 : s.rho0;
    const int tid = threadIdx.x;
    const uint64_t tk = (uint64_t)t << 32;
    const unsigned long long k0 = DCLK();
    unsigned long long k1 = k0, k2 = k0, k3 = k0;
    for (int i = tid; i < HCAP; i += NT) kl->hk[i] = -1;
    if (tid == 0) { sh->nL = 0; sh->nN = 0; sh->nnew = 0; sh->event = 0; sh->npend = 0; }
    __syncthreads();
    // 1. candidates, de-duplicated through the hash, and closure round 0
    //    (touches the inside set of step t-1), fused: entry i is candidate i
    //    of the step's list (a repeat of an earlier candidate leaves a hole,
    //    Lv = -1), handled by the thread that reads it, whose link row is
    //    loaded together with the candidate's key.  The first entry of each
    //    thread keeps its link (ids and pre-step keys) in registers for the
    //    later rounds and the classification.
    const int32_t *cl = s.cand[t & 1];
    const int32_t *pl = s.pend[(t - 1) & 1];
    const int nL = nc + np;
    int n0 = 0, nhole = 0;
    int32_t cnb[GB];
    uint64_t ckn[GB];
    bool cached = false;
    for (int i = tid; i < nL; i += NT) {
        const int32_t x = i < nc ? ldx<CM>(cl + i) : pl[i - nc];
        // crossers of step t were checked against rho_t by the field phase;
        // pending ones are re-checked here
        const uint64_t kx = ldg(s.key + x);
        const double rx = i >= nc ? ldx<CM>(rho + x) : 1.0;
        int32_t nb[GB];
        int32_t b;
        int d;
        const bool row = load_lrow(m, x, nb, b, d);
        kl->Lv[i] = -1;
        kl->Lr[i] = -1;
        if (kx != KEY_OUT || !(rx > p.tau)) { nhole++; continue; }
        bool fresh = false;
        uint32_t h = hslot<CAP>(x);
        for (int g = 0; g < HCAP; ++g) {
            const int32_t old = atomicCAS(&kl->hk[h], -1, x);
            if (old == -1) { kl->hv[h] = i; fresh = true; break; }
            if (old == x) break;
            h = (h + 1) & (HCAP - 1);
        }
        if (!fresh) { nhole++; continue; }
        bool hit = false;
        if (row) {
            uint64_t kn[GB];
#pragma unroll
            for (int j = 0; j < GB; ++j) kn[j] = nb[j] >= 0 ? ldg(s.key + nb[j]) : KEY_OUT;
#pragma unroll
            for (int j = 0; j < GB; ++j) hit = hit || kn[j] < tk;
            // for the classification: which neighbours were inside before
            // step t (keys that this step does not change) and the
            // smallest-ranked of them, so that phase 3 needs no key loads;
            // kept in Lc (bit 24 marks it valid; phase 2 overwrites Lc)
            // until phase 3 replaces it with its own output
            uint32_t om = 0;
            int jm = 31;
            int32_t um = -1;
            uint64_t km = KEY_OUT;
#pragma unroll
            for (int j = 0; j < GB; ++j)
                if (nb[j] >= 0 && kn[j] < tk) {
                    om |= 1u << j;
                    if (um < 0 || rank_lt(kn[j], nb[j], km, um)) { jm = j; um = nb[j]; km = kn[j]; }
                }
            kl->Lc[i] = (int32_t)(om | ((uint32_t)jm << 16) | (1u << 24));
            if (i == tid) {
#pragma unroll
                for (int j = 0; j < GB; ++j) { cnb[j] = nb[j]; ckn[j] = kn[j]; }
                cached = true;
            }
        } else {
            d = ldg(m.rp + x + 1) - b;
            for (int c0 = 0; c0 < d; c0 += GB) {
                uint64_t kn[GB];
                gather_link(m, s.key, b, d, c0, nb, kn);
#pragma unroll
                for (int j = 0; j < GB; ++j) hit = hit || kn[j] < tk;
            }
        }
        kl->Lv[i] = x;
        kl->Lb[i] = b;
        kl->Lg[i] = d;
        kl->Lr[i] = hit ? 0 : -1;
        n0 += hit;
    }
    if (nhole) atomicAdd(&sh->nL, nhole);     // sh->nL counts the holes on this path
    k1 = DCLK();
    if (n0) atomicAdd(&sh->nN, n0);
    __syncthreads();
    const int nreal = nL - sh->nL;
    if (nreal == 0) {
        if (tid == 0) ctl->clk_t[0] += k1 - k0;
        return;
    }
    int nrounds = sh->nN ? 1 : 0;
    // later rounds (rare): touch the previous round, found through the hash
    if (sh->nN && sh->nN < nreal) {
        const unsigned long long kr = DCLK();
        for (int round = 1;; ++round) {
            for (int i = tid; i < nL; i += NT) {
                int flag = 0;
                if (kl->Lr[i] == -1 && kl->Lv[i] >= 0) {
                    if (i == tid && cached) {
#pragma unroll
                        for (int j = 0; j < GB; ++j) {
                            const int q = cnb[j] >= 0 ? hfind(kl, cnb[j]) : -1;
                            if (q >= 0 && kl->Lr[q] == round - 1) flag = 1;
                        }
                    } else {
                        const int32_t b = kl->Lb[i], e = b + kl->Lg[i];
                        for (int32_t j = b; j < e && !flag; ++j) {
                            const int q = hfind(kl, ldg(m.cyc + j));
                            if (q >= 0 && kl->Lr[q] == round - 1) flag = 1;
                        }
                    }
                }
                kl->Lc[i] = flag;
            }
            __syncthreads();
            int mine = 0;
            for (int i = tid; i < nL; i += NT)
                if (kl->Lc[i]) { kl->Lr[i] = round; mine++; }
            if (tid == 0) sh->nnew = 0;
            __syncthreads();
            if (mine) atomicAdd(&sh->nnew, mine);
            __syncthreads();
            const int nnew = sh->nnew;
            if (nnew == 0) break;
            nrounds = round + 1;
            __syncthreads();
            if (tid == 0) sh->nN += nnew;
            __syncthreads();
            if (sh->nN == nreal) break;
        }
        if (tid == 0) {
            ctl->clk_rounds += DCLK() - kr;
            ctl->n_round_steps += 1;
        }
    }
    __syncthreads();
    k2 = DCLK();
    // 3. lower-link classification: a neighbour is lower if it was inside
    //    before step t, or joined in this step with a smaller (round, id)
    for (int i = tid; i < nL; i += NT) {
        const int rv = kl->Lr[i];
        if (rv < 0) continue;
        const int32_t x = kl->Lv[i];
        const int32_t b = kl->Lb[i];
        const int d = kl->Lg[i];
        int nlow = 0, runs = 0, ppos = -1;
        int32_t par = -1;
        uint64_t kp = KEY_OUT;
        bool first = false, prev = false;
        uint64_t mask = 0;
        const int pc = kl->Lc[i];
        if (!(i == tid && cached) && d < ELL_W && ((pc >> 24) & 1)) {
            // phase 1 recorded the neighbours inside before step t and the
            // smallest-ranked of them (the parent when there is one: every
            // earlier vertex ranks below this step's); only the link's ids
            // are loaded, from its row
            int32_t nb[GB];
            {
                const GLOBAL_AS v4i *row = (const GLOBAL_AS v4i *)(m.lrow + (int64_t)x * ELL_W);
#pragma unroll
                for (int q = 0; q < ELL_W / 4; ++q) {
                    const v4i w = row[q];
                    nb[4 * q] = w.x; nb[4 * q + 1] = w.y; nb[4 * q + 2] = w.z; nb[4 * q + 3] = w.w;
                }
            }
            const uint32_t om = (uint32_t)pc & 0xffffu;
            const int jm = (pc >> 16) & 31;
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                if (j >= d) continue;
                const int32_t u = nb[j];
                bool low;
                uint64_t ku = KEY_OUT;
                if ((om >> j) & 1u) {
                    low = true;
                } else {
                    const int q = hfind(kl, u);
                    const int ru = q >= 0 ? kl->Lr[q] : -1;
                    low = ru >= 0 && (ru < rv || (ru == rv && u < x));
                    ku = tk | (uint64_t)(ru < 0 ? 0 : ru);
                }
                if (low) {
                    nlow++;
                    mask |= 1ull << j;
                    if (j > 0 && !prev) runs++;
                    if (jm != 31) {
                        if (j == jm) { par = u; ppos = j; }
                    } else if (par < 0 || rank_lt(ku, u, kp, par)) {
                        par = u; kp = ku; ppos = j;
                    }
                }
                if (j == 0) first = low;
                prev = low;
            }
        } else
        for (int c0 = 0; c0 < d; c0 += GB) {
            int32_t nb[GB];
            uint64_t kn[GB];
            if (i == tid && cached) {
#pragma unroll
                for (int j = 0; j < GB; ++j) { nb[j] = cnb[j]; kn[j] = ckn[j]; }
            } else if (d < ELL_W) {
                gather_link_row(m, s.key, x, nb, kn);
            } else {
                gather_link(m, s.key, b, d, c0, nb, kn);
            }
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                if (c0 + j >= d) continue;
                const int32_t u = nb[j];
                uint64_t ku = kn[j];
                bool low;
                if (ku < tk) {
                    low = true;
                } else {
                    const int q = hfind(kl, u);
                    const int ru = q >= 0 ? kl->Lr[q] : -1;
                    low = ru >= 0 && (ru < rv || (ru == rv && u < x));
                    ku = tk | (uint64_t)(ru < 0 ? 0 : ru);
                }
                if (low) {
                    nlow++;
                    if (c0 + j < 64) mask |= 1ull << (c0 + j);
                    if (c0 + j > 0 && !prev) runs++;
                    if (par < 0 || rank_lt(ku, u, kp, par)) { par = u; kp = ku; ppos = c0 + j; }
                }
                if (c0 + j == 0) first = low;
                prev = low;
            }
        }
        // a run starts at position 0 unless it continues from the last
        // position (cyclic link)
        if (first && !prev) runs++;
        const int cls = nlow == d ? -1 : runs;
        kl->Lc[i] = cls;
        kl->Lp[i] = par;
        kl->Lq[i] = ppos;
        kl->Lm[i] = mask;
        s.key[x] = tk | (uint64_t)rv;
        s.parent[x] = par;
        if (cls != 1) atomicOr(&sh->event, 1);
        if (nlow == 0 || d > MAXDEG) atomicOr(&sh->event, 2);
    }
    // the tag of the half-edge (parent -> x) and the depth of round-0
    // vertices, whose parents were inside before step t (both final
    // already): every entry of the thread at once, so its loads are two
    // round trips in all rather than two per entry (CAP / NT entries at most)
    {
        constexpr int PE = CAP / NT;
        int32_t he[PE], pp[PE], rh[PE], tg[PE], dp[PE];
#pragma unroll
        for (int q = 0; q < PE; ++q) {
            const int i = tid + q * NT;
            he[q] = -1;
            pp[q] = -1;
            if (i < nL && kl->Lr[i] == 0 && kl->Lq[i] >= 0) {
                he[q] = kl->Lb[i] + kl->Lq[i];
                pp[q] = kl->Lp[i];
            }
        }
#pragma unroll
        for (int q = 0; q < PE; ++q) rh[q] = he[q] >= 0 ? ldg(m.rev + he[q]) : -1;
#pragma unroll
        for (int q = 0; q < PE; ++q) {
            tg[q] = rh[q] >= 0 ? ldg(s.lid + rh[q]) : 0;
            dp[q] = pp[q] >= 0 ? ldg(s.depth + pp[q]) : 0;
        }
#pragma unroll
        for (int q = 0; q < PE; ++q)
            if (he[q] >= 0) {
                kl->Lt[tid + q * NT] = tg[q];
                kl->Ld[tid + q * NT] = dp[q] + 1;
            }
    }
    __syncthreads();
    k3 = DCLK();
    if (sh->event & 2) {
        if (tid == 0) fail(s, ST_INVARIANT, 12);
    } else if (!sh->event) {
        // 4a. all insertions regular: the new crossed half-edges take the
        //     tag of the half-edge (parent -> v), round by round
        for (int r = 0; r < nrounds; ++r) {
            for (int i = tid; i < nL; i += NT) {
                if (kl->Lr[i] != r) continue;
                const int32_t v = kl->Lv[i];
                const int32_t b = kl->Lb[i];
                const int d = kl->Lg[i];
                const int32_t par = kl->Lp[i];
                int32_t tag;
                if (r == 0) {
                    tag = kl->Lt[i];
                    s.depth[v] = kl->Ld[i];
                } else {
                    tag = ldg(s.lid + ldg(m.rev + b + kl->Lq[i]));
                    s.depth[v] = ldg(s.depth + par) + 1;
                }
                const uint64_t mask = kl->Lm[i];
                for (int j = 0; j < d; ++j)
                    if (!(mask >> j & 1ull)) s.lid[b + j] = tag;
            }
            __syncthreads();
        }
    } else {
        // 4b. events: rank order, regular runs in parallel, events by wave 0
        const int nN = sh->nN;
        int npow = 1;
        while (npow < nN) npow <<= 1;
        uint64_t *arr = npow <= CAP ? lsort : s.ord;
        for (int i = tid; i < npow; i += NT) arr[i] = ~0ull;
        __syncthreads();
        if (tid == 0) sh->nnew = 0;
        __syncthreads();
        // sort key: round (21 bits) | vertex (31) | table index (11) | event flag
        for (int i = tid; i < nL; i += NT) {
            if (kl->Lr[i] < 0) continue;
            const int slot = atomicAdd(&sh->nnew, 1);
            arr[slot] = ((uint64_t)kl->Lr[i] << 43) | ((uint64_t)kl->Lv[i] << 12) | ((uint64_t)i << 1) |
                        (uint64_t)(kl->Lc[i] != 1);
        }
        __syncthreads();
        block_bitonic(arr, npow);
        // breakpoints of the rank order: events and first entries of a round,
        // gathered in parallel, then ranked (few per step)
        if (tid == 0) sh->nbp = 0;
        __syncthreads();
        for (int i = tid; i < nN; i += NT)
            if ((arr[i] & 1ull) || (i > 0 && (arr[i] >> 43) != (arr[i - 1] >> 43))) {
                const int k = atomicAdd(&sh->nbp, 1);
                if (k < MAXBP) sh->bpu[k] = i;
            }
        __syncthreads();
        const int nbp = sh->nbp < MAXBP ? sh->nbp : MAXBP;
        const bool bp_ok = sh->nbp <= MAXBP;
        for (int i = tid; i < nbp; i += NT) {
            const int x = sh->bpu[i];
            int r = 0;
            for (int j = 0; j < nbp; ++j) r += sh->bpu[j] < x;
            sh->bps[r] = x;
        }
        __syncthreads();
        int pos = 0, kb = 0;
        while (pos < nN) {
            int q, a0 = pos, qr;
            if (bp_ok) {
                // next breakpoint at or after pos; regular entries of one
                // round lie between consecutive breakpoints
                while (kb < nbp && sh->bps[kb] < pos) kb++;
                qr = kb < nbp ? sh->bps[kb] : nN;
                if (qr == pos && !(arr[pos] & 1ull)) {
                    // a round starts here: its range runs to the next breakpoint
                    kb++;
                    qr = kb < nbp ? sh->bps[kb] : nN;
                }
                q = (qr < nN && (arr[qr] & 1ull)) ? qr : nN;
                if (qr < nN && !(arr[qr] & 1ull)) q = -1;     // round change, no event yet
            } else {
                q = pos;
                while (q < nN && !(arr[q] & 1ull)) q++;
                qr = q;
            }
            const int stop = q < 0 ? qr : q;
            while (a0 < stop) {
                const int r = (int)(arr[a0] >> 43);
                int a1 = stop;
                if (!bp_ok) {
                    a1 = a0;
                    while (a1 < stop && (int)(arr[a1] >> 43) == r) a1++;
                }
                // regular insertions from the classification tables; the tag
                // of (parent -> v) is read now (an earlier event of this step
                // may have relabelled it), and the parent is of an earlier
                // round, so its depth is final
                for (int i = a0 + tid; i < a1; i += NT) {
                    const int ix = (int)((arr[i] >> 1) & 0x7ffull);
                    const int32_t v = kl->Lv[ix];
                    const int32_t b = kl->Lb[ix];
                    const int d = kl->Lg[ix];
                    const int32_t par = kl->Lp[ix];
                    const int ppos = kl->Lq[ix];
                    const uint64_t mask = kl->Lm[ix];
                    const int32_t tag = ppos >= 0 ? ldg(s.lid + ldg(m.rev + b + ppos)) : -1;
                    s.depth[v] = par >= 0 ? ldg(s.depth + par) + 1 : 0;
                    for (int j = 0; j < d; ++j)
                        if (!(mask >> j & 1ull)) s.lid[b + j] = tag;
                }
                __syncthreads();
                a0 = a1;
            }
            if (q < 0) {
                pos = qr;              // continue with the next round
                continue;
            }
            if (q < nN) {
                if (tid < WAVE)
                    resolve_event<CM>(m, s, p, t, (int32_t)((arr[q] >> 12) & 0x7fffffffull), sh, rho);
                __syncthreads();
                if (ld_relaxed(&ctl->status) != 0) break;
            }
            pos = q + 1;
        }
        if (tid == 0) {
            ctl->event_steps += 1;
            ctl->clk_ev += DCLK() - k3;
        }
    }
    // 5. crossers not connected this step wait for the next
    for (int i = tid; i < nL; i += NT)
        if (kl->Lr[i] < 0 && kl->Lv[i] >= 0) s.pend[t & 1][atomicAdd(&sh->npend, 1)] = kl->Lv[i];
    __syncthreads();
    if (tid == 0) {
        const unsigned long long k4 = DCLK();
        ctl->clk_t[0] += k1 - k0;
        ctl->clk_t[1] += k2 - k1;
        ctl->clk_t[2] += k3 - k2;
        ctl->clk_t[3] += k4 - k3;
    }
}

template <int CM, int CAP>
__device__ __forceinline__ void phase_topo(const DMesh &m, const DState &s, const DParams &p, int64_t t,
                           KSh *sh, KL<CAP> *kl, uint64_t *lsort) {
    Ctl *ctl = s.ctl;
    const int nc = ld_relaxed(&ctl->cnt_cand[t & 3]);
    const int np = ctl->cnt_pend[(t - 1) & 1];
    if (p.topo_global || nc + np > CAP) {
        // the sort buffer and the candidate tables are contiguous in LDS
        constexpr int kSortCap = 1 << ilog2((int)((CAP * sizeof(uint64_t) + sizeof(KL<CAP>)) / sizeof(uint64_t)));
        phase_topo_global<CM, CAP>(m, s, p, t, sh, lsort, kSortCap);
        if (threadIdx.x == 0) ctl->n_global_steps += 1;
        return;
    }
    phase_topo_lds<CM, CAP>(m, s, p, t, sh, kl, lsort, nc, np);
    if (threadIdx.x == 0) {
        ctl->cnt_pend[t & 1] = sh->npend;
        const int nN = sh->nN;
        ctl->n_inside += nN;
        if (nN) ctl->last_insert = t;
        ctl->steps = t;
        if (ctl->status != 0) {
            ctl->done = 1;
        } else if (ctl->n_inside == m.nv) {
            ctl->done = 1;
        } else if (t - ctl->last_insert >= p.stall_steps || t >= p.max_steps) {
            ctl->status = ST_STALLED;
            ctl->done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// the persistent step kernel
// ---------------------------------------------------------------------------
template <int CM, bool FE = false>
__global__ void __launch_bounds__(NT) k_steps(DMesh m, DState s, DParams p) {
    extern __shared__ __align__(16) unsigned char lds[];
    const unsigned G = gridDim.x;
    unsigned long long epoch = 0;
    Ctl *ctl = s.ctl;
    KSh *ksh = (KSh *)lds;
    uint64_t *lsort = (uint64_t *)(lds + ((sizeof(KSh) + 15) & ~(size_t)15));
    KL<LCAP> *kl = (KL<LCAP> *)(lds + ((sizeof(KSh) + 15) & ~(size_t)15) + LCAP * sizeof(uint64_t));
    if (__hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    unsigned long long c_work = 0, c_wait = 0;
    for (int64_t j = 0;; ++j) {
        const unsigned long long c0 = __builtin_amdgcn_s_memrealtime();
        if (blockIdx.x == 0) {
            if (threadIdx.x == 0) {
                ctl->cnt_act[(j + 3) & 3] = 0;
                ctl->cnt_cand[(j + 2) & 3] = 0;
            }
            if (j >= 1) phase_topo<CM, LCAP>(m, s, p, j, ksh, kl, lsort);
            __syncthreads();
            // publish this iteration's decision in its own slot: the slot is
            // rewritten two iterations later, after every workgroup read it
            if (threadIdx.x == 0)
                ctl->stop[j & 1] = __hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (G == 1) {
                __syncthreads();
                if (FE) phase_field<CM, 1, true>(m, s, p, j + 1, 0, 1);
                else if (p.dense) phase_field_dense<CM>(m, s, p, j + 1, 0, 1, (LDS_AS int32_t *)lsort);
                else phase_field<CM>(m, s, p, j + 1, 0, 1);
            }
        } else {
            if (FE) phase_field<CM, 1, true>(m, s, p, j + 1, blockIdx.x - 1, G - 1);
            else if (p.dense) phase_field_dense<CM>(m, s, p, j + 1, blockIdx.x - 1, G - 1, (LDS_AS int32_t *)lsort);
            else phase_field<CM>(m, s, p, j + 1, blockIdx.x - 1, G - 1);
        }
        // field snapshots of step j (its buffer is not written in this iteration)
        for (int q = 0; q < s.n_ckpt; ++q) {
            if (s.ckpt_steps[q] != j || j == 0) continue;
            const double *src = (j & 1) ? s.rho1 : s.rho0;
            double *dst = s.ckpt + (int64_t)q * m.nv;
            const int nb = G > 1 ? G - 1 : 1;
            const int bi = G > 1 ? (int)blockIdx.x - 1 : 0;
            if (bi < 0) continue;
            for (int64_t i = (int64_t)bi * NT + threadIdx.x; i < m.nv; i += (int64_t)nb * NT) dst[i] = ldx<CM>(src + i);
        }
        const unsigned long long c1 = __builtin_amdgcn_s_memrealtime();
        grid_sync<CM>(ctl, G, epoch);
        const unsigned long long c2 = __builtin_amdgcn_s_memrealtime();
        c_work += c1 - c0;
        c_wait += c2 - c1;
        if (__hip_atomic_load(&ctl->stop[j & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
    if (threadIdx.x == 0 && blockIdx.x <= 1) {
        if (blockIdx.x == 0) { ctl->clk_topo = c_work; ctl->clk_wait0 = c_wait; }
        else { ctl->clk_field = c_work; ctl->clk_wait1 = c_wait; }
    }
}

// ---------------------------------------------------------------------------
// the decoupled step kernel: the field never depends on the fronts, so the
// field workgroups (1..G-1) step on with a barrier among themselves, while
// workgroup 0 runs the topology of step t as soon as field step t is
// complete.  Field step t rewrites the buffer of step t-2 and the crosser
// list of step t-2, so it waits until topology step t-2 is done: the field
// runs at most two steps ahead and never waits on the current topology.
// Every spin has a wall-clock bound that records an error instead of
// hanging.
// ---------------------------------------------------------------------------
#define SPIN_LIMIT 2000000000ull   // s_memrealtime ticks (100 MHz): 20 s
#define KDONE_STOP (1ll << 60)

__device__ __forceinline__ bool spin_ge(const unsigned long long *p, unsigned long long target, const DState &s) {
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_s_memrealtime() - t0 > SPIN_LIMIT) { fail(s, ST_INVARIANT, 20); return false; }
    }
    return true;
}
__device__ __forceinline__ bool spin_ge64(const long long *p, long long target, const DState &s) {
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_s_memrealtime() - t0 > SPIN_LIMIT) { fail(s, ST_INVARIANT, 21); return false; }
    }
    return true;
}

// Hand-off fences between a gang's workgroups.  CM = 0: plain accesses to
// shared data, so full agent-scope fences (release writes back the L2,
// acquire invalidates it: the XCDs' L2s are not coherent with each other).
// CM = 1: shared data moves through agent-scope atomics, so the release only
// writes back the topology's plain stores and the acquire is an ordering
// point; no L2 is invalidated, which keeps the caches of every other
// workgroup on the XCD warm.
template <int CM> __device__ __forceinline__ void hand_off_acquire() {
    if constexpr (CM) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    else __threadfence();
}
template <int CM> __device__ __forceinline__ void hand_off_release() {
    if constexpr (CM) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    else __threadfence();
}

// One mesh advanced by a gang of G >= 2 co-resident workgroups: rank 0 runs
// the topology, ranks 1..G-1 the field.  Entry state: iterations below j0
// complete (topology j0-1 and field j0 done), fbar = 0, kdone <= j0-1,
// stop_step = LLONG_MAX.  Field step t waits for topology t-2 (it rewrites
// that step's field buffer and crosser list) and for field t-1 on every
// field workgroup; topology t waits for field t.  Rank 0 stops after a
// topology step once the mesh is done or the visit has used budget ticks
// of s_memrealtime; the field then completes exactly one more step, so the
// exit state is again "iterations below t+1 complete".  Rank 0 returns the
// next iteration.  Every wait is bounded (an overrun records an error).
template <int CM, int CAP, int FK, bool FE = false>
__device__ __forceinline__ int64_t gang_advance(const DMesh &m, const DState &s, const DParams &p, int rank, int G,
                                                int64_t j0, unsigned long long budget, KSh *ksh, KL<CAP> *kl,
                                                uint64_t *lsort, int &go) {
    const unsigned long long W = (unsigned long long)(G - 1);       // field workgroups
    Ctl *ctl = s.ctl;
    const unsigned long long v0 = __builtin_amdgcn_s_memrealtime();
    unsigned long long c_work = 0, c_wait = 0;
    if (rank == 0) {
        int64_t next = j0;
        for (int64_t t = j0 < 1 ? 1 : j0;; ++t) {
            const unsigned long long c0 = __builtin_amdgcn_s_memrealtime();
            if (threadIdx.x == 0) {
                go = spin_ge(&ctl->fbar, (unsigned long long)(t - j0) * W, s) ? 1 : 0;
                hand_off_acquire<CM>();
            }
            __syncthreads();
            const unsigned long long c1 = __builtin_amdgcn_s_memrealtime();
            if (go) phase_topo<CM, CAP>(m, s, p, t, ksh, kl, lsort);
            __syncthreads();
            if (threadIdx.x == 0) {
                const int d = __hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || !go;
                const int y = !d && __builtin_amdgcn_s_memrealtime() - v0 >= budget;
                hand_off_release<CM>();
                if (d || y) {
                    // the stop step becomes visible before the jump of kdone
                    __hip_atomic_store(&ctl->stop_step, (long long)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    hand_off_release<CM>();
                    __hip_atomic_store(&ctl->kdone, KDONE_STOP, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    __hip_atomic_store(&ctl->kdone, (long long)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                go = d || y;
            }
            __syncthreads();
            const unsigned long long c2 = __builtin_amdgcn_s_memrealtime();
            c_wait += c1 - c0;
            c_work += c2 - c1;
            if (go) { next = t + 1; break; }
        }
        if (threadIdx.x == 0) { ctl->clk_topo += c_work; ctl->clk_wait0 += c_wait; }
        return next;
    }
    const int worker = rank - 1;
    unsigned long long c_bar = 0;
    for (int64_t t = j0 + 1;; ++t) {
        const unsigned long long c0 = __builtin_amdgcn_s_memrealtime();
        if (threadIdx.x == 0) {
            // topology t-2 done (its field buffer and crosser list are free)
            int ok = spin_ge64(&ctl->kdone, t - 2, s);
            hand_off_acquire<CM>();
            const long long stop = __hip_atomic_load(&ctl->stop_step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!ok || stop <= t - 2) {
                go = 0;
            } else {
                // field step t-1 complete on every field workgroup
                const unsigned long long cb = DCLK();
                ok = spin_ge(&ctl->fbar, (unsigned long long)(t - 1 - j0) * W, s);
                hand_off_acquire<CM>();
                c_bar += DCLK() - cb;
                go = ok;
            }
            if (go && worker == 0) {
                ctl->cnt_act[(t + 2) & 3] = 0;
                ctl->cnt_cand[(t + 2) & 3] = 0;
            }
        }
        __syncthreads();
        const unsigned long long c1 = __builtin_amdgcn_s_memrealtime();
        if (!go) break;
        if (FE) phase_field<CM, FK, true>(m, s, p, t, worker, (int)W);
        else if (p.dense) phase_field_dense<CM>(m, s, p, t, worker, (int)W, (LDS_AS int32_t *)lsort);
        else phase_field<CM, FK>(m, s, p, t, worker, (int)W);
        // field snapshot of step t-1 (its buffer is not written by step t)
        for (int q = 0; q < s.n_ckpt; ++q) {
            if (s.ckpt_steps[q] != t - 1 || t == 1) continue;
            const double *src = ((t - 1) & 1) ? s.rho1 : s.rho0;
            double *dst = s.ckpt + (int64_t)q * m.nv;
            for (int64_t i = (int64_t)worker * NT + threadIdx.x; i < m.nv; i += (int64_t)W * NT) dst[i] = ldx<CM>(src + i);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            hand_off_release<CM>();
            atomicAdd(&ctl->fbar, 1ull);
        }
        const unsigned long long c2 = __builtin_amdgcn_s_memrealtime();
        c_wait += c1 - c0;
        c_work += c2 - c1;
    }
    if (threadIdx.x == 0 && worker == 0) {
        ctl->clk_field += c_work;
        ctl->clk_wait1 += c_wait - c_bar;
        ctl->clk_fbar += c_bar;
    }
    return 0;
}

// the decoupled step kernel of one mesh: the whole grid is one gang
template <int CM, bool FE = false>
__global__ void __launch_bounds__(NT) k_steps_dec(DMesh m, DState s, DParams p) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int go;
    KSh *ksh = (KSh *)lds;
    uint64_t *lsort = (uint64_t *)(lds + ((sizeof(KSh) + 15) & ~(size_t)15));
    KL<LCAP> *kl = (KL<LCAP> *)(lds + ((sizeof(KSh) + 15) & ~(size_t)15) + LCAP * sizeof(uint64_t));
    if (__hip_atomic_load(&s.ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    (void)gang_advance<CM, LCAP, FE ? 1 : 2, FE>(m, s, p, (int)blockIdx.x, (int)gridDim.x, 0, ~0ull, ksh, kl, lsort,
                                                  go);
}

// ---------------------------------------------------------------------------
// batched mode: many meshes in one launch
// ---------------------------------------------------------------------------
// Batched mode: a cooperative pool of workgroups takes slots from a shared
// counter; slot k names a task (a mesh) and a rank in that task's gang.
// A task of one workgroup runs the topology of step j and the field of
// step j+1 back to back; a gang of g >= 2 runs the decoupled protocol
// (gang_advance).  Gang slots come first in the slot list and fit in the
// pool, so every gang's members are running together.  A visit ends when
// the mesh is done or, at a step boundary, once it has used budget_ticks of
// s_memrealtime (100 MHz); the next iteration is kept in the mesh's control
// block (biter), so a later launch, with any gang size, continues it with
// the same arithmetic.  done_out[task] reports each visited mesh's state.
__device__ __forceinline__ void zero_dead_counters(Ctl *ctl, int64_t j0) {
    // counters the field steps j0+1 and j0+2 append to; their previous
    // contents were consumed by steps below j0
    ctl->cnt_act[(j0 + 2) & 3] = 0;
    ctl->cnt_act[(j0 + 3) & 3] = 0;
    ctl->cnt_cand[(j0 + 1) & 3] = 0;
    ctl->cnt_cand[(j0 + 2) & 3] = 0;
}

// OCC workgroups per CU: OCC = 1 keeps the solo kernel's LDS topology path
// (LCAP candidates) and two list entries per field thread; OCC = 2 halves
// both (LCAP_BATCH, one entry) so that two workgroups overlap on each CU.
template <int OCC, int CM>
__global__ void __launch_bounds__(NT, OCC) k_batch(const DMesh *ms, const DState *ss, const DParams *ps,
                                              const int32_t *order, const int32_t *task_g, const int32_t *slots,
                                              int nslots, int *next_slot, unsigned long long budget_ticks,
                                              int32_t *done_out, unsigned int epoch) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int cur, yield, go;
    __shared__ long long jstart;
    KSh *ksh = (KSh *)lds;
    uint64_t *lsort = (uint64_t *)(lds + ((sizeof(KSh) + 15) & ~(size_t)15));
    constexpr int CAP = OCC == 2 ? LCAP_BATCH : LCAP;
    constexpr int FKB = OCC == 2 ? 1 : 2;
    KL<CAP> *kl = (KL<CAP> *)(lds + ((sizeof(KSh) + 15) & ~(size_t)15) + CAP * sizeof(uint64_t));
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(next_slot, 1);
        __syncthreads();
        const int k = cur;
        __syncthreads();
        if (k >= nslots) break;
        const int w = slots[2 * k], rank = slots[2 * k + 1];
        const int mi = order[w];
        const int g = task_g[w];
        // descriptors read in place (uniform loads); a local copy would be
        // spilled to scratch because of its per-parity pointer arrays
        const DMesh &m = ms[mi];
        const DState &s = ss[mi];
        const DParams &p = ps[mi];
        Ctl *ctl = s.ctl;
        const unsigned long long c_start = __builtin_amdgcn_s_memrealtime();
        if (g >= 2) {
            // gang hand-off: rank 0 sets this visit's counters, then opens it
            if (threadIdx.x == 0) {
                if (rank == 0) {
                    const int64_t j0 = ctl->biter;
                    const int skip = ctl->done;
                    ctl->fbar = 0;
                    ctl->kdone = j0 - 1;
                    ctl->stop_step = skip ? -1 : LLONG_MAX;
                    ctl->vbase = j0;
                    if (!skip) zero_dead_counters(ctl, j0);
                    jstart = skip ? -1 : j0;
                    __threadfence();
                    __hip_atomic_store(&ctl->gang_epoch, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
                    while (__hip_atomic_load(&ctl->gang_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                        __builtin_amdgcn_s_sleep(1);
                        if (__builtin_amdgcn_s_memrealtime() - t0 > SPIN_LIMIT) { fail(s, ST_INVARIANT, 22); break; }
                    }
                    __threadfence();
                    jstart = __hip_atomic_load(&ctl->gang_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch
                                 ? __hip_atomic_load(&ctl->vbase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
                }
            }
            __syncthreads();
            const long long j0 = jstart;
            if (rank == 0 && j0 < 0) {
                if (threadIdx.x == 0 && done_out) done_out[w] = 1;
            } else if (rank != 0 && j0 < 0) {
                // the visit never opened (error already recorded) or the mesh is done
            } else {
                const int64_t nx = gang_advance<CM, CAP, FKB>(m, s, p, rank, g, j0, budget_ticks, ksh, kl, lsort, go);
                if (rank == 0 && threadIdx.x == 0) {
                    ctl->biter = nx;
                    if (done_out) done_out[w] = ctl->done;
                }
            }
            __syncthreads();
            continue;
        }
        if (!ctl->done) {
            const int64_t j0 = ctl->biter;
            if (threadIdx.x == 0) zero_dead_counters(ctl, j0);
            for (int64_t j = j0;; ++j) {
                if (threadIdx.x == 0)
                    yield = j > j0 && __builtin_amdgcn_s_memrealtime() - c_start >= budget_ticks;
                __syncthreads();
                if (yield) {
                    if (threadIdx.x == 0) ctl->biter = j;
                    break;
                }
                if (threadIdx.x == 0) {
                    ctl->cnt_act[(j + 3) & 3] = 0;
                    ctl->cnt_cand[(j + 2) & 3] = 0;
                }
                __syncthreads();
                if (j >= 1) phase_topo<0, CAP>(m, s, p, j, ksh, kl, lsort);
                // field snapshot of step j (complete since the previous
                // iteration; step j+1 writes the other buffer), taken before
                // the stop test so that the last step's snapshot is kept too
                for (int q = 0; q < s.n_ckpt; ++q) {
                    if (s.ckpt_steps[q] != j || j == 0) continue;
                    const double *src = (j & 1) ? s.rho1 : s.rho0;
                    double *dst = s.ckpt + (int64_t)q * m.nv;
                    for (int64_t i = threadIdx.x; i < m.nv; i += NT) dst[i] = src[i];
                }
                __syncthreads();
                const int stop = ctl->done;
                __syncthreads();
                if (stop) break;
                if (p.dense) phase_field_dense<0>(m, s, p, j + 1, 0, 1, (LDS_AS int32_t *)lsort);
                else phase_field<0, FKB>(m, s, p, j + 1, 0, 1);
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) {
            ctl->clk_topo += __builtin_amdgcn_s_memrealtime() - c_start;
            if (done_out) done_out[w] = ctl->done;
        }
        __syncthreads();
    }
}

hipError_t launch_batch(const DMesh *ms, const DState *ss, const DParams *ps, const int32_t *order,
                        const int32_t *task_g, const int32_t *slots, int nslots, int *next_slot, int grid, size_t lds,
                        unsigned long long budget_ticks, int32_t *done_out, unsigned int epoch, int occ, int cm,
                        hipStream_t st) {
    void *args[] = {&ms, &ss, &ps, &order, &task_g, &slots, &nslots, &next_slot, &budget_ticks, &done_out, &epoch};
    const void *fn = occ == 2 ? (cm ? (const void *)k_batch<2, 1> : (const void *)k_batch<2, 0>)
                              : (cm ? (const void *)k_batch<1, 1> : (const void *)k_batch<1, 0>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(NT), args, (unsigned)lds, st);
}

int max_coresident_batch(size_t lds_bytes, int occ) {
    // the smaller residency of the two sharing modes
    int per_cu = 1 << 30;
    const void *fns[2] = {occ == 2 ? (const void *)k_batch<2, 0> : (const void *)k_batch<1, 0>,
                          occ == 2 ? (const void *)k_batch<2, 1> : (const void *)k_batch<1, 1>};
    for (const void *fn : fns) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, NT, lds_bytes) != hipSuccess) return 0;
        per_cu = n < per_cu ? n : per_cu;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

// ---------------------------------------------------------------------------
// the finite-element operator of a mesh (Section "Mathematical representation
// and data structure", "Implementation details": linear finite elements):
// lumped masses m_v = (sum of the areas of v's triangles, counter-clockwise
// from the smallest neighbour) / 3; cotangent weights k_vu = (cot at the
// link successor a of u + cot at its predecessor b) / 2, the angles facing
// the edge vu; sigma = sqrt(3) * (sum of the masses in id order) / nv, so
// that on equilateral meshes of one valence every coefficient is 1;
// coefficient g = (sigma * k_vu) / m_v per half-edge in ascending-neighbour
// order; the explicit step takes the largest absolute row sum.  Every
// expression is evaluated in the order written, without contraction, and
// every sum runs in the order stated, so the coefficients are the same bits
// wherever they are computed that way.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fem_tri_area(const double *x, int64_t v, int64_t p, int64_t q) {
    const double e0 = x[3 * p] - x[3 * v], e1 = x[3 * p + 1] - x[3 * v + 1], e2 = x[3 * p + 2] - x[3 * v + 2];
    const double f0 = x[3 * q] - x[3 * v], f1 = x[3 * q + 1] - x[3 * v + 1], f2 = x[3 * q + 2] - x[3 * v + 2];
    const double c0 = e1 * f2 - e2 * f1, c1 = e2 * f0 - e0 * f2, c2 = e0 * f1 - e1 * f0;
    return 0.5 * sqrt((c0 * c0 + c1 * c1) + c2 * c2);
}

// cotangent of the angle at `apex` between its edges to v and to u
__device__ __forceinline__ double fem_cot(const double *x, int64_t apex, int64_t v, int64_t u) {
    const double p0 = x[3 * v] - x[3 * apex], p1 = x[3 * v + 1] - x[3 * apex + 1], p2 = x[3 * v + 2] - x[3 * apex + 2];
    const double q0 = x[3 * u] - x[3 * apex], q1 = x[3 * u + 1] - x[3 * apex + 1], q2 = x[3 * u + 2] - x[3 * apex + 2];
    const double dot = (p0 * q0 + p1 * q1) + p2 * q2;
    const double c0 = p1 * q2 - p2 * q1, c1 = p2 * q0 - p0 * q2, c2 = p0 * q1 - p1 * q0;
    return dot / sqrt((c0 * c0 + c1 * c1) + c2 * c2);
}

__global__ void k_fem_mass(DMesh m, double *mass) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m.nv) return;
    const int32_t b0 = m.rp[v], d = m.rp[v + 1] - b0;
    double S = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        const int32_t k1 = k + 1 < d ? k + 1 : 0;
        S = S + fem_tri_area(m.xyz, v, m.cyc[b0 + k], m.cyc[b0 + k1]);
    }
    mass[v] = S / 3.0;
}

// one lane: the masses summed in id order (the order fixes the bits)
__global__ void k_fem_sigma(const double *mass, int64_t nv, double *scal) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double T = 0.0;
    for (int64_t v = 0; v < nv; ++v) T = T + mass[v];
    scal[0] = (sqrt(3.0) * T) / (double)nv;
}

__global__ void k_fem_coef(DMesh m, const double *mass, const double *scal, double *g,
                           unsigned long long *dmax_bits) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m.nv) return;
    const double sigma = scal[0];
    const int32_t b0 = m.rp[v], d = m.rp[v + 1] - b0;
    double D = 0.0;
    for (int32_t i = b0; i < b0 + d; ++i) {
        const int32_t u = m.adj[i];
        int32_t k = 0;
        while (k < d - 1 && m.cyc[b0 + k] != u) ++k;
        const int32_t a = m.cyc[b0 + (k + 1 < d ? k + 1 : 0)], b = m.cyc[b0 + (k > 0 ? k - 1 : d - 1)];
        const double kvu = 0.5 * (fem_cot(m.xyz, a, v, u) + fem_cot(m.xyz, b, v, u));
        const double gi = (sigma * kvu) / mass[v];
        g[i] = gi;
        D = D + fabs(gi);
    }
    // non-negative doubles order as their bit patterns
    atomicMax(dmax_bits, (unsigned long long)__double_as_longlong(D));
}

hipError_t launch_fem_operator(const DMesh &m, double *mass, double *scal, double *g,
                               unsigned long long *dmax_bits, hipStream_t st) {
    const unsigned blocks = (unsigned)((m.nv + NT - 1) / NT);
    hipLaunchKernelGGL(k_fem_mass, dim3(blocks), dim3(NT), 0, st, m, mass);
    hipLaunchKernelGGL(k_fem_sigma, dim3(1), dim3(64), 0, st, (const double *)mass, (int64_t)m.nv, scal);
    hipLaunchKernelGGL(k_fem_coef, dim3(blocks), dim3(NT), 0, st, m, (const double *)mass, (const double *)scal, g,
                       dmax_bits);
    return hipGetLastError();
}

// dynamic LDS of the solo step kernels: topology tables of LCAP candidates
size_t step_lds_bytes(int block, int dmax) {
    (void)block;
    (void)dmax;
    return ((sizeof(KSh) + 15) & ~(size_t)15) + LCAP * sizeof(uint64_t) + sizeof(KL<LCAP>);
}

// dynamic LDS of the batched kernel: LCAP candidates with one workgroup per
// CU, LCAP_BATCH with two
size_t batch_lds_bytes(int occ) {
    if (occ != 2) return ((sizeof(KSh) + 15) & ~(size_t)15) + LCAP * sizeof(uint64_t) + sizeof(KL<LCAP>);
    return ((sizeof(KSh) + 15) & ~(size_t)15) + LCAP_BATCH * sizeof(uint64_t) + sizeof(KL<LCAP_BATCH>);
}

int max_coresident_blocks(int block, size_t lds_bytes) {
    // the smallest residency over every variant the launcher may pick
    const void *fns[8] = {(const void *)k_steps<0>, (const void *)k_steps<1>, (const void *)k_steps_dec<0>,
                          (const void *)k_steps_dec<1>, (const void *)k_steps<0, true>,
                          (const void *)k_steps<1, true>, (const void *)k_steps_dec<0, true>,
                          (const void *)k_steps_dec<1, true>};
    int per_cu = 1 << 30;
    for (const void *f : fns) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds_bytes) != hipSuccess) return 0;
        per_cu = n < per_cu ? n : per_cu;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

hipError_t launch_steps(const DMesh &m, const DState &s, const DParams &p, int grid, int block,
                        hipStream_t st) {
    const size_t lds = step_lds_bytes(block, m.dmax);
    DMesh mm = m;
    DState ss = s;
    DParams pp = p;
    void *args[] = {&mm, &ss, &pp};
    const void *fn;
    if (p.fem) {
        if (p.lockstep || grid < 2) fn = p.coherent ? (const void *)k_steps<1, true> : (const void *)k_steps<0, true>;
        else fn = p.coherent ? (const void *)k_steps_dec<1, true> : (const void *)k_steps_dec<0, true>;
    } else if (p.lockstep || grid < 2) {
        fn = p.coherent ? (const void *)k_steps<1> : (const void *)k_steps<0>;
    } else {
        fn = p.coherent ? (const void *)k_steps_dec<1> : (const void *)k_steps_dec<0>;
    }
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds, st);
}

// ---------------------------------------------------------------------------
// post-pass: Reeb node positions = mean of the distinct vertices of the
// front triangles of the involved loops just before the event vertex joins,
// summed in ascending vertex id
// ---------------------------------------------------------------------------
// Count pass: one wave per event, one lane per involved loop.  Each lane
// walks its loop once (inside set {rank < rank(v)}) and keeps up to RCK
// checkpoints at a power-of-two stride, so the fill pass re-walks short
// segments in parallel.  meta[ev][q] = {length, stride, checkpoints, offset
// of the loop's entries}; cnt[ev] = 3 * total length.
#define RCK 64
// event ev of the mesh (m, s); its outputs at index rel of cnt, ck, meta
__device__ __forceinline__ void reeb_count_one(const DMesh &m, const DState &s, int ev, int64_t rel, int64_t *cnt,
                                               int32_t *ck, int64_t *meta) {
    const int lane = threadIdx.x;
    const int64_t *rec = s.ev + 16 * (int64_t)ev;
    const int32_t v = (int32_t)rec[1];
    const int sN = (int)rec[4];
    const uint64_t kv = s.key[v];
    const int32_t b = m.rp[v];
    int64_t n = 0;
    if (lane < sN && lane < 16) {
        int32_t *cq = ck + (rel * 16 + lane) * RCK;
        const int32_t e0 = m.rev[b + s.ev_rep[16 * (int64_t)ev + lane]];
        Walk w = walk_at(m, e0);
        long long K = 1;
        int nck = 0;
        do {
            if ((n & (K - 1)) == 0) {
                if (nck == RCK) {
                    for (int c = 0; c < RCK / 2; ++c) cq[c] = cq[2 * c];
                    nck = RCK / 2;
                    K *= 2;
                }
                if ((n & (K - 1)) == 0) cq[nck++] = w.e;
            }
            n++;
            walk_step(m, s.key, w, kv, v, false);
        } while (w.e != e0 && n <= m.nnz);
        int64_t *mq = meta + (rel * 16 + lane) * 4;
        mq[0] = n;
        mq[1] = K;
        mq[2] = nck;
    }
    // loop offsets: exclusive prefix of the lengths over the lanes
    int64_t inc = n;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane < sN && lane < 16) meta[(rel * 16 + lane) * 4 + 3] = inc - n;
    if (lane == 63) cnt[rel] = 3 * inc;
}

__global__ void k_reeb_count(DMesh m, DState s, int ev0, int n_events, int64_t *cnt, int32_t *ck, int64_t *meta) {
    // events ev0 .. ev0+n_events-1; cnt, ck, meta indexed from ev0
    if ((int)blockIdx.x >= n_events) return;
    reeb_count_one(m, s, ev0 + (int)blockIdx.x, blockIdx.x, cnt, ck, meta);
}

// many meshes' events in one launch: entry g is event eve[g] of mesh evm[g]
__global__ void k_reeb_count_multi(const DMesh *ms, const DState *ss, const int32_t *evm, const int32_t *eve, int n,
                                   int64_t *cnt, int32_t *ck, int64_t *meta) {
    const int g = (int)blockIdx.x;
    if (g >= n) return;
    const int i = evm[g];
    reeb_count_one(ms[i], ss[i], eve[g], g, cnt, ck, meta);
}

// Fill pass: a workgroup per event; every (loop, checkpoint) segment is
// re-walked by one thread, writing the three vertices of each front
// triangle; then the segment's padding up to its power of two.  The order
// of the entries does not matter (they are sorted before the mean).
// Events ev0 .. ev0+n_events-1: off[] (n_events+1 entries) is relative to
// this launch, cnt/ck/meta are the count pass's arrays shifted to ev0.
__device__ __forceinline__ void reeb_fill_one(const DMesh &m, const DState &s, int ev, int64_t rel, const int64_t *off,
                                              const int64_t *cnt, const int32_t *ck, const int64_t *meta,
                                              int32_t *buf) {
    const int64_t *rec = s.ev + 16 * (int64_t)ev;
    const int32_t v = (int32_t)rec[1];
    const int sN = (int)rec[4] < 16 ? (int)rec[4] : 16;
    const uint64_t kv = s.key[v];
    int32_t *out = buf + off[rel];
    for (int sg = threadIdx.x; sg < sN * RCK; sg += blockDim.x) {
        const int q = sg / RCK, c = sg % RCK;
        const int64_t *mq = meta + (rel * 16 + q) * 4;
        if (c >= (int)mq[2]) continue;
        const int64_t nq = mq[0], Kq = mq[1], base = mq[3];
        Walk w = walk_at(m, ck[(rel * 16 + q) * RCK + c]);
        const int64_t i0 = (int64_t)c * Kq;
        const int64_t i1 = i0 + Kq < nq ? i0 + Kq : nq;
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t o = 3 * (base + i);
            out[o] = w.src;
            out[o + 1] = w.r.w;
            out[o + 2] = w.r.z;
            walk_step(m, s.key, w, kv, v, false);
        }
    }
    for (int64_t i = off[rel] + cnt[rel] + threadIdx.x; i < off[rel + 1]; i += blockDim.x) buf[i] = 0x7fffffff;
}

__global__ void k_reeb_fill(DMesh m, DState s, int ev0, int n_events, const int64_t *off, const int64_t *cnt,
                            const int32_t *ck, const int64_t *meta, int32_t *buf) {
    if ((int)blockIdx.x >= n_events) return;
    reeb_fill_one(m, s, ev0 + (int)blockIdx.x, blockIdx.x, off, cnt, ck, meta, buf);
}

// entries g0 .. g0+n-1 of a multi-mesh event list; off (n+1 entries) is
// relative to g0, cnt / ck / meta are the count pass's arrays shifted to g0
__global__ void k_reeb_fill_multi(const DMesh *ms, const DState *ss, const int32_t *evm, const int32_t *eve, int g0,
                                  int n, const int64_t *off, const int64_t *cnt, const int32_t *ck,
                                  const int64_t *meta, int32_t *buf) {
    const int rel = (int)blockIdx.x;
    if (rel >= n) return;
    const int i = evm[g0 + rel];
    reeb_fill_one(ms[i], ss[i], eve[g0 + rel], rel, off, cnt, ck, meta, buf);
}

template <typename K>
__device__ void block_bitonic_t(K *a, int64_t np) {
    for (int64_t k = 2; k <= np; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t i = threadIdx.x; i < np; i += NT) {
                const int64_t ixj = i ^ j;
                if (ixj > i) {
                    const K x = a[i], y = a[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) { a[i] = y; a[ixj] = x; }
                }
            }
            __syncthreads();
        }
    }
}

#define MEANCAP 16384
// Reeb positions of n_events events: entry ev's mesh positions are
// xyz_of(ev) (one mesh, or the mesh of entry ev of a multi-mesh list)
template <typename XyzOf>
__device__ __forceinline__ void reeb_mean_all(XyzOf xyz_of, int n_events, const int64_t *off, const int64_t *cnt,
                                              int32_t *buf, double *pos, uint32_t *a) {
    for (int ev = blockIdx.x; ev < n_events; ev += gridDim.x) {
        const double *xyz = xyz_of(ev);
        const int64_t o = off[ev], np = off[ev + 1] - off[ev], n = cnt[ev];
        uint32_t *arr;
        if (np <= MEANCAP) {
            for (int64_t i = threadIdx.x; i < np; i += NT) a[i] = (uint32_t)buf[o + i];
            __syncthreads();
            arr = a;
        } else {
            arr = (uint32_t *)(buf + o);
        }
        block_bitonic_t<uint32_t>(arr, np);
        // wave 0 sums the distinct ids' positions in ascending id order: each
        // lane gathers one entry of a 64-entry chunk (64 loads in flight),
        // then every lane adds the chunk's values in lane order from
        // shuffles, so the sum's order, and its bits, are those of one lane
        // walking the sorted list
        if (threadIdx.x < WAVE) {
            const int lane = (int)threadIdx.x;
            double sx = 0.0, sy = 0.0, sz = 0.0;
            long long c = 0;
            for (int64_t c0 = 0; c0 < n; c0 += WAVE) {
                const int64_t i = c0 + lane;
                bool first = false;
                double x0 = 0.0, x1 = 0.0, x2 = 0.0;
                if (i < n) {
                    first = i == 0 || arr[i] != arr[i - 1];
                    if (first) {
                        const double *x = xyz + 3 * (int64_t)arr[i];
                        x0 = x[0];
                        x1 = x[1];
                        x2 = x[2];
                    }
                }
                const unsigned long long fm = __ballot(first);
                for (int l = 0; l < WAVE; ++l) {
                    const double y0 = __shfl(x0, l), y1 = __shfl(x1, l), y2 = __shfl(x2, l);
                    if ((fm >> l) & 1ull) {
                        sx = sx + y0;
                        sy = sy + y1;
                        sz = sz + y2;
                        c++;
                    }
                }
            }
            if (lane == 0) {
                pos[3 * ev] = sx / (double)c;
                pos[3 * ev + 1] = sy / (double)c;
                pos[3 * ev + 2] = sz / (double)c;
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NT) k_reeb_mean(DMesh m, int n_events, const int64_t *off,
                                                   const int64_t *cnt, int32_t *buf, double *pos) {
    __shared__ uint32_t a[MEANCAP];
    const double *xyz = m.xyz;
    reeb_mean_all([=](int) { return xyz; }, n_events, off, cnt, buf, pos, a);
}

__global__ void __launch_bounds__(NT) k_reeb_mean_multi(const DMesh *ms, const int32_t *evm, int g0, int n,
                                                         const int64_t *off, const int64_t *cnt, int32_t *buf,
                                                         double *pos) {
    __shared__ uint32_t a[MEANCAP];
    reeb_mean_all([=](int ev) { return ms[evm[g0 + ev]].xyz; }, n, off, cnt, buf, pos, a);
}

hipError_t launch_reeb_count(const DMesh &m, const DState &s, int ev0, int n_events, int64_t *cnt, int32_t *ck,
                             int64_t *meta, hipStream_t st) {
    if (n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reeb_count, dim3(n_events), dim3(64), 0, st, m, s, ev0, n_events, cnt, ck, meta);
    return hipGetLastError();
}
hipError_t launch_reeb_fill(const DMesh &m, const DState &s, int ev0, int n_events, const int64_t *off,
                            const int64_t *cnt, const int32_t *ck, const int64_t *meta, int32_t *buf,
                            hipStream_t st) {
    if (n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reeb_fill, dim3(n_events), dim3(NT), 0, st, m, s, ev0, n_events, off, cnt, ck, meta, buf);
    return hipGetLastError();
}
hipError_t launch_reeb_mean(const DMesh &m, int n_events, const int64_t *off, const int64_t *cnt,
                            int32_t *buf, double *pos, hipStream_t st) {
    if (n_events <= 0) return hipSuccess;
    int blocks = n_events < 1024 ? n_events : 1024;
    hipLaunchKernelGGL(k_reeb_mean, dim3(blocks), dim3(NT), 0, st, m, n_events, off, cnt, buf, pos);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// post-pass: tunnel candidates v, a_j, ..., common ancestor, ..., a_0
// ---------------------------------------------------------------------------
__device__ int64_t tunnel_path(const DState &s, int i, int32_t *out) {
    const int32_t *tr = s.tn + 4 * (int64_t)i;
    const int32_t v = tr[1];
    int32_t p1 = tr[2], p2 = tr[3];
    int64_t n = 0;
    if (out) out[n] = v;
    n++;
    // climb to equal depth, then together; the a_0 side is written reversed
    int64_t up = 0, down = 0;
    {
        int32_t q1 = p1, q2 = p2;
        while (ldg(s.depth + q1) > ldg(s.depth + q2)) { q1 = ldg(s.parent + q1); up++; }
        while (ldg(s.depth + q2) > ldg(s.depth + q1)) { q2 = ldg(s.parent + q2); down++; }
        while (q1 != q2) { q1 = ldg(s.parent + q1); q2 = ldg(s.parent + q2); up++; down++; }
    }
    if (out) {
        int32_t q = p1;
        for (int64_t i2 = 0; i2 <= up; ++i2) { out[n + i2] = q; q = s.parent[q]; }
        q = p2;
        for (int64_t i2 = 0; i2 < down; ++i2) { out[n + up + down - i2] = q; q = s.parent[q]; }
    }
    return n + up + 1 + down;
}

// tunnel of entry g of a multi-mesh list: tunnel tnt[g] of mesh tnm[g]
__global__ void k_tunnel_count_multi(const DState *ss, const int32_t *tnm, const int32_t *tnt, int n, int64_t *cnt) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x)
        cnt[g] = tunnel_path(ss[tnm[g]], tnt[g], nullptr);
}
// entries g0 .. g0+n-1; off (n+1 entries) and len are relative to g0
__global__ void k_tunnel_fill_multi(const DMesh *ms, const DState *ss, const int32_t *tnm, const int32_t *tnt, int g0,
                                    int n, const int64_t *off, int32_t *out, double *len) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int mi = tnm[g0 + i];
        const int64_t nn = tunnel_path(ss[mi], tnt[g0 + i], out + off[i]);
        const int32_t *c = out + off[i];
        const double *xyz = ms[mi].xyz;
        double L = 0.0;
        for (int64_t q = 0; q < nn; ++q) {
            const double *pa = xyz + 3 * (int64_t)c[q];
            const double *pb = xyz + 3 * (int64_t)c[(q + 1) % nn];
            const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
            L = L + sqrt((dx * dx + dy * dy) + dz * dz);
        }
        len[i] = L;
    }
}

__global__ void k_tunnel_count(DState s, int nt, int64_t *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x)
        cnt[i] = tunnel_path(s, i, nullptr);
}
// tunnels t0 .. t0+nt-1; off (nt+1 entries) and len are relative to t0
__global__ void k_tunnel_fill(DMesh m, DState s, int t0, int nt, const int64_t *off, int32_t *out, double *len) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) {
        const int64_t n = tunnel_path(s, t0 + i, out + off[i]);
        const int32_t *c = out + off[i];
        double L = 0.0;
        for (int64_t q = 0; q < n; ++q) {
            const double *pa = m.xyz + 3 * (int64_t)c[q];
            const double *pb = m.xyz + 3 * (int64_t)c[(q + 1) % n];
            const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
            L = L + sqrt((dx * dx + dy * dy) + dz * dz);
        }
        len[i] = L;
    }
}
hipError_t launch_reeb_count_multi(const DMesh *ms, const DState *ss, const int32_t *evm, const int32_t *eve, int n,
                                   int64_t *cnt, int32_t *ck, int64_t *meta, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reeb_count_multi, dim3(n), dim3(64), 0, st, ms, ss, evm, eve, n, cnt, ck, meta);
    return hipGetLastError();
}
hipError_t launch_reeb_fill_multi(const DMesh *ms, const DState *ss, const int32_t *evm, const int32_t *eve, int g0,
                                  int n, const int64_t *off, const int64_t *cnt, const int32_t *ck,
                                  const int64_t *meta, int32_t *buf, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reeb_fill_multi, dim3(n), dim3(NT), 0, st, ms, ss, evm, eve, g0, n, off, cnt, ck, meta, buf);
    return hipGetLastError();
}
hipError_t launch_reeb_mean_multi(const DMesh *ms, const int32_t *evm, int g0, int n, const int64_t *off,
                                  const int64_t *cnt, int32_t *buf, double *pos, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int blocks = n < 1024 ? n : 1024;
    hipLaunchKernelGGL(k_reeb_mean_multi, dim3(blocks), dim3(NT), 0, st, ms, evm, g0, n, off, cnt, buf, pos);
    return hipGetLastError();
}
hipError_t launch_tunnel_count_multi(const DState *ss, const int32_t *tnm, const int32_t *tnt, int n, int64_t *cnt,
                                     hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tunnel_count_multi, dim3((n + 63) / 64), dim3(64), 0, st, ss, tnm, tnt, n, cnt);
    return hipGetLastError();
}
hipError_t launch_tunnel_fill_multi(const DMesh *ms, const DState *ss, const int32_t *tnm, const int32_t *tnt, int g0,
                                    int n, const int64_t *off, int32_t *out, double *len, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tunnel_fill_multi, dim3((n + 63) / 64), dim3(64), 0, st, ms, ss, tnm, tnt, g0, n, off, out,
                       len);
    return hipGetLastError();
}

hipError_t launch_tunnel_count(const DState &s, int n_tunnels, int64_t *cnt, hipStream_t st) {
    if (n_tunnels <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tunnel_count, dim3((n_tunnels + 63) / 64), dim3(64), 0, st, s, n_tunnels, cnt);
    return hipGetLastError();
}
hipError_t launch_tunnel_fill(const DMesh &m, const DState &s, int t0, int n_tunnels, const int64_t *off, int32_t *out,
                              double *len, hipStream_t st) {
    if (n_tunnels <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tunnel_fill, dim3((n_tunnels + 63) / 64), dim3(64), 0, st, m, s, t0, n_tunnels, off, out, len);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// device scratch of the allocation-free entry point: one array per device,
// held by the code object until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in for the
// symbol); its device address comes from hipGetSymbolAddress, looked up once
// per device with that device current, and is what kernels receive.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch(int device, void **ptr) {
    static std::mutex mu;
    static std::unordered_map<int, void *> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr.emplace(device, p);
    *ptr = p;
    return hipSuccess;
}

}  // namespace vls
