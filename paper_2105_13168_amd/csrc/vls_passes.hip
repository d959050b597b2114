// vls_passes.hip -- the tunnel-loop pass and the handle-refinement pass of
// the variational loop-shrinking method (Section "Tunnel loop pass", Section
// "Handle refinement pass", Section "Performance Considerations": these
// passes hold one layer as a dense vector, its base layer implicit as one
// minus the value, and many of them run at once), and the handle/tunnel
// distinction by offsetting a loop along the surface normals (Section
// "Distinguishing handle and tunnel loops").
//
// A pass diffuses one region on a restricted operator: only domain vertices
// carry a field and are neighbours, and the cut edges (the edges the source
// loop crosses) are not edges of the operator, so the loop is a border.  The
// start side of the loop begins at 1; each step is the initial pass's field
// step (same equation, coefficients, time step, clip and evaluation order)
// over the operator's neighbours in ascending id, then its threshold and
// closure rounds.  Inserted vertices get an arrival time inside their step
// (linear interpolation of the threshold crossing) and a parent: the lower
// operator neighbour over which the arrival time falls fastest per unit
// length.  The pass ends when the other side of the loop is reached; the
// streamline (parent chain) from the vertex reached, closed along the start
// side and across the cut, is the new loop.
//   - tunnel pass of handle loop h (merge at vertex v): domain = the inside
//     set once v has joined; cut = h's crossed edges; start = h's inside
//     vertices; target = h's outside vertices in the domain.
//   - refinement pass of tunnel W: domain = every vertex; cut = the edges
//     from W to the vertices left of it (counter-clockwise from w_{k+1} to
//     w_{k-1} around w_k); start = W; target = left vertices that are not
//     also right of W.
//
// One workgroup runs one pass at a time and takes the next pass from a
// counter; each workgroup owns a slot of per-vertex state that it returns to
// the reset state (touched vertices only) before its next pass.  The field
// is updated over an update list: a vertex that is a fixed point of the step
// (value 0 or 1, every operator neighbour equal) keeps its value exactly, so
// only the non-fixed vertices of step t-1 and their neighbours are listed
// for step t; the results equal a step over the whole domain bit for bit.
//
// Floating point: FP64, evaluated exactly as written (built with
// -ffp-contract=off), neighbour sums in ascending neighbour id.
#include <climits>

#include "vls_internal.h"

namespace vls {
namespace {

constexpr int PT = 256;     // threads per workgroup
enum { PF_START = 1, PF_TARGET = 2, PF_CUTV = 4, PF_LEFT = 8, PF_RIGHT = 16, PF_INW = 32 };
enum { PS_OK = 0, PS_INVALID = -1, PS_STALLED = -7, PS_CAPACITY = -14 };

struct PSh {
    int task, kind, src;
    int nU, nUn, ncand, npn, nnew, nonfixed, nflag, ntouch, nside;
    int bad;
    unsigned long long reached;
    int32_t ev_v;
    uint64_t ev_key;
};

__device__ __forceinline__ bool rank_below(uint64_t ka, int32_t a, uint64_t kb, int32_t b) {
    return ka < kb || (ka == kb && a < b);
}

__device__ __forceinline__ bool in_dom(const PassArgs &A, const PSh &sh, int32_t u) {
    if (sh.kind != 0) return true;
    const uint64_t k = A.s.key[u];
    return k < sh.ev_key || (k == sh.ev_key && u <= sh.ev_v);
}

__device__ __forceinline__ bool cut_he(const PassSlot &S, int64_t i) {
    return (S.cutbits[i >> 5] >> (i & 31)) & 1u;
}

// is neighbour u of v (half-edge i of v's ascending row) an operator neighbour?
__device__ __forceinline__ bool op_nb(const PassArgs &A, const PassSlot &S, const PSh &sh, int fv, int64_t i,
                                      int32_t u) {
    if (!in_dom(A, sh, u)) return false;
    return !((fv & PF_CUTV) && cut_he(S, i));
}

__device__ __forceinline__ int set_flag(const PassSlot &S, PSh &sh, int32_t v, int bits) {
    const int old = atomicOr(&S.flag[v], bits);
    if (old == 0) S.flist[atomicAdd(&sh.nflag, 1)] = v;
    return old;
}

// sets (or clears) the cut bit of half-edge a -> b
__device__ __forceinline__ void cut_he_bit(const PassArgs &A, const PassSlot &S, int32_t a, int32_t b, bool clear) {
    for (int64_t i = A.m.rp[a]; i < A.m.rp[a + 1]; ++i)
        if (A.m.adj[i] == b) {
            const uint32_t bit = 1u << (i & 31);
            if (clear) atomicAnd(&S.cutbits[i >> 5], ~bit);
            else atomicOr(&S.cutbits[i >> 5], bit);
            return;
        }
}

// the undirected edge {a, b} leaves the operator (clear: returns to it;
// the flags are reset separately)
__device__ __forceinline__ void set_cut(const PassArgs &A, const PassSlot &S, PSh &sh, int32_t a, int32_t b,
                                        bool clear = false) {
    cut_he_bit(A, S, a, b, clear);
    cut_he_bit(A, S, b, a, clear);
    if (!clear) {
        set_flag(S, sh, a, PF_CUTV);
        set_flag(S, sh, b, PF_CUTV);
    }
}

// appends y to the update list of step t once (mark = t); records the first
// listing of the pass (the vertex's state is reset at the end)
__device__ __forceinline__ void list_add(const PassSlot &S, PSh &sh, int32_t y, int t, int32_t *L, int *n) {
    const int old = atomicExch(&S.mark[y], t);
    if (old != t) {
        L[atomicAdd(n, 1)] = y;
        if (old == 0) S.touched[atomicAdd(&sh.ntouch, 1)] = y;
    }
}

__device__ __forceinline__ double edge_len(const double *p, int32_t a, int32_t b) {
    const double dx = p[3 * (int64_t)b] - p[3 * (int64_t)a], dy = p[3 * (int64_t)b + 1] - p[3 * (int64_t)a + 1];
    const double dz = p[3 * (int64_t)b + 2] - p[3 * (int64_t)a + 2];
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

// area-weighted normal of w: the cross products of its triangles (w, c_j,
// c_{j+1}) over its counter-clockwise link from the smallest neighbour id,
// summed in that order, normalised
__device__ void vertex_normal(const DMesh &m, int32_t w, double *n) {
    const double *p = m.xyz;
    const int64_t b = m.rp[w], d = m.rp[w + 1] - b;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        const int32_t c0 = m.cyc[b + j], c1 = m.cyc[b + (j + 1) % d];
        const double ax = p[3 * (int64_t)c0] - p[3 * (int64_t)w], ay = p[3 * (int64_t)c0 + 1] - p[3 * (int64_t)w + 1];
        const double az = p[3 * (int64_t)c0 + 2] - p[3 * (int64_t)w + 2];
        const double bx = p[3 * (int64_t)c1] - p[3 * (int64_t)w], by = p[3 * (int64_t)c1 + 1] - p[3 * (int64_t)w + 1];
        const double bz = p[3 * (int64_t)c1 + 2] - p[3 * (int64_t)w + 2];
        sx = sx + (ay * bz - az * by);
        sy = sy + (az * bx - ax * bz);
        sz = sz + (ax * by - ay * bx);
    }
    const double l = sqrt((sx * sx + sy * sy) + sz * sz);
    n[0] = sx / l;
    n[1] = sy / l;
    n[2] = sz / l;
}

// thread 0: streamline from the vertex reached, closed along the start side;
// length and offset test; appended to the output
__device__ void close_loop(const PassArgs &A, const PassSlot &S, PSh &sh, PassResult &R) {
    const DMesh &m = A.m;
    const int32_t x = (int32_t)(sh.reached & 0xffffffffull);
    int64_t n = 0;
    S.buf[n++] = x;
    while (S.key[S.buf[n - 1]] != 0ull) {
        const int32_t p = S.par[S.buf[n - 1]];
        if (p < 0 || n >= m.nv) { R.status = PS_INVALID; return; }
        S.buf[n++] = p;
    }
    const int32_t sstar = S.buf[n - 1];
    const int ns = sh.nside;
    // the shortest walk along the start side from s* to a start vertex that
    // shares a cut edge with x (ties: forward, then the smaller position)
    long long bd = -1;
    int bback = 0, bj = 0, bi = 0;
    for (int j = 0; j < ns; ++j) {
        const int32_t q = S.side[j];
        bool partner = false;
        for (int64_t i = m.rp[x]; i < m.rp[x + 1]; ++i)
            if (m.adj[i] == q) { partner = cut_he(S, i); break; }
        if (!partner) continue;
        for (int i = 0; i < ns; ++i) {
            if (S.side[i] != sstar) continue;
            const int f = ((j - i) % ns + ns) % ns, b = ((i - j) % ns + ns) % ns;
            const int dist = f <= b ? f : b, back = f <= b ? 0 : 1;
            const bool better = bd < 0 || dist < bd || (dist == bd && (back < bback || (back == bback &&
                                (j < bj || (j == bj && i < bi)))));
            if (better) { bd = dist; bback = back; bj = j; bi = i; }
        }
    }
    if (bd < 0) { R.status = PS_INVALID; return; }
    // loop erasure while appending the walk: a vertex met again cuts out
    // the part after its first visit
    for (int64_t k = 0; k < n; ++k) S.pos[S.buf[k]] = (int32_t)k;
    for (long long k = 1; k <= bd; ++k) {
        const int32_t y = S.side[((bi + (bback ? -k : k)) % ns + ns) % ns];
        const int32_t py = S.pos[y];
        if (py >= 0) {
            for (int64_t z = py + 1; z < n; ++z) S.pos[S.buf[z]] = -1;
            n = py + 1;
        } else {
            S.pos[y] = (int32_t)n;
            S.buf[n++] = y;
        }
    }
    for (int64_t k = 0; k < n; ++k) S.pos[S.buf[k]] = -1;
    double L0 = 0.0;
    for (int64_t k = 0; k < n; ++k) L0 = L0 + edge_len(m.xyz, S.buf[k], S.buf[(k + 1) % n]);
    // offset along the normals by rel_eps times the mean edge length
    const double eps = A.rel_eps * L0 / (double)n;
    double q0[3], qp[3], L1 = 0.0;
    for (int64_t k = 0; k <= n; ++k) {
        double q[3];
        if (k < n) {
            const int32_t w = S.buf[k];
            double nn[3];
            vertex_normal(m, w, nn);
            for (int c = 0; c < 3; ++c) q[c] = m.xyz[3 * (int64_t)w + c] + eps * nn[c];
        } else {
            for (int c = 0; c < 3; ++c) q[c] = q0[c];
        }
        if (k == 0) {
            for (int c = 0; c < 3; ++c) q0[c] = q[c];
        } else {
            const double dx = q[0] - qp[0], dy = q[1] - qp[1], dz = q[2] - qp[2];
            L1 = L1 + sqrt((dx * dx + dy * dy) + dz * dz);
        }
        for (int c = 0; c < 3; ++c) qp[c] = q[c];
    }
    const unsigned long long off = atomicAdd(A.out_used, (unsigned long long)n);
    if ((int64_t)(off + n) > A.out_cap) { R.status = PS_CAPACITY; return; }
    for (int64_t k = 0; k < n; ++k) A.out[off + k] = S.buf[k];
    R.off = (int64_t)off;
    R.n = n;
    R.length = L0;
    R.offset_length = L1;
    R.label = L1 > L0 ? 0 : 1;
}

__global__ void __launch_bounds__(PT) k_passes(PassArgs A) {
    __shared__ PSh sh;
    const int tid = threadIdx.x;
    const PassSlot S = A.slots[blockIdx.x];
    const DMesh &m = A.m;
    const double *__restrict__ xyz = m.xyz;
    for (;;) {
        if (tid == 0) {
            sh.task = atomicAdd(A.next, 1);
            sh.nflag = sh.ntouch = sh.nside = 0;
            sh.bad = 0;
            sh.nU = 0;
        }
        __syncthreads();
        const int task = sh.task;
        if (task >= A.ntasks) break;
        const PassTask T = A.tasks[task];
        PassResult R{};
        R.status = PS_OK;
        R.reached = -1;
        R.label = -1;
        // --- set-up: flags, cut edges, start side --------------------------
        if (tid == 0) { sh.kind = T.kind; sh.src = T.src; }
        __syncthreads();
        if (T.kind == 0) {
            const int64_t *lp = A.s.lp + 8 * (int64_t)T.src;
            const int64_t off = lp[3], cnt = lp[4];
            const int32_t v = (int32_t)A.s.ev[16 * lp[0] + 1];
            if (tid == 0) { sh.ev_v = v; sh.ev_key = A.s.key[v]; }
            const int32_t *he = A.s.lp_he + 2 * off;
            for (int64_t k = tid; k < cnt; k += PT) {
                set_cut(A, S, sh, he[2 * k], he[2 * k + 1]);
                set_flag(S, sh, he[2 * k], PF_START);
            }
            __syncthreads();
            for (int64_t k = tid; k < cnt; k += PT) {
                const int32_t x = he[2 * k + 1];
                if (in_dom(A, sh, x) && !(S.flag[x] & PF_START)) set_flag(S, sh, x, PF_TARGET);
            }
            if (tid == 0) {
                // start side in loop order, repeats in a row dropped
                int ns = 0;
                for (int64_t k = 0; k < cnt; ++k)
                    if (ns == 0 || S.side[ns - 1] != he[2 * k]) S.side[ns++] = he[2 * k];
                while (ns > 1 && S.side[0] == S.side[ns - 1]) ns--;
                sh.nside = ns;
            }
        } else {
            const PassResult &Q = A.src_res[T.src];
            const int64_t n = Q.status == PS_OK ? Q.n : 0;
            const int32_t *W = A.src_out + (Q.status == PS_OK ? Q.off : 0);
            if (n < 3) {
                if (tid == 0) sh.bad = 1;
            } else {
                for (int64_t k = tid; k < n; k += PT) {
                    set_flag(S, sh, W[k], PF_INW | PF_START);
                    S.side[k] = W[k];
                }
                if (tid == 0) sh.nside = (int)n;
                __syncthreads();
                for (int64_t k = tid; k < n; k += PT) {
                    const int32_t w = W[k], nx = W[(k + 1) % n], pv = W[(k + n - 1) % n];
                    const int64_t b = m.rp[w];
                    const int d = (int)(m.rp[w + 1] - b);
                    int jn = -1, jp = -1;
                    for (int j = 0; j < d; ++j) {
                        if (m.cyc[b + j] == nx) jn = j;
                        if (m.cyc[b + j] == pv) jp = j;
                    }
                    if (jn < 0 || jp < 0 || jn == jp) { sh.bad = 1; continue; }
                    for (int j = (jn + 1) % d; j != jp; j = (j + 1) % d) {
                        const int32_t y = m.cyc[b + j];
                        if (S.flag[y] & PF_INW) continue;
                        set_flag(S, sh, y, PF_LEFT);
                        set_cut(A, S, sh, w, y);
                    }
                    for (int j = (jp + 1) % d; j != jn; j = (j + 1) % d) {
                        const int32_t y = m.cyc[b + j];
                        if (!(S.flag[y] & PF_INW)) set_flag(S, sh, y, PF_RIGHT);
                    }
                }
                __syncthreads();
                for (int k = tid; k < sh.nflag; k += PT) {
                    const int32_t y = S.flist[k];
                    const int f = S.flag[y];
                    if ((f & PF_LEFT) && !(f & PF_RIGHT)) atomicOr(&S.flag[y], PF_TARGET);
                }
            }
        }
        __syncthreads();
        if (sh.bad) {
            R.status = PS_INVALID;
        } else {
            // start side at 1, inside at step 0; update list of step 1: the
            // start side and its operator neighbours
            int32_t *U1 = S.U[1];
            for (int k = tid; k < sh.nside; k += PT) {
                const int32_t u = S.side[k];
                S.rho[u] = 1.0;
                S.key[u] = 0ull;
                S.ta[u] = 0.0;
                S.par[u] = -1;
            }
            __syncthreads();
            for (int k = tid; k < sh.nside; k += PT) {
                const int32_t u = S.side[k];
                const int fu = S.flag[u];
                list_add(S, sh, u, 1, U1, &sh.nU);
                for (int64_t i = m.rp[u]; i < m.rp[u + 1]; ++i) {
                    const int32_t y = m.adj[i];
                    if (op_nb(A, S, sh, fu, i, y)) list_add(S, sh, y, 1, U1, &sh.nU);
                }
            }
            __syncthreads();
            // --- steps -----------------------------------------------------
            int64_t last_insert = 0;
            int nonfixed_prev = -1, npend = 0;
            int64_t updates = 0;
            for (int64_t t = 1;; ++t) {
                if (t > A.max_steps || (nonfixed_prev == 0 && npend == 0)) {
                    R.status = PS_STALLED;
                    R.steps = t - 1;
                    break;
                }
                const int nU = sh.nU;
                int32_t *U = S.U[t & 1];
                int32_t *Un = S.U[(t + 1) & 1];
                const uint64_t tk = (uint64_t)t << 32;
                if (tid == 0) { sh.nUn = 0; sh.nonfixed = 0; sh.ncand = 0; sh.npn = 0; sh.nnew = 0; sh.reached = ~0ull; }
                __syncthreads();
                // A: new values (Jacobi, over the operator's neighbours in
                //    ascending id); a vertex that is not a fixed point of
                //    the step lists itself and its neighbours for t+1
                int nf = 0;
                for (int i = tid; i < nU; i += PT) {
                    const int32_t v = U[i];
                    const int fv = S.flag[v];
                    const double r = S.rho[v];
                    double sum = 0.0;
                    int64_t deg = 0;
                    bool fixed = r == 0.0 || r == 1.0;
                    for (int64_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
                        const int32_t u = m.adj[j];
                        if (!op_nb(A, S, sh, fv, j, u)) continue;
                        const double ru = S.rho[u];
                        sum = sum + ru;
                        deg++;
                        fixed = fixed && ru == r;
                    }
                    const double lap = sum - (double)deg * r;
                    const double d = (A.a * lap + A.w * (2.0 * r - 1.0)) + A.e * sqrt(r * (1.0 - r));
                    double x = r + A.c * d;
                    if (x < 0.0) x = 0.0;
                    if (x > 1.0) x = 1.0;
                    S.tmp[i] = x;
                    if (!fixed) {
                        nf++;
                        list_add(S, sh, v, (int)t + 1, Un, &sh.nUn);
                        for (int64_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
                            const int32_t u = m.adj[j];
                            if (op_nb(A, S, sh, fv, j, u)) list_add(S, sh, u, (int)t + 1, Un, &sh.nUn);
                        }
                    }
                }
                if (nf) atomicAdd(&sh.nonfixed, nf);
                __syncthreads();
                updates += nU;
                // B: write the values; crossers of the step
                for (int i = tid; i < nU; i += PT) {
                    const int32_t v = U[i];
                    const double x = S.tmp[i];
                    const double old = S.rho[v];
                    S.rho[v] = x;
                    if (S.key[v] == KEY_OUT && x > A.tau) {
                        S.prev[v] = old;
                        S.upd[v] = (int32_t)t;
                        if (atomicExch(&S.cst[v], (int32_t)t) != (int32_t)t) S.cand[atomicAdd(&sh.ncand, 1)] = v;
                    }
                }
                __syncthreads();
                // crossers still waiting from the previous step
                const int32_t *P = S.pend[(t - 1) & 1];
                for (int i = tid; i < npend; i += PT) {
                    const int32_t v = P[i];
                    if (S.key[v] == KEY_OUT && S.rho[v] > A.tau && atomicExch(&S.cst[v], (int32_t)t) != (int32_t)t)
                        S.cand[atomicAdd(&sh.ncand, 1)] = v;
                }
                __syncthreads();
                // C: closure rounds over the operator's edges (round per
                //    candidate in U, the list of this step, free by now)
                const int nc = sh.ncand;
                int32_t *crd = U;
                for (int i = tid; i < nc; i += PT) crd[i] = -1;
                __syncthreads();
                int nins = 0;
                for (int round = 0;; ++round) {
                    const uint64_t want = tk | (uint64_t)(round - 1);
                    for (int i = tid; i < nc; i += PT) {
                        int hit = 0;
                        if (crd[i] < 0) {
                            const int32_t v = S.cand[i];
                            const int fv = S.flag[v];
                            for (int64_t j = m.rp[v]; j < m.rp[v + 1] && !hit; ++j) {
                                const int32_t u = m.adj[j];
                                if (!op_nb(A, S, sh, fv, j, u)) continue;
                                const uint64_t ku = S.key[u];
                                hit = round == 0 ? ku < tk : ku == want;
                            }
                        }
                        S.buf[i] = hit;
                    }
                    __syncthreads();
                    int mine = 0;
                    for (int i = tid; i < nc; i += PT)
                        if (S.buf[i]) {
                            crd[i] = round;
                            S.key[S.cand[i]] = tk | (uint64_t)round;
                            mine++;
                        }
                    if (tid == 0) sh.nnew = 0;
                    __syncthreads();
                    if (mine) atomicAdd(&sh.nnew, mine);
                    __syncthreads();
                    const int nnew = sh.nnew;
                    nins += nnew;
                    __syncthreads();
                    if (nnew == 0) break;
                }
                // D: arrival times of the step's insertions
                for (int i = tid; i < nc; i += PT) {
                    if (crd[i] < 0) continue;
                    const int32_t v = S.cand[i];
                    const double x = S.rho[v];
                    const double pv = S.upd[v] == (int32_t)t ? S.prev[v] : x;
                    const double d = x - pv;
                    double f = d > 0.0 ? (A.tau - pv) / d : 0.0;
                    if (f < 0.0) f = 0.0;
                    if (f > 1.0) f = 1.0;
                    S.ta[v] = (double)(t - 1) + f;
                }
                __syncthreads();
                // E: parents (steepest descent of the arrival time per unit
                //    length over lower operator neighbours), the first target
                //    in rank order, the crossers left waiting
                int32_t *Pn = S.pend[t & 1];
                for (int i = tid; i < nc; i += PT) {
                    const int32_t v = S.cand[i];
                    if (crd[i] < 0) {
                        Pn[atomicAdd(&sh.npn, 1)] = v;
                        continue;
                    }
                    const uint64_t kv = S.key[v];
                    const int fv = S.flag[v];
                    int32_t best = -1;
                    uint64_t kb = 0;
                    double bs = 0.0;
                    for (int64_t j = m.rp[v]; j < m.rp[v + 1]; ++j) {
                        const int32_t u = m.adj[j];
                        if (!op_nb(A, S, sh, fv, j, u)) continue;
                        const uint64_t ku = S.key[u];
                        if (!rank_below(ku, u, kv, v)) continue;
                        const double sl = (S.ta[v] - S.ta[u]) / edge_len(xyz, v, u);
                        if (best < 0 || sl > bs || (sl == bs && rank_below(ku, u, kb, best))) {
                            best = u;
                            kb = ku;
                            bs = sl;
                        }
                    }
                    S.par[v] = best;
                    if (fv & PF_TARGET) atomicMin(&sh.reached, ((unsigned long long)crd[i] << 32) | (uint32_t)v);
                }
                __syncthreads();
                if (sh.reached != ~0ull) {
                    R.steps = t;
                    R.reached = (int32_t)(sh.reached & 0xffffffffull);
                    break;
                }
                if (nins) last_insert = t;
                if (t - last_insert >= A.stall_steps) {
                    R.status = PS_STALLED;
                    R.steps = t;
                    break;
                }
                nonfixed_prev = sh.nonfixed;
                npend = sh.npn;
                __syncthreads();
                if (tid == 0) sh.nU = sh.nUn;
                __syncthreads();
            }
            R.updates = updates;
            if (R.status == PS_OK && tid == 0) close_loop(A, S, sh, R);
        }
        __syncthreads();
        // --- back to the reset state ---------------------------------------
        // cut bits: the set-up's edges again, cleared (the flags that chose
        // them are still set)
        if (T.kind == 0) {
            const int64_t *lp = A.s.lp + 8 * (int64_t)T.src;
            const int32_t *he = A.s.lp_he + 2 * lp[3];
            for (int64_t k = tid; k < lp[4]; k += PT) set_cut(A, S, sh, he[2 * k], he[2 * k + 1], true);
        } else {
            const PassResult &Q = A.src_res[T.src];
            const int64_t n = Q.status == PS_OK ? Q.n : 0;
            const int32_t *W = A.src_out + (Q.status == PS_OK ? Q.off : 0);
            for (int64_t k = tid; k < (n < 3 ? 0 : n); k += PT) {
                const int32_t w = W[k], nx = W[(k + 1) % n], pv = W[(k + n - 1) % n];
                const int64_t b = m.rp[w];
                const int d = (int)(m.rp[w + 1] - b);
                int jn = -1, jp = -1;
                for (int j = 0; j < d; ++j) {
                    if (m.cyc[b + j] == nx) jn = j;
                    if (m.cyc[b + j] == pv) jp = j;
                }
                if (jn < 0 || jp < 0 || jn == jp) continue;
                for (int j = (jn + 1) % d; j != jp; j = (j + 1) % d) {
                    const int32_t y = m.cyc[b + j];
                    if (!(S.flag[y] & PF_INW)) set_cut(A, S, sh, w, y, true);
                }
            }
        }
        __syncthreads();
        for (int k = tid; k < sh.ntouch; k += PT) {
            const int32_t y = S.touched[k];
            S.rho[y] = 0.0;
            S.key[y] = KEY_OUT;
            S.par[y] = -1;
            S.mark[y] = 0;
            S.cst[y] = 0;
            S.upd[y] = 0;
        }
        for (int k = tid; k < sh.nflag; k += PT) S.flag[S.flist[k]] = 0;
        if (tid == 0) A.res[task] = R;
        __syncthreads();
    }
}

__global__ void k_pass_slot_init(PassSlot S, int32_t nv, int64_t nwords) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        S.rho[i] = 0.0;
        S.key[i] = KEY_OUT;
        S.par[i] = -1;
        S.mark[i] = 0;
        S.cst[i] = 0;
        S.upd[i] = 0;
        S.flag[i] = 0;
        S.pos[i] = -1;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) S.cutbits[i] = 0u;
}

}  // namespace

hipError_t launch_pass_slot_init(const PassSlot &s, int32_t nv, int64_t nnz, hipStream_t st) {
    const int64_t nwords = nnz / 32 + 1;
    int64_t n = nv > nwords ? nv : nwords;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pass_slot_init, dim3(blocks), dim3(256), 0, st, s, nv, nwords);
    return hipGetLastError();
}

hipError_t launch_passes(const PassArgs &a, hipStream_t st) {
    if (a.ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_passes, dim3(a.nslots), dim3(PT), 0, st, a);
    return hipGetLastError();
}

int max_coresident_passes() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_passes, PT, 0) != hipSuccess) return 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return n * cus;
}

}  // namespace vls
