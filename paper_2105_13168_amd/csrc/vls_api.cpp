// vls_api.cpp -- host side of the C ABI declared in include/vls.h: mesh
// validation and adjacency construction (step S0), device buffers, the run
// sequence (init, seed, persistent step kernel, post-passes) and the result
// objects.  All arithmetic of the method runs in the kernels of
// vls_kernels.hip; this file only moves data and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vls.h"
#include "vls_internal.h"

using namespace vls;

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct vls_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
};

struct DeviceBuf {
    void *p = nullptr;
    size_t n = 0;
};

struct RunBuffers;   // per-mesh cached device state

struct vls_mesh {
    vls_context *ctx = nullptr;
    int64_t nv = 0, nf = 0, ne = 0, nnz = 0;
    int32_t dmax = 0;
    int32_t euler_genus = 0;
    std::vector<double> xyz;             // host copy (for seed-node position)
    DMesh d{};
    std::vector<void *> allocs;
    RunBuffers *rb = nullptr;
    vls_result *pending = nullptr;       // run whose results still sit in rb
    double fem_sigma = 0.0, fem_dmax = 0.0;   // finite-element operator (d.fem_g) once prepared
};

struct RunPrep;   // one run in flight (defined with the run sequence)

struct Pending {
    bool active = false;                 // bulk results still on the device
    vls_context *ctx = nullptr;
    vls_mesh *mesh = nullptr;            // mesh whose cached run state holds them
    hipStream_t stream = nullptr;
    DState s{};
    Ctl c{};
    std::vector<void *> tmp_allocs;      // checkpoint buffers of hipMalloc'ed runs
    bool rec_field = false;
};

struct vls_result {
    Pending pend;
    RunPrep *launched = nullptr;         // vls_run_async: enqueued, not yet waited for
    vls_status launch_status = VLS_OK;   // status vls_result_wait returns once done
    bool failed = false;                 // the post-passes or copies failed: no outputs
    int static_dev = -1;                 // vls_run_async_noalloc: device whose static scratch it holds
    vls_summary sum{};
    int64_t nv = 0;
    std::vector<int64_t> ev;             // [n][16]
    std::vector<int64_t> ev_ids;
    std::vector<double> node_pos;        // [n_events][3]
    std::vector<double> seed_xyz;        // [3]
    std::vector<int32_t> front_birth, front_death;
    std::vector<int64_t> lp;             // [n_loops][8]
    std::vector<int32_t> lp_he;          // [*][2]
    std::vector<double> lp_pts;          // [*][3]
    std::vector<int32_t> tn;             // [n_tunnels][4]
    std::vector<int64_t> tn_off;         // [n_tunnels+1]
    std::vector<int32_t> tn_v;
    std::vector<double> tn_pts;          // [*][3] positions of the tunnel vertices
    std::vector<double> tn_len;          // [n_tunnels] vertex polyline lengths
    std::vector<int32_t> step, round, parent;
    std::vector<double> rho_final;
    std::vector<int64_t> ckpt_steps;
    std::vector<double> ckpt;            // [n_ckpt][nv]
    std::vector<int32_t> ckpt_ok;
    // tunnel-loop (index 0) and handle-refinement (index 1) passes
    std::vector<PassResult> pres[2];
    std::vector<int32_t> pout[2];
    std::vector<double> pass_xyz;        // mesh positions, kept when the passes ran
    vls_result *refined = nullptr;       // VLS_REEB_REFINE: the pass from the first handle loop (owned)
};

static vls_status set_err(vls_context *ctx, vls_status s, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return s;
}

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_err(ctx, VLS_E_DEVICE, "%s failed: %s (%s:%d)", #call,                 \
                           hipGetErrorString(e_), __FILE__, __LINE__);                         \
    } while (0)

extern "C" {

void vls_params_default(vls_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(vls_params);
    p->dt_mode = 0;
    p->tau = 0.5;
    p->mu = 0.25;
    p->a = 1.0 / 25.0;
    p->w = (1.0 / 25.0) / 5.0;
    p->e = 1.0 / 30.0;
    p->seed_vertex = 0;
    p->rng_seed = 0;
    p->seed_radius = 2;
    p->stall_steps = 200000;
    p->max_steps = 10000000;
    p->flags = 0;
    p->n_ckpt = 0;
    p->ckpt_steps = nullptr;
    p->grid = 0;
    p->block = 256;
}

const char *vls_status_string(vls_status s) {
    switch (s) {
    case VLS_OK: return "VLS_OK";
    case VLS_E_INVALID_ARG: return "VLS_E_INVALID_ARG";
    case VLS_E_MESH_NOT_MANIFOLD: return "VLS_E_MESH_NOT_MANIFOLD";
    case VLS_E_MESH_HAS_BOUNDARY: return "VLS_E_MESH_HAS_BOUNDARY";
    case VLS_E_MESH_NOT_CONNECTED: return "VLS_E_MESH_NOT_CONNECTED";
    case VLS_E_MESH_NOT_ORIENTABLE: return "VLS_E_MESH_NOT_ORIENTABLE";
    case VLS_E_SEED_INVALID: return "VLS_E_SEED_INVALID";
    case VLS_E_STALLED: return "VLS_E_STALLED";
    case VLS_E_OUT_OF_MEMORY: return "VLS_E_OUT_OF_MEMORY";
    case VLS_E_DEVICE: return "VLS_E_DEVICE";
    case VLS_E_BUFFER_TOO_SMALL: return "VLS_E_BUFFER_TOO_SMALL";
    case VLS_E_PENDING: return "VLS_E_PENDING";
    case VLS_E_CANCELLED: return "VLS_E_CANCELLED";
    case VLS_E_INVARIANT: return "VLS_E_INVARIANT";
    case VLS_E_CAPACITY: return "VLS_E_CAPACITY";
    case VLS_E_TOO_LARGE: return "VLS_E_TOO_LARGE";
    default: return "VLS_E_UNKNOWN";
    }
}

const char *vls_last_error(const vls_context *ctx) { return ctx ? ctx->err.c_str() : ""; }

vls_status vls_context_create(int device, void *hip_stream, vls_context **out) {
    if (!out) return VLS_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VLS_E_DEVICE;
    auto *c = new (std::nothrow) vls_context;
    if (!c) return VLS_E_OUT_OF_MEMORY;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return VLS_E_DEVICE; }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return VLS_E_DEVICE; }
        c->own_stream = true;
    }
    *out = c;
    return VLS_OK;
}

vls_status vls_context_destroy(vls_context *ctx) {
    if (!ctx) return VLS_E_INVALID_ARG;
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return VLS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// mesh validation and adjacency (S0)
// ---------------------------------------------------------------------------
namespace {

struct HostAdj {
    std::vector<int32_t> rp, adj, cyc, src, rev, succ, nin, ell, lrow, hrec;
    int32_t dmax = 0;
};

// Builds the counter-clockwise links: triangle (a,b,c) contributes the link
// edge b->c to a, c->a to b, a->b to c.  A closed oriented 2-manifold has,
// at every vertex, link edges forming a single cycle.
vls_status build_adjacency(vls_context *ctx, int64_t nv, int64_t nf, const int32_t *tri, HostAdj &h) {
    for (int64_t i = 0; i < 3 * nf; ++i)
        if (tri[i] < 0 || tri[i] >= nv)
            return set_err(ctx, VLS_E_INVALID_ARG, "triangle %lld references vertex %d outside [0,%lld)",
                           (long long)(i / 3), tri[i], (long long)nv);
    std::vector<int64_t> cnt(nv + 1, 0);
    for (int64_t i = 0; i < 3 * nf; ++i) cnt[tri[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) {
        if (cnt[v + 1] == 0) return set_err(ctx, VLS_E_MESH_NOT_CONNECTED, "vertex %lld is in no triangle", (long long)v);
        cnt[v + 1] += cnt[v];
    }
    const int64_t nnz = cnt[nv];
    if (nnz >= (int64_t)1 << 31) return set_err(ctx, VLS_E_TOO_LARGE, "3*nf = %lld exceeds the 32-bit index range", (long long)nnz);
    std::vector<int32_t> la(nnz), lb(nnz);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t a = tri[3 * f], b = tri[3 * f + 1], c = tri[3 * f + 2];
        if (a == b || b == c || a == c)
            return set_err(ctx, VLS_E_MESH_NOT_MANIFOLD, "triangle %lld repeats a vertex", (long long)f);
        la[fill[a]] = b; lb[fill[a]++] = c;
        la[fill[b]] = c; lb[fill[b]++] = a;
        la[fill[c]] = a; lb[fill[c]++] = b;
    }
    h.rp.resize(nv + 1);
    for (int64_t v = 0; v <= nv; ++v) h.rp[v] = (int32_t)cnt[v];
    h.adj.resize(nnz); h.cyc.resize(nnz); h.src.resize(nnz);
    h.rev.resize(nnz); h.succ.resize(nnz); h.nin.resize(nnz);
    int32_t dmax = 0;
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t b = cnt[v], d = cnt[v + 1] - b;
        if (d < 3) return set_err(ctx, VLS_E_MESH_NOT_MANIFOLD, "vertex %lld has degree %lld", (long long)v, (long long)d);
        if (d > 64) return set_err(ctx, VLS_E_TOO_LARGE, "vertex %lld has degree %lld (limit 64)", (long long)v, (long long)d);
        dmax = std::max<int32_t>(dmax, (int32_t)d);
        // each link vertex must start exactly one link edge
        for (int64_t i = 0; i < d; ++i)
            for (int64_t j = i + 1; j < d; ++j)
                if (la[b + i] == la[b + j]) {
                    // the same directed edge v->la twice: two triangles with equal orientation,
                    // or a non-manifold fan
                    return set_err(ctx, VLS_E_MESH_NOT_ORIENTABLE,
                                   "directed edge %lld->%d occurs twice", (long long)v, la[b + i]);
                }
        int32_t start = la[b];
        for (int64_t i = 1; i < d; ++i) start = std::min(start, la[b + i]);
        int32_t cur = start;
        for (int64_t i = 0; i < d; ++i) {
            h.cyc[b + i] = cur;
            h.src[b + i] = (int32_t)v;
            int64_t hit = -1;
            for (int64_t j = 0; j < d; ++j)
                if (la[b + j] == cur) { hit = j; break; }
            if (hit < 0)
                return set_err(ctx, VLS_E_MESH_HAS_BOUNDARY, "link of vertex %lld is open at %d", (long long)v, cur);
            cur = lb[b + hit];
        }
        if (cur != start)
            return set_err(ctx, VLS_E_MESH_NOT_MANIFOLD, "link of vertex %lld is not a single cycle", (long long)v);
        for (int64_t i = 0; i < d; ++i) {
            h.adj[b + i] = h.cyc[b + i];
            h.succ[b + i] = (int32_t)(i + 1 == d ? b : b + i + 1);
        }
        std::sort(h.adj.begin() + b, h.adj.begin() + b + d);
        for (int64_t i = 1; i < d; ++i)
            if (h.adj[b + i] == h.adj[b + i - 1])
                return set_err(ctx, VLS_E_MESH_NOT_MANIFOLD, "link of vertex %lld repeats vertex %d", (long long)v, h.adj[b + i]);
    }
    h.dmax = dmax;
    // padded rows of the field gather: ascending neighbours, then the vertex
    // itself; a row whose vertex has more than ELL_W neighbours is marked -1
    h.ell.assign((size_t)nv * ELL_W, 0);
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t b = cnt[v], d = cnt[v + 1] - b;
        int32_t *row = h.ell.data() + (size_t)v * ELL_W;
        if (d > ELL_W) {
            for (int j = 0; j < ELL_W; ++j) row[j] = -1;
            continue;
        }
        for (int j = 0; j < ELL_W; ++j) row[j] = j < d ? h.adj[b + j] : (int32_t)v;
    }
    // link rows of the topology: counter-clockwise neighbours, -1 padding,
    // and the first half-edge index in the last slot (-2 first: too wide)
    h.lrow.assign((size_t)nv * ELL_W, -1);
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t b = cnt[v], d = cnt[v + 1] - b;
        int32_t *row = h.lrow.data() + (size_t)v * ELL_W;
        row[ELL_W - 1] = (int32_t)b;
        if (d > ELL_W - 1) {
            row[0] = -2;
            continue;
        }
        for (int j = 0; j < d; ++j) row[j] = h.cyc[b + j];
    }
    // opposite half-edges, and the (y->x) successor
    auto find = [&](int32_t u, int32_t x) -> int64_t {
        for (int64_t j = cnt[u]; j < cnt[u + 1]; ++j)
            if (h.cyc[j] == x) return j;
        return -1;
    };
    for (int64_t v = 0; v < nv; ++v)
        for (int64_t e = cnt[v]; e < cnt[v + 1]; ++e) {
            const int32_t x = h.cyc[e];
            const int64_t r = find(x, (int32_t)v);
            if (r < 0) return set_err(ctx, VLS_E_MESH_HAS_BOUNDARY, "edge %lld-%d has one side only", (long long)v, x);
            h.rev[e] = (int32_t)r;
            const int32_t y = h.cyc[h.succ[e]];
            const int64_t q = find(y, x);
            if (q < 0) return set_err(ctx, VLS_E_MESH_NOT_MANIFOLD, "triangle (%lld,%d,%d) not closed", (long long)v, x, y);
            h.nin[e] = (int32_t)q;
        }
    // walk records: successor, (y->x) half-edge, third vertex y, far end x
    h.hrec.resize(4 * h.cyc.size());
    for (size_t e = 0; e < h.cyc.size(); ++e) {
        h.hrec[4 * e] = h.succ[e];
        h.hrec[4 * e + 1] = h.nin[e];
        h.hrec[4 * e + 2] = h.cyc[h.succ[e]];
        h.hrec[4 * e + 3] = h.cyc[e];
    }
    // connected
    std::vector<int32_t> queue;
    queue.reserve(nv);
    std::vector<char> seen(nv, 0);
    queue.push_back(0);
    seen[0] = 1;
    for (size_t qi = 0; qi < queue.size(); ++qi) {
        const int32_t v = queue[qi];
        for (int64_t e = cnt[v]; e < cnt[v + 1]; ++e)
            if (!seen[h.cyc[e]]) { seen[h.cyc[e]] = 1; queue.push_back(h.cyc[e]); }
    }
    if ((int64_t)queue.size() != nv)
        return set_err(ctx, VLS_E_MESH_NOT_CONNECTED, "mesh has %lld of %lld vertices in the first component",
                       (long long)queue.size(), (long long)nv);
    return VLS_OK;
}

template <typename T>
vls_status upload(vls_mesh *m, const std::vector<T> &h, const T **out) {
    void *p = nullptr;
    const size_t bytes = h.size() * sizeof(T);
    // 16 bytes of tail padding: aligned 16-byte loads of a row array's last
    // partial chunk stay inside the allocation
    if (hipMalloc(&p, bytes + 16) != hipSuccess) return set_err(m->ctx, VLS_E_OUT_OF_MEMORY, "hipMalloc %zu bytes", bytes);
    m->allocs.push_back(p);
    if (bytes && hipMemcpyAsync(p, h.data(), bytes, hipMemcpyHostToDevice, m->ctx->stream) != hipSuccess)
        return set_err(m->ctx, VLS_E_DEVICE, "upload failed");
    *out = (const T *)p;
    return VLS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// device memory of a run: either carved from one caller-provided block (a
// workspace: nothing is allocated) or one hipMalloc per buffer; a counting
// mode sizes a workspace with the same sequence of requests
// ---------------------------------------------------------------------------
struct DevArena {
    enum Mode { MALLOC, CARVE, COUNT } mode = MALLOC;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    std::vector<void *> owned;        // MALLOC mode: freed by release()
    static size_t padded(size_t bytes) {
        // 64 bytes of tail padding (aligned vector loads of a buffer's last
        // partial chunk stay inside it), 256-byte aligned starts
        return (bytes + 64 + 255) & ~(size_t)255;
    }
    size_t left() const { return used <= cap ? cap - used : 0; }
    template <typename T> hipError_t get(T **p, size_t n) {
        const size_t b = padded((n ? n : 1) * sizeof(T));
        if (mode == MALLOC) {
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, b);
            if (e == hipSuccess) owned.push_back(q);
            *p = (T *)q;
            used += b;
            return e;
        }
        if (mode == COUNT) {
            *p = (T *)(uintptr_t)(256 + used);   // never dereferenced
            used += b;
            return hipSuccess;
        }
        if (used + b > cap) { *p = nullptr; return hipErrorOutOfMemory; }
        *p = (T *)(base + used);
        used += b;
        return hipSuccess;
    }
    void release() {
        for (void *q : owned) (void)hipFree(q);
        owned.clear();
        used = 0;
    }
};

// run state of one pass on mesh m (the arrays of DState), from arena A
static hipError_t alloc_state(const vls_mesh *m, DevArena &A, DState &s) {
    s = DState{};
    const size_t nv = (size_t)m->nv, nnz = (size_t)m->nnz;
    size_t npow = 1;
    while (npow < nv) npow <<= 1;
    const int64_t g = std::max<int64_t>(0, m->euler_genus);
    s.tag_cap = (int32_t)std::min<int64_t>((int64_t)nv + 4096, INT32_MAX);
    s.front_cap = s.tag_cap;
    // event records: one per saddle / vanish insertion (at most nv); loop
    // buffers: the involved loops of merges (each at most the whole front)
    s.ev_cap = (int32_t)std::min<int64_t>((int64_t)nv, 65536 + (int64_t)nv / 16);
    s.ev_ids_cap = 4 * (int64_t)s.ev_cap + 64;
    s.lp_cap = (int32_t)(2 * g + 64);
    s.lp_he_cap = (int64_t)nnz / 4 + 65536;
    hipError_t e = hipSuccess;
#define A_(ptr, n) if (e == hipSuccess) e = A.get(&(ptr), (n))
    A_(s.rho0, nv); A_(s.rho1, nv); A_(s.key, nv); A_(s.parent, nv); A_(s.depth, nv);
    A_(s.lid, nnz); A_(s.stamp, nv); A_(s.cstamp, nv); A_(s.mark[0], nv); A_(s.mark[1], nv);
    A_(s.act[0], nv); A_(s.act[1], nv); A_(s.cand[0], nv); A_(s.cand[1], nv);
    A_(s.pend[0], nv); A_(s.pend[1], nv); A_(s.L, nv); A_(s.Lrnd, nv); A_(s.Lcls, nv);
    A_(s.ord, npow);
    A_(s.tag_parent, (size_t)s.tag_cap); A_(s.tag_fid, (size_t)s.tag_cap);
    A_(s.ev, (size_t)s.ev_cap * 16); A_(s.ev_rep, (size_t)s.ev_cap * 16); A_(s.ev_ids, (size_t)s.ev_ids_cap);
    A_(s.front_birth, (size_t)s.front_cap); A_(s.front_death, (size_t)s.front_cap);
    A_(s.lp, (size_t)s.lp_cap * 8); A_(s.lp_he, (size_t)s.lp_he_cap * 2); A_(s.lp_pts, (size_t)s.lp_he_cap * 3);
    A_(s.tn, (size_t)s.lp_cap * 4);
    A_(s.wck, 64 * 64);
    A_(s.wseg, (size_t)s.lp_he_cap);
    A_(s.ctl, 1);
#undef A_
    return e;
}

// Post-pass scratch: event chunks of kPostChunk events (walk checkpoints and
// counts), the fill buffer of the Reeb positions and the tunnel paths.  One
// event's fill needs the next power of two of 3 x (its loops' total length)
// entries; the loops are disjoint sets of crossed edges, so that is below
// 3 * nnz; a tunnel path has at most 2 * nv + 1 vertices.  A workspace of
// post_bytes() therefore always completes the post-passes, chunk by chunk.
constexpr int kPostChunk = 256;
static size_t post_fill_entries(const vls_mesh *m) {
    return (size_t)std::max<int64_t>(3 * m->nnz, 2 * m->nv + 2) + 16;
}
static size_t post_bytes(const vls_mesh *m) {
    const size_t C = kPostChunk;
    const size_t ntn = (size_t)(2 * std::max<int64_t>(0, m->euler_genus) + 64);
    return DevArena::padded((C + 1) * 8) * 2 + DevArena::padded(C * 16 * 64 * 4) + DevArena::padded(C * 16 * 4 * 8) +
           DevArena::padded(C * 3 * 8) + DevArena::padded((ntn + 1) * 8) * 2 + DevArena::padded(ntn * 8) +
           DevArena::padded(post_fill_entries(m) * 4);
}

// per-mesh device run state of vls_run / vls_batch_run (allocated at the
// first run, reused)
struct RunBuffers {
    DevArena arena;
    DState s{};
    int64_t nv = 0, nnz = 0, genus = 0;   // the mesh shape it was sized for
    ~RunBuffers() { arena.release(); }
};

// device bytes of one run's state on mesh m (the server's HBM admission
// charges a request this much plus its checkpoints)
static size_t run_buffer_bytes(const vls_mesh *m) {
    DevArena A;
    A.mode = DevArena::COUNT;
    DState s;
    (void)alloc_state(m, A, s);
    return A.used;
}

static vls_status make_run_buffers(vls_mesh *m, RunBuffers **out) {
    auto rb = std::make_unique<RunBuffers>();
    rb->nv = m->nv;
    rb->nnz = m->nnz;
    rb->genus = m->euler_genus;
    hipError_t e = alloc_state(m, rb->arena, rb->s);
    if (e != hipSuccess) return set_err(m->ctx, VLS_E_OUT_OF_MEMORY, "device allocation failed: %s", hipGetErrorString(e));
    *out = rb.release();
    return VLS_OK;
}

// Copies a run's bulk results from the device; frees the per-run device
// buffers.  Runs once per result (at the end of vls_run, or on first access
// for VLS_DEFER_RESULTS, or before the mesh's buffers are reused).
static vls_status fetch_results(vls_result *r) {
    Pending &pd = r->pend;
    if (!pd.active) return VLS_OK;
    pd.active = false;
    vls_context *ctx = pd.ctx;
    if (pd.mesh && pd.mesh->pending == r) pd.mesh->pending = nullptr;
    const DState &s = pd.s;
    const Ctl &c = pd.c;
    hipStream_t stream = pd.stream;
    const int64_t nv = r->nv;
    const int nev = c.n_events;
    (void)hipSetDevice(ctx->device);
    r->ev.resize((size_t)nev * 16);
    r->ev_ids.resize((size_t)c.ev_ids_used);
    r->front_birth.resize(c.next_front);
    r->front_death.resize(c.next_front);
    r->lp.resize((size_t)c.n_loops * 8);
    r->lp_he.resize((size_t)c.lp_he_used * 2);
    r->lp_pts.resize((size_t)c.lp_he_used * 3);
    std::vector<uint64_t> key(nv);
    r->parent.resize(nv);
    r->rho_final.resize(nv);
    auto cp = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream) : hipSuccess;
    };
    HIPCHK(ctx, cp(r->ev.data(), s.ev, r->ev.size() * 8));
    HIPCHK(ctx, cp(r->ev_ids.data(), s.ev_ids, r->ev_ids.size() * 8));
    HIPCHK(ctx, cp(r->front_birth.data(), s.front_birth, r->front_birth.size() * 4));
    HIPCHK(ctx, cp(r->front_death.data(), s.front_death, r->front_death.size() * 4));
    HIPCHK(ctx, cp(r->lp.data(), s.lp, r->lp.size() * 8));
    HIPCHK(ctx, cp(r->lp_he.data(), s.lp_he, r->lp_he.size() * 4));
    HIPCHK(ctx, cp(r->lp_pts.data(), s.lp_pts, r->lp_pts.size() * 8));
    HIPCHK(ctx, cp(key.data(), s.key, nv * 8));
    HIPCHK(ctx, cp(r->parent.data(), s.parent, nv * 4));
    const int64_t fin = c.steps;
    HIPCHK(ctx, cp(r->rho_final.data(), (fin & 1) ? s.rho1 : s.rho0, nv * 8));
    const int nck = (int)r->ckpt_steps.size();
    if (pd.rec_field) {
        r->ckpt.resize((size_t)nck * nv);
        HIPCHK(ctx, cp(r->ckpt.data(), s.ckpt, r->ckpt.size() * 8));
    }
    HIPCHK(ctx, hipStreamSynchronize(stream));
    for (void *q : pd.tmp_allocs) (void)hipFree(q);
    pd.tmp_allocs.clear();
    r->step.resize(nv);
    r->round.resize(nv);
    for (int64_t v = 0; v < nv; ++v) {
        if (key[v] == KEY_OUT) { r->step[v] = INT32_MAX; r->round[v] = 0; }
        else { r->step[v] = (int32_t)(key[v] >> 32); r->round[v] = (int32_t)(key[v] & 0xffffffffu); }
    }
    if (pd.rec_field) {
        r->ckpt_ok.assign(nck, 0);
        for (int q = 0; q < nck; ++q) {
            const int64_t st = r->ckpt_steps[q];
            r->ckpt_ok[q] = st >= 1 && st <= fin;
        }
    }
    return VLS_OK;
}

static vls_status wait_launched(vls_result *r);

// statuses with which a run still produces a result (partial for a stall)
static bool is_run_status(vls_status st) {
    return st == VLS_E_STALLED || st == VLS_E_SEED_INVALID || st == VLS_E_INVARIANT || st == VLS_E_CAPACITY;
}

static vls_status ensure(const vls_result *r) {
    vls_result *q = const_cast<vls_result *>(r);
    if (q->failed) return q->launch_status;
    if (q->launched) {
        vls_status st = wait_launched(q);
        if (st != VLS_OK && !is_run_status(st)) return st;
    }
    return fetch_results(q);
}

extern "C" {

vls_status vls_mesh_create(vls_context *ctx, int64_t nv, const double *xyz, int64_t nf, const int32_t *tri,
                           vls_mesh **out) {
    if (!ctx || !out || !xyz || !tri || nv < 4 || nf < 4) return set_err(ctx, VLS_E_INVALID_ARG, "bad mesh arguments");
    *out = nullptr;
    if (nv >= INT32_MAX) return set_err(ctx, VLS_E_TOO_LARGE, "nv = %lld", (long long)nv);
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
    HostAdj h;
    vls_status st = build_adjacency(ctx, nv, nf, tri, h);
    if (st) return st;
    auto m = std::make_unique<vls_mesh>();
    m->ctx = ctx;
    m->nv = nv;
    m->nf = nf;
    m->nnz = (int64_t)h.cyc.size();
    m->ne = m->nnz / 2;
    m->dmax = h.dmax;
    const int64_t chi = nv - m->ne + nf;
    m->euler_genus = (int32_t)((2 - chi) / 2);
    m->xyz.assign(xyz, xyz + 3 * nv);
    DMesh &d = m->d;
    d.nv = (int32_t)nv;
    d.dmax = h.dmax;
    d.nnz = m->nnz;
    if ((st = upload(m.get(), h.rp, &d.rp)) || (st = upload(m.get(), h.adj, &d.adj)) ||
        (st = upload(m.get(), h.cyc, &d.cyc)) || (st = upload(m.get(), h.src, &d.src)) ||
        (st = upload(m.get(), h.rev, &d.rev)) || (st = upload(m.get(), h.succ, &d.succ)) ||
        (st = upload(m.get(), h.nin, &d.nin)) || (st = upload(m.get(), h.ell, &d.ell)) ||
        (st = upload(m.get(), h.lrow, &d.lrow)) || (st = upload(m.get(), h.hrec, &d.hrec)) ||
        (st = upload(m.get(), m->xyz, &d.xyz))) {
        for (void *p : m->allocs) (void)hipFree(p);
        return st;
    }
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        for (void *p : m->allocs) (void)hipFree(p);
        return set_err(ctx, VLS_E_DEVICE, "mesh upload failed");
    }
    *out = m.release();
    return VLS_OK;
}

vls_status vls_mesh_info(const vls_mesh *m, int64_t *nv, int64_t *ne, int64_t *nf, int32_t *dmax, int32_t *eg) {
    if (!m) return VLS_E_INVALID_ARG;
    if (nv) *nv = m->nv;
    if (ne) *ne = m->ne;
    if (nf) *nf = m->nf;
    if (dmax) *dmax = m->dmax;
    if (eg) *eg = m->euler_genus;
    return VLS_OK;
}

vls_status vls_mesh_prepare_fem(vls_mesh *m, double *sigma, double *row_sum_max) {
    if (!m) return VLS_E_INVALID_ARG;
    vls_context *ctx = m->ctx;
    if (!m->d.fem_g) {
        if (m->pending) (void)fetch_results(m->pending);
        if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
        void *g = nullptr, *tmp = nullptr;
        const size_t gb = (size_t)m->nnz * sizeof(double) + 64;
        const size_t mb = ((size_t)m->nv * sizeof(double) + 255) & ~(size_t)255;
        if (hipMalloc(&g, gb) != hipSuccess) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "operator coefficients");
        if (hipMalloc(&tmp, mb + 256 + 64) != hipSuccess) {
            (void)hipFree(g);
            return set_err(ctx, VLS_E_OUT_OF_MEMORY, "operator scratch");
        }
        double *mass = (double *)tmp;
        double *scal = (double *)((char *)tmp + mb);
        unsigned long long *bits = (unsigned long long *)((char *)tmp + mb + 128);
        double hs[2] = {0.0, 0.0};
        unsigned long long hb = 0;
        hipStream_t st = ctx->stream;
        hipError_t e = hipMemsetAsync(bits, 0, sizeof(unsigned long long), st);
        if (e == hipSuccess) e = launch_fem_operator(m->d, mass, scal, (double *)g, bits, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hs, scal, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hb, bits, sizeof hb, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(tmp);
        if (e != hipSuccess) {
            (void)hipFree(g);
            return set_err(ctx, VLS_E_DEVICE, "finite-element operator: %s", hipGetErrorString(e));
        }
        std::memcpy(&hs[1], &hb, sizeof(double));
        if (!(hs[1] > 0.0) || !std::isfinite(hs[1])) {
            (void)hipFree(g);
            return set_err(ctx, VLS_E_INVALID_ARG, "finite-element operator is degenerate (largest row sum %g)", hs[1]);
        }
        m->allocs.push_back(g);
        m->d.fem_g = (const double *)g;
        m->fem_sigma = hs[0];
        m->fem_dmax = hs[1];
    }
    if (sigma) *sigma = m->fem_sigma;
    if (row_sum_max) *row_sum_max = m->fem_dmax;
    return VLS_OK;
}

vls_status vls_mesh_fem_coefficients(const vls_mesh *m, int64_t cap, double *g, int64_t *n_out) {
    if (!m || !n_out) return VLS_E_INVALID_ARG;
    if (!m->d.fem_g) return set_err(m->ctx, VLS_E_INVALID_ARG, "the finite-element operator is not prepared");
    *n_out = m->nnz;
    if (cap == 0) return VLS_OK;
    if (cap < m->nnz || !g) return VLS_E_BUFFER_TOO_SMALL;
    if (hipSetDevice(m->ctx->device) != hipSuccess) return set_err(m->ctx, VLS_E_DEVICE, "hipSetDevice");
    if (hipMemcpyAsync(g, m->d.fem_g, (size_t)m->nnz * sizeof(double), hipMemcpyDeviceToHost, m->ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(m->ctx->stream) != hipSuccess)
        return set_err(m->ctx, VLS_E_DEVICE, "coefficient copy failed");
    return VLS_OK;
}

vls_status vls_mesh_destroy(vls_mesh *m) {
    if (!m) return VLS_E_INVALID_ARG;
    if (m->pending) (void)fetch_results(m->pending);
    (void)hipSetDevice(m->ctx->device);
    delete m->rb;
    for (void *p : m->allocs) (void)hipFree(p);
    delete m;
    return VLS_OK;
}

static uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

}  // extern "C"

// One run in flight: everything prepared on the host before the launch of
// the step kernel, and what finishing it needs afterwards.
struct RunPrep {
    vls_mesh *m = nullptr;
    bool priv = false;          // device state owned by the caller (server request), not by the mesh
    bool ws = false;            // run state carved from a caller workspace: nothing allocated
    hipStream_t stream = nullptr;
    DState s{};
    DParams dp{};
    int64_t seed = 0;
    bool rec_field = false;
    std::vector<void *> tmp_allocs;
    DevArena post;              // post-pass scratch: the workspace's tail (ws) or hipMalloc
    vls_params params{};        // vls_run_async: parameters kept for the wait
    std::vector<int64_t> ckpt;  // vls_run_async: checkpoint list kept for the wait
    int grid = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    // post-pass outputs computed for many runs at once (vls_batch_run)
    bool post_given = false;
    std::vector<double> g_node_pos, g_tn_len;
    std::vector<int32_t> g_tn, g_tn_v;
    std::vector<int64_t> g_tn_off;
    ~RunPrep() {
        for (void *q : tmp_allocs) (void)hipFree(q);
        post.release();
        for (hipEvent_t e : {e0, e1, e2, e3}) if (e) (void)hipEventDestroy(e);
    }
};

// checks, device buffers, parameters; enqueues init + seed on rp.stream.
// priv: the caller's run state (server request); ws: a workspace arena the
// run state, checkpoints and post-pass scratch are carved from (no
// allocation, no events).
static vls_status prepare_run(vls_context *ctx, vls_mesh *m, const vls_params *p, RunPrep &rp,
                              RunBuffers *priv = nullptr, DevArena *ws = nullptr,
                              const int32_t *d_seed_set = nullptr, int32_t n_seed_set = 0) {
    if (p->struct_size != sizeof(vls_params)) return set_err(ctx, VLS_E_INVALID_ARG, "vls_params.struct_size mismatch");
    if (!priv && !ws && m->pending) {
        vls_status fs = fetch_results(m->pending);
        if (fs) return fs;
    }
    const int64_t nv = m->nv;
    int64_t seed = p->seed_vertex;
    if (seed < 0) seed = (int64_t)(splitmix64(p->rng_seed) % (uint64_t)nv);
    if (seed >= nv) return set_err(ctx, VLS_E_INVALID_ARG, "seed vertex %lld >= nv", (long long)seed);
    if (p->seed_radius < 0 || p->seed_radius > 1000) return set_err(ctx, VLS_E_INVALID_ARG, "seed_radius");
    if (p->max_steps < 1 || p->max_steps >= INT32_MAX) return set_err(ctx, VLS_E_INVALID_ARG, "max_steps");
    if (p->stall_steps < 1) return set_err(ctx, VLS_E_INVALID_ARG, "stall_steps");
    if (p->block != 0 && p->block != 256) return set_err(ctx, VLS_E_INVALID_ARG, "block must be 256");
    if ((p->flags & VLS_DENSE_FIELD) && nv >= (int64_t)1 << 29)
        return set_err(ctx, VLS_E_INVALID_ARG, "VLS_DENSE_FIELD needs fewer than 2^29 vertices");
    if (p->n_ckpt < 0 || p->pass_slots < 0) return set_err(ctx, VLS_E_INVALID_ARG, "n_ckpt / pass_slots");
    if ((p->flags & (VLS_TUNNEL_PASS | VLS_REFINE_PASS | VLS_REEB_REFINE)) && (priv || ws))
        return set_err(ctx, VLS_E_INVALID_ARG,
                       "the tunnel-loop, refinement and Reeb refinement passes run with vls_run only");
    const bool fem = (p->flags & VLS_FEM_LAPLACIAN) != 0;
    if (fem) {
        if (p->flags & (VLS_DENSE_FIELD | VLS_TUNNEL_PASS | VLS_REFINE_PASS))
            return set_err(ctx, VLS_E_INVALID_ARG,
                           "VLS_FEM_LAPLACIAN runs with the update-list field step of the initial pass only");
        if (priv) return set_err(ctx, VLS_E_INVALID_ARG, "VLS_FEM_LAPLACIAN is not served");
        if (!m->d.fem_g) {
            if (ws) return set_err(ctx, VLS_E_INVALID_ARG, "VLS_FEM_LAPLACIAN: call vls_mesh_prepare_fem first");
            if (vls_status fs = vls_mesh_prepare_fem(m, nullptr, nullptr)) return fs;
        }
    }
    rp.m = m;
    rp.seed = seed;
    rp.rec_field = (p->flags & VLS_RECORD_FIELD) && p->n_ckpt > 0 && p->ckpt_steps;
    if (!rp.stream) rp.stream = ctx->stream;
    if (ws) {
        rp.ws = true;
        if (alloc_state(m, *ws, rp.s) != hipSuccess) return set_err(ctx, VLS_E_BUFFER_TOO_SMALL, "workspace too small");
    } else if (priv) {
        rp.priv = true;
        rp.s = priv->s;
    } else {
        if (!m->rb) {
            vls_status st = make_run_buffers(m, &m->rb);
            if (st) return st;
        }
        rp.s = m->rb->s;
    }
    DState &s = rp.s;
    hipStream_t stream = rp.stream;
    s.n_ckpt = 0;
    s.ckpt = nullptr;
    s.ckpt_steps = nullptr;
    if (rp.rec_field) {
        double *a = nullptr;
        int64_t *b = nullptr;
        if (ws) {
            if (ws->get(&a, (size_t)p->n_ckpt * nv) != hipSuccess || ws->get(&b, (size_t)p->n_ckpt) != hipSuccess)
                return set_err(ctx, VLS_E_BUFFER_TOO_SMALL, "workspace too small for the checkpoints");
        } else {
            if (hipMalloc(&a, (size_t)p->n_ckpt * nv * sizeof(double)) != hipSuccess) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "checkpoint buffers");
            rp.tmp_allocs.push_back(a);
            if (hipMalloc(&b, (size_t)p->n_ckpt * sizeof(int64_t)) != hipSuccess) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "checkpoint buffers");
            rp.tmp_allocs.push_back(b);
        }
        s.ckpt = a;
        s.ckpt_steps = b;
        s.n_ckpt = p->n_ckpt;
        HIPCHK(ctx, hipMemcpyAsync(b, p->ckpt_steps, (size_t)p->n_ckpt * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    }
    if (ws) {
        // the rest of the workspace is the post-pass scratch
        rp.post.mode = DevArena::CARVE;
        rp.post.base = ws->base + ws->used;
        rp.post.cap = ws->left();
        if (rp.post.cap < post_bytes(m)) return set_err(ctx, VLS_E_BUFFER_TOO_SMALL, "workspace too small for the post-passes");
    }
    DParams &dp = rp.dp;
    const double dmx = fem ? m->fem_dmax : (double)m->dmax;
    const double dt = p->dt_mode == 1 ? 0.25 / dmx : 50.0 / dmx;
    dp.tau = p->tau;
    dp.a = p->a;
    dp.w = p->w;
    dp.e = p->e;
    dp.c = dt * (p->mu / 2.0);
    dp.seed = seed;
    dp.r0 = p->seed_radius;
    dp.stall_steps = p->stall_steps;
    dp.max_steps = p->max_steps;
    dp.topo_global = (p->flags & VLS_TOPO_GLOBAL_PATH) ? 1 : 0;
    dp.coherent = (p->flags & VLS_COHERENT_SHARING) ? 1 : 0;
    dp.lockstep = (p->flags & VLS_LOCKSTEP) ? 1 : 0;
    dp.dense = (p->flags & VLS_DENSE_FIELD) ? 1 : 0;
    dp.fem = fem ? 1 : 0;
    dp.n_seed_set = n_seed_set;
    dp.seed_set = d_seed_set;
    if (!ws) {
        HIPCHK(ctx, hipEventCreate(&rp.e0));
        HIPCHK(ctx, hipEventCreate(&rp.e1));
        HIPCHK(ctx, hipEventCreate(&rp.e2));
        HIPCHK(ctx, hipEventCreate(&rp.e3));
        HIPCHK(ctx, hipEventRecord(rp.e0, stream));
    }
    HIPCHK(ctx, launch_init(m->d, s, m->nnz, stream));
    HIPCHK(ctx, launch_seed(m->d, s, dp, stream));
    if (!ws) HIPCHK(ctx, hipEventRecord(rp.e1, stream));
    return VLS_OK;
}

// Reeb positions and tunnel paths of a finished run, into r (host), with
// post-pass scratch from rp.post: one chunk of events / tunnels when the
// scratch is hipMalloc'ed, as many chunks as the workspace needs otherwise.
static vls_status post_passes(vls_context *ctx, RunPrep &rp, const Ctl &c, vls_result &r) {
    vls_mesh *m = rp.m;
    const DState &s = rp.s;
    hipStream_t stream = rp.stream;
    DevArena &A = rp.post;
    const bool carve = A.mode == DevArena::CARVE;
    const int nev = c.n_events, ntn = c.n_tunnels;
    r.node_pos.assign((size_t)nev * 3, 0.0);
    r.tn.resize((size_t)ntn * 4);
    r.tn_off.assign(ntn + 1, 0);
    r.tn_len.assign(ntn, 0.0);
    const size_t mark = A.used;
    auto toolarge = [&](const char *what) {
        return set_err(ctx, VLS_E_CAPACITY, "post-pass scratch too small for %s", what);
    };
    if (nev > 0) {
        const int C = carve ? std::min(nev, kPostChunk) : nev;
        int64_t *dcnt = nullptr, *doff = nullptr, *dmeta = nullptr;
        int32_t *dck = nullptr;
        double *dpos = nullptr;
        if (A.get(&dcnt, C + 1) || A.get(&doff, C + 1) || A.get(&dck, (size_t)C * 16 * 64) ||
            A.get(&dmeta, (size_t)C * 16 * 4) || A.get(&dpos, (size_t)C * 3))
            return carve ? toolarge("event chunks") : set_err(ctx, VLS_E_OUT_OF_MEMORY, "post-pass buffers");
        int32_t *dbuf = nullptr;
        size_t fill_cap = 0;   // entries
        if (carve) {
            fill_cap = A.left() / 4 > 64 ? A.left() / 4 - 64 : 0;
            dbuf = (int32_t *)(A.base + A.used);
        }
        std::vector<int64_t> cnt(C + 1, 0), off;
        for (int c0 = 0; c0 < nev; c0 += C) {
            const int nc = std::min(C, nev - c0);
            HIPCHK(ctx, launch_reeb_count(m->d, s, c0, nc, dcnt, dck, dmeta, stream));
            HIPCHK(ctx, hipMemcpyAsync(cnt.data(), dcnt, nc * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
            HIPCHK(ctx, hipStreamSynchronize(stream));
            std::vector<int64_t> np(nc);
            int64_t tot = 0;
            for (int i = 0; i < nc; ++i) {
                int64_t q = 1;
                while (q < cnt[i]) q <<= 1;
                np[i] = q;
                tot += q;
            }
            if (!carve) {
                // one fill over the whole chunk
                if (A.get(&dbuf, (size_t)tot + 16)) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "post-pass fill buffer");
                fill_cap = (size_t)tot + 16;
            }
            for (int a = 0; a < nc;) {
                int b = a;
                int64_t used = 0;
                while (b < nc && used + np[b] <= (int64_t)fill_cap) used += np[b++];
                if (b == a) return toolarge("one event's front triangles");
                off.assign(b - a + 1, 0);
                for (int i = a; i < b; ++i) off[i - a + 1] = off[i - a] + np[i];
                HIPCHK(ctx, hipMemcpyAsync(doff, off.data(), (b - a + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream));
                HIPCHK(ctx, launch_reeb_fill(m->d, s, c0 + a, b - a, doff, dcnt + a, dck + (size_t)a * 16 * 64,
                                             dmeta + (size_t)a * 16 * 4, dbuf, stream));
                HIPCHK(ctx, launch_reeb_mean(m->d, b - a, doff, dcnt + a, dbuf, dpos + 3 * a, stream));
                // the offsets are re-uploaded by the next sub-chunk: wait for this one
                HIPCHK(ctx, hipStreamSynchronize(stream));
                a = b;
            }
            HIPCHK(ctx, hipMemcpyAsync(r.node_pos.data() + 3 * (size_t)c0, dpos, (size_t)nc * 3 * sizeof(double),
                                       hipMemcpyDeviceToHost, stream));
        }
        HIPCHK(ctx, hipStreamSynchronize(stream));
    }
    if (!carve) A.release();
    A.used = mark;
    if (ntn > 0) {
        HIPCHK(ctx, hipMemcpyAsync(r.tn.data(), s.tn, (size_t)ntn * 4 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        int64_t *dtcnt = nullptr, *dtoff = nullptr;
        double *dtlen = nullptr;
        if (A.get(&dtcnt, ntn + 1) || A.get(&dtoff, ntn + 1) || A.get(&dtlen, ntn))
            return carve ? toolarge("tunnel counts") : set_err(ctx, VLS_E_OUT_OF_MEMORY, "post-pass buffers");
        std::vector<int64_t> tcnt(ntn + 1, 0);
        HIPCHK(ctx, launch_tunnel_count(s, ntn, dtcnt, stream));
        HIPCHK(ctx, hipMemcpyAsync(tcnt.data(), dtcnt, ntn * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        for (int i = 0; i < ntn; ++i) r.tn_off[i + 1] = r.tn_off[i] + tcnt[i];
        r.tn_v.resize((size_t)r.tn_off[ntn]);
        int32_t *dtn = nullptr;
        size_t cap = 0;
        if (carve) {
            cap = A.left() / 4 > 64 ? A.left() / 4 - 64 : 0;
            dtn = (int32_t *)(A.base + A.used);
        } else {
            if (A.get(&dtn, (size_t)r.tn_off[ntn] + 16)) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "tunnel buffer");
            cap = (size_t)r.tn_off[ntn] + 16;
        }
        std::vector<int64_t> toff;
        for (int a = 0; a < ntn;) {
            int b = a;
            while (b < ntn && r.tn_off[b + 1] - r.tn_off[a] <= (int64_t)cap) ++b;
            if (b == a) return toolarge("one tunnel path");
            toff.assign(b - a + 1, 0);
            for (int i = a; i <= b; ++i) toff[i - a] = r.tn_off[i] - r.tn_off[a];
            HIPCHK(ctx, hipMemcpyAsync(dtoff, toff.data(), (b - a + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream));
            HIPCHK(ctx, launch_tunnel_fill(m->d, s, a, b - a, dtoff, dtn, dtlen + a, stream));
            HIPCHK(ctx, hipMemcpyAsync(r.tn_v.data() + r.tn_off[a], dtn, (size_t)(r.tn_off[b] - r.tn_off[a]) * 4,
                                       hipMemcpyDeviceToHost, stream));
            HIPCHK(ctx, hipStreamSynchronize(stream));
            a = b;
        }
        HIPCHK(ctx, hipMemcpyAsync(r.tn_len.data(), dtlen, ntn * sizeof(double), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        r.tn_pts.resize(r.tn_v.size() * 3);
        for (size_t q = 0; q < r.tn_v.size(); ++q)
            std::memcpy(r.tn_pts.data() + 3 * q, m->xyz.data() + 3 * (size_t)r.tn_v[q], 3 * sizeof(double));
    }
    if (!carve) A.release();
    A.used = mark;
    return VLS_OK;
}

// Post-passes of many runs at once (a batch, or the server's completed
// requests): the events (and tunnels) of every run are listed together and
// each pass is one launch over a chunk of that list, so the runs' short
// dependent walks run side by side instead of run after run with a
// synchronisation between each.  The outputs are those of post_passes (the
// same kernels' bodies, one entry per block or thread), handed to
// finish_run through the RunPreps.  dm / ds: device arrays of the runs'
// meshes and states; cs: each run's control block.  Scratch: chunk arrays of
// fixed size, a fill buffer and a path buffer (multi_post_bytes), from A.
constexpr int kMultiEvents = 4096;
constexpr int kMultiTunnels = 65536;
static void multi_post_caps(const std::vector<const vls_mesh *> &meshes, size_t &fill_cap, size_t &path_cap) {
    fill_cap = (size_t)1 << 22;
    path_cap = (size_t)1 << 22;
    for (const vls_mesh *m : meshes) {
        fill_cap = std::max(fill_cap, post_fill_entries(m));
        path_cap = std::max(path_cap, (size_t)(2 * m->nv + 2));
    }
}
static size_t multi_post_bytes(size_t fill_cap, size_t path_cap) {
    const size_t C = kMultiEvents, TC = kMultiTunnels;
    return DevArena::padded(C * 4) * 2 + DevArena::padded((C + 1) * 8) * 2 + DevArena::padded(C * 16 * 64 * 4) +
           DevArena::padded(C * 16 * 4 * 8) + DevArena::padded(C * 3 * 8) + DevArena::padded((fill_cap + 16) * 4) +
           DevArena::padded(TC * 4) * 2 + DevArena::padded((TC + 1) * 8) * 2 + DevArena::padded(TC * 8) +
           DevArena::padded((path_cap + 16) * 4);
}
static vls_status multi_post_passes(vls_context *ctx, const std::vector<const vls_mesh *> &meshes,
                                    const std::vector<RunPrep *> &preps, const std::vector<Ctl> &cs, const DMesh *dm,
                                    const DState *ds, DevArena &A, hipStream_t stream) {
    const int n = (int)preps.size();
    std::vector<int32_t> evm, eve, tnm, tnt;
    size_t fill_cap, path_cap;
    multi_post_caps(meshes, fill_cap, path_cap);
    for (int i = 0; i < n; ++i) {
        RunPrep &rp = *preps[i];
        const int nev = cs[i].n_events, ntn = cs[i].n_tunnels;
        rp.g_node_pos.assign((size_t)nev * 3, 0.0);
        rp.g_tn.resize((size_t)ntn * 4);
        rp.g_tn_off.assign(ntn + 1, 0);
        rp.g_tn_len.assign(ntn, 0.0);
        rp.g_tn_v.clear();
        for (int e = 0; e < nev; ++e) { evm.push_back(i); eve.push_back(e); }
        for (int e = 0; e < ntn; ++e) { tnm.push_back(i); tnt.push_back(e); }
        if (ntn)
            HIPCHK(ctx, hipMemcpyAsync(rp.g_tn.data(), rp.s.tn, (size_t)ntn * 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                       stream));
    }
    const int E = (int)evm.size(), T = (int)tnm.size();
    const int C = kMultiEvents, TC = kMultiTunnels;
    int32_t *devm = nullptr, *deve = nullptr, *dtnm = nullptr, *dtnt = nullptr, *dck = nullptr, *dbuf = nullptr,
            *dpath = nullptr;
    int64_t *dcnt = nullptr, *doff = nullptr, *dmeta = nullptr, *dtcnt = nullptr, *dtoff = nullptr;
    double *dpos = nullptr, *dlen = nullptr;
    const size_t mark = A.used;
    struct Rel {
        DevArena *a;
        size_t mark;
        ~Rel() {
            if (a->mode == DevArena::MALLOC) a->release();
            a->used = mark;
        }
    } rel{&A, mark};
    if (A.get(&devm, C) || A.get(&deve, C) || A.get(&dcnt, C + 1) || A.get(&doff, C + 1) ||
        A.get(&dck, (size_t)C * 16 * 64) || A.get(&dmeta, (size_t)C * 16 * 4) || A.get(&dpos, (size_t)C * 3) ||
        A.get(&dbuf, fill_cap + 16) || A.get(&dtnm, TC) || A.get(&dtnt, TC) || A.get(&dtcnt, TC + 1) ||
        A.get(&dtoff, TC + 1) || A.get(&dlen, TC) || A.get(&dpath, path_cap + 16))
        return set_err(ctx, VLS_E_OUT_OF_MEMORY, "multi-run post-pass buffers");
    std::vector<int64_t> cnt(C + 1), np(C), off;
    std::vector<double> pos((size_t)C * 3);
    for (int g0 = 0; g0 < E; g0 += C) {
        const int nc = std::min(C, E - g0);
        HIPCHK(ctx, hipMemcpyAsync(devm, evm.data() + g0, (size_t)nc * 4, hipMemcpyHostToDevice, stream));
        HIPCHK(ctx, hipMemcpyAsync(deve, eve.data() + g0, (size_t)nc * 4, hipMemcpyHostToDevice, stream));
        HIPCHK(ctx, launch_reeb_count_multi(dm, ds, devm, deve, nc, dcnt, dck, dmeta, stream));
        HIPCHK(ctx, hipMemcpyAsync(cnt.data(), dcnt, nc * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        for (int i = 0; i < nc; ++i) {
            int64_t q = 1;
            while (q < cnt[i]) q <<= 1;
            np[i] = q;
        }
        for (int a = 0; a < nc;) {
            int b = a;
            int64_t used = 0;
            while (b < nc && used + np[b] <= (int64_t)fill_cap) used += np[b++];
            if (b == a) return set_err(ctx, VLS_E_CAPACITY, "post-pass scratch too small for one event's front triangles");
            off.assign(b - a + 1, 0);
            for (int i = a; i < b; ++i) off[i - a + 1] = off[i - a] + np[i];
            HIPCHK(ctx, hipMemcpyAsync(doff, off.data(), (b - a + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream));
            HIPCHK(ctx, launch_reeb_fill_multi(dm, ds, devm, deve, a, b - a, doff, dcnt + a, dck + (size_t)a * 16 * 64,
                                               dmeta + (size_t)a * 16 * 4, dbuf, stream));
            HIPCHK(ctx, launch_reeb_mean_multi(dm, devm, a, b - a, doff, dcnt + a, dbuf, dpos + 3 * (size_t)a, stream));
            // the offsets are re-uploaded by the next sub-chunk: wait for this one
            HIPCHK(ctx, hipStreamSynchronize(stream));
            a = b;
        }
        HIPCHK(ctx, hipMemcpyAsync(pos.data(), dpos, (size_t)nc * 3 * sizeof(double), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        for (int i = 0; i < nc; ++i)
            std::memcpy(preps[evm[g0 + i]]->g_node_pos.data() + 3 * (size_t)eve[g0 + i], pos.data() + 3 * (size_t)i,
                        3 * sizeof(double));
    }
    std::vector<int64_t> tc(TC + 1), toff;
    std::vector<int32_t> path;
    std::vector<double> len(TC);
    for (int g0 = 0; g0 < T; g0 += TC) {
        const int nt = std::min(TC, T - g0);
        HIPCHK(ctx, hipMemcpyAsync(dtnm, tnm.data() + g0, (size_t)nt * 4, hipMemcpyHostToDevice, stream));
        HIPCHK(ctx, hipMemcpyAsync(dtnt, tnt.data() + g0, (size_t)nt * 4, hipMemcpyHostToDevice, stream));
        HIPCHK(ctx, launch_tunnel_count_multi(ds, dtnm, dtnt, nt, dtcnt, stream));
        HIPCHK(ctx, hipMemcpyAsync(tc.data(), dtcnt, nt * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        for (int a = 0; a < nt;) {
            int b = a;
            int64_t used = 0;
            while (b < nt && used + tc[b] <= (int64_t)path_cap) used += tc[b++];
            if (b == a) return set_err(ctx, VLS_E_CAPACITY, "post-pass scratch too small for one tunnel path");
            toff.assign(b - a + 1, 0);
            for (int i = a; i < b; ++i) toff[i - a + 1] = toff[i - a] + tc[i];
            HIPCHK(ctx, hipMemcpyAsync(dtoff, toff.data(), (b - a + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream));
            HIPCHK(ctx, launch_tunnel_fill_multi(dm, ds, dtnm, dtnt, a, b - a, dtoff, dpath, dlen + a, stream));
            path.resize((size_t)toff[b - a]);
            HIPCHK(ctx, hipMemcpyAsync(path.data(), dpath, path.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
            HIPCHK(ctx, hipStreamSynchronize(stream));
            // tunnels of one run are consecutive in the list and in order
            for (int i = a; i < b; ++i) {
                RunPrep &rp = *preps[tnm[g0 + i]];
                const int k = tnt[g0 + i];
                rp.g_tn_off[k + 1] = rp.g_tn_off[k] + tc[i];
                rp.g_tn_v.insert(rp.g_tn_v.end(), path.begin() + toff[i - a], path.begin() + toff[i - a + 1]);
            }
            a = b;
        }
        HIPCHK(ctx, hipMemcpyAsync(len.data(), dlen, nt * sizeof(double), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        for (int i = 0; i < nt; ++i) preps[tnm[g0 + i]]->g_tn_len[tnt[g0 + i]] = len[i];
    }
    HIPCHK(ctx, hipStreamSynchronize(stream));
    for (RunPrep *rp : preps) rp->post_given = true;
    return VLS_OK;
}

// Tunnel-loop passes of every handle loop and, with VLS_REFINE_PASS, the
// refinement pass of every tunnel, after the initial pass (vls_run only).
// As many passes run at once as there are co-resident workgroups and slots
// of per-vertex state within half of the free device memory (the paper's
// rule: as many passes as memory allows).
static vls_status run_passes(vls_context *ctx, RunPrep &rp, const vls_params *p, const Ctl &c, vls_result &r) {
    const bool refine = (p->flags & VLS_REFINE_PASS) != 0;
    if (!(p->flags & VLS_TUNNEL_PASS) && !refine) return VLS_OK;
    vls_mesh *m = rp.m;
    hipStream_t stream = rp.stream;
    const int nl = c.n_loops;
    std::vector<int64_t> lp((size_t)nl * 8);
    if (nl) HIPCHK(ctx, hipMemcpyAsync(lp.data(), rp.s.lp, lp.size() * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(ctx, hipStreamSynchronize(stream));
    std::vector<PassTask> tun;
    for (int i = 0; i < nl; ++i)
        if (lp[8 * (size_t)i + 2]) tun.push_back(PassTask{0, i});
    const int nt = (int)tun.size();
    vls_summary &S = r.sum;
    S.n_tunnel_passes = nt;
    S.n_refine_passes = refine ? nt : 0;
    if (nt == 0) return VLS_OK;
    // slots
    const int64_t nv = m->nv, nnz = m->nnz;
    DevArena cnt;
    cnt.mode = DevArena::COUNT;
    PassSlot tmpl{};
    auto alloc_slot = [&](DevArena &A, PassSlot &q) -> hipError_t {
        hipError_t e = hipSuccess;
#define P_(ptr, n) if (e == hipSuccess) e = A.get(&(ptr), (size_t)(n))
        P_(q.rho, nv); P_(q.tmp, nv); P_(q.ta, nv); P_(q.prev, nv); P_(q.key, nv); P_(q.par, nv);
        P_(q.mark, nv); P_(q.cst, nv); P_(q.upd, nv); P_(q.flag, nv); P_(q.pos, nv); P_(q.U[0], nv);
        P_(q.U[1], nv); P_(q.cand, nv); P_(q.pend[0], nv); P_(q.pend[1], nv); P_(q.touched, nv);
        P_(q.flist, nv); P_(q.buf, nv); P_(q.side, nv); P_(q.cutbits, nnz / 32 + 1);
#undef P_
        return e;
    };
    (void)alloc_slot(cnt, tmpl);
    const size_t slot_bytes = cnt.used;
    size_t free_b = 0, total_b = 0;
    HIPCHK(ctx, hipMemGetInfo(&free_b, &total_b));
    const int maxg = max_coresident_passes();
    if (maxg <= 0) return set_err(ctx, VLS_E_DEVICE, "occupancy query of the pass kernel failed");
    int64_t ns = std::min<int64_t>({(int64_t)nt, (int64_t)maxg, (int64_t)(free_b / 2 / slot_bytes)});
    if (p->pass_slots > 0) ns = std::min<int64_t>(ns, p->pass_slots);
    if (ns < 1) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "no memory for one pass slot (%zu bytes)", slot_bytes);
    DevArena A;   // hipMalloc'ed, released on return
    struct Rel { DevArena &a; ~Rel() { a.release(); } } rel{A};
    std::vector<PassSlot> slots((size_t)ns);
    for (auto &q : slots) {
        if (alloc_slot(A, q) != hipSuccess) return set_err(ctx, VLS_E_OUT_OF_MEMORY, "pass slots");
        HIPCHK(ctx, launch_pass_slot_init(q, (int32_t)nv, nnz, stream));
    }
    PassSlot *dslots = nullptr;
    PassTask *dtasks = nullptr;
    PassResult *dres[2] = {nullptr, nullptr};
    int32_t *dout[2] = {nullptr, nullptr};
    int *dnext = nullptr;
    unsigned long long *dused = nullptr;
    const int64_t out_cap = 2 * nv + (1 << 20);
    if (A.get(&dslots, (size_t)ns) || A.get(&dtasks, (size_t)nt) || A.get(&dres[0], (size_t)nt) ||
        A.get(&dres[1], (size_t)nt) || A.get(&dout[0], (size_t)out_cap) || A.get(&dout[1], (size_t)out_cap) ||
        A.get(&dnext, 2) || A.get(&dused, 2))
        return set_err(ctx, VLS_E_OUT_OF_MEMORY, "pass buffers");
    HIPCHK(ctx, hipMemcpyAsync(dslots, slots.data(), slots.size() * sizeof(PassSlot), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemsetAsync(dnext, 0, 2 * sizeof(int), stream));
    HIPCHK(ctx, hipMemsetAsync(dused, 0, 2 * sizeof(unsigned long long), stream));
    PassArgs a{};
    a.m = m->d;
    a.s = rp.s;
    a.nslots = (int)ns;
    a.slots = dslots;
    a.out_cap = out_cap;
    a.tau = rp.dp.tau;
    a.a = rp.dp.a;
    a.w = rp.dp.w;
    a.e = rp.dp.e;
    a.c = rp.dp.c;
    a.max_steps = p->max_steps;
    a.stall_steps = p->stall_steps;
    a.rel_eps = 0.1;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    struct EvRel { hipEvent_t *e; ~EvRel() { for (int i = 0; i < 3; ++i) if (e[i]) (void)hipEventDestroy(e[i]); } } evrel{ev};
    for (auto &e : ev) HIPCHK(ctx, hipEventCreate(&e));
    HIPCHK(ctx, hipEventRecord(ev[0], stream));
    for (int k = 0; k < (refine ? 2 : 1); ++k) {
        std::vector<PassTask> tasks(tun);
        if (k == 1)
            for (int i = 0; i < nt; ++i) tasks[i] = PassTask{1, i};
        HIPCHK(ctx, hipMemcpyAsync(dtasks, tasks.data(), nt * sizeof(PassTask), hipMemcpyHostToDevice, stream));
        a.tasks = dtasks;
        a.ntasks = nt;
        a.next = dnext + k;
        a.res = dres[k];
        a.out = dout[k];
        a.out_used = dused + k;
        a.src_res = dres[0];
        a.src_out = dout[0];
        HIPCHK(ctx, launch_passes(a, stream));
        HIPCHK(ctx, hipEventRecord(ev[k + 1], stream));
    }
    unsigned long long used[2] = {0, 0};
    HIPCHK(ctx, hipMemcpyAsync(used, dused, sizeof used, hipMemcpyDeviceToHost, stream));
    for (int k = 0; k < (refine ? 2 : 1); ++k) {
        r.pres[k].resize(nt);
        HIPCHK(ctx, hipMemcpyAsync(r.pres[k].data(), dres[k], nt * sizeof(PassResult), hipMemcpyDeviceToHost, stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(stream));
    for (int k = 0; k < (refine ? 2 : 1); ++k) {
        const int64_t nu = std::min<int64_t>((int64_t)used[k], out_cap);
        r.pout[k].resize((size_t)nu);
        if (nu) HIPCHK(ctx, hipMemcpyAsync(r.pout[k].data(), dout[k], nu * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(stream));
    float ms0 = 0.f, ms1 = 0.f;
    (void)hipEventElapsedTime(&ms0, ev[0], ev[1]);
    if (refine) (void)hipEventElapsedTime(&ms1, ev[1], ev[2]);
    S.tunnel_pass_ms = ms0;
    S.refine_pass_ms = ms1;
    S.pass_slots = (int32_t)ns;
    r.pass_xyz = m->xyz;
    for (int k = 0; k < 2; ++k)
        for (const PassResult &q : r.pres[k]) {
            S.pass_vertex_updates += q.updates;
            if (q.status == 0) (k ? S.n_refined_loops : S.n_tunnel_loops) += 1;
        }
    return VLS_OK;
}

// after the step kernel: post-passes, summary, result object r (bulk
// results deferred until fetched unless copied here)
static vls_status finish_run(vls_context *ctx, RunPrep &rp, const vls_params *p, int grid, int block,
                             double kernel_ms_override, vls_result &R) {
    vls_mesh *m = rp.m;
    const DState &s = rp.s;
    hipStream_t stream = rp.stream;
    const int64_t nv = m->nv;
    Ctl c{};
    HIPCHK(ctx, hipMemcpyAsync(&c, s.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIPCHK(ctx, hipStreamSynchronize(stream));
    vls_result *r = &R;
    r->nv = nv;
    if (rp.post_given) {
        r->node_pos = std::move(rp.g_node_pos);
        r->tn = std::move(rp.g_tn);
        r->tn_off = std::move(rp.g_tn_off);
        r->tn_v = std::move(rp.g_tn_v);
        r->tn_len = std::move(rp.g_tn_len);
        r->tn_pts.resize(r->tn_v.size() * 3);
        for (size_t q = 0; q < r->tn_v.size(); ++q)
            std::memcpy(r->tn_pts.data() + 3 * q, m->xyz.data() + 3 * (size_t)r->tn_v[q], 3 * sizeof(double));
    } else if (vls_status ps = post_passes(ctx, rp, c, *r)) {
        return ps;
    }
    if (c.status == 0)
        if (vls_status ps = run_passes(ctx, rp, p, c, *r)) return ps;
    float ms_k = 0.f, ms_t = 0.f;
    if (!rp.ws) {
        HIPCHK(ctx, hipEventRecord(rp.e3, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        (void)hipEventElapsedTime(&ms_k, rp.e1, rp.e2);
        (void)hipEventElapsedTime(&ms_t, rp.e0, rp.e3);
    }
    // bulk results stay on the device until fetched
    Pending &pd = r->pend;
    pd.active = true;
    pd.ctx = ctx;
    pd.mesh = (rp.priv || rp.ws) ? nullptr : m;
    pd.stream = stream;
    pd.s = s;
    pd.c = c;
    pd.tmp_allocs = rp.tmp_allocs;
    rp.tmp_allocs.clear();
    pd.rec_field = rp.rec_field;
    if (rp.rec_field) r->ckpt_steps.assign(p->ckpt_steps, p->ckpt_steps + p->n_ckpt);
    if (pd.mesh) m->pending = r;
    r->seed_xyz.assign(m->xyz.begin() + 3 * rp.seed, m->xyz.begin() + 3 * rp.seed + 3);
    vls_summary &S = r->sum;
    S.n_handles = (int32_t)c.gsum_h;
    S.n_tunnels = c.n_tunnels;
    S.euler_genus = m->euler_genus;
    S.swept_genus = (int32_t)((2 - c.chi - c.b) / 2);
    S.reeb_nodes = c.n_events + 1;
    S.reeb_edges = c.next_front;
    S.n_degenerate = c.n_degenerate;
    S.n_events = c.n_events;
    S.steps = c.steps;
    S.active_vertex_updates = c.active_updates;
    S.active_degree_sum = c.active_deg;
    S.n_inside = c.n_inside;
    S.seed_vertex = rp.seed;
    S.run_status = c.status;
    S.grid = grid;
    S.block = block;
    S.kernel_ms = kernel_ms_override >= 0 ? kernel_ms_override : ms_k;
    S.total_ms = ms_t;
    S.topo_ms = (double)c.clk_topo * 1e-5;
    S.wait0_ms = (double)c.clk_wait0 * 1e-5;
    S.field_ms = (double)c.clk_field * 1e-5;
    S.wait1_ms = (double)c.clk_wait1 * 1e-5;
    S.event_steps = c.event_steps;
    for (int q = 0; q < 4; ++q) S.topo_split_ms[q] = (double)c.clk_t[q] * 1e-5;
    S.topo_event_ms = (double)c.clk_ev * 1e-5;
    S.topo_rounds_ms = (double)c.clk_rounds * 1e-5;
    S.topo_round_steps = c.n_round_steps;
    S.topo_global_steps = c.n_global_steps;
    S.field_barrier_ms = (double)c.clk_fbar * 1e-5;
    for (int q = 0; q < 4; ++q) S.event_split_ms[q] = (double)c.clk_evp[q] * 1e-5;
    for (int q = 0; q < 4; ++q) S.topo_global_split_ms[q] = (double)c.clk_g[q] * 1e-5;
    vls_status rs = c.status;
    if (rs == VLS_E_INVARIANT || rs == VLS_E_CAPACITY)
        set_err(ctx, rs, "device reported %s (detail %d) at step %lld", vls_status_string(rs), c.err_code, (long long)c.steps);
    else if (rs == VLS_E_STALLED)
        set_err(ctx, rs, "front stalled at step %lld (%lld of %lld vertices inside)", (long long)c.steps,
                (long long)c.n_inside, (long long)nv);
    else if (rs == VLS_E_SEED_INVALID)
        set_err(ctx, rs, "seed region around vertex %lld is not a disk-like region", (long long)rp.seed);
    // results of caller-owned state (server requests, workspaces) are
    // copied now: that state is not kept for a later fetch
    if (rp.priv || rp.ws || !(p->flags & VLS_DEFER_RESULTS)) {
        vls_status fs = fetch_results(r);
        if (fs) return fs;
    }
    return rs;
}

// Launch plan of the batched kernel.  Tasks (meshes) run largest first; a
// mesh of nv vertices wants a gang of nv / gv workgroups (gv its gang
// granularity, kGangVerts when 0; at most kGangMax, and at least 2 to be a
// gang).  Gangs are granted in task order (largest first, the longest runs)
// while they fit in the pool less a reserve for the tasks too small for a
// gang (a quarter of the pool, or one workgroup each when there are fewer
// of them); a task whose full gang no longer fits gets what is left if that
// is at least 2.  Otherwise it runs on one workgroup, or, with defer (a
// launch that a later one continues) once some gang is granted, it sits the
// launch out (task_g 0): a mesh that wants a gang advances too slowly on one
// workgroup to repay the L2 its band takes from the others.  So all gangs
// run at once, and the tail of the launch is not set by a large mesh on one
// workgroup.  The slot list holds every gang member first (rank 0 first),
// then the one-workgroup tasks.
namespace {
constexpr int64_t kGangVerts = 65536;
constexpr int kGangMax = 64;
std::atomic<unsigned int> g_epoch{0};

struct BatchPlan {
    std::vector<int32_t> order, task_g, slots;
    int nslots = 0, grid = 0;
};

void plan_batch(const std::vector<int64_t> &nv, const std::vector<int64_t> &gv, int pool, BatchPlan &bp,
                bool defer = false) {
    const int n = (int)nv.size();
    bp.order.resize(n);
    for (int i = 0; i < n; ++i) bp.order[i] = i;
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](int32_t a, int32_t b) { return nv[a] > nv[b]; });
    bp.task_g.assign(n, 1);
    std::vector<int64_t> want(n);
    int64_t small = 0;
    for (int w = 0; w < n; ++w) {
        const int64_t gw = gv[bp.order[w]] > 0 ? gv[bp.order[w]] : kGangVerts;
        want[w] = std::min<int64_t>(kGangMax, nv[bp.order[w]] / gw);
        small += want[w] < 2;
    }
    int64_t left = (int64_t)pool - std::min<int64_t>(small, pool / 4);
    bool granted = false;
    for (int w = 0; w < n; ++w) {
        if (want[w] < 2) continue;
        const int64_t g = std::min(want[w], left);
        if (g >= 2) { bp.task_g[w] = (int32_t)g; left -= g; granted = true; }
    }
    if (defer && granted)
        for (int w = 0; w < n; ++w)
            if (want[w] >= 2 && bp.task_g[w] < 2) bp.task_g[w] = 0;
    bp.slots.clear();
    for (int w = 0; w < n; ++w)
        if (bp.task_g[w] >= 2)
            for (int r = 0; r < bp.task_g[w]; ++r) { bp.slots.push_back(w); bp.slots.push_back(r); }
    for (int w = 0; w < n; ++w)
        if (bp.task_g[w] == 1) { bp.slots.push_back(w); bp.slots.push_back(0); }
    bp.nslots = (int)(bp.slots.size() / 2);
    bp.grid = std::max(1, std::min(pool, bp.nslots));
}
}  // namespace

extern "C" {

// Reeb junction refinement (Section "Reeb Graph Extraction": a second pass
// improves where the junctions sit; Section "Introduction": a Reeb graph from
// a diffusion initiated at a detected handle loop).  The initial pass runs
// again from the first kept handle loop of r: its initial region is every
// vertex within seed_radius hops of the loop's inside vertices, ranked by hop
// distance inside that region from the smallest of them.  That pass's result
// (events, Reeb graph with band-mean junctions, loops) is kept in r->refined;
// nothing is run when r has no handle loop.
static int solo_grid(const vls_mesh *m, const vls_params *p);
static vls_status reeb_refine(vls_context *ctx, vls_mesh *m, const vls_params *p, vls_result &r) {
    if (vls_status fs = ensure(&r)) return fs;
    const int64_t nl = (int64_t)r.lp.size() / 8;
    std::vector<int32_t> set;
    for (int64_t q = 0; q < nl; ++q) {
        if (!r.lp[8 * q + 2]) continue;
        const int64_t off = r.lp[8 * q + 3], n = r.lp[8 * q + 4];
        for (int64_t k = 0; k < n; ++k) set.push_back(r.lp_he[2 * (off + k)]);
        break;
    }
    if (set.empty()) return VLS_OK;
    std::sort(set.begin(), set.end());
    set.erase(std::unique(set.begin(), set.end()), set.end());
    vls_params p2 = *p;
    p2.flags &= ~(VLS_REEB_REFINE | VLS_TUNNEL_PASS | VLS_REFINE_PASS | VLS_RECORD_FIELD | VLS_DEFER_RESULTS);
    p2.n_ckpt = 0;
    p2.ckpt_steps = nullptr;
    p2.seed_vertex = set[0];
    int32_t *d_set = nullptr;
    HIPCHK(ctx, hipMalloc(&d_set, set.size() * sizeof(int32_t)));
    struct Free { int32_t *q; ~Free() { if (q) (void)hipFree(q); } } guard{d_set};
    HIPCHK(ctx, hipMemcpy(d_set, set.data(), set.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    RunPrep rp;
    vls_status st = prepare_run(ctx, m, &p2, rp, nullptr, nullptr, d_set, (int32_t)set.size());
    if (st) return st;
    const int grid = solo_grid(m, &p2);
    if (grid <= 0) return set_err(ctx, VLS_E_DEVICE, "occupancy query failed");
    hipError_t le = launch_steps(m->d, rp.s, rp.dp, grid, 256, ctx->stream);
    if (le != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "step kernel launch: %s", hipGetErrorString(le));
    HIPCHK(ctx, hipEventRecord(rp.e2, ctx->stream));
    auto r2 = std::make_unique<vls_result>();
    vls_status rs = finish_run(ctx, rp, &p2, grid, 256, -1.0, *r2);
    if (rs != VLS_OK && !is_run_status(rs)) {
        if (m->pending == r2.get()) m->pending = nullptr;
        return rs;
    }
    if (vls_status fs = ensure(r2.get())) return fs;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    r.refined = r2.release();
    return VLS_OK;
}

// launch shape of a one-mesh run: p->grid if set, else about one workgroup
// per 34k vertices, 16..128.  The field's share of a step grows with the
// band, but every field workgroup also loads the memory system the
// topology's dependent chains run through: on the 256^3 pretzel 64
// workgroups beat 99 (456 against 491 ms per pass) although the field alone
// runs faster at 99.  The dense step streams the whole mesh: every
// co-resident workgroup.  0 when the occupancy query fails.
static int solo_grid(const vls_mesh *m, const vls_params *p) {
    const size_t lds = step_lds_bytes(256, m->dmax);
    const int maxg = max_coresident_blocks(256, lds);
    if (maxg <= 0) return 0;
    int grid = p->grid > 0 ? p->grid : (int)std::min<int64_t>(128, std::max<int64_t>(16, m->nv / 34000));
    if (p->grid <= 0 && (p->flags & VLS_DENSE_FIELD)) grid = maxg;
    return std::min(grid, maxg);
}

vls_status vls_run(vls_context *ctx, const vls_mesh *mc, const vls_params *p, vls_result **out) {
    if (!ctx || !mc || !p || !out) return set_err(ctx, VLS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    vls_mesh *m = const_cast<vls_mesh *>(mc);
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
    RunPrep rp;
    vls_status st = prepare_run(ctx, m, p, rp);
    if (st) return st;
    const int block = 256;
    const int grid = solo_grid(m, p);
    if (grid <= 0) return set_err(ctx, VLS_E_DEVICE, "occupancy query failed");
    hipError_t le = launch_steps(m->d, rp.s, rp.dp, grid, block, ctx->stream);
    if (le != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "step kernel launch: %s", hipGetErrorString(le));
    HIPCHK(ctx, hipEventRecord(rp.e2, ctx->stream));
    auto r = std::make_unique<vls_result>();
    vls_status rs = finish_run(ctx, rp, p, grid, block, -1.0, *r);
    if (rs != VLS_OK && !is_run_status(rs)) {
        if (m->pending == r.get()) m->pending = nullptr;
        return rs;
    }
    if (rs == VLS_OK && (p->flags & VLS_REEB_REFINE)) {
        vls_status fs = reeb_refine(ctx, m, p, *r);
        if (fs) {
            if (m->pending == r.get()) m->pending = nullptr;
            (void)vls_result_destroy(r.release());
            return fs;
        }
    }
    *out = r.release();
    return rs;
}

vls_status vls_workspace_size(const vls_mesh *m, const vls_params *p, size_t *bytes) {
    if (!m || !p || !bytes) return VLS_E_INVALID_ARG;
    if (p->struct_size != sizeof(vls_params)) return VLS_E_INVALID_ARG;
    DevArena A;
    A.mode = DevArena::COUNT;
    DState s;
    (void)alloc_state(m, A, s);
    if ((p->flags & VLS_RECORD_FIELD) && p->n_ckpt > 0 && p->ckpt_steps) {
        double *a;
        int64_t *b;
        (void)A.get(&a, (size_t)p->n_ckpt * (size_t)m->nv);
        (void)A.get(&b, (size_t)p->n_ckpt);
    }
    *bytes = A.used + post_bytes(m);
    return VLS_OK;
}

}  // extern "C"

// enqueues a whole pass on `stream` with every device buffer carved from
// [base, base + bytes); the result waits for it on first use
static vls_status run_in_workspace(vls_context *ctx, const vls_mesh *mc, const vls_params *p, void *base,
                                   size_t bytes, hipStream_t stream, vls_result **out) {
    if (!ctx || !mc || !p || !out || !base) return set_err(ctx, VLS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (((uintptr_t)base & 255) != 0) return set_err(ctx, VLS_E_INVALID_ARG, "workspace must be 256-byte aligned");
    vls_mesh *m = const_cast<vls_mesh *>(mc);
    if (p->struct_size != sizeof(vls_params)) return set_err(ctx, VLS_E_INVALID_ARG, "vls_params.struct_size mismatch");
    size_t need = 0;
    (void)vls_workspace_size(m, p, &need);
    if (bytes < need)
        return set_err(ctx, VLS_E_BUFFER_TOO_SMALL, "workspace of %zu bytes, %zu needed", bytes, need);
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
    const int grid = solo_grid(m, p);
    if (grid <= 0) return set_err(ctx, VLS_E_DEVICE, "occupancy query failed");
    auto rp = std::make_unique<RunPrep>();
    rp->stream = stream ? stream : ctx->stream;
    rp->params = *p;
    const bool rec = (p->flags & VLS_RECORD_FIELD) && p->n_ckpt > 0 && p->ckpt_steps;
    if (rec) rp->ckpt.assign(p->ckpt_steps, p->ckpt_steps + p->n_ckpt);
    rp->params.ckpt_steps = rec ? rp->ckpt.data() : nullptr;
    rp->params.n_ckpt = rec ? p->n_ckpt : 0;
    rp->grid = grid;
    DevArena ws;
    ws.mode = DevArena::CARVE;
    ws.base = (char *)base;
    ws.cap = bytes;
    vls_status st = prepare_run(ctx, m, &rp->params, *rp, nullptr, &ws);
    if (st) return st;
    hipError_t le = launch_steps(m->d, rp->s, rp->dp, grid, 256, rp->stream);
    if (le != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "step kernel launch: %s", hipGetErrorString(le));
    auto r = std::make_unique<vls_result>();
    r->pend.ctx = ctx;
    r->launched = rp.release();
    *out = r.release();
    return VLS_OK;
}

// the static scratch of a device serves one run at a time: claimed by
// vls_run_async_noalloc, released once that run's result has been waited
// for or destroyed
static std::mutex g_static_mu;
static std::unordered_map<int, bool> g_static_busy;
static bool static_claim(int dev) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    bool &b = g_static_busy[dev];
    if (b) return false;
    b = true;
    return true;
}
static void static_release(vls_result *r) {
    if (r->static_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_busy[r->static_dev] = false;
    r->static_dev = -1;
}

// the second half of a workspace run: the step kernel's end, post-passes,
// every result copied to the host; the workspace is free afterwards
static vls_status wait_launched(vls_result *r) {
    RunPrep *rp = r->launched;
    if (!rp) return r->launch_status;
    r->launched = nullptr;
    std::unique_ptr<RunPrep> own(rp);
    vls_context *ctx = r->pend.ctx;
    (void)hipSetDevice(ctx->device);
    vls_status rs = finish_run(ctx, *rp, &rp->params, rp->grid, 256, -1.0, *r);
    if (rs != VLS_OK && !is_run_status(rs)) {
        // the device work may still be queued: let it end before the
        // workspace is given back
        (void)hipStreamSynchronize(rp->stream);
        r->failed = true;
    }
    r->launch_status = rs;
    static_release(r);
    return rs;
}

extern "C" {

vls_status vls_run_async(vls_context *ctx, const vls_mesh *m, const vls_params *p, void *d_workspace,
                         size_t bytes, void *hip_stream, vls_result **out) {
    return run_in_workspace(ctx, m, p, d_workspace, bytes, (hipStream_t)hip_stream, out);
}

vls_status vls_run_async_noalloc(vls_context *ctx, const vls_mesh *m, const vls_params *p, void *hip_stream,
                                 vls_result **out) {
    if (!ctx || !m || !p || !out) return set_err(ctx, VLS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (p->struct_size != sizeof(vls_params)) return set_err(ctx, VLS_E_INVALID_ARG, "vls_params.struct_size mismatch");
    size_t need = 0;
    (void)vls_workspace_size(m, p, &need);
    if (need > STATIC_SCRATCH_BYTES)
        return set_err(ctx, VLS_E_BUFFER_TOO_SMALL, "the run needs %zu bytes of workspace; the static scratch holds %zu",
                       need, (size_t)STATIC_SCRATCH_BYTES);
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
    void *base = nullptr;
    hipError_t e = static_scratch(ctx->device, &base);
    if (e != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "static scratch address: %s", hipGetErrorString(e));
    if (!static_claim(ctx->device))
        return set_err(ctx, VLS_E_PENDING, "the static scratch of device %d is held by a result not yet waited for",
                       ctx->device);
    vls_status st = run_in_workspace(ctx, m, p, base, STATIC_SCRATCH_BYTES, (hipStream_t)hip_stream, out);
    if (st != VLS_OK) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[ctx->device] = false;
        return st;
    }
    (*out)->static_dev = ctx->device;
    return VLS_OK;
}

vls_status vls_result_wait(vls_result *r) {
    if (!r) return VLS_E_INVALID_ARG;
    if (r->failed) return r->launch_status;
    if (r->launched) return wait_launched(r);
    return r->sum.run_status;
}

vls_status vls_batch_run(vls_context *ctx, int32_t n, const vls_mesh *const *meshes, const vls_params *per_mesh,
                         vls_result **out) {
    if (!ctx || n <= 0 || !meshes || !per_mesh || !out) return set_err(ctx, VLS_E_INVALID_ARG, "bad batch arguments");
    for (int32_t i = 0; i < n; ++i) {
        out[i] = nullptr;
        if (!meshes[i]) return set_err(ctx, VLS_E_INVALID_ARG, "mesh %d is NULL", i);
        for (int32_t j = 0; j < i; ++j)
            if (meshes[j] == meshes[i]) return set_err(ctx, VLS_E_INVALID_ARG, "mesh %d appears twice in the batch", i);
    }
    for (int32_t i = 0; i < n; ++i) {
        if (per_mesh[i].flags & (VLS_TUNNEL_PASS | VLS_REFINE_PASS | VLS_REEB_REFINE))
            return set_err(ctx, VLS_E_INVALID_ARG,
                           "the tunnel-loop, refinement and Reeb refinement passes run with vls_run only");
        if (per_mesh[i].flags & VLS_FEM_LAPLACIAN)
            return set_err(ctx, VLS_E_INVALID_ARG, "VLS_FEM_LAPLACIAN runs with vls_run and the workspace calls only");
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
    hipStream_t stream = ctx->stream;
    std::vector<RunPrep> preps(n);
    std::vector<DMesh> hm(n);
    std::vector<DState> hs(n);
    std::vector<DParams> hp(n);
    size_t lds = 0;
    for (int32_t i = 0; i < n; ++i) {
        vls_mesh *m = const_cast<vls_mesh *>(meshes[i]);
        vls_status st = prepare_run(ctx, m, &per_mesh[i], preps[i]);
        if (st) return st;
        hm[i] = m->d;
        hs[i] = preps[i].s;
        hp[i] = preps[i].dp;
    }
    const int occ = (per_mesh[0].flags & VLS_BATCH_TWO_PER_CU) ? 2 : 1;
    lds = batch_lds_bytes(occ);
    const int maxg = max_coresident_batch(lds, occ);
    if (maxg <= 0) return set_err(ctx, VLS_E_DEVICE, "occupancy query failed");
    const int pool = per_mesh[0].grid > 0 ? std::min(per_mesh[0].grid, maxg) : maxg;
    std::vector<int64_t> nvs(n);
    for (int32_t i = 0; i < n; ++i) nvs[i] = meshes[i]->nv;
    BatchPlan bp;
    plan_batch(nvs, std::vector<int64_t>(n, per_mesh[0].gang_vertices), pool, bp);
    const int grid = bp.grid;
    void *dm = nullptr, *ds = nullptr, *dpp = nullptr, *dord = nullptr, *dnext = nullptr, *dtg = nullptr,
         *dsl = nullptr;
    struct Guard {
        std::vector<void **> ptrs;
        ~Guard() { for (void **q : ptrs) if (*q) (void)hipFree(*q); }
    } guard{{&dm, &ds, &dpp, &dord, &dnext, &dtg, &dsl}};
    HIPCHK(ctx, hipMalloc(&dm, n * sizeof(DMesh)));
    HIPCHK(ctx, hipMalloc(&ds, n * sizeof(DState)));
    HIPCHK(ctx, hipMalloc(&dpp, n * sizeof(DParams)));
    HIPCHK(ctx, hipMalloc(&dord, n * sizeof(int32_t)));
    HIPCHK(ctx, hipMalloc(&dtg, n * sizeof(int32_t)));
    HIPCHK(ctx, hipMalloc(&dsl, bp.slots.size() * sizeof(int32_t)));
    HIPCHK(ctx, hipMalloc(&dnext, sizeof(int)));
    HIPCHK(ctx, hipMemcpyAsync(dm, hm.data(), n * sizeof(DMesh), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(ds, hs.data(), n * sizeof(DState), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(dpp, hp.data(), n * sizeof(DParams), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(dord, bp.order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(dtg, bp.task_g.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemcpyAsync(dsl, bp.slots.data(), bp.slots.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIPCHK(ctx, hipMemsetAsync(dnext, 0, sizeof(int), stream));
    hipEvent_t b0 = nullptr, b1 = nullptr;
    HIPCHK(ctx, hipEventCreate(&b0));
    HIPCHK(ctx, hipEventCreate(&b1));
    HIPCHK(ctx, hipEventRecord(b0, stream));
    hipError_t le = launch_batch((const DMesh *)dm, (const DState *)ds, (const DParams *)dpp, (const int32_t *)dord,
                                 (const int32_t *)dtg, (const int32_t *)dsl, bp.nslots, (int *)dnext, grid, lds, ~0ull,
                                 nullptr, ++g_epoch, occ, (per_mesh[0].flags & VLS_COHERENT_SHARING) ? 1 : 0, stream);
    if (le != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "batch kernel launch: %s", hipGetErrorString(le));
    HIPCHK(ctx, hipEventRecord(b1, stream));
    HIPCHK(ctx, hipEventSynchronize(b1));
    float ms_b = 0.f;
    (void)hipEventElapsedTime(&ms_b, b0, b1);
    (void)hipEventDestroy(b0);
    (void)hipEventDestroy(b1);
    {
        std::vector<Ctl> cs(n);
        for (int32_t i = 0; i < n; ++i)
            HIPCHK(ctx, hipMemcpyAsync(&cs[i], preps[i].s.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        std::vector<const vls_mesh *> mv(meshes, meshes + n);
        std::vector<RunPrep *> pv(n);
        for (int32_t i = 0; i < n; ++i) pv[i] = &preps[i];
        DevArena A;
        if (vls_status ps = multi_post_passes(ctx, mv, pv, cs, (const DMesh *)dm, (const DState *)ds, A, stream))
            return ps;
    }
    vls_status first = VLS_OK;
    for (int32_t i = 0; i < n; ++i) {
        HIPCHK(ctx, hipEventRecord(preps[i].e2, stream));
        auto r = std::make_unique<vls_result>();
        vls_status rs = finish_run(ctx, preps[i], &per_mesh[i], grid, 256, ms_b, *r);
        if (rs != VLS_OK && !is_run_status(rs)) {
            vls_mesh *mi = const_cast<vls_mesh *>(meshes[i]);
            if (mi->pending == r.get()) mi->pending = nullptr;
            for (int32_t j = 0; j < i; ++j) { (void)vls_result_destroy(out[j]); out[j] = nullptr; }
            return rs;
        }
        if (rs && !first) first = rs;
        out[i] = r.release();
    }
    return first;
}

vls_status vls_result_summary(const vls_result *r, vls_summary *s) {
    if (!r || !s) return VLS_E_INVALID_ARG;
    vls_result *q = const_cast<vls_result *>(r);
    if (q->launched) {
        vls_status st = wait_launched(q);
        if (st != VLS_OK && !is_run_status(st)) return st;
    }
    if (q->failed) return q->launch_status;
    *s = r->sum;
    return VLS_OK;
}

vls_status vls_result_events(const vls_result *r, int64_t cap, int64_t *rec, int64_t *n_out) {
    if (!r || !n_out) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    const int64_t n = (int64_t)r->ev.size() / 16;
    *n_out = n;
    if (cap == 0) return VLS_OK;
    if (cap < n || !rec) return VLS_E_BUFFER_TOO_SMALL;
    std::memcpy(rec, r->ev.data(), r->ev.size() * 8);
    return VLS_OK;
}

vls_status vls_result_event_fronts(const vls_result *r, int64_t cap, int64_t *ids, int64_t *n_out) {
    if (!r || !n_out) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    const int64_t n = (int64_t)r->ev_ids.size();
    *n_out = n;
    if (cap == 0) return VLS_OK;
    if (cap < n || !ids) return VLS_E_BUFFER_TOO_SMALL;
    std::memcpy(ids, r->ev_ids.data(), n * 8);
    return VLS_OK;
}

static bool loop_index(const vls_result *r, int32_t kind, int32_t i, int64_t *li) {
    const int64_t nl = (int64_t)r->lp.size() / 8;
    if (kind == 2) {
        if (i < 0 || i >= nl) return false;
        *li = i;
        return true;
    }
    int64_t c = 0;
    for (int64_t q = 0; q < nl; ++q)
        if (r->lp[8 * q + 2]) {
            if (c == i) { *li = q; return true; }
            c++;
        }
    return false;
}

vls_status vls_result_loop(const vls_result *r, int32_t kind, int32_t i, int64_t cap, int32_t *edges_uv,
                           double *pts, double *length, int64_t *n_out) {
    if (!r || !n_out) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    if (kind == 0 || kind == 2) {
        int64_t li;
        if (!loop_index(r, kind, i, &li)) return VLS_E_INVALID_ARG;
        const int64_t off = r->lp[8 * li + 3], n = r->lp[8 * li + 4];
        *n_out = n;
        if (length) { double L; int64_t bits = r->lp[8 * li + 6]; std::memcpy(&L, &bits, 8); *length = L; }
        if (cap == 0) return VLS_OK;
        if (cap < n) return VLS_E_BUFFER_TOO_SMALL;
        if (edges_uv) std::memcpy(edges_uv, r->lp_he.data() + 2 * off, n * 2 * sizeof(int32_t));
        if (pts) std::memcpy(pts, r->lp_pts.data() + 3 * off, n * 3 * sizeof(double));
        return VLS_OK;
    }
    if (kind == 3 || kind == 4) {
        const std::vector<PassResult> &v = r->pres[kind - 3];
        if (i < 0 || i >= (int32_t)v.size()) return VLS_E_INVALID_ARG;
        const PassResult &q = v[i];
        const int64_t n = q.status == 0 ? q.n : 0;
        *n_out = n;
        if (length) *length = q.status == 0 ? q.length : 0.0;
        if (cap == 0 || n == 0) return VLS_OK;
        if (cap < n) return VLS_E_BUFFER_TOO_SMALL;
        const int32_t *c = r->pout[kind - 3].data() + q.off;
        const double *xyz = r->pass_xyz.data();
        for (int64_t k = 0; k < n; ++k) {
            if (edges_uv) { edges_uv[2 * k] = c[k]; edges_uv[2 * k + 1] = c[(k + 1) % n]; }
            if (pts) std::memcpy(pts + 3 * k, xyz + 3 * (int64_t)c[k], 3 * sizeof(double));
        }
        return VLS_OK;
    }
    if (kind == 1) {
        const int64_t nt = (int64_t)r->tn.size() / 4;
        if (i < 0 || i >= nt) return VLS_E_INVALID_ARG;
        const int64_t off = r->tn_off[i], n = r->tn_off[i + 1] - off;
        *n_out = n;
        if (length) *length = r->tn_len[i];
        if (cap == 0) return VLS_OK;
        if (cap < n) return VLS_E_BUFFER_TOO_SMALL;
        for (int64_t q = 0; q < n; ++q) {
            const int32_t a = r->tn_v[off + q], b = r->tn_v[off + (q + 1) % n];
            if (edges_uv) { edges_uv[2 * q] = a; edges_uv[2 * q + 1] = b; }
            if (pts) std::memcpy(pts + 3 * q, r->tn_pts.data() + 3 * (off + q), 3 * sizeof(double));
        }
        return VLS_OK;
    }
    return VLS_E_INVALID_ARG;
}

vls_status vls_result_pass_info(const vls_result *r, int32_t kind, int32_t i, int32_t *status, int64_t *steps,
                                int32_t *reached, int32_t *label, double *length, double *offset_length) {
    if (!r || (kind != 3 && kind != 4)) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    const std::vector<PassResult> &v = r->pres[kind - 3];
    if (i < 0 || i >= (int32_t)v.size()) return VLS_E_INVALID_ARG;
    const PassResult &q = v[i];
    if (status) *status = q.status;
    if (steps) *steps = q.steps;
    if (reached) *reached = q.reached;
    if (label) *label = q.status == 0 ? q.label : -1;
    if (length) *length = q.status == 0 ? q.length : 0.0;
    if (offset_length) *offset_length = q.status == 0 ? q.offset_length : 0.0;
    return VLS_OK;
}

vls_status vls_result_loop_info(const vls_result *r, int32_t kind, int32_t i, int64_t *event, int64_t *front_id,
                                int32_t *kept) {
    if (!r || (kind != 0 && kind != 2)) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    int64_t li;
    if (!loop_index(r, kind, i, &li)) return VLS_E_INVALID_ARG;
    if (event) *event = r->lp[8 * li];
    if (front_id) *front_id = r->lp[8 * li + 1];
    if (kept) *kept = (int32_t)r->lp[8 * li + 2];
    return VLS_OK;
}

vls_status vls_result_reeb(const vls_result *r, int64_t cap_n, vls_reeb_node *nodes, int64_t cap_e,
                           vls_reeb_edge *edges, int64_t *n_nodes, int64_t *n_edges) {
    if (!r || !n_nodes || !n_edges) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    const int64_t nev = (int64_t)r->ev.size() / 16;
    const int64_t nn = nev + 1, ne = (int64_t)r->front_birth.size();
    *n_nodes = nn;
    *n_edges = ne;
    if (cap_n == 0 && cap_e == 0) return VLS_OK;
    if (cap_n < nn || cap_e < ne || !nodes || !edges) return VLS_E_BUFFER_TOO_SMALL;
    int32_t b0 = 0;
    for (int64_t f = 0; f < ne; ++f) b0 += r->front_birth[f] == 0;
    vls_reeb_node &s0 = nodes[0];
    std::memset(&s0, 0, sizeof s0);
    s0.type = VLS_NODE_SEED;
    s0.vertex = (int32_t)r->sum.seed_vertex;
    s0.in_deg = 0;
    s0.out_deg = b0;
    s0.step = 0;
    std::memcpy(s0.xyz, r->seed_xyz.data(), 3 * sizeof(double));
    for (int64_t i = 0; i < nev; ++i) {
        const int64_t *e = r->ev.data() + 16 * i;
        vls_reeb_node &n = nodes[i + 1];
        std::memset(&n, 0, sizeof n);
        n.type = (int32_t)e[2];
        n.vertex = (int32_t)e[1];
        n.in_deg = (int32_t)e[4];
        n.out_deg = (int32_t)e[5];
        n.extra_cycles = (int32_t)e[7];
        n.step = e[0];
        std::memcpy(n.xyz, r->node_pos.data() + 3 * i, 3 * sizeof(double));
    }
    for (int64_t f = 0; f < ne; ++f) {
        edges[f].src = r->front_birth[f];
        edges[f].dst = r->front_death[f];
        edges[f].front_id = (int32_t)f;
    }
    return VLS_OK;
}

vls_status vls_result_field(const vls_result *r, int64_t step, double *rho) {
    if (!r || !rho) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    if (step < 0) {
        std::memcpy(rho, r->rho_final.data(), r->nv * sizeof(double));
        return VLS_OK;
    }
    for (size_t q = 0; q < r->ckpt_steps.size(); ++q)
        if (r->ckpt_steps[q] == step && r->ckpt_ok[q]) {
            std::memcpy(rho, r->ckpt.data() + q * r->nv, r->nv * sizeof(double));
            return VLS_OK;
        }
    return VLS_E_INVALID_ARG;
}

vls_status vls_result_vertices(const vls_result *r, int32_t *step, int32_t *round, int32_t *parent) {
    if (!r) return VLS_E_INVALID_ARG;
    if (vls_status fs = ensure(r)) return fs;
    if (step) std::memcpy(step, r->step.data(), r->nv * sizeof(int32_t));
    if (round) std::memcpy(round, r->round.data(), r->nv * sizeof(int32_t));
    if (parent) std::memcpy(parent, r->parent.data(), r->nv * sizeof(int32_t));
    return VLS_OK;
}

vls_status vls_result_fetch(vls_result *r) {
    if (!r) return VLS_E_INVALID_ARG;
    return fetch_results(r);
}

vls_status vls_result_refined(const vls_result *r, const vls_result **second) {
    if (!r || !second) return VLS_E_INVALID_ARG;
    *second = r->refined;
    return VLS_OK;
}

vls_status vls_result_destroy(vls_result *r) {
    if (!r) return VLS_E_INVALID_ARG;
    if (r->refined) {
        (void)vls_result_destroy(r->refined);
        r->refined = nullptr;
    }
    if (r->launched) {
        // enqueued and never waited for: let the device work end first (it
        // uses the caller's workspace)
        (void)hipStreamSynchronize(r->launched->stream);
        delete r->launched;
        r->launched = nullptr;
    }
    static_release(r);
    Pending &pd = r->pend;
    if (pd.active) {
        // never fetched: drop the device copies without reading them
        pd.active = false;
        if (pd.mesh && pd.mesh->pending == r) pd.mesh->pending = nullptr;
        (void)hipSetDevice(pd.ctx->device);
        for (void *q : pd.tmp_allocs) (void)hipFree(q);
    }
    delete r;
    return VLS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving: continuous batching over bounded launches of the batched kernel
// ---------------------------------------------------------------------------
namespace {

using Clock = std::chrono::steady_clock;

struct SrvReq {
    uint64_t ticket = 0;
    vls_mesh *m = nullptr;
    vls_params p{};
    std::vector<int64_t> ckpt;
    size_t bytes = 0;
    std::unique_ptr<RunBuffers> rb;
    std::unique_ptr<RunPrep> prep;
    vls_status status = VLS_E_PENDING;
    vls_result *res = nullptr;
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct vls_server {
    vls_context ctx;                 // private stream on the caller's device
    size_t budget = 0;
    int max_slots = 0;
    int occ = 1;                     // workgroups per CU of the step launches
    int cm = 0;                      // 1: gangs share through coherent atomics
    unsigned long long slice_ticks = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<SrvReq *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<SrvReq>> reqs;
    std::vector<SrvReq *> active;    // touched by the scheduler thread only
    uint64_t next_ticket = 1;
    bool stop = false;
    size_t used = 0;
    int64_t launches = 0, completed = 0;
    std::thread th;
    // launch descriptors on the device, rebuilt when the running set changes
    void *dm = nullptr, *ds = nullptr, *dp = nullptr, *dord = nullptr, *dnext = nullptr, *ddone = nullptr,
         *dtg = nullptr, *dsl = nullptr;
    int cap = 0;
    std::vector<int32_t> hdone;
    std::string thread_err;
    // run state of finished requests kept for the next request of the same
    // mesh shape (no allocation on admission), up to pool_cap bytes; one
    // post-pass scratch reused by every completion (grown when needed)
    std::unordered_map<const vls_mesh *, std::vector<std::unique_ptr<RunBuffers>>> pool;
    size_t pooled = 0, pool_cap = 0;
    void *post_buf = nullptr;
    size_t post_cap = 0;
    // completions taken together: their meshes and run states on the device
    // (kCompleteBatch entries), and the multi-run post-pass scratch in
    // post_buf (grown when needed)
    DMesh *cdm = nullptr;
    DState *cds = nullptr;
    // host time of the scheduler's phases (ms): admissions, launches incl.
    // their wait; and of the completion thread's work
    double t_admit_ms = 0.0, t_launch_ms = 0.0, t_complete_ms = 0.0;
    // completions (post-passes, results to the host) run on their own thread
    // and stream, beside the next slices
    vls_context cctx;
    std::thread cth;
    std::deque<SrvReq *> cq;
    std::condition_variable ccv;
    bool cstop = false;
    std::mutex pool_mu;

    ~vls_server() {
        for (void *q : {dm, ds, dp, dord, dnext, ddone, dtg, dsl}) if (q) (void)hipFree(q);
        pool.clear();
        if (post_buf) (void)hipFree(post_buf);
        if (cdm) (void)hipFree(cdm);
        if (cds) (void)hipFree(cds);
        if (ctx.own_stream && ctx.stream) (void)hipStreamDestroy(ctx.stream);
        if (cctx.own_stream && cctx.stream) (void)hipStreamDestroy(cctx.stream);
    }
    std::unique_ptr<RunBuffers> take_buffers(const vls_mesh *m) {
        std::lock_guard<std::mutex> lk(pool_mu);
        auto it = pool.find(m);
        if (it == pool.end()) return nullptr;
        while (!it->second.empty()) {
            std::unique_ptr<RunBuffers> rb = std::move(it->second.back());
            it->second.pop_back();
            const size_t b = rb->arena.used;
            pooled -= b;
            if (rb->nv == m->nv && rb->nnz == m->nnz && rb->genus == m->euler_genus) return rb;
        }
        return nullptr;
    }
    void give_buffers(const vls_mesh *m, std::unique_ptr<RunBuffers> rb) {
        if (!rb) return;
        std::lock_guard<std::mutex> lk(pool_mu);
        const size_t b = rb->arena.used;
        if (pooled + b > pool_cap) return;       // freed
        pooled += b;
        pool[m].push_back(std::move(rb));
    }
    void finish(SrvReq *q, vls_status st, vls_result *r);
    void complete(std::vector<SrvReq *> &qs);
    bool admit_one(SrvReq *q);
    bool launch_slice();
    void loop();
    void complete_loop();
};

// marks q done (status, result), releases its admission charge
void vls_server::finish(SrvReq *q, vls_status st, vls_result *r) {
    if (st == VLS_OK || is_run_status(st)) give_buffers(q->m, std::move(q->rb));
    q->rb.reset();
    q->prep.reset();
    std::lock_guard<std::mutex> lk(mu);
    q->status = st;
    q->res = r;
    q->t_done = Clock::now();
    if (r) {
        r->sum.server_queue_ms = ms_between(q->t_submit, q->t_admit);
        r->sum.server_latency_ms = ms_between(q->t_submit, q->t_done);
    }
    q->done = true;
    used -= q->bytes;
    completed += 1;
}

// requests whose step kernels finished: post-passes of all of them
// together, then each one's results to the host
constexpr int kCompleteBatch = 256;
void vls_server::complete(std::vector<SrvReq *> &qs) {
    const int k = (int)qs.size();
    auto fail_all = [&](vls_status st) {
        for (SrvReq *q : qs) finish(q, st, nullptr);
    };
    // the requests' device work ended with the slices that finished them;
    // the post-passes and copies go on the completion stream
    std::vector<const vls_mesh *> mv(k);
    std::vector<RunPrep *> pv(k);
    std::vector<DMesh> hm(k);
    std::vector<DState> hs(k);
    std::vector<Ctl> cs(k);
    hipStream_t st = cctx.stream;
    for (int i = 0; i < k; ++i) {
        RunPrep &rp = *qs[i]->prep;
        rp.stream = st;
        mv[i] = qs[i]->m;
        pv[i] = &rp;
        hm[i] = qs[i]->m->d;
        hs[i] = rp.s;
        if (hipMemcpyAsync(&cs[i], rp.s.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st) != hipSuccess) {
            fail_all(VLS_E_DEVICE);
            return;
        }
    }
    size_t fill_cap, path_cap;
    multi_post_caps(mv, fill_cap, path_cap);
    const size_t need = multi_post_bytes(fill_cap, path_cap);
    if (need > post_cap) {
        if (post_buf) (void)hipFree(post_buf);
        post_buf = nullptr;
        post_cap = 0;
        if (hipMalloc(&post_buf, need) != hipSuccess) { post_buf = nullptr; fail_all(VLS_E_OUT_OF_MEMORY); return; }
        post_cap = need;
    }
    if ((!cdm && hipMalloc(&cdm, kCompleteBatch * sizeof(DMesh)) != hipSuccess) ||
        (!cds && hipMalloc(&cds, kCompleteBatch * sizeof(DState)) != hipSuccess)) {
        fail_all(VLS_E_OUT_OF_MEMORY);
        return;
    }
    if (hipMemcpyAsync(cdm, hm.data(), k * sizeof(DMesh), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(cds, hs.data(), k * sizeof(DState), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        fail_all(VLS_E_DEVICE);
        return;
    }
    DevArena A;
    A.mode = DevArena::CARVE;
    A.base = (char *)post_buf;
    A.cap = post_cap;
    if (vls_status ps = multi_post_passes(&cctx, mv, pv, cs, cdm, cds, A, st)) {
        fail_all(ps);
        return;
    }
    for (SrvReq *q : qs) {
        auto r = std::make_unique<vls_result>();
        vls_status rs = finish_run(&cctx, *q->prep, &q->p, 0, 256, -1.0, *r);
        if (rs != VLS_OK && !is_run_status(rs)) { finish(q, rs, nullptr); continue; }
        finish(q, rs, r.release());
    }
}

void vls_server::complete_loop() {
    (void)hipSetDevice(cctx.device);
    for (;;) {
        std::vector<SrvReq *> qs;
        {
            std::unique_lock<std::mutex> lk(mu);
            ccv.wait(lk, [&] { return cstop || !cq.empty(); });
            if (cq.empty()) break;
            while (!cq.empty() && (int)qs.size() < kCompleteBatch) {
                qs.push_back(cq.front());
                cq.pop_front();
            }
        }
        const auto t0 = Clock::now();
        complete(qs);
        const double ms = ms_between(t0, Clock::now());
        {
            std::lock_guard<std::mutex> lk(mu);
            t_complete_ms += ms;
        }
        cv.notify_one();       // budget freed: the scheduler may admit more
    }
}

// device run state and seed initialisation of a newly admitted request
bool vls_server::admit_one(SrvReq *q) {
    q->t_admit = Clock::now();
    q->rb = take_buffers(q->m);
    vls_status st = VLS_OK;
    if (!q->rb) {
        RunBuffers *rb = nullptr;
        st = make_run_buffers(q->m, &rb);
        if (st) { finish(q, st, nullptr); return false; }
        q->rb.reset(rb);
    }
    q->prep = std::make_unique<RunPrep>();
    vls_params pp = q->p;
    pp.ckpt_steps = q->ckpt.empty() ? nullptr : q->ckpt.data();
    q->p = pp;
    st = prepare_run(&ctx, q->m, &q->p, *q->prep, q->rb.get());
    if (st) { finish(q, st, nullptr); return false; }
    return true;
}

// one bounded launch over the running requests (largest first); false on a
// device error (every running request then fails)
bool vls_server::launch_slice() {
    const auto tl = Clock::now();
    const int n = (int)active.size();
    if (n > cap) {
        for (void *q : {dm, ds, dp, dord, dnext, ddone, dtg, dsl}) if (q) (void)hipFree(q);
        dm = ds = dp = dord = dnext = ddone = dtg = dsl = nullptr;
        cap = 0;   // a failed allocation below is retried by the next slice
        int c = 64;
        while (c < n) c <<= 1;
        if (hipMalloc(&dm, c * sizeof(DMesh)) || hipMalloc(&ds, c * sizeof(DState)) ||
            hipMalloc(&dp, c * sizeof(DParams)) || hipMalloc(&dord, c * sizeof(int32_t)) ||
            hipMalloc(&dnext, sizeof(int)) || hipMalloc(&ddone, c * sizeof(int32_t)) ||
            hipMalloc(&dtg, c * sizeof(int32_t)) || hipMalloc(&dsl, 2 * (size_t)(c + 4096) * sizeof(int32_t)))
            return false;
        cap = c;
    }
    std::vector<DMesh> hm(n);
    std::vector<DState> hs(n);
    std::vector<DParams> hp(n);
    std::vector<int64_t> nvs(n), gvs(n);
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        hm[i] = active[i]->m->d;
        hs[i] = active[i]->prep->s;
        hp[i] = active[i]->prep->dp;
        nvs[i] = active[i]->m->nv;
        gvs[i] = active[i]->p.gang_vertices;
    }
    lds = batch_lds_bytes(occ);
    const int maxg = max_coresident_batch(lds, occ);
    if (maxg <= 0) return false;
    BatchPlan bp;
    plan_batch(nvs, gvs, maxg, bp, true);
    if (bp.nslots > cap + 4096) return false;      // slot buffer holds cap + 4096 slots
    const std::vector<int32_t> &order = bp.order;
    hipStream_t st = ctx.stream;
    if (hipMemcpyAsync(dm, hm.data(), n * sizeof(DMesh), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(ds, hs.data(), n * sizeof(DState), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(dp, hp.data(), n * sizeof(DParams), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(dord, order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(dtg, bp.task_g.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(dsl, bp.slots.data(), bp.slots.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) ||
        hipMemsetAsync(dnext, 0, sizeof(int), st))
        return false;
    if (launch_batch((const DMesh *)dm, (const DState *)ds, (const DParams *)dp, (const int32_t *)dord,
                     (const int32_t *)dtg, (const int32_t *)dsl, bp.nslots, (int *)dnext, bp.grid, lds, slice_ticks,
                     (int32_t *)ddone, ++g_epoch, occ, cm, st) != hipSuccess)
        return false;
    hdone.assign(n, 0);
    if (hipMemcpyAsync(hdone.data(), ddone, n * sizeof(int32_t), hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st))
        return false;
    launches += 1;
    const auto tc = Clock::now();
    t_launch_ms += ms_between(tl, tc);
    // done_out is indexed by visit order
    std::vector<SrvReq *> still;
    std::vector<SrvReq *> fin;
    std::vector<int32_t> flag(n, 0);
    for (int w = 0; w < n; ++w) flag[order[w]] = bp.task_g[w] > 0 && hdone[w];   // task_g 0: not visited
    for (int i = 0; i < n; ++i) (flag[i] ? fin : still).push_back(active[i]);
    active.swap(still);
    for (SrvReq *q : fin) {
        // kernel time of the request ends with this slice
        if (hipEventRecord(q->prep->e2, st) != hipSuccess) return false;
    }
    if (!fin.empty()) {
        {
            std::lock_guard<std::mutex> lk(mu);
            for (SrvReq *q : fin) cq.push_back(q);
        }
        ccv.notify_one();
    }
    (void)tc;
    return true;
}

void vls_server::loop() {
    (void)hipSetDevice(ctx.device);
    for (;;) {
        std::vector<SrvReq *> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            // a request fits when its run state fits the budget beside what is
            // admitted (running or still completing), or when nothing is
            cv.wait(lk, [&] {
                return stop || !active.empty() ||
                       (!queue.empty() && (used + queue.front()->bytes <= budget || used == 0));
            });
            if (stop) break;
            while (!queue.empty() && (int)(active.size() + admit.size()) < max_slots) {
                SrvReq *q = queue.front();
                if (used + q->bytes > budget && !(used == 0 && admit.empty())) break;
                queue.pop_front();
                used += q->bytes;
                admit.push_back(q);
            }
        }
        const auto ta = Clock::now();
        for (SrvReq *q : admit)
            if (admit_one(q)) active.push_back(q);
        t_admit_ms += ms_between(ta, Clock::now());
        if (active.empty()) continue;
        if (!launch_slice()) {
            thread_err = "device error in the server's step launch";
            for (SrvReq *q : active) finish(q, VLS_E_DEVICE, nullptr);
            active.clear();
        }
    }
}

extern "C" {

vls_status vls_server_create(vls_context *ctx, size_t hbm_budget_bytes, int32_t max_slots, int64_t slice_us,
                             uint32_t flags, vls_server **out) {
    if (!ctx || !out || max_slots < 1 || slice_us < 1 || hbm_budget_bytes == 0 ||
        (flags & ~(VLS_BATCH_TWO_PER_CU | VLS_COHERENT_SHARING)))
        return set_err(ctx, VLS_E_INVALID_ARG, "bad server arguments");
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, VLS_E_DEVICE, "hipSetDevice");
    auto s = std::make_unique<vls_server>();
    s->ctx.device = ctx->device;
    if (hipStreamCreateWithFlags(&s->ctx.stream, hipStreamNonBlocking) != hipSuccess)
        return set_err(ctx, VLS_E_DEVICE, "server stream");
    s->ctx.own_stream = true;
    s->cctx.device = ctx->device;
    if (hipStreamCreateWithFlags(&s->cctx.stream, hipStreamNonBlocking) != hipSuccess)
        return set_err(ctx, VLS_E_DEVICE, "server completion stream");
    s->cctx.own_stream = true;
    s->budget = hbm_budget_bytes;
    s->pool_cap = hbm_budget_bytes / 4;
    s->max_slots = max_slots;
    s->slice_ticks = (unsigned long long)slice_us * 100ull;    // s_memrealtime runs at 100 MHz
    s->occ = (flags & VLS_BATCH_TWO_PER_CU) ? 2 : 1;
    s->cm = (flags & VLS_COHERENT_SHARING) ? 1 : 0;
    vls_server *raw = s.get();
    try {
        s->cth = std::thread([raw] { raw->complete_loop(); });
    } catch (...) {
        return set_err(ctx, VLS_E_OUT_OF_MEMORY, "server thread");
    }
    try {
        s->th = std::thread([raw] { raw->loop(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->cstop = true;
        }
        s->ccv.notify_all();
        s->cth.join();
        return set_err(ctx, VLS_E_OUT_OF_MEMORY, "server thread");
    }
    *out = s.release();
    return VLS_OK;
}

vls_status vls_server_submit(vls_server *srv, const vls_mesh *m, const vls_params *p, uint64_t *ticket) {
    if (!srv || !m || !p || !ticket) return VLS_E_INVALID_ARG;
    if (p->struct_size != sizeof(vls_params)) return VLS_E_INVALID_ARG;
    if (p->flags & (VLS_TUNNEL_PASS | VLS_REFINE_PASS | VLS_REEB_REFINE | VLS_FEM_LAPLACIAN)) return VLS_E_INVALID_ARG;
    auto q = std::make_unique<SrvReq>();
    q->m = const_cast<vls_mesh *>(m);
    q->p = *p;
    q->p.flags &= ~VLS_DEFER_RESULTS;
    const bool rec = (p->flags & VLS_RECORD_FIELD) && p->n_ckpt > 0 && p->ckpt_steps;
    if (rec) q->ckpt.assign(p->ckpt_steps, p->ckpt_steps + p->n_ckpt);
    else { q->p.n_ckpt = 0; q->p.ckpt_steps = nullptr; q->p.flags &= ~VLS_RECORD_FIELD; }
    q->bytes = run_buffer_bytes(q->m) + (rec ? (size_t)p->n_ckpt * (size_t)m->nv * sizeof(double) : 0);
    q->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return VLS_E_CANCELLED;
        q->ticket = srv->next_ticket++;
        *ticket = q->ticket;
        srv->queue.push_back(q.get());
        srv->reqs.emplace(q->ticket, std::move(q));
    }
    srv->cv.notify_one();
    return VLS_OK;
}

vls_status vls_server_poll(vls_server *srv, uint64_t ticket, vls_result **out) {
    if (!srv || !out) return VLS_E_INVALID_ARG;
    *out = nullptr;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return VLS_E_INVALID_ARG;
    SrvReq *q = it->second.get();
    if (!q->done) return VLS_E_PENDING;
    const vls_status st = q->status;
    *out = q->res;
    srv->reqs.erase(it);
    return st;
}

vls_status vls_server_stats(const vls_server *srv, int64_t *launches, int64_t *completed, int64_t *admitted_bytes,
                            int32_t *queued, int32_t *running) {
    if (!srv) return VLS_E_INVALID_ARG;
    vls_server *s = const_cast<vls_server *>(srv);
    std::lock_guard<std::mutex> lk(s->mu);
    if (launches) *launches = s->launches;
    if (completed) *completed = s->completed;
    if (admitted_bytes) *admitted_bytes = (int64_t)s->used;
    if (queued) *queued = (int32_t)s->queue.size();
    if (running) {
        int32_t r = 0;
        for (auto &kv : s->reqs) r += !kv.second->done;
        *running = r - (int32_t)s->queue.size();
    }
    return VLS_OK;
}

vls_status vls_server_timing(const vls_server *srv, double *admit_ms, double *launch_ms, double *complete_ms) {
    if (!srv) return VLS_E_INVALID_ARG;
    vls_server *s = const_cast<vls_server *>(srv);
    std::lock_guard<std::mutex> lk(s->mu);
    if (admit_ms) *admit_ms = s->t_admit_ms;
    if (launch_ms) *launch_ms = s->t_launch_ms;
    if (complete_ms) *complete_ms = s->t_complete_ms;
    return VLS_OK;
}

vls_status vls_server_shutdown(vls_server *srv) {
    if (!srv) return VLS_E_INVALID_ARG;
    std::vector<SrvReq *> queued;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop && !srv->th.joinable()) return VLS_OK;
        srv->stop = true;
        queued.assign(srv->queue.begin(), srv->queue.end());
        srv->queue.clear();
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    // requests that finished on the device are completed normally
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->cstop = true;
    }
    srv->ccv.notify_all();
    if (srv->cth.joinable()) srv->cth.join();
    // the scheduler has stopped after its last launch: the requests it was
    // running and those still queued end as cancelled (their polls say so)
    (void)hipSetDevice(srv->ctx.device);
    (void)hipStreamSynchronize(srv->ctx.stream);
    std::vector<SrvReq *> drop(srv->active.begin(), srv->active.end());
    srv->active.clear();
    for (SrvReq *q : drop) { q->rb.reset(); q->prep.reset(); }
    std::lock_guard<std::mutex> lk(srv->mu);
    for (SrvReq *q : drop) {
        q->status = VLS_E_CANCELLED;
        q->done = true;
        q->t_done = Clock::now();
        srv->used -= q->bytes;
    }
    for (SrvReq *q : queued) {
        q->status = VLS_E_CANCELLED;
        q->done = true;
        q->t_done = Clock::now();
    }
    return VLS_OK;
}

vls_status vls_server_destroy(vls_server *srv) {
    if (!srv) return VLS_E_INVALID_ARG;
    (void)vls_server_shutdown(srv);
    for (auto &kv : srv->reqs)
        if (kv.second->res) (void)vls_result_destroy(kv.second->res);
    srv->reqs.clear();
    delete srv;
    return VLS_OK;
}

}  // extern "C"
