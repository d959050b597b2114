// vls_internal.h -- device-side data layout shared by the host part of the
// library (vls_api.cpp) and its HIP kernels (vls_kernels.hip).  Not part of
// the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vls {

// ---------------------------------------------------------------------------
// Mesh in HBM.  Half-edges are stored per owner vertex in counter-clockwise
// link order (triangles (u, cyc[e], cyc[succ[e]]) are the mesh triangles
// around u); the ascending neighbour list adj[] is kept separately because
// the field sum runs over ascending neighbour ids.
// ---------------------------------------------------------------------------
struct DMesh {
    int32_t nv;
    int32_t dmax;
    int64_t nnz;
    const int32_t *rp;    // [nv+1] row offsets (both layouts share them)
    const int32_t *adj;   // [nnz]  neighbours, ascending id
    const int32_t *cyc;   // [nnz]  neighbours, counter-clockwise from the smallest id
    const int32_t *src;   // [nnz]  owner vertex of half-edge e
    const int32_t *rev;   // [nnz]  index of the opposite half-edge
    const int32_t *succ;  // [nnz]  next half-edge of the same owner (ccw, wrapping)
    const int32_t *nin;   // [nnz]  e=(u->x), y=cyc[succ[e]]: index of half-edge (y->x)
    const int32_t *ell;   // [nv][ELL_W] ascending neighbours padded with the vertex itself;
                          //   first entry -1 when the degree exceeds ELL_W
    const int32_t *hrec;  // [nnz][4] per half-edge e: succ[e], nin[e], cyc[succ[e]], cyc[e]
    const int32_t *lrow;  // [nv][ELL_W] counter-clockwise neighbours from the smallest id,
                          //   padded with -1, first half-edge index in the last slot;
                          //   first entry -2 when the degree exceeds ELL_W - 1
    const double *xyz;    // [nv][3]
    const double *fem_g;  // [nnz] finite-element operator coefficients, ascending-neighbour order
                          //   (sigma * cot weight / lumped mass); null until prepared
};

constexpr int ELL_W = 16;             // width of the padded neighbour rows (64 B)
constexpr uint64_t KEY_OUT = ~0ull;   // rank key of a vertex not yet inside

// control block (device memory), zeroed by the host before a run
struct Ctl {
    unsigned long long bar;  // grid barrier arrivals (monotonic)
    unsigned long long fbar; // field-step completions (decoupled kernel): W per step
    long long kdone;         // last topology step completed (decoupled kernel)
    long long stop_step;     // step at which the topology stopped (decoupled kernel)
    int32_t stop[2];         // per-iteration exit decision, slot j&1
    int32_t done;
    int32_t status;
    int32_t err_code;        // detail for VLS_E_INVARIANT / VLS_E_CAPACITY
    int32_t cnt_act[4];      // update-list counts, slot t&3 for step t
    int32_t cnt_cand[4];     // crosser-candidate counts, slot t&3 for step t
    int32_t cnt_pend[2];     // pending crossers, slot t&1
    int32_t n_events;
    int32_t next_front;
    int32_t n_tags;
    int32_t n_loops;
    int32_t n_tunnels;
    int32_t n_degenerate;
    int64_t steps;
    int64_t n_inside;
    int64_t last_insert;
    int64_t active_updates;
    int64_t active_deg;
    int64_t lp_he_used;
    int64_t ev_ids_used;
    int64_t chi;
    int64_t b;
    int64_t gsum_h;
    int64_t gsum_x;
    int64_t event_steps;     // steps that needed the sequential event path
    // phase clocks (s_memrealtime ticks, 100 MHz): workgroup 0 topology,
    // workgroup 0 barrier wait, workgroup 1 field, workgroup 1 barrier wait
    unsigned long long clk_topo, clk_wait0, clk_field, clk_wait1;
    // finer split of the topology: candidates, closure, classification,
    // insertion (of which: steps with events, closure rounds after round 0)
    unsigned long long clk_t[4];
    unsigned long long clk_ev, clk_rounds;
    unsigned long long clk_fbar;   // field workgroup 1: wait for the other field workgroups
    unsigned long long clk_evp[4]; // events: merge walks, split walkers, relabel walks, the rest
    unsigned long long clk_ev0;
    unsigned long long clk_g[4];   // global-memory topology path: candidates, closure, classification, insertion
    int32_t n_round_steps, n_global_steps;
    // batched mode: next iteration to run (a mesh may be advanced over
    // several launches, each visit bounded in time), the first iteration of
    // the current gang visit, and the launch epoch that opened it
    int64_t biter;
    int64_t vbase;
    unsigned int gang_epoch;
};

// run state in HBM
struct DState {
    double *rho0, *rho1;     // field double buffer: step t lives in rho[t&1]
    uint64_t *key;           // [nv] (step << 32) | round, KEY_OUT if outside
    int32_t *parent;         // [nv]
    int32_t *depth;          // [nv]
    int32_t *lid;            // [nnz] front tag of a crossed half-edge (inside -> outside)
    int32_t *stamp;          // [nv] claims of new list entries (step number)
    int32_t *mark[2];        // [nv] update-set membership per step parity (step number)
    int32_t *cstamp;         // [nv] candidate de-duplication (step number)
    int32_t *act[2];         // [nv] update lists (step parity)
    int32_t *cand[2];        // [nv] crosser candidates (step parity)
    int32_t *pend[2];        // [nv] crossers not yet connected
    int32_t *L;              // [nv] topology-phase list
    int32_t *Lrnd;           // [nv] closure round per entry (-1: not connected)
    int32_t *Lcls;           // [nv] lower arcs per entry (-1: full link)
    uint64_t *ord;           // [nv] rank-sort scratch
    int32_t *tag_parent;     // [tag_cap] union-find over front tags
    int32_t *tag_fid;        // [tag_cap] front id of a root tag
    int32_t tag_cap;
    int32_t ev_cap;
    int64_t *ev;             // [ev_cap][16] event records
    int32_t *ev_rep;         // [ev_cap][16] one lower-run position per involved front
    int64_t *ev_ids;         // [ev_ids_cap] involved / new front ids
    int64_t ev_ids_cap;
    int32_t *front_birth;    // [front_cap]
    int32_t *front_death;    // [front_cap]
    int32_t front_cap;
    int32_t lp_cap;
    int64_t *lp;             // [lp_cap][8]: event, front id, kept, off, count, a-vertex, len bits, pad
    int32_t *lp_he;          // [lp_he_cap][2]
    double *lp_pts;          // [lp_he_cap][3]
    int64_t lp_he_cap;
    int32_t *tn;             // [lp_cap][4]: loop index, v, a_j, a_0
    int32_t *wck;            // [64][64] walk checkpoints of an event's involved loops
    double *wseg;            // [lp_he_cap] segment lengths of the loop being written
    double *ckpt;            // [n_ckpt][nv]
    const int64_t *ckpt_steps;  // (device) [n_ckpt]
    int32_t n_ckpt;
    int32_t pad1;
    Ctl *ctl;
};

struct DParams {
    double tau, a, w, e, c;  // c = dt * mu / 2
    int64_t seed;
    int32_t r0;
    int32_t stall_steps;
    int64_t max_steps;
    int32_t topo_global;     // 1: always use the global-memory topology path
    int32_t coherent;        // 1: coherent atomic shared accesses, release-only barrier
    int32_t lockstep;        // 1: one grid barrier per step instead of the decoupled kernel
    int32_t dense;           // 1: the field step updates every vertex (no update list)
    int32_t fem;             // 1: the finite-element operator (m.fem_g) in place of the graph Laplacian
    int32_t n_seed_set;      // > 0: the initial region grows from seed_set (ascending, unique; seed = its first)
    const int32_t *seed_set; // device
};

// ---------------------------------------------------------------------------
// tunnel-loop and handle-refinement passes (vls_passes.hip): one pass per
// workgroup at a time, each workgroup with its own slot of per-vertex state
// ---------------------------------------------------------------------------
struct PassSlot {
    double *rho;             // [nv] the pass's field (one buffer: Jacobi values go through tmp)
    double *tmp;             // [nv] new values of the update list, by list position
    double *ta;              // [nv] arrival time of inserted vertices
    double *prev;            // [nv] value before the step of a vertex that crossed the threshold
    uint64_t *key;           // [nv] (step << 32) | round, KEY_OUT outside
    int32_t *par;            // [nv] streamline parent
    int32_t *mark;           // [nv] update-list membership (step number; 0 = never listed)
    int32_t *cst;            // [nv] candidate de-duplication (step number)
    int32_t *upd;            // [nv] step of the last update that crossed the threshold
    int32_t *flag;           // [nv] PF_* bits
    int32_t *pos;            // [nv] loop-erasure positions (-1)
    int32_t *U[2];           // [nv] update lists (step parity)
    int32_t *cand;           // [nv] crossers of the step
    int32_t *pend[2];        // [nv] crossers not yet connected (step parity)
    int32_t *touched;        // [nv] every vertex listed at least once (reset at the end)
    int32_t *flist;          // [nv] every vertex with a flag (reset at the end)
    int32_t *buf;            // [nv] streamline, then the closed loop
    int32_t *side;           // [nv] the start side in loop order
    uint32_t *cutbits;       // [nnz/32 + 1] cut half-edges, ascending-row layout
};
struct PassTask {
    int32_t kind;            // 0: tunnel pass of a handle loop; 1: refinement pass of a tunnel
    int32_t src;             // kind 0: loop index (every involved loop of every merge); kind 1: tunnel task
};
struct PassResult {
    int32_t status;          // 0, VLS_E_STALLED, VLS_E_INVALID_ARG (no usable input), VLS_E_CAPACITY
    int32_t reached;         // vertex the pass reached on the other side (-1)
    int32_t label;           // 0 handle, 1 tunnel (offset along the normals), -1 none
    int32_t pad;
    int64_t steps, off, n, updates;
    double length, offset_length;
};
struct PassArgs {
    DMesh m;
    DState s;                // the initial pass's results: keys, events, loops
    const PassTask *tasks;
    int ntasks;
    int nslots;
    int *next;               // task counter
    const PassSlot *slots;   // [nslots]
    PassResult *res;         // [ntasks]
    int32_t *out;            // closed loops, appended
    int64_t out_cap;
    unsigned long long *out_used;
    const PassResult *src_res;   // refinement passes: the tunnel passes' results
    const int32_t *src_out;      //   and loops
    double tau, a, w, e, c;
    int64_t max_steps, stall_steps;
    double rel_eps;          // offset of the handle/tunnel test, times the mean edge length of the loop
};
hipError_t launch_passes(const PassArgs &a, hipStream_t st);
hipError_t launch_pass_slot_init(const PassSlot &s, int32_t nv, int64_t nnz, hipStream_t st);
int max_coresident_passes();

// host launchers (vls_kernels.hip)
hipError_t launch_init(const DMesh &m, const DState &s, int64_t nnz, hipStream_t st);
hipError_t launch_seed(const DMesh &m, const DState &s, const DParams &p, hipStream_t st);
// the finite-element operator of a mesh: lumped masses (scratch [nv]),
// scal = {sigma, largest absolute row sum} (scratch [2]), coefficients g
// [nnz]; dmax_bits [1] zeroed by the caller
hipError_t launch_fem_operator(const DMesh &m, double *mass, double *scal, double *g,
                               unsigned long long *dmax_bits, hipStream_t st);
hipError_t launch_steps(const DMesh &m, const DState &s, const DParams &p, int grid, int block,
                        hipStream_t st);
int max_coresident_blocks(int block, size_t lds_bytes);
hipError_t launch_batch(const DMesh *ms, const DState *ss, const DParams *ps, const int32_t *order,
                        const int32_t *task_g, const int32_t *slots, int nslots, int *next_slot, int grid, size_t lds,
                        unsigned long long budget_ticks, int32_t *done_out, unsigned int epoch, int occ, int cm,
                        hipStream_t st);
int max_coresident_batch(size_t lds_bytes, int occ);
size_t batch_lds_bytes(int occ);
size_t step_lds_bytes(int block, int dmax);
hipError_t launch_reeb_count(const DMesh &m, const DState &s, int ev0, int n_events, int64_t *cnt, int32_t *ck,
                             int64_t *meta, hipStream_t st);
hipError_t launch_reeb_fill(const DMesh &m, const DState &s, int ev0, int n_events, const int64_t *off,
                            const int64_t *cnt, const int32_t *ck, const int64_t *meta, int32_t *buf,
                            hipStream_t st);
hipError_t launch_reeb_mean(const DMesh &m, int n_events, const int64_t *off, const int64_t *cnt,
                            int32_t *buf, double *pos, hipStream_t st);
hipError_t launch_tunnel_count(const DState &s, int n_tunnels, int64_t *cnt, hipStream_t st);
// the same post-passes over the events / tunnels of many meshes at once:
// entry g is event eve[g] (tunnel tnt[g]) of mesh evm[g] (tnm[g]) of the
// device arrays ms / ss
hipError_t launch_reeb_count_multi(const DMesh *ms, const DState *ss, const int32_t *evm, const int32_t *eve, int n,
                                   int64_t *cnt, int32_t *ck, int64_t *meta, hipStream_t st);
hipError_t launch_reeb_fill_multi(const DMesh *ms, const DState *ss, const int32_t *evm, const int32_t *eve, int g0,
                                  int n, const int64_t *off, const int64_t *cnt, const int32_t *ck,
                                  const int64_t *meta, int32_t *buf, hipStream_t st);
hipError_t launch_reeb_mean_multi(const DMesh *ms, const int32_t *evm, int g0, int n, const int64_t *off,
                                  const int64_t *cnt, int32_t *buf, double *pos, hipStream_t st);
hipError_t launch_tunnel_count_multi(const DState *ss, const int32_t *tnm, const int32_t *tnt, int n, int64_t *cnt,
                                     hipStream_t st);
hipError_t launch_tunnel_fill_multi(const DMesh *ms, const DState *ss, const int32_t *tnm, const int32_t *tnt, int g0,
                                    int n, const int64_t *off, int32_t *out, double *len, hipStream_t st);
hipError_t launch_tunnel_fill(const DMesh &m, const DState &s, int t0, int n_tunnels, const int64_t *off, int32_t *out,
                              double *len, hipStream_t st);

// bytes of the per-device static scratch of vls_run_async_noalloc, and its
// device address on `device` (hipGetSymbolAddress, once per device)
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
hipError_t static_scratch(int device, void **ptr);

}  // namespace vls
