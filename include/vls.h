/*
 * vls.h -- C ABI of the MI355X library for the initial pass of the
 * variational loop-shrinking method (Weinrauch, Seidel, Mlakar, Steinberger,
 * Zayer, "A Variational Loop Shrinking Analogy for Handle and Tunnel
 * Detection and Reeb Graph Construction on Surfaces", ACM TOG).
 *
 * Problem statement (Introduction; Section "Variational Loop Shrinking"):
 * a closed orientable triangle mesh goes in; handle loops, tunnel loops and
 * the Reeb graph swept by a diffusion front grown from one seed location
 * come out.  Every computing step runs in HIP kernels on the GPU; the host
 * side only validates the mesh, builds its adjacency, launches, and copies
 * results back.
 *
 * Conventions
 *   - Plain C, no exceptions cross the ABI.  Every call returns a
 *     vls_status (0 = VLS_OK, negative = error); the context keeps a
 *     human-readable detail for its last failure (vls_last_error).
 *   - Inputs are copied at *_create; handles are opaque and owned by the
 *     library until *_destroy.  Result arrays are caller-allocated and use a
 *     two-call protocol: call with cap = 0 to get the size in *n_out, then
 *     again with enough capacity; too small a capacity fails with
 *     VLS_E_BUFFER_TOO_SMALL and still reports the size.
 *   - Host pointers are marked (host); device pointers (device).
 *   - Results depend only on (mesh, params): not on launch shape, stream or
 *     other work on the device.  The field is computed in FP64 with a fixed
 *     evaluation order (no contraction, IEEE sqrt), so it is reproducible
 *     bit for bit.
 *   - One context per host thread.
 */
#ifndef VLS_H
#define VLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vls_status;
enum {
    VLS_OK = 0,
    VLS_E_INVALID_ARG = -1,
    VLS_E_MESH_NOT_MANIFOLD = -2,     /* a vertex link is not one cycle, or a degenerate triangle */
    VLS_E_MESH_HAS_BOUNDARY = -3,     /* an edge lacks its opposite half-edge                    */
    VLS_E_MESH_NOT_CONNECTED = -4,    /* more than one component, or an unused vertex            */
    VLS_E_MESH_NOT_ORIENTABLE = -5,   /* a directed edge occurs twice                            */
    VLS_E_SEED_INVALID = -6,          /* the initial region has swept genus != 0 or no boundary  */
    VLS_E_STALLED = -7,               /* no insertion for stall_steps, or max_steps reached      */
    VLS_E_OUT_OF_MEMORY = -8,
    VLS_E_DEVICE = -9,                /* a HIP runtime call failed                               */
    VLS_E_BUFFER_TOO_SMALL = -10,
    VLS_E_PENDING = -11,              /* server request / async run not finished yet             */
    VLS_E_CANCELLED = -12,            /* server request dropped by vls_server_shutdown / _destroy */
    VLS_E_INVARIANT = -13,            /* a topological invariant failed (see vls_last_error)     */
    VLS_E_CAPACITY = -14,             /* an internal device buffer bound was exceeded            */
    VLS_E_TOO_LARGE = -15             /* mesh beyond the index range or the degree limit (64)    */
};

/* Reeb node types (Section "Initial Pass": branching and collision;
   Section "Reeb Graph Extraction"). */
enum { VLS_NODE_SEED = 0, VLS_NODE_SPLIT = 1, VLS_NODE_MERGE = 2, VLS_NODE_VANISH = 3,
       VLS_NODE_DEGENERATE = 4 };

/* flags */
#define VLS_RECORD_FIELD 1u   /* keep FP64 snapshots of the field at ckpt_steps */
#define VLS_DEFER_RESULTS 2u  /* vls_run returns once the device work is done; bulk results
                                 are copied to the host by vls_result_fetch or on first access */
#define VLS_TOPO_GLOBAL_PATH 4u  /* always run the topology phase from global memory (the path
                                    otherwise taken only by steps with more candidates than the
                                    LDS tables hold: 2048 solo, 1024 in two-per-CU launches);
                                    results are identical, the flag exists for testing */
#define VLS_COHERENT_SHARING 8u  /* share data between workgroups through coherent atomic accesses
                                    and release-only hand-offs instead of plain accesses and full
                                    agent-scope fences (vls_run; vls_batch_run through the flags of
                                    per_mesh[0]; the server through its creation flags); identical
                                    results */
#define VLS_LOCKSTEP 16u         /* one grid barrier per step (topology of t beside field of t+1)
                                    instead of the decoupled kernel; identical results, for testing */
#define VLS_DENSE_FIELD 64u      /* the field step updates every vertex in id order instead of the
                                    update list (streams the whole mesh each step; vls_run's default
                                    grid is then every co-resident workgroup); identical results;
                                    meshes below 2^29 vertices (else VLS_E_INVALID_ARG) */
#define VLS_TUNNEL_PASS 128u     /* vls_run only: after the initial pass, a tunnel-loop pass for every
                                    handle loop (Section "Tunnel loop pass"): loops of kind 3 */
#define VLS_REFINE_PASS 256u     /* vls_run only: also a handle-refinement pass for every tunnel of the
                                    tunnel-loop pass (Section "Handle refinement pass"): loops of
                                    kind 4; implies VLS_TUNNEL_PASS */
#define VLS_FEM_LAPLACIAN 512u   /* vls_run and the workspace calls: the field step uses the Laplacian of
                                    linear finite elements (Section "Mathematical representation and
                                    data structure", "Implementation details") in place of the uniform
                                    graph Laplacian: cotangent weights over lumped masses, scaled by
                                    sqrt(3) x the mean lumped mass (so that on a mesh of equilateral
                                    triangles of one valence it is the graph Laplacian), dt = 50 (or
                                    0.25) over its largest absolute row sum; see vls_mesh_prepare_fem.
                                    Not with VLS_DENSE_FIELD, the passes, vls_batch_run or the server
                                    (VLS_E_INVALID_ARG) */
#define VLS_REEB_REFINE 1024u    /* vls_run only: Reeb junction refinement (Section "Reeb Graph
                                    Extraction": a second pass improves where the junctions sit;
                                    Section "Introduction": a Reeb graph from a diffusion initiated at
                                    a detected handle loop).  When the pass ends with a handle loop,
                                    the initial pass runs again from the first kept one: its initial
                                    region is every vertex within seed_radius hops of the loop's inside
                                    vertices, ranked by hop distance inside that region from the
                                    smallest of them.  That second result (its Reeb graph has the
                                    refined junctions at its band means) is read with
                                    vls_result_refined.  The first result is fetched before the second
                                    pass starts, so VLS_DEFER_RESULTS has no effect; the secondary
                                    passes and field checkpoints apply to the first pass only.  Not with
                                    vls_batch_run, the server or the workspace calls
                                    (VLS_E_INVALID_ARG) */
#define VLS_BATCH_TWO_PER_CU 32u /* vls_batch_run (flags of per_mesh[0]) and the server (creation
                                    flags): two workgroups per CU, each with a 1024-candidate LDS
                                    topology path and one list entry per field thread; default: one
                                    per CU with the solo kernel's 2048 candidates and two entries */

/*
 * Parameters.  Defaults (vls_params_default) are the paper's coefficients
 * (Section "Mathematical representation and data structure", "Implementation
 * details": e = 1/30, mu = 1/4, a = 1/25, w = a/5) and the readings of the
 * points it leaves open: threshold tau = 0.5, time step dt = 50/dmax
 * (dt_mode 0) or the literal 0.25/dmax (dt_mode 1), seed region = hop ball
 * of radius 2 around seed_vertex.
 */
typedef struct vls_params {
    uint32_t struct_size;      /* sizeof(vls_params)                                      */
    int32_t dt_mode;           /* 0: dt = 50/dmax, 1: dt = 0.25/dmax                     */
    double tau, mu, a, w, e;   /* threshold and equation coefficients                    */
    int64_t seed_vertex;       /* >= 0: seed vertex id; < 0: chosen from rng_seed        */
    uint64_t rng_seed;         /* seed_vertex = splitmix64(rng_seed) mod nv when < 0      */
    int32_t seed_radius;       /* hop radius of the initial region (>= 0)                */
    int32_t stall_steps;       /* VLS_E_STALLED after this many steps without insertion  */
    int64_t max_steps;         /* VLS_E_STALLED when reached                              */
    uint32_t flags;            /* VLS_RECORD_FIELD                                        */
    int32_t n_ckpt;            /* number of entries in ckpt_steps                         */
    const int64_t *ckpt_steps; /* (host) steps whose field is kept (with VLS_RECORD_FIELD) */
    int32_t grid;              /* persistent workgroups; 0 = chosen by the library: about
                                  one per 34k vertices, 16..128, at most what is co-resident;
                                  vls_batch_run: pool size of per_mesh[0]                 */
    int32_t block;             /* threads per workgroup: 256 (0 = default)                */
    int64_t gang_vertices;     /* vls_batch_run (per_mesh[0], for every mesh) and each server
                                  request (its own): a mesh gets one workgroup per this many
                                  vertices (at least 2 to form a gang, at most 64); 0 = 65536 */
    int32_t pass_slots;        /* tunnel-loop / refinement passes run at once (each on one
                                  workgroup with its own per-vertex state, about 100 B per
                                  vertex); 0 = as many as co-resident workgroups and half of
                                  the free device memory allow */
    int32_t reserved;
} vls_params;

struct vls_context;
struct vls_mesh;
struct vls_result;

void vls_params_default(vls_params *p);
const char *vls_status_string(vls_status s);
/* detail text of the last failing call on ctx (never NULL; "" if none) */
const char *vls_last_error(const struct vls_context *ctx);

/* Context: binds a HIP device and a stream.  hip_stream is a hipStream_t
   (e.g. PyTorch's current stream); NULL creates a private stream.  All
   library work of this context is enqueued on that stream. */
vls_status vls_context_create(int device, void *hip_stream, struct vls_context **out);
vls_status vls_context_destroy(struct vls_context *ctx);

/*
 * Mesh setup (step S0: closed, connected, orientable 2-manifold; the paper
 * precomputes the mesh operator once, Section "Mathematical representation
 * and data structure", "Implementation details").
 *   nv   number of vertices, xyz (host) [nv][3] FP64 positions
 *   nf   number of triangles, tri (host) [nf][3] vertex ids, consistently
 *        oriented (counter-clockwise seen from outside)
 * Copies, validates, builds the adjacency (ascending and counter-clockwise
 * vertex links, reverse and successor half-edge maps) and uploads it.
 * Limits: every vertex degree is 3..64, nv < 2^31 - 1 and 3*nf < 2^31.
 * Errors: VLS_E_MESH_* when the mesh is not a closed connected orientable
 * manifold; VLS_E_TOO_LARGE when 3*nf >= 2^31 or a vertex has degree > 64.
 */
vls_status vls_mesh_create(struct vls_context *ctx, int64_t nv, const double *xyz,
                           int64_t nf, const int32_t *tri, struct vls_mesh **out);
/* ne = edges, dmax = maximum vertex degree, euler_genus = (2 - (V-E+F))/2 */
vls_status vls_mesh_info(const struct vls_mesh *m, int64_t *nv, int64_t *ne, int64_t *nf,
                         int32_t *dmax, int32_t *euler_genus);
vls_status vls_mesh_destroy(struct vls_mesh *m);

/*
 * The Laplacian of linear finite elements on the mesh (Section
 * "Mathematical representation and data structure", "Implementation
 * details": the fields are discretised with standard linear finite elements
 * and the mesh's Laplacian matrix is computed once), for runs with
 * VLS_FEM_LAPLACIAN.  Computed on the device and kept with the mesh
 * (8 bytes per half-edge) until vls_mesh_destroy; later calls return the
 * kept values.  For vertex v with counter-clockwise link c_0..c_{d-1}:
 *   lumped mass  m_v = (sum over k of area(v, c_k, c_{k+1})) / 3,
 *   weight       k_vu = (cot(angle at a) + cot(angle at b)) / 2, a and b the
 *                link successor and predecessor of u (the two vertices
 *                facing the edge vu),
 *   coefficient  g_vu = sigma * k_vu / m_v,  sigma = sqrt(3) * mean(m_v),
 * and the field step's Laplacian is sum over ascending neighbours u of
 * g_vu * (rho_u - rho_v).  *sigma and *row_sum_max (the largest sum of
 * |g_vu| over a row; the step size is 50 / row_sum_max) may be NULL.
 * vls_run prepares the operator by itself; the workspace calls, which
 * allocate nothing, need it prepared first.  Errors: VLS_E_OUT_OF_MEMORY,
 * VLS_E_DEVICE, VLS_E_INVALID_ARG for a degenerate operator (a zero or
 * non-finite row sum, from degenerate triangles).
 */
vls_status vls_mesh_prepare_fem(struct vls_mesh *m, double *sigma, double *row_sum_max);

/*
 * The prepared coefficients g_vu, nnz of them, in CSR order of ascending
 * neighbours (row v holds v's neighbours in increasing id).  cap = 0 only
 * reports *n_out = nnz; a smaller positive cap gives VLS_E_BUFFER_TOO_SMALL;
 * VLS_E_INVALID_ARG before vls_mesh_prepare_fem.
 */
vls_status vls_mesh_fem_coefficients(const struct vls_mesh *m, int64_t cap, double *g, int64_t *n_out);

/*
 * The initial pass (Section "Initial Pass"), blocking.  Runs the seed
 * initialisation, then the persistent step kernel until every vertex is
 * inside, then the Reeb-position and tunnel post-passes, and copies the
 * results to host memory owned by *out.  A run that stalls still returns a
 * result whose summary carries run_status = VLS_E_STALLED and the events
 * recorded so far; the call then returns VLS_E_STALLED.
 */
vls_status vls_run(struct vls_context *ctx, const struct vls_mesh *m, const vls_params *p,
                   struct vls_result **out);

/*
 * The same pass on caller-owned device memory and a caller stream: PyTorch
 * (or any caller) allocates the workspace and owns the stream; the library
 * allocates no device memory for the run (Introduction: mesh in, loops and
 * Reeb graph out; the memory-budgeted concurrency of Section "Performance
 * Considerations" is the caller's to plan with vls_workspace_size).
 *
 * vls_workspace_size: bytes of device workspace a vls_run_async of mesh m
 *   with parameters p needs: the run state (per vertex and per half-edge
 *   arrays, event and loop buffers), the field checkpoints of p, and the
 *   post-pass scratch (Reeb positions and tunnel paths, processed in chunks
 *   that always fit it).  Depends on the mesh and on p's checkpoint count
 *   only.
 * vls_run_async: enqueues the seed initialisation and the persistent step
 *   kernel on hip_stream (a hipStream_t; NULL = the context's stream) and
 *   returns at once with *out in the launched state.  d_workspace (device,
 *   256-byte aligned, at least vls_workspace_size bytes) is borrowed: it
 *   must stay allocated and untouched by other work until vls_result_wait
 *   (or the first accessor, or vls_result_destroy) has returned; its
 *   initial contents do not matter.  p and its checkpoint list are copied.
 *   The mesh's own cached run state is not used, so several async runs of
 *   one mesh may be in flight, each with its own workspace.
 * vls_result_wait: waits for the step kernel, runs the post-passes on the
 *   same stream in the workspace, copies every result to host memory owned
 *   by the result, and returns the run status (as vls_run would).  Every
 *   accessor waits implicitly; a stream synchronisation alone does not run
 *   the post-passes.  For a result of vls_run it returns its run status.
 * Errors: VLS_E_BUFFER_TOO_SMALL (workspace too small), VLS_E_INVALID_ARG
 *   (misaligned or NULL workspace, bad parameters), VLS_E_DEVICE.
 */
vls_status vls_workspace_size(const struct vls_mesh *m, const vls_params *p, size_t *bytes);
vls_status vls_run_async(struct vls_context *ctx, const struct vls_mesh *m, const vls_params *p,
                         void *d_workspace, size_t bytes, void *hip_stream, struct vls_result **out);
vls_status vls_result_wait(struct vls_result *r);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the pass
 * of vls_run_async with its workspace replaced by a static device array of
 * 64 MiB per device, which the library holds until the process ends.  No
 * hipMalloc, hipFree, event or stream creation happens in this call or in
 * the wait; the result and its arrays are host memory.  The mesh (created
 * beforehand) and the result are the caller's inputs and outputs.
 *   - Meshes whose vls_workspace_size exceeds 64 MiB (about 120-150k vertices)
 *     fail with VLS_E_BUFFER_TOO_SMALL.
 *   - Every call on one device shares that device's array: a call made
 *     while an earlier call's result has not been waited for (or
 *     destroyed) fails with VLS_E_PENDING; calls that bypass this check
 *     (another process's copy of the library aside, which has its own
 *     array) would race on the array.  The array keeps the last run's
 *     contents; the run clears what must start at zero itself.
 */
vls_status vls_run_async_noalloc(struct vls_context *ctx, const struct vls_mesh *m, const vls_params *p,
                                 void *hip_stream, struct vls_result **out);

typedef struct {
    int32_t n_handles;         /* handle loops emitted (merges: fronts involved minus one)   */
    int32_t n_tunnels;         /* tunnel candidates, one per handle loop                      */
    int32_t euler_genus;       /* (2 - chi(mesh))/2                                           */
    int32_t swept_genus;       /* (2 - chi_t - b_t)/2 at the last step                        */
    int32_t reeb_nodes, reeb_edges, n_degenerate;
    int32_t n_events;
    int64_t steps;             /* diffusion steps taken                                       */
    int64_t active_vertex_updates;  /* sum over steps of the updated vertex count             */
    int64_t active_degree_sum;      /* sum of the degrees of those updates                    */
    int64_t n_inside;
    int64_t seed_vertex;
    vls_status run_status;
    int32_t grid, block;       /* launch shape used                                           */
    double kernel_ms;          /* device time of the persistent step kernel (HIP events)     */
    double total_ms;           /* device time of the whole pass, seed to post-passes          */
    /* device clock (s_memrealtime) split of the step kernel: workgroup 0
       topology work and its barrier wait, workgroup 1 field work and wait */
    double topo_ms, wait0_ms, field_ms, wait1_ms;
    int64_t event_steps;       /* steps resolved through the sequential event path           */
    double topo_split_ms[4];   /* topology: candidates, closure, classification, insert/events */
    double topo_event_ms;      /* topology: time in steps with events (rank-ordered insertion) */
    double topo_rounds_ms;     /* topology: closure rounds after round 0                       */
    int32_t topo_round_steps;  /* steps that needed closure rounds after round 0               */
    int32_t topo_global_steps; /* steps whose candidates took the global-memory path           */
    /* server requests only (0 otherwise), host wall clock: submission to
       admission (queueing) and submission to result ready (latency) */
    double server_queue_ms, server_latency_ms;
    /* decoupled kernel: field workgroup 1's wait for the other field
       workgroups (wait1_ms is then its wait for the topology) */
    double field_barrier_ms;
    /* event resolution split: merge loop walks and output, split walkers,
       relabel walks, the rest (classification, ids, records) */
    double event_split_ms[4];
    /* tunnel-loop / handle-refinement passes (VLS_TUNNEL_PASS, VLS_REFINE_PASS):
       passes run and passes that produced a loop, passes run at once,
       device time of each kind's launch, and the vertex updates of all */
    int32_t n_tunnel_passes, n_tunnel_loops, n_refine_passes, n_refined_loops;
    int32_t pass_slots, pass_pad;
    double tunnel_pass_ms, refine_pass_ms;
    int64_t pass_vertex_updates;
    /* topology steps on the global-memory path: candidates, closure,
       classification, insertion and events (device clock) */
    double topo_global_split_ms[4];
} vls_summary;
vls_status vls_result_summary(const struct vls_result *r, vls_summary *s);

/* Event log: one record of 16 int64 per saddle/vanish insertion, in rank
   order: step, vertex, node type, k (lower arcs; 0 for vanish), s (fronts
   involved), m (fronts after), h (handles), x (extra cycles), Reeb node
   index, closure round, vanish flag, offset into the front-id list,
   reserved[4].  The front-id list holds, per event, its s involved front
   ids (ascending) followed by its m new front ids. */
vls_status vls_result_events(const struct vls_result *r, int64_t cap, int64_t *rec,
                             int64_t *n_out);
vls_status vls_result_event_fronts(const struct vls_result *r, int64_t cap, int64_t *ids,
                                   int64_t *n_out);

/*
 * Loops.  kind 0 = handle loop i: the ordered crossed edges
 * (inside, outside) of the front just before the merge, starting at the
 * smallest (inside*nv + outside) key (Section "Initial Pass": the involved
 * fronts before the merge, the longest one ignored); pts = crossing points
 * on those edges at the threshold, length = closed polyline length.
 * kind 1 = tunnel candidate i (the streamline traced back against the
 * diffusion, Introduction / Section "Tunnel loop pass"): a closed vertex
 * cycle v, a_i, parent(a_i), ..., common ancestor, ..., a_0 written into
 * edges_uv[*][0] (edges_uv[*][1] = next vertex); pts/length for its vertex
 * polyline.  kind 2 = every involved loop of every merge (handle loops and
 * the ignored longest one), in event order.
 * kind 3 = the tunnel loop of handle loop i from the tunnel-loop pass, kind
 * 4 = the refined handle loop of tunnel i from the handle-refinement pass
 * (with VLS_TUNNEL_PASS / VLS_REFINE_PASS): closed vertex paths, written as
 * kind 1 (edges_uv[*][0] the vertices, pts their positions, length the
 * closed polyline's); n_out = 0 when that pass produced no loop.
 */
vls_status vls_result_loop(const struct vls_result *r, int32_t kind, int32_t i, int64_t cap,
                           int32_t *edges_uv, double *pts, double *length, int64_t *n_out);
/*
 * Outcome of pass i of kind 3 (tunnel-loop) or 4 (handle-refinement)
 * (Sections "Tunnel loop pass", "Handle refinement pass", "Distinguishing
 * handle and tunnel loops"): status (0; VLS_E_STALLED when the diffusion
 * stopped before reaching the other side; VLS_E_INVALID_ARG when its
 * source loop was missing or degenerate; VLS_E_CAPACITY when the loop
 * buffer overflowed), diffusion steps, the vertex reached first on the
 * other side, and the normal-offset test: label 0 = handle (the loop grows
 * when moved along the surface normals by a tenth of its mean edge length),
 * 1 = tunnel (it shrinks), -1 = no loop; length and offset length.
 * Any output pointer may be NULL.
 */
vls_status vls_result_pass_info(const struct vls_result *r, int32_t kind, int32_t i, int32_t *status,
                                int64_t *steps, int32_t *reached, int32_t *label, double *length,
                                double *offset_length);
/* per-loop info for kind 0 or 2: event index, front id, kept (1 = handle loop) */
vls_status vls_result_loop_info(const struct vls_result *r, int32_t kind, int32_t i,
                                int64_t *event, int64_t *front_id, int32_t *kept);

typedef struct { int32_t type, vertex, in_deg, out_deg, extra_cycles; int32_t pad; int64_t step; double xyz[3]; } vls_reeb_node;
typedef struct { int32_t src, dst, front_id; } vls_reeb_edge;
/* Reeb graph (Section "Reeb Graph Extraction"): node 0 is the seed, node
   i+1 the i-th event; a node sits at the mean position of the distinct
   vertices of the front triangles of the fronts involved; edge = front,
   from its birth node to its death node (dst = -1 if still alive). */
vls_status vls_result_reeb(const struct vls_result *r, int64_t cap_n, vls_reeb_node *nodes,
                           int64_t cap_e, vls_reeb_edge *edges, int64_t *n_nodes, int64_t *n_edges);

/* Field snapshot at step (one of ckpt_steps, with VLS_RECORD_FIELD), or the
   final field for step < 0.  rho (host) [nv] FP64. */
vls_status vls_result_field(const struct vls_result *r, int64_t step, double *rho);
/* Per vertex: insertion step (INT32_MAX if never inside), closure round,
   parent (streamline predecessor, -1 for the seed).  Any pointer may be NULL. */
vls_status vls_result_vertices(const struct vls_result *r, int32_t *step, int32_t *round,
                               int32_t *parent);
/*
 * Batched initial passes (many meshes, one launch): each mesh is advanced by
 * one workgroup of a persistent pool, the largest meshes first; a mesh's
 * results are identical to a vls_run of that mesh alone.  meshes[n] must be
 * distinct (a mesh holds one run's device state); per_mesh[n] parameters
 * (grid of per_mesh[0] = pool size, 0 = as many as fit); out[n] receives one
 * result per mesh (kernel_ms of each = the whole batch kernel).  Returns the
 * first non-OK run status, VLS_OK if all succeeded.
 */
vls_status vls_batch_run(struct vls_context *ctx, int32_t n, const struct vls_mesh *const *meshes,
                         const vls_params *per_mesh, struct vls_result **out);

/*
 * Serving: a request loop over one device with continuous batching.  The
 * paper runs its secondary passes concurrently up to what GPU memory allows
 * (Section "Tunnel loop pass", "Implementation details"); here whole
 * initial passes of different meshes share the device the same way.
 *
 * vls_server_create: a scheduler thread with its own stream on ctx's
 *   device.  hbm_budget_bytes caps the device run state of the admitted
 *   requests (per request: the per-vertex and per-half-edge run arrays,
 *   event/loop buffers and checkpoints; the mesh itself is the caller's);
 *   max_slots caps how many run at once.  A request larger than the budget
 *   is admitted only when nothing else runs.  flags: VLS_BATCH_TWO_PER_CU
 *   (two workgroups per CU in the step launches; default one) and
 *   VLS_COHERENT_SHARING (gangs share through coherent atomics); any other
 *   bit is VLS_E_INVALID_ARG.
 * vls_server_submit: queues an initial pass of mesh m with parameters p
 *   (copied, checkpoint list included); thread-safe; *ticket identifies it.
 *   The mesh must stay alive until the request is polled; one mesh may be
 *   in several requests at once (each has its own run state).
 * Scheduling: admitted requests advance together in bounded launches of
 *   the batched step kernel (one workgroup per mesh, each visit bounded to
 *   slice_us microseconds of device time at a step boundary); between
 *   launches finished requests are completed (post-passes, results to host)
 *   and queued ones admitted as slots and budget free up.  A request's
 *   results are identical to a vls_run of the same mesh and parameters.
 *   The run state of finished requests is kept for later requests of the
 *   same mesh (up to a quarter of hbm_budget_bytes, outside the budget), so
 *   a repeated mesh is admitted without allocating.
 * vls_server_poll: VLS_E_PENDING until the request is done; then *out
 *   receives its result (owned by the caller) and the call returns the run
 *   status; the ticket is then forgotten.  Thread-safe.
 * vls_server_shutdown: stops the scheduler after its current launch; every
 *   request still queued or running is cancelled: its poll returns
 *   VLS_E_CANCELLED with *out = NULL.  Finished requests keep their results
 *   until polled; later submits return VLS_E_CANCELLED.  Idempotent.
 * vls_server_destroy: vls_server_shutdown, then frees the server and every
 *   result that was never polled; the handle and its tickets are invalid
 *   afterwards.
 * Errors: VLS_E_INVALID_ARG (bad handle/ticket), VLS_E_DEVICE.
 */
struct vls_server;
vls_status vls_server_create(struct vls_context *ctx, size_t hbm_budget_bytes, int32_t max_slots,
                             int64_t slice_us, uint32_t flags, struct vls_server **out);
vls_status vls_server_submit(struct vls_server *srv, const struct vls_mesh *m, const vls_params *p,
                             uint64_t *ticket);
vls_status vls_server_poll(struct vls_server *srv, uint64_t ticket, struct vls_result **out);
/* counters: launches of the step kernel, requests completed, device run
   state currently admitted (bytes), requests queued and running */
vls_status vls_server_stats(const struct vls_server *srv, int64_t *launches, int64_t *completed,
                            int64_t *admitted_bytes, int32_t *queued, int32_t *running);
/* host time the scheduler thread has spent admitting requests (run state,
   seed initialisation), launching slices (including the wait for each), and
   completing finished requests (post-passes, results to host), in ms */
vls_status vls_server_timing(const struct vls_server *srv, double *admit_ms, double *launch_ms,
                             double *complete_ms);
vls_status vls_server_shutdown(struct vls_server *srv);
vls_status vls_server_destroy(struct vls_server *srv);

/* Copies the bulk results of a VLS_DEFER_RESULTS run to the host (no-op
   otherwise).  Called implicitly by every accessor, by the next vls_run on
   the same mesh and by vls_mesh_destroy, since a mesh keeps one run's
   device state at a time.  A deferred result must be fetched or destroyed
   before its context is destroyed. */
vls_status vls_result_fetch(struct vls_result *r);
/* The second pass of VLS_REEB_REFINE (Section "Reeb Graph Extraction"): *second is a result owned by
   r (read it with the accessors above; destroyed with r, never by the caller), or NULL when the flag
   was not given or the pass found no handle loop. */
vls_status vls_result_refined(const struct vls_result *r, const struct vls_result **second);
/* Frees a result; a deferred result that was never fetched is discarded
   without copying it. */
vls_status vls_result_destroy(struct vls_result *r);

#ifdef __cplusplus
}
#endif
#endif /* VLS_H */
