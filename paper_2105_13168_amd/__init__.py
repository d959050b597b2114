"""Python binding of libvls.so, the MI355X library for the initial pass of the
variational loop-shrinking method (handle loops, tunnel loops and Reeb graph
of a closed orientable triangle mesh).

Only argument marshalling lives here: every step of the method runs in the
HIP kernels behind the C ABI of ``include/vls.h``.  The functions keep the C
names (``vls_context_create``, ``vls_mesh_create``, ``vls_run``, ...); the
small ``Context`` / ``Mesh`` / ``Result`` classes wrap them for tests and the
benchmark.  The library must have been built (``python
paper_2105_13168_amd/build.py``); importing fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvls.so")

VLS_OK = 0
VLS_E_INVALID_ARG = -1
VLS_E_STALLED = -7
VLS_E_BUFFER_TOO_SMALL = -10
VLS_E_PENDING = -11
VLS_E_CANCELLED = -12
VLS_E_INVARIANT = -13
VLS_E_CAPACITY = -14
VLS_E_TOO_LARGE = -15
VLS_RECORD_FIELD = 1
VLS_DEFER_RESULTS = 2
VLS_TOPO_GLOBAL_PATH = 4
VLS_COHERENT_SHARING = 8
VLS_LOCKSTEP = 16
VLS_BATCH_TWO_PER_CU = 32
VLS_DENSE_FIELD = 64
VLS_TUNNEL_PASS = 128
VLS_REFINE_PASS = 256
VLS_FEM_LAPLACIAN = 512
VLS_REEB_REFINE = 1024
NODE_SEED, NODE_SPLIT, NODE_MERGE, NODE_VANISH, NODE_DEGENERATE = range(5)


class vls_params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("dt_mode", C.c_int32),
                ("tau", C.c_double), ("mu", C.c_double), ("a", C.c_double),
                ("w", C.c_double), ("e", C.c_double),
                ("seed_vertex", C.c_int64), ("rng_seed", C.c_uint64),
                ("seed_radius", C.c_int32), ("stall_steps", C.c_int32),
                ("max_steps", C.c_int64), ("flags", C.c_uint32), ("n_ckpt", C.c_int32),
                ("ckpt_steps", C.POINTER(C.c_int64)), ("grid", C.c_int32), ("block", C.c_int32),
                ("gang_vertices", C.c_int64), ("pass_slots", C.c_int32), ("reserved", C.c_int32)]


class vls_summary(C.Structure):
    _fields_ = [("n_handles", C.c_int32), ("n_tunnels", C.c_int32), ("euler_genus", C.c_int32),
                ("swept_genus", C.c_int32), ("reeb_nodes", C.c_int32), ("reeb_edges", C.c_int32),
                ("n_degenerate", C.c_int32), ("n_events", C.c_int32), ("steps", C.c_int64),
                ("active_vertex_updates", C.c_int64), ("active_degree_sum", C.c_int64),
                ("n_inside", C.c_int64), ("seed_vertex", C.c_int64), ("run_status", C.c_int32),
                ("grid", C.c_int32), ("block", C.c_int32), ("kernel_ms", C.c_double),
                ("total_ms", C.c_double), ("topo_ms", C.c_double), ("wait0_ms", C.c_double),
                ("field_ms", C.c_double), ("wait1_ms", C.c_double), ("event_steps", C.c_int64),
                ("topo_split_ms", C.c_double * 4), ("topo_event_ms", C.c_double),
                ("topo_rounds_ms", C.c_double), ("topo_round_steps", C.c_int32),
                ("topo_global_steps", C.c_int32), ("server_queue_ms", C.c_double),
                ("server_latency_ms", C.c_double), ("field_barrier_ms", C.c_double),
                ("event_split_ms", C.c_double * 4),
                ("n_tunnel_passes", C.c_int32), ("n_tunnel_loops", C.c_int32),
                ("n_refine_passes", C.c_int32), ("n_refined_loops", C.c_int32),
                ("pass_slots", C.c_int32), ("pass_pad", C.c_int32),
                ("tunnel_pass_ms", C.c_double), ("refine_pass_ms", C.c_double),
                ("pass_vertex_updates", C.c_int64), ("topo_global_split_ms", C.c_double * 4)]


class vls_reeb_node(C.Structure):
    _fields_ = [("type", C.c_int32), ("vertex", C.c_int32), ("in_deg", C.c_int32),
                ("out_deg", C.c_int32), ("extra_cycles", C.c_int32), ("pad", C.c_int32),
                ("step", C.c_int64), ("xyz", C.c_double * 3)]


class vls_reeb_edge(C.Structure):
    _fields_ = [("src", C.c_int32), ("dst", C.c_int32), ("front_id", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2105_13168_amd/build.py`")
# PyTorch ships its own HIP runtime under the same soname as the system one
# the library links against.  Loaded after PyTorch, the library binds to
# that runtime (one runtime per process: PyTorch's streams and memory are
# valid here); loaded first, it would pull in the system runtime and
# PyTorch's would then fail to find the device.  So PyTorch goes first.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)
_I64P = C.POINTER(C.c_int64)
_sig = {
    "vls_params_default": (None, [C.POINTER(vls_params)]),
    "vls_status_string": (C.c_char_p, [C.c_int32]),
    "vls_last_error": (C.c_char_p, [_P]),
    "vls_context_create": (C.c_int32, [C.c_int, _P, _PP]),
    "vls_context_destroy": (C.c_int32, [_P]),
    "vls_mesh_create": (C.c_int32, [_P, C.c_int64, _P, C.c_int64, _P, _PP]),
    "vls_mesh_info": (C.c_int32, [_P, _I64P, _I64P, _I64P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "vls_mesh_destroy": (C.c_int32, [_P]),
    "vls_mesh_prepare_fem": (C.c_int32, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vls_mesh_fem_coefficients": (C.c_int32, [_P, C.c_int64, _P, _I64P]),
    "vls_run": (C.c_int32, [_P, _P, C.POINTER(vls_params), _PP]),
    "vls_workspace_size": (C.c_int32, [_P, C.POINTER(vls_params), C.POINTER(C.c_size_t)]),
    "vls_run_async": (C.c_int32, [_P, _P, C.POINTER(vls_params), _P, C.c_size_t, _P, _PP]),
    "vls_result_wait": (C.c_int32, [_P]),
    "vls_run_async_noalloc": (C.c_int32, [_P, _P, C.POINTER(vls_params), _P, _PP]),
    "vls_batch_run": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "vls_result_summary": (C.c_int32, [_P, C.POINTER(vls_summary)]),
    "vls_result_events": (C.c_int32, [_P, C.c_int64, _P, _I64P]),
    "vls_result_event_fronts": (C.c_int32, [_P, C.c_int64, _P, _I64P]),
    "vls_result_loop": (C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int64, _P, _P,
                                    C.POINTER(C.c_double), _I64P]),
    "vls_result_loop_info": (C.c_int32, [_P, C.c_int32, C.c_int32, _I64P, _I64P, C.POINTER(C.c_int32)]),
    "vls_result_pass_info": (C.c_int32, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), _I64P,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]),
    "vls_result_reeb": (C.c_int32, [_P, C.c_int64, _P, C.c_int64, _P, _I64P, _I64P]),
    "vls_result_field": (C.c_int32, [_P, C.c_int64, _P]),
    "vls_result_vertices": (C.c_int32, [_P, _P, _P, _P]),
    "vls_result_fetch": (C.c_int32, [_P]),
    "vls_result_refined": (C.c_int32, [_P, C.POINTER(C.c_void_p)]),
    "vls_result_destroy": (C.c_int32, [_P]),
    "vls_server_create": (C.c_int32, [_P, C.c_size_t, C.c_int32, C.c_int64, C.c_uint32, _PP]),
    "vls_server_submit": (C.c_int32, [_P, _P, C.POINTER(vls_params), C.POINTER(C.c_uint64)]),
    "vls_server_poll": (C.c_int32, [_P, C.c_uint64, _PP]),
    "vls_server_stats": (C.c_int32, [_P, _I64P, _I64P, _I64P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "vls_server_timing": (C.c_int32, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vls_server_shutdown": (C.c_int32, [_P]),
    "vls_server_destroy": (C.c_int32, [_P]),
}
for _n, (_rt, _at) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _rt
    _f.argtypes = _at
    globals()[_n] = _f

EXPORTED = tuple(_sig)


class VLSError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = int(status)
        name = vls_status_string(status).decode()
        super().__init__(f"{name}: {detail}" if detail else name)


def default_params(**kw) -> vls_params:
    p = vls_params()
    vls_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "ckpt_steps":
            continue
        setattr(p, k, v)
    return p


class Context:
    """A device plus the stream all work is enqueued on (``stream`` is a
    hipStream_t as an int, e.g. ``torch.cuda.current_stream().cuda_stream``;
    None = a private stream)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        h = C.c_void_p()
        st = vls_context_create(device, C.c_void_p(stream) if stream else None, C.byref(h))
        if st != VLS_OK:
            raise VLSError(st, "context")
        self.h = h

    def last_error(self) -> str:
        return vls_last_error(self.h).decode()

    def close(self):
        if self.h:
            vls_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, xyz: np.ndarray, tri: np.ndarray):
        self.ctx = ctx
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = C.c_void_p()
        st = vls_mesh_create(ctx.h, self.xyz.shape[0], self.xyz.ctypes.data, self.tri.shape[0],
                             self.tri.ctypes.data, C.byref(h))
        if st != VLS_OK:
            raise VLSError(st, ctx.last_error())
        self.h = h
        nv, ne, nf = C.c_int64(), C.c_int64(), C.c_int64()
        dmax, eg = C.c_int32(), C.c_int32()
        vls_mesh_info(h, C.byref(nv), C.byref(ne), C.byref(nf), C.byref(dmax), C.byref(eg))
        self.nv, self.ne, self.nf, self.dmax, self.euler_genus = nv.value, ne.value, nf.value, dmax.value, eg.value

    def run(self, seed_vertex: int = 0, ckpt_steps=(), raise_on_error: bool = True, **kw) -> "Result":
        ck = np.ascontiguousarray(np.asarray(ckpt_steps, dtype=np.int64).reshape(-1))
        p = default_params(seed_vertex=seed_vertex, **kw)
        if ck.size:
            p.flags |= VLS_RECORD_FIELD
            p.n_ckpt = ck.size
            p.ckpt_steps = ck.ctypes.data_as(_I64P)
        h = C.c_void_p()
        st = vls_run(self.ctx.h, self.h, C.byref(p), C.byref(h))
        if not h:
            raise VLSError(st, self.ctx.last_error())
        r = Result(h, self, ck)
        r.status = int(st)
        r.error = self.ctx.last_error() if st != VLS_OK else ""
        if st != VLS_OK and raise_on_error and st != -7:
            raise VLSError(st, r.error)
        return r

    def prepare_fem(self):
        """The finite-element operator of the mesh (computed once on the
        device): returns (sigma, largest absolute row sum)."""
        sg, dm = C.c_double(), C.c_double()
        st = vls_mesh_prepare_fem(self.h, C.byref(sg), C.byref(dm))
        if st != VLS_OK:
            raise VLSError(st, self.ctx.last_error())
        return sg.value, dm.value

    def fem_coefficients(self) -> np.ndarray:
        """The operator's coefficient per half-edge, CSR order of ascending
        neighbours."""
        n = C.c_int64()
        st = vls_mesh_fem_coefficients(self.h, 0, None, C.byref(n))
        if st != VLS_OK:
            raise VLSError(st, self.ctx.last_error())
        g = np.empty(n.value, dtype=np.float64)
        st = vls_mesh_fem_coefficients(self.h, n.value, g.ctypes.data, C.byref(n))
        if st != VLS_OK:
            raise VLSError(st, self.ctx.last_error())
        return g

    def close(self):
        if getattr(self, "h", None):
            vls_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Result:
    """Host copies of a run's outputs as numpy arrays."""

    def __init__(self, h, mesh: Mesh, ckpt_steps, own: bool = True):
        self.h = h
        self.mesh = mesh
        s = vls_summary()
        vls_result_summary(h, C.byref(s))
        self.summary = {f: getattr(s, f) for f, _ in vls_summary._fields_}
        n = C.c_int64()
        vls_result_events(h, 0, None, C.byref(n))
        self.events = np.zeros((n.value, 16), dtype=np.int64)
        if n.value:
            vls_result_events(h, n.value, self.events.ctypes.data, C.byref(n))
        vls_result_event_fronts(h, 0, None, C.byref(n))
        ids = np.zeros(n.value, dtype=np.int64)
        if n.value:
            vls_result_event_fronts(h, n.value, ids.ctypes.data, C.byref(n))
        self.event_in, self.event_out = [], []
        for ev in self.events:
            o, s_, m_ = int(ev[11]), int(ev[4]), int(ev[5])
            self.event_in.append(ids[o:o + s_])
            self.event_out.append(ids[o + s_:o + s_ + m_])
        nv = mesh.nv
        self.step = np.zeros(nv, dtype=np.int32)
        self.round = np.zeros(nv, dtype=np.int32)
        self.parent = np.zeros(nv, dtype=np.int32)
        vls_result_vertices(h, self.step.ctypes.data, self.round.ctypes.data, self.parent.ctypes.data)
        self.rho = np.zeros(nv, dtype=np.float64)
        vls_result_field(h, -1, self.rho.ctypes.data)
        self.ckpt = {}
        for st in ckpt_steps.tolist():
            a = np.zeros(nv, dtype=np.float64)
            if vls_result_field(h, int(st), a.ctypes.data) == VLS_OK:
                self.ckpt[int(st)] = a
        # loops of merges (kind 2) and tunnels (kind 1)
        self.loops = []
        i = 0
        while True:
            ev, fid, kept = C.c_int64(), C.c_int64(), C.c_int32()
            if vls_result_loop_info(h, 2, i, C.byref(ev), C.byref(fid), C.byref(kept)) != VLS_OK:
                break
            cnt, L = C.c_int64(), C.c_double()
            vls_result_loop(h, 2, i, 0, None, None, C.byref(L), C.byref(cnt))
            he = np.zeros((cnt.value, 2), dtype=np.int32)
            pts = np.zeros((cnt.value, 3), dtype=np.float64)
            vls_result_loop(h, 2, i, cnt.value, he.ctypes.data, pts.ctypes.data, C.byref(L), C.byref(cnt))
            self.loops.append(dict(event=ev.value, front_id=fid.value, kept=bool(kept.value),
                                   he=he, pts=pts, length=L.value))
            i += 1
        self.tunnels = []
        for i in range(self.summary["n_tunnels"]):
            cnt, L = C.c_int64(), C.c_double()
            vls_result_loop(h, 1, i, 0, None, None, C.byref(L), C.byref(cnt))
            uv = np.zeros((cnt.value, 2), dtype=np.int32)
            vls_result_loop(h, 1, i, cnt.value, uv.ctypes.data, None, C.byref(L), C.byref(cnt))
            self.tunnels.append(uv[:, 0].copy())
        # tunnel-loop (kind 3) and handle-refinement (kind 4) passes
        self.passes = {3: [], 4: []}
        for kind, cnt in ((3, self.summary["n_tunnel_passes"]), (4, self.summary["n_refine_passes"])):
            for i in range(cnt):
                st, steps, reached, label = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32()
                L, L1 = C.c_double(), C.c_double()
                vls_result_pass_info(h, kind, i, C.byref(st), C.byref(steps), C.byref(reached), C.byref(label),
                                     C.byref(L), C.byref(L1))
                n = C.c_int64()
                vls_result_loop(h, kind, i, 0, None, None, None, C.byref(n))
                uv = np.zeros((n.value, 2), dtype=np.int32)
                if n.value:
                    vls_result_loop(h, kind, i, n.value, uv.ctypes.data, None, None, C.byref(n))
                self.passes[kind].append(dict(status=st.value, steps=steps.value, reached=reached.value,
                                              label=label.value, length=L.value, offset_length=L1.value,
                                              cycle=uv[:, 0].copy()))
        nn, ne = C.c_int64(), C.c_int64()
        vls_result_reeb(h, 0, None, 0, None, C.byref(nn), C.byref(ne))
        nodes = (vls_reeb_node * max(1, nn.value))()
        edges = (vls_reeb_edge * max(1, ne.value))()
        vls_result_reeb(h, nn.value, nodes, ne.value, edges, C.byref(nn), C.byref(ne))
        self.reeb_nodes = [(n.type, n.vertex, n.step, n.in_deg, n.out_deg, n.extra_cycles,
                            n.xyz[0], n.xyz[1], n.xyz[2]) for n in nodes[:nn.value]]
        self.reeb_edges = [(e.src, e.dst, e.front_id) for e in edges[:ne.value]]
        # the Reeb refinement's second pass (VLS_REEB_REFINE), owned by h
        h2 = C.c_void_p()
        self.refined = None
        if vls_result_refined(h, C.byref(h2)) == VLS_OK and h2.value:
            self.refined = Result(h2, mesh, np.zeros(0, dtype=np.int64), own=False)
        if own:
            vls_result_destroy(h)
        self.h = None

    def handle_loops(self):
        return [l for l in self.loops if l["kept"]]


def batch_run(ctx: Context, meshes, seeds, raise_on_error: bool = True, per_mesh=None, **kw):
    """Many meshes in one launch (one workgroup per mesh); returns one
    Result per mesh, in input order.  ``kw`` applies to every mesh,
    ``per_mesh`` (a list of dicts, ckpt_steps allowed) to one mesh each."""
    n = len(meshes)
    hm = (C.c_void_p * n)(*[m.h.value for m in meshes])
    ps = (vls_params * n)()
    cks = []
    for i in range(n):
        d = dict(kw)
        if per_mesh is not None:
            d.update(per_mesh[i])
        ck = np.ascontiguousarray(np.asarray(d.pop("ckpt_steps", ()), dtype=np.int64).reshape(-1))
        cks.append(ck)
        ps[i] = default_params(seed_vertex=int(seeds[i]), **d)
        if ck.size:
            ps[i].flags |= VLS_RECORD_FIELD
            ps[i].n_ckpt = ck.size
            ps[i].ckpt_steps = ck.ctypes.data_as(_I64P)
    outs = (C.c_void_p * n)()
    st = vls_batch_run(ctx.h, n, hm, ps, outs)
    if st != VLS_OK and (raise_on_error and st != -7 or not outs[0]):
        for i in range(n):
            if outs[i]:
                vls_result_destroy(C.c_void_p(outs[i]))
        raise VLSError(st, ctx.last_error())
    res = []
    for i in range(n):
        r = Result(C.c_void_p(outs[i]), meshes[i], cks[i])
        r.status = r.summary["run_status"]
        r.error = ""
        res.append(r)
    return res


class Server:
    """Request loop with continuous batching on one device: submit()
    returns a ticket, poll() returns None while the request runs and its
    Result once done.  A mesh must stay open until its requests are polled."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 1024, slice_us: int = 20000,
                 flags: int = 0):
        h = C.c_void_p()
        st = vls_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), int(slice_us), int(flags), C.byref(h))
        if st != VLS_OK:
            raise VLSError(st, ctx.last_error())
        self.h = h
        self.ctx = ctx
        self._meshes = {}
        self._ck = {}

    def submit(self, mesh: Mesh, seed_vertex: int = 0, ckpt_steps=(), **kw) -> int:
        ck = np.ascontiguousarray(np.asarray(ckpt_steps, dtype=np.int64).reshape(-1))
        p = default_params(seed_vertex=seed_vertex, **kw)
        if ck.size:
            p.flags |= VLS_RECORD_FIELD
            p.n_ckpt = ck.size
            p.ckpt_steps = ck.ctypes.data_as(_I64P)
        t = C.c_uint64()
        st = vls_server_submit(self.h, mesh.h, C.byref(p), C.byref(t))
        if st != VLS_OK:
            raise VLSError(st, "submit")
        self._meshes[t.value] = mesh
        self._ck[t.value] = ck
        return t.value

    def poll(self, ticket: int):
        h = C.c_void_p()
        st = vls_server_poll(self.h, C.c_uint64(ticket), C.byref(h))
        if st == VLS_E_PENDING:
            return None
        mesh = self._meshes.pop(ticket)
        ck = self._ck.pop(ticket)
        if not h:
            raise VLSError(st, "request failed")
        r = Result(h, mesh, ck)
        r.status = int(st)
        r.error = ""
        return r

    def shutdown(self):
        """Stops scheduling; unfinished requests then poll as cancelled."""
        st = vls_server_shutdown(self.h)
        if st != VLS_OK:
            raise VLSError(st, "shutdown")

    def stats(self) -> dict:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        q, r = C.c_int32(), C.c_int32()
        vls_server_stats(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(q), C.byref(r))
        x, y, z = C.c_double(), C.c_double(), C.c_double()
        vls_server_timing(self.h, C.byref(x), C.byref(y), C.byref(z))
        return {"launches": a.value, "completed": b.value, "admitted_bytes": c.value,
                "queued": q.value, "running": r.value, "admit_ms": x.value, "launch_ms": y.value,
                "complete_ms": z.value}

    def close(self):
        if getattr(self, "h", None):
            vls_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(xyz, tri, seed_vertex=0, device=0, stream=None, **kw) -> Result:
    """One-shot convenience: context, mesh, run."""
    ctx = Context(device, stream)
    m = Mesh(ctx, xyz, tri)
    try:
        return m.run(seed_vertex=seed_vertex, **kw)
    finally:
        m.close()
        ctx.close()
