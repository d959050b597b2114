"""CPU oracle of the initial pass (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links,
loads or calls it, and it shares no code with the GPU path: the C oracle in
``vls_oracle.c`` is compiled with gcc on its own, and ``field_step_numpy``
below is an independent vectorised restatement of the field update used to
pin the C field step.

``run(mesh, ...)`` returns a plain dict of numpy arrays with the oracle's
results (see ``OracleResult`` field names).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vls_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "vls_passes.c")]
_LIB = os.path.join(_HERE, "_vls_oracle.so")

# node types (Reeb graph)
NODE_SEED, NODE_SPLIT, NODE_MERGE, NODE_VANISH, NODE_DEGENERATE = range(5)

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "MESH_NOT_MANIFOLD", -3: "MESH_HAS_BOUNDARY",
          -4: "MESH_NOT_CONNECTED", -5: "MESH_NOT_ORIENTABLE", -6: "SEED_INVALID",
          -7: "STALLED", -8: "OUT_OF_MEMORY", -13: "INVARIANT"}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c99", "-shared", "-fPIC", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("mu", C.c_double), ("a", C.c_double),
                ("w", C.c_double), ("e", C.c_double), ("dt_mode", C.c_int32),
                ("seed_radius", C.c_int32), ("seed_vertex", C.c_int64),
                ("max_steps", C.c_int64), ("stall_steps", C.c_int64),
                ("dense", C.c_int32), ("n_ckpt", C.c_int32),
                ("ckpt_steps", C.POINTER(C.c_int64)), ("fem", C.c_int32),
                ("n_seed_set", C.c_int64), ("seed_set", C.POINTER(C.c_int32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_run.restype = P
        lib.orc_run.argtypes = [C.c_int64, P, C.c_int64, P, C.POINTER(_Params)]
        lib.orc_status.restype = C.c_int32
        lib.orc_status.argtypes = [P]
        lib.orc_summary.argtypes = [P, P]
        lib.orc_free.argtypes = [P]
        for name, rt in [("orc_T", C.POINTER(C.c_int64)), ("orc_rnd", C.POINTER(C.c_int32)),
                         ("orc_parent", C.POINTER(C.c_int32)), ("orc_rho", C.POINTER(C.c_double)),
                         ("orc_cyc", C.POINTER(C.c_int32)), ("orc_rp", C.POINTER(C.c_int64)),
                         ("orc_event_pos", C.POINTER(C.c_double)),
                         ("orc_front_death", C.POINTER(C.c_int64)),
                         ("orc_loop_len", C.POINTER(C.c_double)),
                         ("orc_loop_pts", C.POINTER(C.c_double))]:
            f = getattr(lib, name)
            f.restype = rt
            f.argtypes = [P]
        lib.orc_fem_operator.restype = C.c_int32
        lib.orc_fem_operator.argtypes = [C.c_int64, P, C.c_int64, P, P, P, P, P, P]
        lib.orc_ckpt.restype = C.POINTER(C.c_double)
        lib.orc_ckpt.argtypes = [P, C.c_int32]
        for name in ["orc_steplog", "orc_events", "orc_event_ids", "orc_front_birth",
                     "orc_loops", "orc_loop_he", "orc_tunnels", "orc_tunnel_v"]:
            f = getattr(lib, name)
            f.restype = C.POINTER(C.c_int64)
            f.argtypes = [P, C.POINTER(C.c_int64)]
        _lib = lib
    return _lib


def _arr(ptr, n, dtype, shape=None):
    if n == 0 or not ptr:
        return np.zeros(shape if shape is not None else (0,), dtype=dtype)
    a = np.ctypeslib.as_array(ptr, shape=(int(n),)).copy().astype(dtype, copy=False)
    return a.reshape(shape) if shape is not None else a


@dataclass
class OracleResult:
    status: int
    steps: int = 0
    n_events: int = 0
    n_handles: int = 0
    chi_mesh: int = 0
    chi_final: int = 0
    b_final: int = 0
    n_inside: int = 0
    dmax: int = 0
    n_fronts: int = 0
    active_updates: int = 0
    T: np.ndarray = None
    rnd: np.ndarray = None
    parent: np.ndarray = None
    rho: np.ndarray = None
    ckpt: dict = field(default_factory=dict)
    steplog: np.ndarray = None        # [steps,3]: chi_t, b_t, |N_t|
    events: np.ndarray = None         # [n,14]
    event_in: list = None             # per event: in front ids
    event_out: list = None            # per event: out front ids
    event_pos: np.ndarray = None      # [n,3]
    front_birth: np.ndarray = None
    front_death: np.ndarray = None
    loops: np.ndarray = None          # [nl,6]: event, front id, kept, off, count, a-vertex
    loop_len: np.ndarray = None
    loop_he: np.ndarray = None        # [*,2]
    loop_pts: np.ndarray = None       # [*,3]
    tunnels: np.ndarray = None        # [nt,3]: loop index, off, count
    tunnel_v: np.ndarray = None

    @property
    def status_name(self):
        return STATUS.get(self.status, str(self.status))

    @property
    def genus(self):
        return (2 - self.chi_mesh) // 2

    def handle_loops(self):
        """[(event, front id, he[n,2], pts[n,3], length)] of emitted handle loops."""
        out = []
        for i, (ev, fid, kept, off, cnt, av) in enumerate(self.loops):
            if kept:
                out.append((int(ev), int(fid), self.loop_he[off:off + cnt],
                            self.loop_pts[off:off + cnt], float(self.loop_len[i])))
        return out

    def tunnel_loops(self):
        return [self.tunnel_v[off:off + cnt] for (_, off, cnt) in self.tunnels]

    def reeb(self):
        """Nodes [(type, vertex, step, in, out, extra, x, y, z)] and edges
        [(src, dst, front id)]."""
        ev = self.events
        nodes = []
        # seed node
        nodes.append(None)
        for i in range(ev.shape[0]):
            nodes.append((int(ev[i, 2]), int(ev[i, 1]), int(ev[i, 0]), int(ev[i, 4]),
                          int(ev[i, 5]), int(ev[i, 7]), *map(float, self.event_pos[i])))
        edges = [(int(self.front_birth[f]), int(self.front_death[f]), f)
                 for f in range(self.front_birth.size)]
        return nodes, edges


def default_params(**kw):
    p = dict(tau=0.5, mu=0.25, a=1.0 / 25.0, w=(1.0 / 25.0) / 5.0, e=1.0 / 30.0,
             dt_mode=0, seed_radius=2, seed_vertex=0, max_steps=10_000_000,
             stall_steps=200_000, dense=0, ckpt_steps=(), fem=0, seed_set=())
    p.update(kw)
    return p


def run(xyz, tri, **kw) -> OracleResult:
    lib = _load()
    p = default_params(**kw)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    ck = np.ascontiguousarray(np.asarray(p["ckpt_steps"], dtype=np.int64).reshape(-1))
    ss = np.ascontiguousarray(np.asarray(p["seed_set"], dtype=np.int32).reshape(-1))
    cp = _Params(p["tau"], p["mu"], p["a"], p["w"], p["e"], int(p["dt_mode"]),
                 int(p["seed_radius"]), int(p["seed_vertex"]), int(p["max_steps"]),
                 int(p["stall_steps"]), int(p["dense"]), int(ck.size),
                 ck.ctypes.data_as(C.POINTER(C.c_int64)) if ck.size else None, int(p["fem"]),
                 int(ss.size), ss.ctypes.data_as(C.POINTER(C.c_int32)) if ss.size else None)
    h = lib.orc_run(xyz.shape[0], xyz.ctypes.data, tri.shape[0], tri.ctypes.data, C.byref(cp))
    if not h:
        raise MemoryError("oracle allocation failed")
    try:
        s = np.zeros(16, dtype=np.int64)
        lib.orc_summary(h, s.ctypes.data)
        r = OracleResult(status=int(s[0]), steps=int(s[1]), n_events=int(s[2]),
                         n_handles=int(s[3]), chi_mesh=int(s[4]), chi_final=int(s[5]),
                         b_final=int(s[6]), n_inside=int(s[7]), dmax=int(s[8]),
                         n_fronts=int(s[9]), active_updates=int(s[10]))
        if r.status in (-1, -2, -3, -4, -5, -8):
            return r
        nv = xyz.shape[0]
        nnz = int(s[11])
        r.T = _arr(lib.orc_T(h), nv, np.int64)
        r.rnd = _arr(lib.orc_rnd(h), nv, np.int32)
        r.parent = _arr(lib.orc_parent(h), nv, np.int32)
        r.rho = _arr(lib.orc_rho(h), nv, np.float64)
        for i, st in enumerate(ck.tolist()):
            ptr = lib.orc_ckpt(h, i)
            if ptr:
                r.ckpt[int(st)] = _arr(ptr, nv, np.float64)
        n = C.c_int64()
        ptr = lib.orc_steplog(h, C.byref(n))
        r.steplog = _arr(ptr, 3 * n.value, np.int64, (n.value, 3))
        ptr = lib.orc_events(h, C.byref(n))
        ne = n.value
        r.events = _arr(ptr, 14 * ne, np.int64, (ne, 14))
        ptr = lib.orc_event_ids(h, C.byref(n))
        ids = _arr(ptr, n.value, np.int64)
        r.event_in, r.event_out = [], []
        o = 0
        for i in range(ne):
            sN, mN = int(r.events[i, 4]), int(r.events[i, 5])
            r.event_in.append(ids[o:o + sN]); o += sN
            r.event_out.append(ids[o:o + mN]); o += mN
        r.event_pos = _arr(lib.orc_event_pos(h), 3 * ne, np.float64, (ne, 3))
        ptr = lib.orc_front_birth(h, C.byref(n))
        r.front_birth = _arr(ptr, n.value, np.int64)
        r.front_death = _arr(lib.orc_front_death(h), n.value, np.int64)
        ptr = lib.orc_loops(h, C.byref(n))
        nl = n.value
        r.loops = _arr(ptr, 6 * nl, np.int64, (nl, 6))
        r.loop_len = _arr(lib.orc_loop_len(h), nl, np.float64)
        ptr = lib.orc_loop_he(h, C.byref(n))
        r.loop_he = _arr(ptr, 2 * n.value, np.int64, (n.value, 2))
        r.loop_pts = _arr(lib.orc_loop_pts(h), 3 * n.value, np.float64, (n.value, 3))
        ptr = lib.orc_tunnels(h, C.byref(n))
        r.tunnels = _arr(ptr, 3 * n.value, np.int64, (n.value, 3))
        ptr = lib.orc_tunnel_v(h, C.byref(n))
        r.tunnel_v = _arr(ptr, n.value, np.int64)
        r._nnz = nnz
        return r
    finally:
        lib.orc_free(h)


def fem_operator(xyz, tri):
    """The oracle's finite-element operator of a closed mesh: (rp, adj, g,
    mass, sigma, dmax) with g[i] the coefficient of half-edge v -> adj[i]
    (sigma * cot weight / lumped mass) for i in rp[v]:rp[v+1]."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nv, nf = xyz.shape[0], tri.shape[0]
    rp = np.zeros(nv + 1, dtype=np.int64)
    adj = np.zeros(3 * nf, dtype=np.int32)
    g = np.zeros(3 * nf, dtype=np.float64)
    mass = np.zeros(nv, dtype=np.float64)
    scal = np.zeros(2, dtype=np.float64)
    rc = lib.orc_fem_operator(nv, xyz.ctypes.data, nf, tri.ctypes.data, rp.ctypes.data, adj.ctypes.data,
                              g.ctypes.data, mass.ctypes.data, scal.ctypes.data)
    if rc:
        raise ValueError(f"oracle mesh check failed: {STATUS.get(rc, rc)}")
    return rp, adj, g, mass, float(scal[0]), float(scal[1])


# ---------------------------------------------------------------------------
# independent numpy restatement of the field step (pins the C field step)
# ---------------------------------------------------------------------------
def ascending_ell(tri: np.ndarray, nv: int):
    """Neighbour table padded with -1: row v lists N(v) ascending by id."""
    t = np.asarray(tri, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    key = np.unique(e[:, 0] * nv + e[:, 1])
    u, x = np.divmod(key, nv)
    deg = np.bincount(u, minlength=nv)
    dmax = int(deg.max())
    start = np.concatenate([[0], np.cumsum(deg)[:-1]])
    pos = np.arange(u.size) - start[u]
    ell = np.full((nv, dmax), -1, dtype=np.int64)
    ell[u, pos] = x
    return ell, deg


def field_step_numpy(rho, ell, deg, dmax_mesh, dt_mode=0, a=1.0 / 25.0,
                     w=(1.0 / 25.0) / 5.0, e=1.0 / 30.0, mu=0.25):
    """One explicit Euler step of the two-phase field with the clip, summing
    each row's neighbours in ascending id order (vectorised over rows)."""
    dt = 0.25 / float(dmax_mesh) if dt_mode == 1 else 50.0 / float(dmax_mesh)
    c = dt * (mu / 2.0)
    s = rho[ell[:, 0]].copy()
    for k in range(1, ell.shape[1]):
        col = ell[:, k]
        has = col >= 0
        s[has] = s[has] + rho[col[has]]
    r = rho
    lap = s - deg.astype(np.float64) * r
    d = (a * lap + w * (2.0 * r - 1.0)) + e * np.sqrt(r * (1.0 - r))
    x = r + c * d
    return np.minimum(np.maximum(x, 0.0), 1.0)


def refinement_seed_set(result) -> np.ndarray:
    """The seed set of the Reeb refinement pass: the inside endpoints of the
    first kept handle loop's crossed edges, ascending (empty without one)."""
    loops = result.handle_loops()
    if not loops:
        return np.zeros(0, dtype=np.int32)
    return np.unique(np.asarray(loops[0][2])[:, 0]).astype(np.int32)


def reeb_refined(xyz, tri, **kw):
    """Reeb junction refinement (Section "Reeb Graph Extraction": the second
    pass relocates the junctions).  Reading: the initial pass is run again
    from the first kept handle loop instead of a random point (the diffusion
    initiated at a detected handle loop, Section "Introduction"): its
    initial region is every vertex within seed_radius hops of the loop's
    inside vertices, ranked by hop distance inside that region from its
    smallest vertex.  The refined Reeb graph is that pass's graph, junctions
    at its band means.  Returns (first pass, second pass or None)."""
    first = run(xyz, tri, **kw)
    ss = refinement_seed_set(first) if first.status == 0 else np.zeros(0, dtype=np.int32)
    if ss.size == 0:
        return first, None
    kw2 = dict(kw)
    kw2["seed_set"] = ss
    kw2["seed_vertex"] = int(ss[0])
    return first, run(xyz, tri, **kw2)

