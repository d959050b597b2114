"""Oracle of the tunnel-loop pass, the handle-refinement pass and the
handle/tunnel distinction (Section "Tunnel loop pass", Section "Handle
refinement pass", Section "Distinguishing handle and tunnel loops").

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline of bench.py; shares no code with the GPU library.  The diffusion of
each pass runs in plain C (orc_pass_run in vls_passes.c); this module builds
each pass's inputs from the loop it starts from and turns the traced
streamline into a closed loop.

Tunnel-loop pass of handle loop h (a loop of crossed edges (u, x), u inside,
found when the fronts merged at vertex v):
  * domain: the area covered when h was detected, the vertices of rank at
    most rank(v) (the inside set once v has joined);
  * cut: the edges h crosses; start: h's inside vertices (one side);
  * target: h's outside vertices in the domain (the other side), which is v.
Handle-refinement pass of a tunnel loop W (a closed vertex path):
  * domain: every vertex (restricted by the tunnel loop only);
  * cut: the edges from W to the vertices on its left (the link of w_k
    counter-clockwise from w_{k+1} to w_{k-1}, seen from outside);
  * start: W itself; target: the vertices on W's left that are not also on
    its right.
The loop is closed from the streamline x*, parent(x*), ..., s* (s* on the
start side): along the start side from s* to the start vertex q that shares
a cut edge with x*, the shorter way round (ties: forward, then the smaller
position), then back to x* over that cut edge; a vertex visited twice cuts
out the part between its visits.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _load

PASS_STALLED = -7


class _PassParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("mu", C.c_double), ("a", C.c_double),
                ("w", C.c_double), ("e", C.c_double), ("dt_mode", C.c_int32),
                ("n_ckpt", C.c_int32), ("max_steps", C.c_int64), ("stall_steps", C.c_int64),
                ("ckpt_steps", C.POINTER(C.c_int64))]


def _lib():
    lib = _load()
    if not getattr(lib, "_pass_sig", False):
        P = C.c_void_p
        lib.orc_pass_run.restype = C.c_int
        lib.orc_pass_run.argtypes = [C.c_int64, C.c_int32, P, P, P, P, P, C.c_int64, P, C.c_int64, P,
                                     C.POINTER(_PassParams), P, P, P, P, P, P, P]
        lib._pass_sig = True
    return lib


class MeshGraph:
    """Ascending adjacency and counter-clockwise links of a closed oriented
    triangle mesh (ccw seen from outside)."""

    def __init__(self, xyz, tri):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int64)
        nv = self.xyz.shape[0]
        self.nv = nv
        t = self.tri
        e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
        e = np.concatenate([e, e[:, ::-1]])
        key = np.unique(e[:, 0] * nv + e[:, 1])
        src, dst = key // nv, key % nv
        self.rp = np.zeros(nv + 1, dtype=np.int64)
        np.add.at(self.rp, src + 1, 1)
        self.rp = np.cumsum(self.rp)
        self.adj = np.ascontiguousarray(dst.astype(np.int32))
        self.dmax = int(np.max(np.diff(self.rp)))
        # link successor: triangle (a, b, c) gives b -> c around a
        self._succ = {}
        for a, b, c in t.tolist():
            self._succ.setdefault(a, {})[b] = c
            self._succ.setdefault(b, {})[c] = a
            self._succ.setdefault(c, {})[a] = b

    def neighbours(self, v):
        return self.adj[self.rp[v]:self.rp[v + 1]]

    def ccw_after(self, w, start, stop):
        """Link vertices of w strictly after `start` and before `stop`,
        counter-clockwise."""
        out = []
        s = self._succ[w]
        x = s[start]
        n = 0
        while x != stop:
            out.append(x)
            x = s[x]
            n += 1
            if n > len(s):
                raise ValueError("not a link cycle")
        return out


def _run_pass(g: MeshGraph, dom, cut_pairs, start, target, ckpt_steps=(), max_steps=10_000_000,
              stall_steps=200_000, tau=0.5, mu=0.25, a=1.0 / 25.0, w=(1.0 / 25.0) / 5.0, e=1.0 / 30.0, dt_mode=0):
    lib = _lib()
    nv = g.nv
    dom = np.ascontiguousarray(dom, dtype=np.uint8)
    target = np.ascontiguousarray(target, dtype=np.uint8)
    if len(cut_pairs):
        cp = np.asarray(cut_pairs, dtype=np.int64).reshape(-1, 2)
        cut = np.unique(np.minimum(cp[:, 0], cp[:, 1]) * nv + np.maximum(cp[:, 0], cp[:, 1]))
    else:
        cut = np.zeros(0, dtype=np.int64)
    cut = np.ascontiguousarray(cut, dtype=np.int64)
    start = np.ascontiguousarray(np.unique(np.asarray(start, dtype=np.int64)).astype(np.int32))
    ck = np.ascontiguousarray(np.asarray(ckpt_steps, dtype=np.int64).reshape(-1))
    p = _PassParams(tau, mu, a, w, e, dt_mode, int(ck.size), int(max_steps), int(stall_steps),
                    ck.ctypes.data_as(C.POINTER(C.c_int64)) if ck.size else None)
    T = np.zeros(nv, dtype=np.int64)
    rnd = np.zeros(nv, dtype=np.int32)
    parent = np.zeros(nv, dtype=np.int32)
    rho = np.zeros(nv, dtype=np.float64)
    ta = np.zeros(nv, dtype=np.float64)
    ckpt = np.zeros((max(1, ck.size), nv), dtype=np.float64)
    res = np.zeros(4, dtype=np.int64)
    lib.orc_pass_run(nv, g.dmax, g.rp.ctypes.data, g.adj.ctypes.data, g.xyz.ctypes.data, dom.ctypes.data, cut.ctypes.data,
                     cut.size, start.ctypes.data, start.size, target.ctypes.data, C.byref(p), T.ctypes.data,
                     rnd.ctypes.data, parent.ctypes.data, rho.ctypes.data, ta.ctypes.data, ckpt.ctypes.data,
                     res.ctypes.data)
    out = dict(status=int(res[0]), steps=int(res[1]), reached=int(res[2]), updates=int(res[3]),
               T=T, rnd=rnd, parent=parent, rho=rho, arrival=ta, cut=cut, start=start,
               ckpt={int(s): ckpt[i].copy() for i, s in enumerate(ck.tolist())})
    return out


def _dedup_cyclic(seq):
    out = []
    for x in seq:
        if not out or out[-1] != x:
            out.append(x)
    while len(out) > 1 and out[0] == out[-1]:
        out.pop()
    return out


def _close(side, path, partners):
    """Closed loop from the streamline `path` (x* ... s*) along the cyclic
    start-side sequence `side` to a partner of x*."""
    n = len(side)
    s_star = path[-1]
    best = None
    pos_s = [i for i, q in enumerate(side) if q == s_star]
    pos_q = [j for j, q in enumerate(side) if q in partners]
    for i in pos_s:
        for j in pos_q:
            f, b = (j - i) % n, (i - j) % n
            cand = (f, 0, j, i) if f <= b else (b, 1, j, i)
            if best is None or cand < best:
                best = cand
    if best is None:
        return None
    dist, back, j, i = best
    step = -1 if back else 1
    walk = [side[(i + step * k) % n] for k in range(dist + 1)]
    cyc = list(path) + walk[1:]
    # loop erasure: a vertex visited twice cuts out what lies between
    out, where = [], {}
    for x in cyc:
        if x in where:
            k = where[x]
            for y in out[k + 1:]:
                del where[y]
            out = out[:k + 1]
        else:
            where[x] = len(out)
            out.append(x)
    return out


def _trace(parent, T, reached):
    path = [reached]
    while T[path[-1]] != 0:
        path.append(int(parent[path[-1]]))
    return path


def loop_length(xyz, cyc):
    L = 0.0
    n = len(cyc)
    for k in range(n):
        pa, pb = xyz[cyc[k]], xyz[cyc[(k + 1) % n]]
        dx, dy, dz = pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]
        L = L + math.sqrt((dx * dx + dy * dy) + dz * dz)
    return L


def _finish(g, r, side, cut_set, **_):
    if r["status"] != 0:
        return dict(r, cycle=None, length=None)
    x = r["reached"]
    path = _trace(r["parent"], r["T"], x)
    nv = g.nv
    partners = {q for q in side if (min(q, x) * nv + max(q, x)) in cut_set}
    cyc = _close(side, path, partners)
    return dict(r, path=path, cycle=cyc, length=loop_length(g.xyz, cyc) if cyc else None)


def tunnel_pass(g: MeshGraph, init, li: int, **kw):
    """Tunnel-loop pass of loop li (kind 2 numbering: every involved loop of
    every merge) of the initial pass's oracle result `init`."""
    ev, fid, kept, off, cnt, _av = (int(q) for q in init.loops[li])
    he = init.loop_he[off:off + cnt]
    v = int(init.events[ev, 1])
    nv = g.nv
    Tv, Rv = int(init.T[v]), int(init.rnd[v])
    T, R = init.T, init.rnd.astype(np.int64)
    dom = (T < Tv) | ((T == Tv) & ((R < Rv) | ((R == Rv) & (np.arange(nv) <= v))))
    u, x = he[:, 0].astype(np.int64), he[:, 1].astype(np.int64)
    target = np.zeros(nv, dtype=np.uint8)
    target[x[dom[x]]] = 1
    target[u] = 0
    side = _dedup_cyclic(u.tolist())
    r = _run_pass(g, dom, np.stack([u, x], 1), u, target, **kw)
    cut_set = set(r["cut"].tolist())
    return _finish(g, r, side, cut_set)


def refine_pass(g: MeshGraph, cycle, **kw):
    """Handle-refinement pass of a closed vertex path `cycle` (a tunnel)."""
    W = list(cycle)
    n = len(W)
    inW = set(W)
    left, right, cut = set(), set(), []
    for k in range(n):
        w, nxt, prv = W[k], W[(k + 1) % n], W[(k - 1) % n]
        la = g.ccw_after(w, nxt, prv)
        ra = g.ccw_after(w, prv, nxt)
        for y in la:
            if y not in inW:
                left.add(y)
                cut.append((w, y))
        for y in ra:
            if y not in inW:
                right.add(y)
    nv = g.nv
    dom = np.ones(nv, dtype=np.uint8)
    target = np.zeros(nv, dtype=np.uint8)
    for y in left - right:
        target[y] = 1
    r = _run_pass(g, dom, np.array(cut, dtype=np.int64).reshape(-1, 2), W, target, **kw)
    cut_set = set(r["cut"].tolist())
    return _finish(g, r, W, cut_set)


def vertex_normals(g: MeshGraph):
    """Area-weighted vertex normals: the cross products of a vertex's
    triangles (w, c_j, c_j+1) over its counter-clockwise link from its
    smallest neighbour id, summed in that order, normalised."""
    p = g.xyz
    n = np.zeros_like(p)
    for w in range(g.nv):
        s = g._succ[w]
        c0 = min(s)
        link = [c0]
        while len(link) < len(s):
            link.append(s[link[-1]])
        sx = sy = sz = 0.0
        for j in range(len(link)):
            a = p[link[j]] - p[w]
            b = p[link[(j + 1) % len(link)]] - p[w]
            sx = sx + (a[1] * b[2] - a[2] * b[1])
            sy = sy + (a[2] * b[0] - a[0] * b[2])
            sz = sz + (a[0] * b[1] - a[1] * b[0])
        ln = math.sqrt((sx * sx + sy * sy) + sz * sz)
        n[w] = (sx / ln, sy / ln, sz / ln)
    return n


def offset_label(g: MeshGraph, cycle, normals, rel_eps=0.1):
    """Section "Distinguishing handle and tunnel loops": offset the loop
    along the surface normals by rel_eps times its mean edge length and
    compare lengths: a handle loop grows, a tunnel loop shrinks.  Returns
    ("handle" | "tunnel", length, offset length)."""
    L0 = loop_length(g.xyz, cycle)
    eps = rel_eps * L0 / len(cycle)
    q = g.xyz.copy()
    idx = np.asarray(cycle)
    q[idx] = g.xyz[idx] + eps * normals[idx]
    L1 = loop_length(q, cycle)
    return ("handle" if L1 > L0 else "tunnel"), L0, L1
