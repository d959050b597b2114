"""Brute-force topology of an inside set on a closed triangle mesh.

Independent of both the oracle and the GPU library: everything here is
recomputed from scratch from the triangle list and an inside mask with
numpy/scipy, so it can check the incremental bookkeeping of either.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


class MeshTopo:
    def __init__(self, tri, nv):
        self.tri = np.asarray(tri, dtype=np.int64)
        self.nv = int(nv)
        t = self.tri
        e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
        e.sort(axis=1)
        key = e[:, 0] * nv + e[:, 1]
        self.ekey, inv = np.unique(key, return_inverse=True)
        self.eu, self.ex = np.divmod(self.ekey, nv)
        # triangle -> its three edge ids
        self.tedge = inv.reshape(3, -1).T
        # edge -> its two triangles
        order = np.argsort(inv, kind="stable")
        tri_of = (order % t.shape[0])
        self.etri = tri_of.reshape(-1, 2)

    def euler_char(self, inside):
        inside = np.asarray(inside, dtype=bool)
        V = int(inside.sum())
        E = int((inside[self.eu] & inside[self.ex]).sum())
        F = int(inside[self.tri].all(axis=1).sum())
        return V - E + F

    def crossed_mask(self, inside):
        return inside[self.eu] != inside[self.ex]

    def loops(self, inside):
        """Connected components of front triangles (1 or 2 inside vertices)
        joined through shared crossed edges.  Returns (n_loops, label per
        crossed edge id, crossed edge ids)."""
        inside = np.asarray(inside, dtype=bool)
        cm = self.crossed_mask(inside)
        ce = np.flatnonzero(cm)
        if ce.size == 0:
            return 0, np.zeros(0, dtype=np.int64), ce
        t0 = self.etri[ce, 0]
        t1 = self.etri[ce, 1]
        ntri = self.tri.shape[0]
        g = coo_matrix((np.ones(ce.size), (t0, t1)), shape=(ntri, ntri))
        n, lab = connected_components(g, directed=False)
        ft = np.zeros(ntri, dtype=bool)
        ft[t0] = True
        ft[t1] = True
        # components restricted to front triangles
        labs = np.unique(lab[ft])
        remap = -np.ones(n, dtype=np.int64)
        remap[labs] = np.arange(labs.size)
        return int(labs.size), remap[lab[t0]], ce

    def edge_id(self, u, x):
        a, b = (u, x) if u < x else (x, u)
        k = a * self.nv + b
        i = np.searchsorted(self.ekey, k)
        assert self.ekey[i] == k
        return int(i)

    def graph_connected_without(self, removed_edge_ids):
        keep = np.ones(self.ekey.size, dtype=bool)
        keep[np.asarray(removed_edge_ids, dtype=np.int64)] = False
        g = coo_matrix((np.ones(int(keep.sum())), (self.eu[keep], self.ex[keep])),
                       shape=(self.nv, self.nv))
        n, _ = connected_components(g, directed=False)
        return n == 1


def rank_key(T, rnd):
    """Total order of insertion: (step, round, id)."""
    T = np.asarray(T, dtype=np.int64)
    rnd = np.asarray(rnd, dtype=np.int64)
    return np.lexsort((np.arange(T.size), rnd, T))


def hop_ball(tri, nv, s, r0):
    t = np.asarray(tri, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    g = coo_matrix((np.ones(e.shape[0]), (e[:, 0], e[:, 1])), shape=(nv, nv)).tocsr()
    hop = -np.ones(nv, dtype=np.int64)
    hop[s] = 0
    frontier = np.array([s])
    for h in range(1, r0 + 1):
        nb = np.unique(g[frontier].indices)
        nb = nb[hop[nb] < 0]
        hop[nb] = h
        frontier = nb
    return hop


def events_bruteforce(m, r):
    """Every event's s (fronts on the lower link), m (loops through the new
    crossed edges) and h (from the Euler characteristic and loop count
    before and after the insertion) recomputed from the insertion order."""
    topo = MeshTopo(m.tri, m.nv)
    order = rank_key(r.T, r.rnd)
    pos = np.empty(m.nv, dtype=np.int64)
    pos[order] = np.arange(m.nv)
    # neighbours
    t = m.tri.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    nbr = [[] for _ in range(m.nv)]
    for u, x in e:
        nbr[u].append(x)
    # counter-clockwise link edges a -> b of each vertex (triangle (v, a, b))
    link = [[] for _ in range(m.nv)]
    for a_, b_, c_ in t:
        link[a_].append((b_, c_))
        link[b_].append((c_, a_))
        link[c_].append((a_, b_))
    for ev in r.events:
        step, v, typ, k, s, mm, h, x = (int(q) for q in ev[:8])
        pre = pos < pos[v]
        post = pre.copy()
        post[v] = True
        # lower arcs of v's link: a link edge leaving the upper part into the
        # lower part starts one; a full lower link is recorded as k = 0
        full = all(pre[a_] for a_, _ in link[v])
        k_bf = 0 if full else sum(1 for a_, b_ in link[v] if not pre[a_] and pre[b_])
        assert k_bf == k, (ev, k_bf)
        nb, lab, ce = topo.loops(pre)
        na, laba, cea = topo.loops(post)
        # loops through v's star before: labels of crossed edges (u, v)
        lab_of = dict(zip(ce.tolist(), lab.tolist()))
        s_bf = len({lab_of[topo.edge_id(u, v)] for u in nbr[v] if pre[u]})
        laba_of = dict(zip(cea.tolist(), laba.tolist()))
        m_bf = len({laba_of[topo.edge_id(u, v)] for u in nbr[v] if not post[u]})
        assert s_bf == s, (ev, s_bf)
        assert m_bf == mm, (ev, m_bf)
        dchi = topo.euler_char(post) - topo.euler_char(pre)
        db = na - nb
        assert dchi + db == -2 * h
        # node type and extra cycles from (full link, s, h)
        x_bf = 0 if full else h - (s - 1)
        assert x_bf == x, (ev, x_bf)
        typ_bf = 3 if full else (4 if x_bf > 0 else (2 if s >= 2 else 1))
        assert typ_bf == typ, (ev, typ_bf)
