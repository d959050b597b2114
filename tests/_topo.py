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
