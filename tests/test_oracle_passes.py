"""Pins of the oracle's tunnel-loop and handle-refinement passes and of the
handle/tunnel distinction (Section "Tunnel loop pass", Section "Handle
refinement pass", Section "Distinguishing handle and tunnel loops"), from
facts outside the pass oracle:

* with every vertex in the domain, no cut and the seed hop ball as its start
  side, a pass grows exactly as the initial pass does (same field, same
  insertion steps and rounds): the pass's field step and growth reduce to
  the initial pass's, which its own pins fix;
* the insertion step, round and arrival time of every vertex, recomputed by
  brute force from the pass's per-step field snapshots over the restricted
  operator (domain and cut), and parents recomputed as the steepest descent
  of the arrival time; no parent edge is a cut edge;
* the torus: the tunnel loop winds once around the axis and not around the
  tube (a longitude), the refined handle loop once around the tube and not
  around the axis (a meridian), both close to the shortest such curves
  (2 pi (R - r) and 2 pi r), the tunnel shorter than the initial pass's
  streamline candidate; each crosses the loop it came from exactly once;
  offsetting along the normals shrinks the tunnel and grows the handle;
* genus-g surfaces: every handle loop gets a tunnel that crosses it once and
  a refined handle that crosses that tunnel once; the loops are simple
  closed vertex paths whose consecutive vertices are mesh neighbours.
"""
import math

import numpy as np
import pytest

import meshgen as mg

from _topo import hop_ball

R_TORUS, r_TORUS = 1.0, 0.35


def _torus48():
    return mg.sdf_surface(mg.sdf_torus(R=R_TORUS, r=r_TORUS), (-1.4, -1.4, -0.4), (1.4, 1.4, 0.4), 48, 1e-4, 0)


def _winding(xyz, cyc, R):
    c = list(cyc) + [cyc[0]]
    th = np.arctan2(xyz[c, 1], xyz[c, 0])
    ph = np.arctan2(xyz[c, 2], np.hypot(xyz[c, 0], xyz[c, 1]) - R)
    d1 = (np.diff(th) + np.pi) % (2 * np.pi) - np.pi
    d2 = (np.diff(ph) + np.pi) % (2 * np.pi) - np.pi
    return int(round(d1.sum() / (2 * np.pi))), int(round(d2.sum() / (2 * np.pi)))


def _is_simple_cycle(g, cyc):
    if len(set(cyc)) != len(cyc) or len(cyc) < 3:
        return False
    nb = [set(g.neighbours(v).tolist()) for v in cyc]
    return all(cyc[(k + 1) % len(cyc)] in nb[k] for k in range(len(cyc)))


def _crossings(cyc, cut, nv):
    n = len(cyc)
    keys = {min(cyc[k], cyc[(k + 1) % n]) * nv + max(cyc[k], cyc[(k + 1) % n]) for k in range(n)}
    return len(keys & set(cut.tolist()))


def test_pass_without_domain_or_cut_grows_as_the_initial_pass(oracle_mod):
    from oracle import passes as P
    m = mg.torus_grid(rng_seed=0)
    g = P.MeshGraph(m.xyz, m.tri)
    nsteps = 300
    init = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, max_steps=nsteps, ckpt_steps=[nsteps])
    ball = np.flatnonzero(hop_ball(m.tri, m.nv, m.seed, 2) >= 0)
    r = P._run_pass(g, np.ones(m.nv), [], ball, np.zeros(m.nv), max_steps=nsteps, ckpt_steps=[nsteps])
    assert r["status"] == P.PASS_STALLED and r["steps"] == nsteps
    assert np.array_equal(r["ckpt"][nsteps].view(np.int64), init.ckpt[nsteps].view(np.int64))
    T_init = np.where(init.T == np.iinfo(np.int64).max, -1, init.T)
    T_pass = np.where(r["T"] == np.iinfo(np.int64).max, -1, r["T"])
    assert np.array_equal(T_pass, T_init)
    grown = T_init > 0
    assert grown.sum() > 500
    assert np.array_equal(r["rnd"][grown], init.rnd[grown])


def _growth_bruteforce(g, dom, cut, start, snaps, steps, tau=0.5):
    nv = g.nv
    cutk = set(cut.tolist())
    op = [[u for u in g.neighbours(v).tolist()
           if dom[u] and dom[v] and (min(u, v) * nv + max(u, v)) not in cutk] for v in range(nv)]
    T = np.full(nv, np.iinfo(np.int64).max, dtype=np.int64)
    rnd = np.zeros(nv, dtype=np.int64)
    ta = np.zeros(nv)
    T[start] = 0
    prev = np.zeros(nv)
    prev[start] = 1.0
    for t in range(1, steps + 1):
        rho = snaps[t]
        cand = {v for v in range(nv) if dom[v] and T[v] > t and rho[v] > tau}
        layer = {v for v in cand if any(T[u] < t for u in op[v])}
        j = 0
        while layer:
            for v in layer:
                T[v], rnd[v] = t, j
                d = rho[v] - prev[v]
                f = min(max((tau - prev[v]) / d if d > 0 else 0.0, 0.0), 1.0)
                ta[v] = (t - 1) + f
            cand -= layer
            j += 1
            layer = {v for v in cand if any(T[u] == t and rnd[u] == j - 1 for u in op[v])}
        prev = rho
    return op, T, rnd, ta


@pytest.mark.parametrize("which", ["tunnel", "refine"])
def test_pass_growth_and_streamline_bruteforce(oracle_mod, which):
    from oracle import passes as P
    m = mg.torus_grid(40, 20, R=1.0, r=0.4, jitter=1e-3, rng_seed=3)
    g = P.MeshGraph(m.xyz, m.tri)
    init = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
    li = int(np.flatnonzero(init.loops[:, 2] == 1)[0])
    first = P.tunnel_pass(g, init, li)
    assert first["status"] == 0
    if which == "refine":
        first = P.refine_pass(g, first["cycle"])
        assert first["status"] == 0
    steps = first["steps"]
    # the same pass again, with a field snapshot at every step
    if which == "tunnel":
        r = P.tunnel_pass(g, init, li, ckpt_steps=list(range(1, steps + 1)))
        ev, _f, _k, off, cnt, _a = (int(q) for q in init.loops[li])
        v = int(init.events[ev, 1])
        key = list(zip(init.T.tolist(), init.rnd.tolist(), range(m.nv)))
        dom = np.array([key[w] <= key[v] for w in range(m.nv)])
    else:
        r = P.refine_pass(g, P.tunnel_pass(g, init, li)["cycle"], ckpt_steps=list(range(1, steps + 1)))
        dom = np.ones(m.nv, dtype=bool)
    op, T, rnd, ta = _growth_bruteforce(g, dom, r["cut"], r["start"], r["ckpt"], steps)
    assert np.array_equal(T, r["T"])
    ins = T <= steps
    assert np.array_equal(rnd[ins], r["rnd"][ins].astype(np.int64))
    assert np.array_equal(ta[ins].view(np.int64), r["arrival"][ins].view(np.int64))
    # parents: steepest descent of the arrival time over lower operator
    # neighbours; never across a cut edge
    rank = list(zip(T.tolist(), rnd.tolist(), range(m.nv)))
    for v in np.flatnonzero(ins & (T > 0)).tolist():
        best, bs = -1, 0.0
        for u in op[v]:
            if rank[u] >= rank[v]:
                continue
            d = m.xyz[u] - m.xyz[v]
            sl = (ta[v] - ta[u]) / math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
            if best < 0 or sl > bs or (sl == bs and rank[u] < rank[best]):
                best, bs = u, sl
        assert r["parent"][v] == best, v
    assert r["reached"] >= 0 and T[r["reached"]] == steps


def test_torus_tunnel_and_refined_handle_are_tight(oracle_mod):
    from oracle import passes as P
    m = _torus48()
    g = P.MeshGraph(m.xyz, m.tri)
    init = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
    assert init.n_handles == 1
    li = int(np.flatnonzero(init.loops[:, 2] == 1)[0])
    tp = P.tunnel_pass(g, init, li)
    assert tp["status"] == 0
    tun = tp["cycle"]
    assert _is_simple_cycle(g, tun)
    assert abs(_winding(m.xyz, tun, R_TORUS)[0]) == 1 and _winding(m.xyz, tun, R_TORUS)[1] == 0
    assert tp["length"] <= 1.2 * 2 * math.pi * (R_TORUS - r_TORUS)
    init_tunnel = P.loop_length(m.xyz, list(init.tunnel_loops()[0]))
    assert tp["length"] < init_tunnel
    # the tunnel crosses the handle loop it came from once
    assert _crossings(tun, tp["cut"], m.nv) == 1
    hp = P.refine_pass(g, tun)
    assert hp["status"] == 0
    han = hp["cycle"]
    assert _is_simple_cycle(g, han)
    w = _winding(m.xyz, han, R_TORUS)
    assert w[0] == 0 and abs(w[1]) == 1
    assert hp["length"] <= 1.6 * 2 * math.pi * r_TORUS
    assert _crossings(han, hp["cut"], m.nv) == 1
    nrm = P.vertex_normals(g)
    assert P.offset_label(g, tun, nrm)[0] == "tunnel"
    assert P.offset_label(g, han, nrm)[0] == "handle"


@pytest.mark.parametrize("case", ["double_torus", "pretzel"])
def test_every_handle_gets_a_tunnel_and_a_refined_handle(oracle_mod, case):
    from oracle import passes as P
    m = mg.multi_torus(2, 28, rng_seed=3) if case == "double_torus" else mg.pretzel(32, rng_seed=2)
    g = P.MeshGraph(m.xyz, m.tri)
    init = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
    kept = np.flatnonzero(init.loops[:, 2] == 1)
    assert kept.size == init.genus >= 2
    for li in kept.tolist():
        tp = P.tunnel_pass(g, init, li)
        assert tp["status"] == 0, li
        assert _is_simple_cycle(g, tp["cycle"])
        assert _crossings(tp["cycle"], tp["cut"], m.nv) == 1
        hp = P.refine_pass(g, tp["cycle"])
        assert hp["status"] == 0, li
        assert _is_simple_cycle(g, hp["cycle"])
        assert _crossings(hp["cycle"], hp["cut"], m.nv) == 1
