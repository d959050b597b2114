"""Pins of the CPU oracle against facts fixed by the paper and by topology,
not by the oracle itself.

* closed-form first step on a 6-regular mesh (hand-derived from the
  two-phase evolution equation with the paper's coefficients, Section
  "Mathematical representation and data structure", "Implementation
  details"), stored with its derivation in tests/golden;
* an independent numpy restatement of the field step, bit-equal;
* the continuum travelling-wave speed mu*e/(2k), k = sqrt(2w/a_eff), of the
  same equation on a quasi-1D strip;
* genus counts: a sphere sweeps no loop, a torus one handle + one tunnel,
  a genus-g surface g of each (Introduction; Section "Results": same number
  of pairs as the genus) for several seeds (Section "Robustness to initial
  seed placement");
* the Euler identity of every step and every event's (s, m, h) recomputed
  by brute force from the insertion order;
* first Betti number of the Reeb graph equals the genus;
* handle loops are non-separating; each tunnel candidate crosses its handle
  loop exactly once; on the torus the handle is a meridian and the tunnel a
  longitude (Introduction: the front folds around the tube first);
* mesh validation errors and an invalid seed region.
"""
import os

import numpy as np
import pytest

import meshgen as mg

from _topo import MeshTopo, events_bruteforce, hop_ball

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _torus():
    return mg.torus_grid()


def _winding_z(p):
    """Winding number of the closed polygon p[0], p[1], ..., p[0] around
    the z axis."""
    th = np.arctan2(p[:, 1], p[:, 0])
    d = np.diff(np.concatenate([th, th[:1]]))
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return d.sum() / (2 * np.pi)


# ---------------------------------------------------------------------------
# field
# ---------------------------------------------------------------------------
def _load_closed_form():
    vals = {}
    with open(os.path.join(GOLDEN, "field_first_step_regular6.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            kind, n, num, den = line.split()
            vals[(kind, int(n))] = int(num) / int(den)
    return vals


def test_field_first_step_closed_form(oracle_mod):
    m = _torus()                                   # 6-regular, dmax = 6
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, dense=1, ckpt_steps=[1])
    rho1 = r.ckpt[1]
    hop = hop_ball(m.tri, m.nv, m.seed, 2)
    ball = hop >= 0
    ell, deg = oracle_mod.ascending_ell(m.tri, m.nv)
    n_in = ball[ell].sum(axis=1)
    vals = _load_closed_form()
    checked = 0
    for v in range(m.nv):
        if ball[v]:
            want = vals[("inside", 6 - n_in[v])]
        else:
            want = vals[("outside", n_in[v])]
        assert abs(rho1[v] - want) <= 4e-16, (v, rho1[v], want)
        checked += 1
    assert checked == m.nv
    # the cases that actually occur include partial neighbourhoods
    assert len(set(n_in[~ball].tolist())) >= 3


def test_field_numpy_twin_bit_equal(oracle_mod):
    for m in (_torus(), mg.pretzel(40, rng_seed=3)):
        steps = [1, 2, 3, 5, 8, 16, 40, 100]
        r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, dense=1, ckpt_steps=steps)
        ell, deg = oracle_mod.ascending_ell(m.tri, m.nv)
        hop = hop_ball(m.tri, m.nv, m.seed, 2)
        rho = (hop >= 0).astype(np.float64)
        for t in range(1, steps[-1] + 1):
            rho = oracle_mod.field_step_numpy(rho, ell, deg, int(deg.max()))
            if t in r.ckpt:
                assert np.array_equal(rho.view(np.int64), r.ckpt[t].view(np.int64)), t


def test_dense_and_active_set_identical(oracle_mod):
    m = mg.pretzel(40, rng_seed=5)
    ck = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]
    a = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, dense=0, ckpt_steps=ck)
    d = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, dense=1, ckpt_steps=ck)
    assert a.status == d.status == 0
    assert a.steps == d.steps
    for t in ck:
        assert np.array_equal(a.ckpt[t].view(np.int64), d.ckpt[t].view(np.int64))
    assert np.array_equal(a.rho.view(np.int64), d.rho.view(np.int64))
    assert np.array_equal(a.T, d.T) and np.array_equal(a.rnd, d.rnd)
    assert np.array_equal(a.events, d.events)
    assert a.active_updates < d.active_updates


def test_travelling_wave_speed(oracle_mod):
    """A planar front on a quasi-1D strip moves at the continuum speed
    |v| = mu*e/(2k) of the two-phase equation (profile (1+sin kx)/2 with
    k = sqrt(2w/a_eff)); on the strip the graph Laplacian of a function of
    the column index is 2*(second difference), so a_eff = 2a.  Per step
    v*dt with dt = 50/6.  The lattice slows the front by a few percent."""
    a, w, e, mu = 1 / 25, 1 / 125, 1 / 30, 1 / 4
    k = np.sqrt(2 * w / (2 * a))
    v_cont = mu * e / (2 * k) * (50.0 / 6.0)          # columns per step
    nM, nm = 400, 6
    m = mg.torus_grid(nM, nm, R=10.0, r=0.2, jitter=0.0, rng_seed=0)
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=0)
    assert r.status == 0 and r.n_handles == 1
    full = r.T.reshape(nM, nm).max(axis=1)
    speed = (160 - 40) / (full[160] - full[40])
    assert 0.80 * v_cont < speed < 1.05 * v_cont, (speed, v_cont)


# ---------------------------------------------------------------------------
# topology
# ---------------------------------------------------------------------------
GENUS_CASES = [
    ("sphere", lambda s: mg.sdf_surface(mg.sdf_sphere(), (-1, -1, -1), (1, 1, 1), 16, 1e-4, s), 0),
    ("box", lambda s: mg.sdf_surface(mg.sdf_box((1, .5, .3)), (-1, -.5, -.3), (1, .5, .3), 20, 1e-4, s), 0),
    ("torus_grid", lambda s: mg.torus_grid(rng_seed=s), 1),
    ("torus_mt", lambda s: mg.sdf_surface(mg.sdf_torus(), (-1.35, -1.35, -.35), (1.35, 1.35, .35), 24, 1e-4, s), 1),
    ("double_torus", lambda s: mg.multi_torus(2, 32, rng_seed=s), 2),
    ("pretzel", lambda s: mg.pretzel(40, rng_seed=s), 3),
    # strut lattices: genus = struts - nodes + 1 (5 for one cell, 28 for 2^3)
    ("lattice1", lambda s: mg.lattice(1, 24, rng_seed=s), mg.lattice_genus(1)),
    ("lattice2", lambda s: mg.lattice(2, 40, rng_seed=s), mg.lattice_genus(2)),
]


@pytest.mark.parametrize("name,make,g", GENUS_CASES, ids=[c[0] for c in GENUS_CASES])
def test_genus_counts_over_seeds(oracle_mod, name, make, g):
    for seed in (0, 1, 2):
        m = make(seed)
        r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        assert r.status == 0, r.status_name
        assert r.genus == g
        assert r.n_handles == g
        assert len(r.tunnel_loops()) == g
        assert r.n_inside == m.nv and r.b_final == 0
        nodes, edges = r.reeb()
        extra = int(r.events[:, 7].sum()) if r.n_events else 0
        assert len(edges) - len(nodes) + 1 + extra == g


def test_event_semantics_bruteforce(oracle_mod):
    for m in (_torus(), mg.multi_torus(2, 24, rng_seed=1), mg.pretzel(32, rng_seed=2)):
        r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        assert r.status == 0
        events_bruteforce(m, r)


def test_euler_identity_every_step_bruteforce(oracle_mod):
    m = mg.multi_torus(2, 24, rng_seed=4)
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
    topo = MeshTopo(m.tri, m.nv)
    g_prev = 0
    for t in range(1, r.steps + 1):
        inside = r.T <= t
        chi = topo.euler_char(inside)
        b, _, _ = topo.loops(inside)
        assert (chi, b) == tuple(r.steplog[t - 1, :2]), t
        assert (2 - chi - b) % 2 == 0
        g = (2 - chi - b) // 2
        assert g >= g_prev
        g_prev = g
    assert g_prev == 2


def test_handle_loops_nonseparating_and_tunnel_crossing(oracle_mod):
    for m in (_torus(), mg.multi_torus(2, 28, rng_seed=7), mg.pretzel(40, rng_seed=1)):
        r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        topo = MeshTopo(m.tri, m.nv)
        hl = r.handle_loops()
        tl = r.tunnel_loops()
        assert len(hl) == len(tl) == r.genus
        ekeys = set()
        for (ev, fid, he, pts, L), tv in zip(hl, tl):
            eids = [topo.edge_id(int(u), int(x)) for u, x in he]
            assert topo.graph_connected_without(eids)      # non-separating
            # consecutive half-edges are joined by a front triangle
            n = len(he)
            assert n >= 3
            # points lie on their edges
            for (u, x), p in zip(he, pts):
                a_, b_ = m.xyz[u], m.xyz[x]
                tt = np.dot(p - a_, b_ - a_) / np.dot(b_ - a_, b_ - a_)
                assert -1e-12 <= tt <= 1 + 1e-12
            seg = np.linalg.norm(np.roll(pts, -1, axis=0) - pts, axis=1).sum()
            assert abs(seg - L) <= 1e-9 * max(1.0, L)
            # tunnel: closed vertex path crossing the handle loop once
            cyc = np.concatenate([tv, tv[:1]])
            es = set(eids)
            crossings = 0
            for a_, b_ in zip(cyc[:-1], cyc[1:]):
                eid = topo.edge_id(int(a_), int(b_))
                crossings += eid in es
            assert crossings == 1
            ekeys.update(eids)


def test_torus_handle_is_meridian_tunnel_is_longitude(oracle_mod):
    for seed in (0, 1, 2):
        m = mg.torus_grid(rng_seed=seed)
        r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        (ev, fid, he, pts, L), = r.handle_loops()
        tv, = r.tunnel_loops()
        assert round(abs(_winding_z(pts))) == 0
        assert round(abs(_winding_z(m.xyz[tv]))) == 1
        # the meridian of a tube of radius 0.4 has length about 2*pi*0.4
        assert 2 * np.pi * 0.4 * 0.9 < L < 2 * np.pi * 0.4 * 1.4


def test_seed_invalid_and_mesh_errors(oracle_mod):
    # on a 5x4 torus grid the radius-2 hop ball already contains a handle
    # (its swept genus is not 0), so it is not a valid initial region
    m = mg.torus_grid(5, 4, R=1.0, r=0.3, jitter=0.0)
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=0)
    assert r.status_name == "SEED_INVALID"
    m = _torus()
    # boundary
    r = oracle_mod.run(m.xyz, m.tri[1:], seed_vertex=0)
    assert r.status_name in ("MESH_HAS_BOUNDARY", "MESH_NOT_CONNECTED")
    # one flipped triangle: a directed edge repeats
    t = m.tri.copy()
    t[5] = t[5, ::-1]
    r = oracle_mod.run(m.xyz, t, seed_vertex=0)
    assert r.status_name == "MESH_NOT_ORIENTABLE"
    # two disjoint tori
    t2 = np.concatenate([m.tri, m.tri + m.nv])
    x2 = np.concatenate([m.xyz, m.xyz + 5.0])
    r = oracle_mod.run(x2, t2, seed_vertex=0)
    assert r.status_name == "MESH_NOT_CONNECTED"
    # stall by step limit
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=0, max_steps=10)
    assert r.status_name == "STALLED"


def test_golden_summaries(oracle_mod):
    """Regression against summaries written by tests/golden/make_golden.py
    (which calls only the oracle)."""
    import json
    with open(os.path.join(GOLDEN, "oracle_summaries.json")) as f:
        gold = json.load(f)
    from golden.make_golden import CASES, summarize
    for name, make in CASES.items():
        m = make()
        r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        assert summarize(r) == gold[name], name
