"""Pins of the oracle's event path, rank order and loop geometry that do not
come from the oracle itself.

* Meshes on which the method's rare event cases occur (found by searching
  unjittered symmetric surfaces with the oracle on the CPU): a voxel cube
  frame where the seed front splits into three at a monkey saddle and three
  fronts later merge at one vertex (Section "Initial Pass": branching,
  collision, "layers involved minus one"), and the 7-vertex torus, whose
  single handle is swept at one monkey saddle of one front (a DEGENERATE
  node, extra cycle x = 1).  Each test asserts that its case occurs, then
  recomputes every event's k, s, m, h, x and node type by brute force.
* The inside set's growth (threshold, then closure rounds; Section
  "Performance Considerations": vertices above the threshold) recomputed
  from the oracle's per-step field snapshots: insertion step, round and
  parent of every vertex, with a threshold that some vertex's field value
  hits exactly (so a non-strict comparison would show).
* Reeb node positions (Section "Reeb Graph Extraction": mean of the band)
  recomputed from the front triangles of the involved loops, found by
  connected components of triangles rather than by walks.
* Crossing points and lengths of every involved loop (Section "Initial
  Pass": the fronts just before they merge) recomputed from the field
  snapshot of the event's step.
* The loop that is not reported is the longest (Section "Initial Pass":
  the longest boundary loop is ignored; ties go to the larger front id).
"""
import numpy as np
import pytest

import meshgen as mg

from _topo import MeshTopo, events_bruteforce, hop_ball, rank_key

TAU = 0.5


def _voxel_frame():
    return mg.voxel_frame(1, 2, 1, center=True)


EDGE_CASES = [
    # name, mesh, run parameters
    ("voxel_frame", _voxel_frame, dict(seed_vertex=0, seed_radius=1)),
    ("csaszar7", mg.csaszar_torus, dict(seed_vertex=5, seed_radius=0)),
    ("lattice1_32_diag", lambda: mg.pick_seed(mg.lattice(1, 32), 0),
     dict(seed_vertex=760, seed_radius=2)),
]


def _run(oracle_mod, name, ck=()):
    make, kw = {c[0]: (c[1], c[2]) for c in EDGE_CASES}[name]
    m = make()
    return m, oracle_mod.run(m.xyz, m.tri, ckpt_steps=ck, **kw), kw


def test_voxel_frame_reaches_three_way_events(oracle_mod):
    m, r, _ = _run(oracle_mod, "voxel_frame")
    assert r.status == 0 and r.genus == 5 and r.n_handles == 5
    ev = r.events
    # a monkey saddle that splits the seed front into three
    assert ((ev[:, 3] == 3) & (ev[:, 4] == 1) & (ev[:, 5] == 3) & (ev[:, 2] == 1)).any()
    # three fronts merging at one vertex: two handle loops, one of three dropped
    i3 = np.flatnonzero((ev[:, 4] == 3) & (ev[:, 2] == 2))
    assert i3.size == 1 and ev[i3[0], 6] == 2 and ev[i3[0], 7] == 0
    loops = r.loops[r.loops[:, 0] == i3[0]]
    assert loops.shape[0] == 3 and int(loops[:, 2].sum()) == 2
    events_bruteforce(m, r)


def test_csaszar_torus_reaches_degenerate_event(oracle_mod):
    m, r, _ = _run(oracle_mod, "csaszar7")
    assert r.status == 0 and r.genus == 1
    ev = r.events
    d = np.flatnonzero(ev[:, 2] == 4)
    assert d.size == 1
    k, s, mm, h, x = (int(q) for q in ev[d[0], 3:8])
    assert (k, s, mm, h, x) == (3, 1, 1, 1, 1)
    # the handle is swept without a merge: no handle loop, and the Reeb
    # graph's first Betti number counts the extra cycle
    assert r.n_handles == 0 and len(r.tunnel_loops()) == 0
    nodes, edges = r.reeb()
    assert len(edges) - len(nodes) + 1 + int(ev[:, 7].sum()) == 1
    events_bruteforce(m, r)


def test_marching_tets_lattice_monkey_saddle_split(oracle_mod):
    m, r, _ = _run(oracle_mod, "lattice1_32_diag")
    assert r.status == 0 and r.n_handles == r.genus == 5
    ev = r.events
    assert ((ev[:, 3] == 3) & (ev[:, 5] == 3)).any()
    events_bruteforce(m, r)


# ---------------------------------------------------------------------------
# rank order: threshold and closure rounds from the field snapshots
# ---------------------------------------------------------------------------
def _neighbours(tri, nv):
    t = np.asarray(tri, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    nb = [set() for _ in range(nv)]
    for u, x in e:
        nb[u].add(int(x))
        nb[x].add(int(u))
    return [sorted(s) for s in nb]


def _growth_bruteforce(m, seed, r0, tau, snaps, steps):
    """Insertion step, closure round and parent of every vertex: the seed
    hop ball at step 0 (round = hop); at step t, the outside vertices whose
    field is strictly above tau join in rounds, round 0 touching the inside
    set of step t-1 and round j touching round j-1; the parent is the
    neighbour of smallest rank (step, round, id) that is already inside."""
    nv = m.nv
    nb = _neighbours(m.tri, nv)
    hop = hop_ball(m.tri, nv, seed, r0)
    T = np.full(nv, np.iinfo(np.int64).max, dtype=np.int64)
    rnd = np.zeros(nv, dtype=np.int64)
    T[hop >= 0] = 0
    rnd[hop >= 0] = hop[hop >= 0]
    for t in range(1, steps + 1):
        rho = snaps[t]
        cand = set(np.flatnonzero((T > t) & (rho > tau)).tolist())
        prev = {v for v in cand if any(T[u] < t for u in nb[v])}
        j = 0
        while prev:
            for v in prev:
                T[v] = t
                rnd[v] = j
            cand -= prev
            j += 1
            prev = {v for v in cand if any(T[u] == t and rnd[u] == j - 1 for u in nb[v])}
    parent = np.full(nv, -1, dtype=np.int64)
    for v in range(nv):
        if v == seed or T[v] > steps:
            continue
        low = [u for u in nb[v] if (T[u], rnd[u], u) < (T[v], rnd[v], v)]
        parent[v] = min(low, key=lambda u: (T[u], rnd[u], u))
    return T, rnd, parent


@pytest.mark.parametrize("case", ["torus", "pretzel32", "voxel_frame", "exact_tie", "rounds"])
def test_closure_rounds_bruteforce(oracle_mod, case):
    tau = TAU
    r0 = 2
    mu = 0.25
    if case == "rounds":
        # a steeper front (mu = 0.9) and a high threshold: some vertices go
        # above tau before a neighbour nearer the inside set does, and join
        # in closure rounds after round 0
        m = mg.torus_grid(rng_seed=0)
        seed, mu, tau = m.seed, 0.9, 0.9
    elif case == "torus":
        m = mg.torus_grid(rng_seed=0)
        seed = m.seed
    elif case == "pretzel32":
        m = mg.pretzel(32, rng_seed=2)
        seed = m.seed
    elif case == "voxel_frame":
        m = _voxel_frame()
        seed, r0 = 0, 1
    else:
        # threshold equal to a value the field takes exactly at step 1 (an
        # outside vertex next to the seed ball, on the 6-regular torus the
        # same value at every vertex with the same number of inside
        # neighbours): those vertices are not crossers at step 1
        m = mg.torus_grid(rng_seed=0)
        seed = m.seed
        r1 = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, max_steps=1, ckpt_steps=[1])
        rho1 = r1.ckpt[1]
        out = (hop_ball(m.tri, m.nv, seed, r0) < 0) & (rho1 > 0.0) & (rho1 < 1.0)
        tau = float(np.max(rho1[out]))
        assert 0.0 < tau < 0.5
    pre = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, seed_radius=r0, tau=tau, mu=mu)
    assert pre.status == 0
    steps = pre.steps
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, seed_radius=r0, tau=tau, mu=mu,
                       ckpt_steps=list(range(1, steps + 1)))
    T, rnd, parent = _growth_bruteforce(m, seed, r0, tau, r.ckpt, steps)
    assert np.array_equal(T, r.T)
    assert np.array_equal(rnd, r.rnd.astype(np.int64))
    assert np.array_equal(parent, r.parent.astype(np.int64))
    if case == "rounds":
        # closure rounds beyond round 0 occur, so the round-0 rule (touching
        # the inside set of the previous step only) is exercised
        assert (rnd[T > 0] >= 1).sum() >= 5
    if case == "exact_tie":
        hit = np.flatnonzero(r.ckpt[1] == tau)
        assert hit.size > 0 and (T[hit] > 1).all()


# ---------------------------------------------------------------------------
# Reeb positions, loop points and lengths, the dropped loop
# ---------------------------------------------------------------------------
def _geometry_cases():
    return [
        ("torus", mg.torus_grid(rng_seed=1), dict()),
        ("double_torus", mg.multi_torus(2, 24, rng_seed=1), dict()),
        ("pretzel32", mg.pretzel(32, rng_seed=2), dict()),
        ("voxel_frame", _voxel_frame(), dict(seed_radius=1)),
        ("lattice1_24", mg.lattice(1, 24, rng_seed=3), dict()),
    ]


def _seq_sum(vals):
    s = 0.0
    for v in vals:
        s = s + float(v)
    return s


@pytest.mark.parametrize("idx", range(5), ids=[c[0] for c in _geometry_cases()])
def test_reeb_positions_from_front_triangles(oracle_mod, idx):
    name, m, kw = _geometry_cases()[idx]
    seed = m.seed if name != "voxel_frame" else 0
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, **kw)
    assert r.status == 0 and r.n_events > 0
    topo = MeshTopo(m.tri, m.nv)
    order = rank_key(r.T, r.rnd)
    pos = np.empty(m.nv, dtype=np.int64)
    pos[order] = np.arange(m.nv)
    nb = _neighbours(m.tri, m.nv)
    tri = topo.tri
    for i, ev in enumerate(r.events):
        v = int(ev[1])
        pre = pos < pos[v]
        _, lab, ce = topo.loops(pre)
        lab_of = dict(zip(ce.tolist(), lab.tolist()))
        involved = {lab_of[topo.edge_id(u, v)] for u in nb[v] if pre[u]}
        # front triangles of the involved loops: the triangles on either side
        # of their crossed edges
        sel = np.array([lab_of[c] in involved for c in ce.tolist()])
        ts = np.unique(np.concatenate([topo.etri[ce[sel], 0], topo.etri[ce[sel], 1]]))
        verts = np.unique(tri[ts].ravel())
        n = float(verts.size)
        want = [_seq_sum(m.xyz[verts, q]) / n for q in range(3)]
        got = r.event_pos[i]
        assert np.array_equal(np.array(want).view(np.int64), got.view(np.int64)), (name, i, want, got)


@pytest.mark.parametrize("idx", range(5), ids=[c[0] for c in _geometry_cases()])
def test_loop_points_lengths_and_dropped_loop(oracle_mod, idx):
    name, m, kw = _geometry_cases()[idx]
    seed = m.seed if name != "voxel_frame" else 0
    first = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, **kw)
    ev_steps = sorted({int(first.events[int(e), 0]) for e in first.loops[:, 0]})
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, ckpt_steps=ev_steps, **kw)
    assert r.status == 0 and r.loops.shape[0] > 0
    topo = MeshTopo(m.tri, m.nv)
    order = rank_key(r.T, r.rnd)
    pos = np.empty(m.nv, dtype=np.int64)
    pos[order] = np.arange(m.nv)
    by_event = {}
    for li, (e, fid, kept, off, cnt, av) in enumerate(r.loops):
        ev = r.events[int(e)]
        t, v = int(ev[0]), int(ev[1])
        rho = r.ckpt[t]
        pre = pos < pos[v]
        he = r.loop_he[off:off + cnt]
        pts = r.loop_pts[off:off + cnt]
        u, x = he[:, 0], he[:, 1]
        # crossed edges of the state just before v joins, inside -> outside
        assert pre[u].all() and not pre[x].any()
        # a closed cycle: consecutive crossed edges share a triangle; the
        # first edge has the smallest key inside*nv + outside
        for k in range(cnt):
            a = topo.edge_id(int(u[k]), int(x[k]))
            b = topo.edge_id(int(u[(k + 1) % cnt]), int(x[(k + 1) % cnt]))
            assert set(topo.etri[a]) & set(topo.etri[b])
        keys = u * m.nv + x
        assert keys[0] == keys.min() and np.unique(keys).size == cnt
        # crossing parameter from the field of the event's step
        ru, rx = rho[u], rho[x]
        den = ru - rx
        tt = np.where(den <= 0.0, 0.5, np.clip((ru - TAU) / np.where(den <= 0.0, 1.0, den), 0.0, 1.0))
        pu, px = m.xyz[u], m.xyz[x]
        want = pu + tt[:, None] * (px - pu)
        assert np.array_equal(want.view(np.int64), pts.view(np.int64)), (name, li)
        # closed polyline length, summed in loop order
        L = 0.0
        for k in range(cnt):
            d = pts[(k + 1) % cnt] - pts[k]
            L = L + float(np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]))
        assert L == r.loop_len[li], (name, li)
        by_event.setdefault(int(e), []).append((float(r.loop_len[li]), int(fid), int(kept)))
    for e, ls in by_event.items():
        assert len(ls) == int(r.events[e, 4]) >= 2
        dropped = [l for l in ls if not l[2]]
        assert len(dropped) == 1
        # the dropped loop is the longest; an exact tie drops the larger id
        assert max(ls, key=lambda l: (l[0], l[1])) == dropped[0]
