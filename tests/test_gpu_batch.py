"""Batched mode: many uneven meshes in one launch, one workgroup per mesh.
Every mesh's result equals the oracle's and the solo run's, element by
element (the mix changes nothing)."""
import pytest

import meshgen as mg
from _parity import compare

pytestmark = pytest.mark.gpu


def _meshes():
    out = []
    for s in range(3):
        out.append(mg.torus_grid(rng_seed=s))
    out.append(mg.torus_grid(96, 48, rng_seed=7))
    out.append(mg.sdf_surface(mg.sdf_sphere(), (-1, -1, -1), (1, 1, 1), 16, 1e-4, 0))
    out.append(mg.multi_torus(2, 28, rng_seed=3))
    out.append(mg.multi_torus(4, 40, rng_seed=4))
    out.append(mg.pretzel(40, rng_seed=5))
    out.append(mg.pretzel(64, rng_seed=6))
    return out


def test_batch_matches_oracle_and_solo(oracle_mod):
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = _meshes()
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    res = vls.batch_run(ctx, M, [m.seed for m in ms])
    for m, g in zip(ms, res):
        o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        bad = compare(g, o, m.nv)
        assert not bad, (m.name, bad)
    # solo runs of two of them give the same outputs
    for i in (3, 8):
        solo = M[i].run(seed_vertex=ms[i].seed)
        o = oracle_mod.run(ms[i].xyz, ms[i].tri, seed_vertex=ms[i].seed)
        assert not compare(solo, o, ms[i].nv)
        assert (solo.events == res[i].events).all()
    for x in M:
        x.close()
    ctx.close()


def test_batch_repeat_is_deterministic():
    import numpy as np
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = _meshes()[:6]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    a = vls.batch_run(ctx, M, [m.seed for m in ms])
    b = vls.batch_run(ctx, M, [m.seed for m in ms], grid=3)
    for x, y in zip(a, b):
        assert np.array_equal(x.rho.view(np.int64), y.rho.view(np.int64))
        assert np.array_equal(x.events, y.events)
    for x in M:
        x.close()
    ctx.close()


_GANG_ORACLE = {}


@pytest.mark.parametrize("dense", [False, True])
@pytest.mark.parametrize("two_per_cu", [False, True])
@pytest.mark.parametrize("pool", [0, 6])
def test_batch_gangs_match_oracle(oracle_mod, pool, two_per_cu, dense):
    """Meshes of >= 2^17 vertices get gangs of workgroups (one topology
    workgroup, the rest field) inside the batched launch; with a pool of 6
    the gangs are scaled down to fit.  Results equal the oracle's, with the
    band-limited and with the dense field step."""
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = [mg.pretzel(96, rng_seed=2), mg.lattice(3, 96, rng_seed=3), mg.pretzel(72, rng_seed=1),
          mg.torus_grid(rng_seed=4), mg.multi_torus(2, 28, rng_seed=5)]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    flags = (vls.VLS_BATCH_TWO_PER_CU if two_per_cu else 0) | (vls.VLS_DENSE_FIELD if dense else 0)
    res = vls.batch_run(ctx, M, [m.seed for m in ms], grid=pool, flags=flags)
    for m, g in zip(ms, res):
        if m.name not in _GANG_ORACLE:
            _GANG_ORACLE[m.name] = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        o = _GANG_ORACLE[m.name]
        bad = compare(g, o, m.nv)
        assert not bad, (m.name, bad)
    for x in M:
        x.close()
    ctx.close()


@pytest.mark.parametrize("two_per_cu", [False, True])
def test_batch_gangs_coherent_sharing_match_oracle(oracle_mod, two_per_cu):
    """Gangs whose workgroups share the field through coherent atomics
    (ordering-point fences instead of L2 invalidation at each hand-off)
    give the oracle's results, next to one-workgroup meshes."""
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = [mg.pretzel(96, rng_seed=2), mg.lattice(3, 96, rng_seed=3), mg.pretzel(72, rng_seed=1),
          mg.torus_grid(rng_seed=4), mg.multi_torus(2, 28, rng_seed=5)]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    flags = vls.VLS_COHERENT_SHARING | (vls.VLS_BATCH_TWO_PER_CU if two_per_cu else 0)
    res = vls.batch_run(ctx, M, [m.seed for m in ms], flags=flags)
    for m, g in zip(ms, res):
        if m.name not in _GANG_ORACLE:
            _GANG_ORACLE[m.name] = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        bad = compare(g, _GANG_ORACLE[m.name], m.nv)
        assert not bad, (m.name, bad)
    for x in M:
        x.close()
    ctx.close()


def test_batch_schedule_changes_no_result():
    """Every schedule the tuner may pick (pool shape, vertices per gang
    workgroup) gives bit-identical results; the tuner returns one of them."""
    import numpy as np
    import paper_2105_13168_amd as vls
    from paper_2105_13168_amd.tune import tune_batch
    ctx = vls.Context(0)
    ms = [mg.pretzel(96, rng_seed=2), mg.pretzel(72, rng_seed=1), mg.torus_grid(rng_seed=4),
          mg.multi_torus(2, 28, rng_seed=5)]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    seeds = [m.seed for m in ms]
    ref = vls.batch_run(ctx, M, seeds)
    for two, gv in ((False, 32768), (True, 131072), (True, 16384)):
        res = vls.batch_run(ctx, M, seeds, gang_vertices=gv, flags=vls.VLS_BATCH_TWO_PER_CU if two else 0)
        for a, b in zip(ref, res):
            assert np.array_equal(a.rho.view(np.int64), b.rho.view(np.int64))
            assert np.array_equal(a.events, b.events) and np.array_equal(a.step, b.step)
    t = tune_batch(ctx, M, seeds, candidates=((False, 65536), (True, 32768)))
    assert (t["two_per_cu"], t["gang_vertices"]) in ((False, 65536), (True, 32768))
    for x in M:
        x.close()
    ctx.close()


def test_batch_edge_events_and_final_checkpoint(oracle_mod):
    """The rare event meshes (3-way merge and 1-to-3 splits, a DEGENERATE
    node, monkey-saddle splits) batched with tori, each with its own seed
    parameters, and field snapshots that include each mesh's last step (the
    step at which its pass stops): every output equals the oracle's."""
    import paper_2105_13168_amd as vls
    from test_oracle_edge_events import EDGE_CASES
    ctx = vls.Context(0)
    ms, kws = [], []
    for _name, make, kw in EDGE_CASES:
        ms.append(make())
        kws.append(dict(kw))
    for s in range(2):
        t = mg.torus_grid(rng_seed=s)
        ms.append(t)
        kws.append(dict(seed_vertex=t.seed))
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    orc = []
    for m, kw in zip(ms, kws):
        rk = {k: v for k, v in kw.items() if k != "seed_vertex"}
        o = oracle_mod.run(m.xyz, m.tri, seed_vertex=kw["seed_vertex"], **rk)
        ck = sorted({1, max(1, o.steps // 3), o.steps})
        kw["ckpt_steps"] = ck
        orc.append(oracle_mod.run(m.xyz, m.tri, seed_vertex=kw["seed_vertex"], ckpt_steps=ck, **rk))
    per = [{k: v for k, v in kw.items() if k != "seed_vertex"} for kw in kws]
    try:
        res = vls.batch_run(ctx, M, [kw["seed_vertex"] for kw in kws], per_mesh=per)
        for m, g, o in zip(ms, res, orc):
            assert o.steps in g.ckpt
            bad = compare(g, o, m.nv)
            assert not bad, (m.name, bad)
    finally:
        for x in M:
            x.close()
        ctx.close()


def test_batch1024_digests_match_oracle():
    """The bench's batch of 1024 uneven meshes (tori with V ~ logU[1e3, 2e5]
    and chains of 2..10 tori), one batched launch: every mesh's outputs
    equal the oracle's, by a combined digest per mesh recorded by
    tests/golden/make_golden.py --batch from the oracle alone."""
    import json
    import os
    import paper_2105_13168_amd as vls
    from _digest import canon_gpu, digests
    from golden.make_golden import combined_digest
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "oracle_batch1024.json")))["meshes"]
    ms = mg.batch_workload(1024, base_seed=0)
    assert [m.nv for m in ms] == [g["nv"] for g in gold]
    ctx = vls.Context(0)
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    try:
        res = vls.batch_run(ctx, M, [m.seed for m in ms])
        bad = []
        for i, (g, want) in enumerate(zip(res, gold)):
            d = digests(canon_gpu(g))
            if (d["steps"], d["n_events"], d["n_handles"]) != (want["steps"], want["n_events"], want["n_handles"]) \
                    or combined_digest(d) != want["digest"]:
                bad.append(i)
        assert not bad, f"{len(bad)} meshes differ from the oracle, first {bad[:10]}"
    finally:
        for x in M:
            x.close()
        ctx.close()
