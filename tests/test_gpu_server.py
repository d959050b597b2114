"""Serving: requests submitted while others run are admitted as slots and
HBM budget free up and advance together in bounded launches (each mesh's
visit cut at a step boundary, then continued by a later launch).  Every
result equals the oracle's element by element, and equals the same mesh
run alone, whatever the mix, the slice length or the admission order."""
import time

import numpy as np
import pytest

import meshgen as mg
from _parity import compare

pytestmark = pytest.mark.gpu


def _meshes():
    return [
        mg.torus_grid(rng_seed=0),
        mg.torus_grid(96, 48, rng_seed=7),
        mg.sdf_surface(mg.sdf_sphere(), (-1, -1, -1), (1, 1, 1), 16, 1e-4, 0),
        mg.multi_torus(2, 28, rng_seed=3),
        mg.pretzel(40, rng_seed=5),
        mg.multi_torus(4, 40, rng_seed=4),
    ]


def _wait(srv, tickets, timeout=90.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, f"server requests not done after {timeout} s: {srv.stats()}"
        time.sleep(0.002)
    return [out[t] for t in tickets]


def _same(a, b):
    assert a.summary["steps"] == b.summary["steps"]
    assert np.array_equal(a.rho.view(np.int64), b.rho.view(np.int64))
    assert np.array_equal(a.step, b.step) and np.array_equal(a.parent, b.parent)
    assert np.array_equal(a.events, b.events)
    assert len(a.loops) == len(b.loops)
    for x, y in zip(a.loops, b.loops):
        assert np.array_equal(x["he"], y["he"]) and x["length"] == y["length"]
    assert len(a.tunnels) == len(b.tunnels)
    for x, y in zip(a.tunnels, b.tunnels):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("shape", ["one_per_cu", "two_per_cu", "coherent"])
@pytest.mark.parametrize("slice_us", [150, 5000])
def test_server_mix_matches_oracle_and_solo(oracle_mod, slice_us, shape):
    import paper_2105_13168_amd as vls
    flags = {"one_per_cu": 0, "two_per_cu": vls.VLS_BATCH_TWO_PER_CU, "coherent": vls.VLS_COHERENT_SHARING}[shape]
    ctx = vls.Context(0)
    ms = _meshes()
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    srv = vls.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=64, slice_us=slice_us, flags=flags)
    try:
        # staggered arrivals; the first torus twice at once (own run state
        # per request); checkpoints on one request
        tickets = []
        for i, (m, h) in enumerate(zip(ms, M)):
            ck = [1, 100, 300] if i == 0 else ()
            tickets.append(srv.submit(h, seed_vertex=m.seed, ckpt_steps=ck))
            if i == 2:
                tickets.append(srv.submit(M[0], seed_vertex=ms[0].seed))
            time.sleep(0.003)
        res = _wait(srv, tickets)
        st = srv.stats()
        assert st["completed"] == len(tickets) and st["admitted_bytes"] == 0
        if slice_us < 1000:
            assert st["launches"] > 2        # visits were cut and continued
        order = list(range(len(ms)))
        order.insert(3, 0)
        for k, r in zip(order, res):
            m = ms[k]
            assert r.summary["run_status"] == 0
            assert r.summary["server_latency_ms"] >= r.summary["server_queue_ms"] >= 0
            o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, ckpt_steps=[1, 100, 300] if r is res[0] else ())
            bad = compare(r, o, m.nv)
            assert not bad, (m.name, bad)
        for k in (0, 5):
            solo = M[k].run(seed_vertex=ms[k].seed)
            _same(solo, res[order.index(k)])
        _same(res[0], res[3])
    finally:
        srv.close()
        for x in M:
            x.close()
        ctx.close()


def test_server_budget_admission_one_at_a_time(oracle_mod):
    """A budget below any one request's run state admits one request at a
    time (the oversize rule); results are unchanged."""
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = _meshes()[:4]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    srv = vls.Server(ctx, hbm_budget_bytes=1, max_slots=8, slice_us=1000)
    try:
        tickets = [srv.submit(h, seed_vertex=m.seed) for m, h in zip(ms, M)]
        seen_running = 0
        t0 = time.time()
        while srv.stats()["completed"] < len(tickets) and time.time() - t0 < 60:
            seen_running = max(seen_running, srv.stats()["running"])
            time.sleep(0.0005)
        assert seen_running <= 1
        res = _wait(srv, tickets)
        for m, r in zip(ms, res):
            bad = compare(r, oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed), m.nv)
            assert not bad, (m.name, bad)
    finally:
        srv.close()
        for x in M:
            x.close()
        ctx.close()


def test_server_rejects_bad_arguments():
    """Unknown flag bits, no slots, a zero slice or a zero budget are
    VLS_E_INVALID_ARG at creation; no server is made."""
    import ctypes as C
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    try:
        for budget, slots, slice_us, flags in ((1 << 30, 8, 1000, 1 << 10), (1 << 30, 8, 1000, vls.VLS_DENSE_FIELD),
                                               (1 << 30, 0, 1000, 0), (1 << 30, 8, 0, 0), (0, 8, 1000, 0)):
            h = C.c_void_p()
            st = vls.vls_server_create(ctx.h, budget, slots, slice_us, flags, C.byref(h))
            assert st == vls.VLS_E_INVALID_ARG and not h.value, (budget, slots, slice_us, flags, st)
    finally:
        ctx.close()


def test_server_destroy_with_work_in_flight():
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    m = mg.pretzel(48, rng_seed=1)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    srv = vls.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=2, slice_us=200)
    for _ in range(6):
        srv.submit(M, seed_vertex=m.seed)
    time.sleep(0.01)
    srv.close()
    # the context and mesh still work afterwards
    r = M.run(seed_vertex=m.seed)
    assert r.summary["run_status"] == 0
    M.close()
    ctx.close()


@pytest.mark.parametrize("two_per_cu", [False, True])
def test_server_gangs_resize_and_switch(oracle_mod, two_per_cu):
    """Many large requests at once: the planner grants meshes of >= 2^17
    vertices gangs of workgroups, largest first, within the pool less the
    reserve for small meshes (256 or 512 workgroups at one or two per CU);
    the requests that no longer fit sit the launch out.  As requests finish
    the rest are re-planned, so a request waits, then runs in gangs of
    changing sizes.  Every result equals the oracle's."""
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    big = [mg.pretzel(72, rng_seed=s) for s in (0, 1)] + [mg.pretzel(96, rng_seed=2), mg.lattice(3, 96, rng_seed=3)]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in big]
    srv = vls.Server(ctx, hbm_budget_bytes=64 << 30, max_slots=512, slice_us=300,
                     flags=vls.VLS_BATCH_TWO_PER_CU if two_per_cu else 0)
    try:
        reqs = [(k % 2, srv.submit(M[k % 2], seed_vertex=big[k % 2].seed)) for k in range(200)]
        reqs += [(2, srv.submit(M[2], seed_vertex=big[2].seed)), (3, srv.submit(M[3], seed_vertex=big[3].seed))]
        res = _wait(srv, [t for _, t in reqs], timeout=110.0)
        assert srv.stats()["launches"] > 3
        oracle_res = {}
        for (k, _), r in zip(reqs, res):
            if k not in oracle_res:
                m = big[k]
                o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
                bad = compare(r, o, m.nv)
                assert not bad, (m.name, bad)
                oracle_res[k] = r
            else:
                _same(r, oracle_res[k])
    finally:
        srv.close()
        for x in M:
            x.close()
        ctx.close()


def test_server_request_gang_granularity(oracle_mod):
    """Each request's own gang_vertices sets its gang: the same meshes
    submitted at 2048, 8192 and the default 65536 vertices per gang
    workgroup (gangs of up to a few dozen workgroups, and one workgroup) in
    one mix give results equal to each other and to the oracle's."""
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = [mg.torus_grid(96, 48, rng_seed=7), mg.multi_torus(4, 40, rng_seed=4), mg.pretzel(40, rng_seed=5)]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    srv = vls.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=64, slice_us=300)
    try:
        reqs = []
        for gv in (2048, 8192, 0):
            for i, (m, h) in enumerate(zip(ms, M)):
                assert m.nv // 2048 >= 2
                reqs.append((i, srv.submit(h, seed_vertex=m.seed, gang_vertices=gv)))
        res = _wait(srv, [t for _, t in reqs])
        first = {}
        for (i, _), r in zip(reqs, res):
            if i not in first:
                m = ms[i]
                o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
                bad = compare(r, o, m.nv)
                assert not bad, (m.name, bad)
                first[i] = r
            else:
                _same(r, first[i])
    finally:
        srv.close()
        for x in M:
            x.close()
        ctx.close()


def test_server_stalled_request_in_the_mix(oracle_mod):
    """A request that stops at its step limit returns VLS_E_STALLED with the
    partial results the oracle gives for the same limit, including the field
    at its last step; the requests around it are unchanged (equal to the
    oracle)."""
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    ms = _meshes()[:4]
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    srv = vls.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=16, slice_us=400)
    try:
        tickets = []
        for i, (m, h) in enumerate(zip(ms, M)):
            tickets.append(srv.submit(h, seed_vertex=m.seed))
            if i == 1:
                tickets.append(srv.submit(M[0], seed_vertex=ms[0].seed, max_steps=300, ckpt_steps=[1, 150, 300]))
        res = _wait(srv, tickets)
        order = [0, 1, 0, 2, 3]
        for k, (i, r) in enumerate(zip(order, res)):
            m = ms[i]
            if k == 2:
                assert r.status == vls.VLS_E_STALLED and r.summary["run_status"] == vls.VLS_E_STALLED
                o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, max_steps=300, ckpt_steps=[1, 150, 300])
                assert o.status == vls.VLS_E_STALLED and 300 in r.ckpt
            else:
                assert r.summary["run_status"] == 0
                o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
            bad = compare(r, o, m.nv)
            assert not bad, (k, m.name, bad)
    finally:
        srv.close()
        for x in M:
            x.close()
        ctx.close()


def test_server_shutdown_cancels_pending_requests():
    """vls_server_shutdown: queued and running requests poll as
    VLS_E_CANCELLED (no result), finished ones keep their results, and later
    submits are refused with VLS_E_CANCELLED."""
    import ctypes as C
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    small = mg.torus_grid(rng_seed=0)
    big = mg.pretzel(72, rng_seed=1)
    Ms = vls.Mesh(ctx, small.xyz, small.tri)
    Mb = vls.Mesh(ctx, big.xyz, big.tri)
    srv = vls.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=2, slice_us=200)
    try:
        first = srv.submit(Ms, seed_vertex=small.seed)
        (r0,) = _wait(srv, [first])
        assert r0.summary["run_status"] == 0
        tickets = [srv.submit(Mb, seed_vertex=big.seed) for _ in range(8)]
        srv.shutdown()
        cancelled = 0
        for t in tickets:
            h = C.c_void_p()
            st = vls.vls_server_poll(srv.h, C.c_uint64(t), C.byref(h))
            assert st in (0, vls.VLS_E_CANCELLED), st
            if st == vls.VLS_E_CANCELLED:
                assert not h.value
                cancelled += 1
            else:
                vls.vls_result_destroy(h)
        assert cancelled >= 6          # two slots: most requests never started
        p = vls.default_params(seed_vertex=small.seed)
        tk = C.c_uint64()
        assert vls.vls_server_submit(srv.h, Ms.h, C.byref(p), C.byref(tk)) == vls.VLS_E_CANCELLED
        srv.shutdown()                 # idempotent
    finally:
        srv.close()
        Ms.close()
        Mb.close()
        ctx.close()
