"""Reeb junction refinement on the GPU (VLS_REEB_REFINE): the second initial
pass, started from the first kept handle loop, equals the oracle's pass from
the same seed set element by element (events, insertion steps, rounds and
parents, loops, tunnels, Reeb nodes with their band-mean positions and
edges), and the first pass is unchanged by the flag."""
import numpy as np
import pytest

import meshgen as mg
from _parity import compare

pytestmark = pytest.mark.gpu

CASES = [
    ("torus64x32", lambda: mg.torus_grid(rng_seed=0)),
    ("torus_mt48", lambda: mg.sdf_surface(mg.sdf_torus(R=1.0, r=0.35), (-1.4, -1.4, -0.4), (1.4, 1.4, 0.4), 48,
                                          1e-4, 0)),
    ("double_torus28", lambda: mg.multi_torus(2, 28, rng_seed=3)),
    ("pretzel40", lambda: mg.pretzel(40, rng_seed=5)),
    ("torus_chain4_40", lambda: mg.multi_torus(4, 40, rng_seed=4)),
    ("lattice2_40", lambda: mg.lattice(2, 40, rng_seed=1)),
    ("lattice3_64", lambda: mg.lattice(3, 64, rng_seed=2)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_refined_pass_matches_oracle(oracle_mod, name, make):
    import paper_2105_13168_amd as vls
    m = make()
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE)
        plain = M.run(seed_vertex=m.seed)
    finally:
        M.close()
        ctx.close()
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed)
    bad = compare(g, first, m.nv)
    assert not bad, (name, "first pass", bad)
    assert plain.refined is None
    assert np.array_equal(plain.events, g.events) and plain.reeb_nodes == g.reeb_nodes
    assert second is not None and g.refined is not None
    bad = compare(g.refined, second, m.nv)
    assert not bad, (name, "refined pass", bad)
    ss = oracle_mod.refinement_seed_set(first)
    assert g.refined.summary["seed_vertex"] == int(ss[0])
    assert g.refined.summary["n_handles"] == first.n_handles


def test_no_handle_no_refined_pass(oracle_mod):
    import paper_2105_13168_amd as vls
    m = mg.sdf_surface(mg.sdf_sphere(), (-1, -1, -1), (1, 1, 1), 16, 1e-4, 0)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE)
    finally:
        M.close()
        ctx.close()
    assert g.summary["n_handles"] == 0 and g.refined is None
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed)
    assert second is None and not compare(g, first, m.nv)


def test_refinement_only_through_vls_run():
    import ctypes as C
    import paper_2105_13168_amd as vls
    m = mg.torus_grid(rng_seed=0)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        p = vls.default_params(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE)
        outs = (C.c_void_p * 1)()
        meshes = (C.c_void_p * 1)(M.h)
        ps = (vls.vls_params * 1)(p)
        assert vls.vls_batch_run(ctx.h, 1, meshes, ps, outs) == vls.VLS_E_INVALID_ARG
        srv = vls.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=4, slice_us=1000)
        try:
            tk = C.c_uint64()
            assert vls.vls_server_submit(srv.h, M.h, C.byref(p), C.byref(tk)) == vls.VLS_E_INVALID_ARG
        finally:
            srv.close()
    finally:
        M.close()
        ctx.close()


def test_refined_pass_with_the_finite_element_operator(oracle_mod):
    """The second pass inherits the field operator: with VLS_FEM_LAPLACIAN
    both passes equal the oracle's finite-element runs."""
    import paper_2105_13168_amd as vls
    m = mg.relaxed(mg.pretzel(32, rng_seed=2), mg.pretzel_sdf(), 10)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE | vls.VLS_FEM_LAPLACIAN)
    finally:
        M.close()
        ctx.close()
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed, fem=1)
    assert not compare(g, first, m.nv)
    assert second is not None and g.refined is not None
    assert second.n_handles == 3
    bad = compare(g.refined, second, m.nv)
    assert not bad, bad


@pytest.mark.parametrize("radius", [0, 1, 3])
def test_refined_pass_seed_radius(oracle_mod, radius):
    """The seed radius sets how far the second pass's initial region reaches
    around the loop's inside vertices (0: the vertices themselves); the
    result equals the oracle's for each."""
    import paper_2105_13168_amd as vls
    m = mg.multi_torus(2, 28, rng_seed=3)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE, seed_radius=radius, raise_on_error=False)
    finally:
        M.close()
        ctx.close()
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed, seed_radius=radius)
    assert not compare(g, first, m.nv)
    if second is None:
        assert g.refined is None
        return
    assert g.refined is not None
    bad = compare(g.refined, second, m.nv)
    assert not bad, bad


@pytest.mark.parametrize("variant", ["VLS_TOPO_GLOBAL_PATH", "VLS_DENSE_FIELD", "VLS_LOCKSTEP", "VLS_COHERENT_SHARING"])
def test_refined_pass_kernel_variants(oracle_mod, variant):
    """The second pass runs with the first pass's kernel variant (global
    topology path, dense field step, lockstep, coherent sharing); every
    variant gives the oracle's result."""
    import paper_2105_13168_amd as vls
    m = mg.pretzel(40, rng_seed=5)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE | getattr(vls, variant))
    finally:
        M.close()
        ctx.close()
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed)
    assert not compare(g, first, m.nv)
    assert g.refined is not None
    bad = compare(g.refined, second, m.nv)
    assert not bad, (variant, bad)
