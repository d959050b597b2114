"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on
the same seeded inputs, element by element.

Bars (stated in tests/_parity.py): integer, index and topology outputs
bit-exact; the FP64 field within 1e-12 and, since both sides evaluate the
same expressions in the same order without contraction, bit-identical, as
are crossing points, loop lengths and Reeb node positions.
"""
import numpy as np
import pytest

import meshgen as mg
from _parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2105_13168_amd as vls
    c = vls.Context(0)
    yield c
    c.close()


def _run_both(ctx, oracle_mod, m, ck=(), **kw):
    import paper_2105_13168_amd as vls
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, ckpt_steps=ck, raise_on_error=False, **kw)
    finally:
        M.close()
    okw = {k: v for k, v in kw.items() if k not in ("grid", "flags")}
    o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, ckpt_steps=ck, **okw)
    return g, o


SMALL = [
    ("torus64x32_s0", lambda: mg.torus_grid(rng_seed=0), [1, 2, 4, 8, 16, 32, 64, 128, 250, 256, 450, 502]),
    ("torus64x32_s1", lambda: mg.torus_grid(rng_seed=1), [1, 100, 300]),
    ("torus64x32_s2", lambda: mg.torus_grid(rng_seed=2), [1, 500]),
    ("sphere16", lambda: mg.sdf_surface(mg.sdf_sphere(), (-1, -1, -1), (1, 1, 1), 16, 1e-4, 0), [1, 50]),
    ("box20", lambda: mg.sdf_surface(mg.sdf_box((1, .5, .3)), (-1, -.5, -.3), (1, .5, .3), 20, 1e-4, 3), [7]),
    ("double_torus32", lambda: mg.multi_torus(2, 32), [1, 500, 1000]),
    ("pretzel48", lambda: mg.pretzel(48), [1, 1000, 2000, 3000]),
    ("thin_strip400x6", lambda: mg.torus_grid(400, 6, R=10.0, r=0.2, jitter=1e-3, rng_seed=0), [1, 1000]),
    ("lattice2_40", lambda: mg.lattice(2, 40, rng_seed=1), [1, 700, 1500]),
    ("lattice3_48", lambda: mg.lattice(3, 48, rng_seed=0), [1, 1000, 2500]),
    # poles of degree 40: wide padded rows, wide link rows, the event path at
    # a large full link, and the one-tile-deep dense step
    ("uvsphere30x40", lambda: mg.uv_sphere(30, 40, rng_seed=0), [1, 60]),
]


@pytest.mark.parametrize("name,make,ck", SMALL, ids=[c[0] for c in SMALL])
def test_parity_small(ctx, oracle_mod, name, make, ck):
    m = make()
    g, o = _run_both(ctx, oracle_mod, m, ck)
    assert g.summary["run_status"] == 0
    bad = compare(g, o, m.nv)
    assert not bad, bad


@pytest.mark.parametrize("grid", [1, 2, 3, 17, 64])
def test_parity_independent_of_launch_shape(ctx, oracle_mod, grid):
    m = mg.multi_torus(2, 28, rng_seed=3)
    g, o = _run_both(ctx, oracle_mod, m, [1, 300, 900], grid=grid)
    assert g.summary["grid"] == grid
    bad = compare(g, o, m.nv)
    assert not bad, bad


@pytest.mark.parametrize("name,make,ck", SMALL[:1] + SMALL[5:7] + SMALL[10:11],
                         ids=["torus", "double_torus", "pretzel48", "uvsphere"])
def test_parity_global_topology_path(ctx, oracle_mod, name, make, ck):
    """The global-memory topology path (taken by steps with more than 1024
    crossers) forced on every step gives the same results."""
    import paper_2105_13168_amd as vls
    m = make()
    g, o = _run_both(ctx, oracle_mod, m, ck, flags=vls.VLS_TOPO_GLOBAL_PATH)
    bad = compare(g, o, m.nv)
    assert not bad, bad


@pytest.mark.parametrize("name,make,ck", [SMALL[0], SMALL[6]], ids=["torus", "pretzel48"])
def test_parity_coherent_sharing_variant(ctx, oracle_mod, name, make, ck):
    """Sharing data between workgroups through coherent atomic accesses and
    a release-only barrier gives the same results as the default (plain
    accesses, full fences)."""
    import paper_2105_13168_amd as vls
    m = make()
    g, o = _run_both(ctx, oracle_mod, m, ck, flags=vls.VLS_COHERENT_SHARING)
    bad = compare(g, o, m.nv)
    assert not bad, bad


@pytest.mark.parametrize("flags", ["lockstep", "lockstep+coherent", "coherent", "dense", "lockstep+dense",
                                   "dense+coherent"])
@pytest.mark.parametrize("name,make,ck", [SMALL[0], SMALL[6], SMALL[10]], ids=["torus", "pretzel48", "uvsphere"])
def test_parity_step_kernel_variants(ctx, oracle_mod, name, make, ck, flags):
    """The lockstep step kernel (one grid barrier per step, topology of step
    t beside the field of step t+1) and the decoupled default (the field
    runs ahead up to two steps, the topology follows each completed field
    step) give the same results, with either sharing mode, and so does the
    dense field step (every vertex each step instead of the update set)."""
    import paper_2105_13168_amd as vls
    f = 0
    if "lockstep" in flags:
        f |= vls.VLS_LOCKSTEP
    if "coherent" in flags:
        f |= vls.VLS_COHERENT_SHARING
    if "dense" in flags:
        f |= vls.VLS_DENSE_FIELD
    m = make()
    g, o = _run_both(ctx, oracle_mod, m, ck, flags=f)
    bad = compare(g, o, m.nv)
    assert not bad, bad


def test_parity_dt_literal_and_radius(ctx, oracle_mod):
    # literal dt = 0.25/dmax on a tiny torus; and a radius-1 / radius-3 seed
    m = mg.torus_grid(16, 8, R=1.0, r=0.4, jitter=1e-3, rng_seed=5)
    for kw in (dict(dt_mode=1), dict(seed_radius=1), dict(seed_radius=3)):
        g, o = _run_both(ctx, oracle_mod, m, [1, 10], **kw)
        bad = compare(g, o, m.nv)
        assert not bad, (kw, bad)


def test_error_paths(ctx, oracle_mod):
    import paper_2105_13168_amd as vls
    # seed region containing a handle
    m = mg.torus_grid(5, 4, R=1.0, r=0.3, jitter=0.0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    g = M.run(seed_vertex=0, raise_on_error=False)
    assert g.status == -6 and g.summary["run_status"] == -6
    M.close()
    # stall by step limit: partial results equal the oracle's
    m = mg.torus_grid()
    g, o = _run_both(ctx, oracle_mod, m, [5], max_steps=300)
    assert g.summary["run_status"] == -7 and o.status == -7
    assert not compare(g, o, m.nv)
    # invalid meshes are rejected at setup
    with pytest.raises(vls.VLSError):
        vls.Mesh(ctx, m.xyz, m.tri[1:])
    t = m.tri.copy()
    t[3] = t[3, ::-1]
    with pytest.raises(vls.VLSError):
        vls.Mesh(ctx, m.xyz, t)


# the method's rare event cases (found with the oracle on the CPU): 1-to-3
# splits at monkey saddles, a 3-way merge (two handle loops, the longest of
# three dropped) and a DEGENERATE node (a handle swept at one saddle of one
# front, extra cycle x = 1)
from test_oracle_edge_events import EDGE_CASES  # noqa: E402


@pytest.mark.parametrize("variant", ["default", "global_topology", "dense", "lockstep"])
@pytest.mark.parametrize("name,make,kw", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_parity_edge_events(ctx, oracle_mod, name, make, kw, variant):
    import paper_2105_13168_amd as vls
    flags = {"default": 0, "global_topology": vls.VLS_TOPO_GLOBAL_PATH, "dense": vls.VLS_DENSE_FIELD,
             "lockstep": vls.VLS_LOCKSTEP}[variant]
    m = make()
    seed = kw["seed_vertex"]
    rk = {k: v for k, v in kw.items() if k != "seed_vertex"}
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        o = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, **rk)
        ck = [1, max(1, o.steps // 2), o.steps]
        o = oracle_mod.run(m.xyz, m.tri, seed_vertex=seed, ckpt_steps=ck, **rk)
        g = M.run(seed_vertex=seed, ckpt_steps=ck, raise_on_error=False, flags=flags, **rk)
    finally:
        M.close()
    ev = o.events
    # the case occurs
    if name == "voxel_frame":
        assert ((ev[:, 4] == 3) & (ev[:, 2] == 2)).any() and ((ev[:, 3] == 3) & (ev[:, 5] == 3)).any()
    elif name == "csaszar7":
        assert (ev[:, 2] == 4).any()
    else:
        assert ((ev[:, 3] == 3) & (ev[:, 5] == 3)).any()
    assert g.summary["run_status"] == 0
    bad = compare(g, o, m.nv)
    assert not bad, bad
    assert g.summary["n_degenerate"] == int((ev[:, 2] == 4).sum())
