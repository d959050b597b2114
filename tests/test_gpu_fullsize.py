"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (default grid of vls_run): every output's digest equals the oracle's
(recorded by tests/golden/make_golden.py from the oracle alone), and the
sampled per-vertex values match one by one.

* 256^3 pretzel (V = 2,188,952), with the band-limited field step (the
  default) and with the dense one.
* the 10^3-cell strut lattice (genus 2300) on 256^3, 512^3 and 1024^3 grids
  (V = 5.8M, 23.8M, 95.3M); besides the digests, properties that hold at
  any size: every vertex inside, handle loops = tunnel loops = swept genus
  = Euler genus, one Reeb node per event plus the seed.
"""
import json
import os

import numpy as np
import pytest

import meshgen as mg
from _digest import canon_gpu, digests

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_full.json")))


def _check(d, gold):
    # sampled values first (a mismatch there says where)
    idx = np.array(gold["sample_idx"])
    assert d["sample_idx"] == gold["sample_idx"]
    bad_T = np.flatnonzero(np.array(d["sample_T"]) != np.array(gold["sample_T"]))
    assert bad_T.size == 0, f"insertion step differs at vertices {idx[bad_T][:10].tolist()}"
    rg = np.array([float.fromhex(x) for x in d["sample_rho"]])
    ro = np.array([float.fromhex(x) for x in gold["sample_rho"]])
    assert np.max(np.abs(rg - ro)) <= 1e-12
    for k in ("steps", "status", "n_events", "n_handles", "n_loops", "n_tunnels", "sample_parent",
              "sample_rho", "loop_lengths", "T", "rnd", "parent", "rho", "events", "fronts", "reeb_pos",
              "reeb_edges", "loops", "tunnels"):
        assert d[k] == gold[k], k


def _run(m, flags=0):
    import paper_2105_13168_amd as vls
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=flags)
        return g, digests(canon_gpu(g))
    finally:
        M.close()
        ctx.close()


@pytest.mark.parametrize("field_step", ["band", "dense"])
def test_pretzel256_digests_match_oracle(field_step):
    import paper_2105_13168_amd as vls
    gold = GOLD["pretzel256_s0"]
    m = mg.pretzel(256, rng_seed=0)
    assert m.nv == gold["nv"] and m.seed == gold["seed_vertex"]
    _g, d = _run(m, vls.VLS_DENSE_FIELD if field_step == "dense" else 0)
    _check(d, gold)


@pytest.mark.parametrize("grid", [256, 512, 1024])
def test_lattice10_digests_match_oracle(grid):
    name = f"lattice10_{grid}_s0"
    if name not in GOLD:
        pytest.skip(f"no oracle digest recorded for {name} (tests/golden/make_golden.py --full {name})")
    gold = GOLD[name]
    m = mg.lattice(10, grid, rng_seed=0)
    assert m.nv == gold["nv"] and m.seed == gold["seed_vertex"]
    g_expect = mg.lattice_genus(10)
    g, d = _run(m)
    s = g.summary
    assert s["run_status"] == 0
    assert s["euler_genus"] == g_expect and s["swept_genus"] == g_expect
    assert s["n_inside"] == m.nv
    assert s["n_handles"] == g_expect and s["n_tunnels"] == g_expect
    assert len(g.reeb_nodes) == s["n_events"] + 1
    _check(d, gold)


def test_pretzel128_relaxed_fem_digests_match_oracle():
    """The finite-element operator variant at the largest size the oracle
    finishes in minutes: the relaxed 128^3 pretzel (the explicit step of the
    cotangent operator is tens of times shorter than the graph Laplacian's,
    so the pass takes that many more steps)."""
    import paper_2105_13168_amd as vls
    name = "pretzel128_relaxed_fem_s0"
    if name not in GOLD:
        pytest.skip(f"no oracle digest recorded for {name} (tests/golden/make_golden.py --full {name})")
    gold = GOLD[name]
    m = mg.relaxed(mg.pretzel(128, rng_seed=0), mg.pretzel_sdf(), 10)
    from golden.make_golden import xyz_digest
    assert xyz_digest(m.xyz) == gold["xyz_sha256"], "relaxed mesh differs from the one the digests were taken on"
    assert m.nv == gold["nv"] and m.seed == gold["seed_vertex"]
    g, d = _run(m, vls.VLS_FEM_LAPLACIAN)
    s = g.summary
    assert s["run_status"] == 0 and s["n_handles"] == 3 and s["n_tunnels"] == 3
    _check(d, gold)


@pytest.mark.parametrize("name,make", [
    ("pretzel256_refined_s0", lambda: mg.pretzel(256, rng_seed=0)),
    ("lattice10_256_refined_s0", lambda: mg.lattice(10, 256, rng_seed=0)),
    ("lattice10_512_refined_s0", lambda: mg.lattice(10, 512, rng_seed=0)),
])
def test_reeb_refined_pass_digests_match_oracle(name, make):
    """The Reeb junction refinement's second pass at full size: started from
    the first kept handle loop of the ordinary pass, every output of that
    pass equals the oracle's."""
    import paper_2105_13168_amd as vls
    if name not in GOLD:
        pytest.skip(f"no oracle digest recorded for {name} (tests/golden/make_golden.py --full {name})")
    gold = GOLD[name]
    m = make()
    assert m.nv == gold["nv"] and m.seed == gold["seed_vertex"]
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE)
    finally:
        M.close()
        ctx.close()
    assert g.refined is not None
    assert g.refined.summary["seed_vertex"] == gold["refined_seed_vertex"]
    _check(digests(canon_gpu(g.refined)), gold)
