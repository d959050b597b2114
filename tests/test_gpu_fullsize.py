"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (default grid of vls_run).

* 256^3 pretzel (V = 2,188,952): every output's digest equals the oracle's
  (recorded by tests/golden/make_golden.py from the oracle alone), and the
  sampled per-vertex values match one by one; with the band-limited field
  step (the default) and with the dense one.
* 10^3-cell strut lattice on a 256^3 grid (V = 5,845,474, genus 2300): the
  oracle is not run at this size; properties that hold at any size are
  checked: every vertex inside, handle loops = tunnel loops = swept genus =
  Euler genus, one Reeb node per event plus the seed.
"""
import json
import os

import numpy as np
import pytest

import meshgen as mg
from _digest import canon_gpu, digests

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("field_step", ["band", "dense"])
def test_pretzel256_digests_match_oracle(field_step):
    import paper_2105_13168_amd as vls
    flags = vls.VLS_DENSE_FIELD if field_step == "dense" else 0
    gold = json.load(open(os.path.join(HERE, "golden", "oracle_full.json")))["pretzel256_s0"]
    m = mg.pretzel(256, rng_seed=0)
    assert m.nv == gold["nv"] and m.seed == gold["seed_vertex"]
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=flags)
        d = digests(canon_gpu(g))
    finally:
        M.close()
        ctx.close()
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


def test_lattice10_grid256_properties():
    import paper_2105_13168_amd as vls
    m = mg.lattice(10, 256, rng_seed=0)
    g_expect = mg.lattice_genus(10)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        r = M.run(seed_vertex=m.seed)
        s = r.summary
        assert s["run_status"] == 0
        assert s["euler_genus"] == g_expect
        assert s["n_inside"] == m.nv
        assert s["n_handles"] == g_expect and s["n_tunnels"] == g_expect
        assert s["swept_genus"] == g_expect
        assert len(r.reeb_nodes) == s["n_events"] + 1
        assert (r.step < np.iinfo(np.int32).max).all()
    finally:
        M.close()
        ctx.close()
