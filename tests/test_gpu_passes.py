"""GPU parity of the tunnel-loop and handle-refinement passes and of the
handle/tunnel label (Sections "Tunnel loop pass", "Handle refinement pass",
"Distinguishing handle and tunnel loops"): for every handle loop, the HIP
pass kernel's status, diffusion steps, vertex reached, closed loop (vertex
for vertex), length and offset length (bit for bit) and label equal the
oracle's, with many passes running at once and workgroups reusing their
per-vertex state from one pass to the next."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu

CASES = [
    ("torus_mt48", lambda: mg.sdf_surface(mg.sdf_torus(R=1.0, r=0.35), (-1.4, -1.4, -0.4), (1.4, 1.4, 0.4), 48,
                                          1e-4, 0), 0),
    ("torus40x20", lambda: mg.torus_grid(40, 20, R=1.0, r=0.4, jitter=1e-3, rng_seed=3), 0),
    ("double_torus28", lambda: mg.multi_torus(2, 28, rng_seed=3), 0),
    ("pretzel32", lambda: mg.pretzel(32, rng_seed=2), 0),
    # 28 handles on 3 workgroups: each workgroup runs about ten passes in turn
    ("lattice2_40_3slots", lambda: mg.lattice(2, 40, rng_seed=1), 3),
]


def _bits(x):
    return np.array([x], dtype=np.float64).view(np.int64)[0]


@pytest.mark.parametrize("name,make,slots", CASES, ids=[c[0] for c in CASES])
def test_passes_match_oracle(oracle_mod, name, make, slots):
    import paper_2105_13168_amd as vls
    from oracle import passes as P
    m = make()
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        g = M.run(seed_vertex=m.seed, flags=vls.VLS_REFINE_PASS, pass_slots=slots)
    finally:
        M.close()
        ctx.close()
    s = g.summary
    assert s["run_status"] == 0
    if slots:
        assert s["pass_slots"] == slots
    o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
    G = P.MeshGraph(m.xyz, m.tri)
    nrm = P.vertex_normals(G)
    kept = np.flatnonzero(o.loops[:, 2] == 1).tolist()
    assert s["n_tunnel_passes"] == len(kept) == s["n_refine_passes"] == o.n_handles
    for i, li in enumerate(kept):
        tp = P.tunnel_pass(G, o, li)
        hp = P.refine_pass(G, tp["cycle"]) if tp["status"] == 0 else None
        for kind, want in ((3, tp), (4, hp)):
            got = g.passes[kind][i]
            if want is None:
                assert got["status"] != 0
                continue
            assert got["status"] == want["status"], (kind, i, got["status"], want["status"])
            assert got["steps"] == want["steps"], (kind, i, got["steps"], want["steps"])
            assert got["reached"] == want["reached"], (kind, i)
            if want["status"] != 0:
                continue
            assert got["cycle"].tolist() == want["cycle"], (kind, i)
            assert _bits(got["length"]) == _bits(want["length"]), (kind, i)
            label, L0, L1 = P.offset_label(G, want["cycle"], nrm)
            assert _bits(L0) == _bits(got["length"])
            assert _bits(L1) == _bits(got["offset_length"]), (kind, i, L1, got["offset_length"])
            assert got["label"] == (0 if label == "handle" else 1)
    assert s["n_tunnel_loops"] == sum(p["status"] == 0 for p in g.passes[3])


def test_passes_only_through_vls_run():
    import ctypes as C
    import paper_2105_13168_amd as vls
    m = mg.torus_grid(rng_seed=0)
    ctx = vls.Context(0)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    try:
        with pytest.raises(vls.VLSError):
            vls.batch_run(ctx, [M], [m.seed], flags=vls.VLS_TUNNEL_PASS)
        p = vls.default_params(seed_vertex=m.seed, flags=vls.VLS_TUNNEL_PASS)
        need = C.c_size_t()
        vls.vls_workspace_size(M.h, C.byref(p), C.byref(need))
        h = C.c_void_p()
        assert vls.vls_run_async(ctx.h, M.h, C.byref(p), None, need, None, C.byref(h)) == vls.VLS_E_INVALID_ARG
    finally:
        M.close()
        ctx.close()
