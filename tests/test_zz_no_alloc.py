"""The allocation-free entry point (vls_run_async_noalloc), through the C
ABI: its outputs equal those of vls_run_async on a caller workspace (the
entry point it is a variant of) and the oracle's, on two calls in a row,
the second with a smaller mesh; a call while the previous result is not yet
waited for is refused; a mesh beyond the static scratch is refused."""
import ctypes as C

import numpy as np
import pytest

import meshgen as mg
from _parity import compare

pytestmark = pytest.mark.gpu


def _params(vls, seed, ck):
    ck = np.ascontiguousarray(np.asarray(ck, dtype=np.int64))
    p = vls.default_params(seed_vertex=seed)
    if ck.size:
        p.flags |= vls.VLS_RECORD_FIELD
        p.n_ckpt = ck.size
        p.ckpt_steps = ck.ctypes.data_as(C.POINTER(C.c_int64))
    return p, ck


def test_noalloc_matches_workspace_path_and_oracle(oracle_mod):
    import torch
    import paper_2105_13168_amd as vls
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = vls.Context(0, stream=stream.cuda_stream)
    cases = [(mg.pretzel(48), [1, 1000, 3000]), (mg.torus_grid(rng_seed=2), [1, 250])]
    assert cases[1][0].nv < cases[0][0].nv            # the second call is smaller
    try:
        for m, ck in cases:
            M = vls.Mesh(ctx, m.xyz, m.tri)
            try:
                p, cka = _params(vls, m.seed, ck)
                need = C.c_size_t()
                assert vls.vls_workspace_size(M.h, C.byref(p), C.byref(need)) == 0
                assert need.value <= 64 << 20
                h = C.c_void_p()
                st = vls.vls_run_async_noalloc(ctx.h, M.h, C.byref(p), C.c_void_p(stream.cuda_stream), C.byref(h))
                assert st == 0, (st, ctx.last_error())
                # the array is held until this result is waited for
                h2 = C.c_void_p()
                st2 = vls.vls_run_async_noalloc(ctx.h, M.h, C.byref(p), None, C.byref(h2))
                assert st2 == vls.VLS_E_PENDING and not h2.value
                assert vls.vls_result_wait(h) == 0
                g = vls.Result(h, M, cka)
                # the existing entry point on a PyTorch workspace
                ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
                hw = C.c_void_p()
                st = vls.vls_run_async(ctx.h, M.h, C.byref(p), C.c_void_p(ws.data_ptr()), need, None, C.byref(hw))
                assert st == 0, (st, ctx.last_error())
                w = vls.Result(hw, M, cka)
                o = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, ckpt_steps=ck)
                bad = compare(g, o, m.nv)
                assert not bad, (m.name, bad)
                assert not compare(w, o, m.nv)
                assert np.array_equal(g.rho.view(np.int64), w.rho.view(np.int64))
                assert np.array_equal(g.events, w.events) and np.array_equal(g.parent, w.parent)
                for a, b in zip(g.tunnels, w.tunnels):
                    assert np.array_equal(a, b)
                del ws
            finally:
                M.close()
        # beyond the static scratch: refused, nothing launched
        big = mg.pretzel(160, rng_seed=0)
        M = vls.Mesh(ctx, big.xyz, big.tri)
        try:
            p, _ = _params(vls, big.seed, [])
            h = C.c_void_p()
            st = vls.vls_run_async_noalloc(ctx.h, M.h, C.byref(p), None, C.byref(h))
            assert st == vls.VLS_E_BUFFER_TOO_SMALL and not h.value
        finally:
            M.close()
    finally:
        ctx.close()
