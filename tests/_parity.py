"""Element-by-element comparison of a GPU run (paper_2105_13168_amd) with the
CPU oracle on the same seeded input.  Returns a list of mismatch strings
(empty = parity).

Bars: integer / index outputs bit-exact; FP64 field values, crossing points,
loop lengths and Reeb positions bit-exact as well (both sides evaluate the
same expressions in the same order without contraction) -- the field bar of
1e-12 is checked separately so that a failure says which bar broke.
"""
from __future__ import annotations

import numpy as np

FIELD_TOL = 1e-12


def _bits_equal(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def compare(g, o, nv) -> list[str]:
    """g: paper_2105_13168_amd.Result, o: oracle.OracleResult."""
    bad = []
    s = g.summary
    if s["run_status"] != o.status:
        bad.append(f"status gpu={s['run_status']} oracle={o.status}")
        return bad
    if s["steps"] != o.steps:
        bad.append(f"steps gpu={s['steps']} oracle={o.steps}")
    # insertion order
    T = np.where(o.T == np.iinfo(np.int64).max, np.iinfo(np.int32).max, o.T).astype(np.int64)
    if not np.array_equal(g.step.astype(np.int64), T):
        d = np.flatnonzero(g.step.astype(np.int64) != T)
        bad.append(f"insertion step differs at {d.size} vertices, first {d[:5].tolist()}")
    if not np.array_equal(g.round, o.rnd):
        d = np.flatnonzero(g.round != o.rnd)
        bad.append(f"closure round differs at {d.size} vertices")
    if not np.array_equal(g.parent, o.parent):
        d = np.flatnonzero(g.parent != o.parent)
        bad.append(f"parent differs at {d.size} vertices")
    # field
    err = float(np.max(np.abs(g.rho - o.rho))) if nv else 0.0
    if err > FIELD_TOL:
        bad.append(f"final field max |diff| = {err:.3e} > {FIELD_TOL}")
    elif not _bits_equal(g.rho, o.rho):
        bad.append(f"final field not bit-identical (max |diff| {err:.3e})")
    for st, a in o.ckpt.items():
        if st not in g.ckpt:
            bad.append(f"checkpoint {st} missing on GPU")
            continue
        e = float(np.max(np.abs(g.ckpt[st] - a)))
        if e > FIELD_TOL or not _bits_equal(g.ckpt[st], a):
            bad.append(f"checkpoint {st}: max |diff| {e:.3e}")
    # events (fields 0..10 are defined identically on both sides)
    ge, oe = g.events, o.events
    if ge.shape[0] != oe.shape[0]:
        bad.append(f"event count gpu={ge.shape[0]} oracle={oe.shape[0]}")
    else:
        for i in range(ge.shape[0]):
            if not np.array_equal(ge[i, :11], oe[i, :11]):
                bad.append(f"event {i}: gpu {ge[i, :11].tolist()} oracle {oe[i, :11].tolist()}")
                break
            if not (np.array_equal(g.event_in[i], o.event_in[i]) and np.array_equal(g.event_out[i], o.event_out[i])):
                bad.append(f"event {i} front ids: gpu {g.event_in[i]}->{g.event_out[i]} oracle {o.event_in[i]}->{o.event_out[i]}")
                break
        if ge.shape[0] and not _bits_equal(np.array([n[6:9] for n in g.reeb_nodes[1:]]), o.event_pos):
            d = np.max(np.abs(np.array([n[6:9] for n in g.reeb_nodes[1:]]) - o.event_pos))
            bad.append(f"Reeb node positions differ (max |diff| {d:.3e})")
    # Reeb edges
    oedges = [(int(o.front_birth[f]), int(o.front_death[f]), f) for f in range(o.front_birth.size)]
    if [tuple(e) for e in g.reeb_edges] != oedges:
        bad.append("Reeb edges differ")
    # merge loops (handle loops and the ignored longest one)
    ol = o.loops
    if len(g.loops) != ol.shape[0]:
        bad.append(f"loop count gpu={len(g.loops)} oracle={ol.shape[0]}")
    else:
        for i, gl in enumerate(g.loops):
            ev, fid, kept, off, cnt, av = (int(x) for x in ol[i])
            if (gl["event"], gl["front_id"], int(gl["kept"])) != (ev, fid, kept):
                bad.append(f"loop {i} header differs")
                continue
            ohe = o.loop_he[off:off + cnt]
            if not np.array_equal(gl["he"].astype(np.int64), ohe):
                bad.append(f"loop {i} edges differ")
                continue
            if not _bits_equal(gl["pts"], o.loop_pts[off:off + cnt]):
                bad.append(f"loop {i} points differ")
            if not _bits_equal(np.array([gl["length"]]), np.array([o.loop_len[i]])):
                bad.append(f"loop {i} length gpu {gl['length']!r} oracle {o.loop_len[i]!r}")
    # tunnels
    ot = o.tunnel_loops()
    if len(g.tunnels) != len(ot):
        bad.append(f"tunnel count gpu={len(g.tunnels)} oracle={len(ot)}")
    else:
        for i, (a, b) in enumerate(zip(g.tunnels, ot)):
            if not np.array_equal(a.astype(np.int64), b):
                bad.append(f"tunnel {i} differs")
    if s["n_handles"] != o.n_handles:
        bad.append(f"handles gpu={s['n_handles']} oracle={o.n_handles}")
    return bad
