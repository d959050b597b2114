"""Canonical form of a run's outputs (oracle or HIP result) and its digests,
for parity at sizes where storing every value as a fixture is not sensible:
a committed script records the oracle's digests plus sampled values, and a
GPU test recomputes the same digests from the HIP path's result."""
from __future__ import annotations

import hashlib

import numpy as np

_I64MAX = np.iinfo(np.int64).max
_I32MAX = np.iinfo(np.int32).max


def _h(parts) -> str:
    h = hashlib.sha256()
    for a in parts:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def canon_oracle(o) -> dict:
    loops = []
    for i, (ev, fid, kept, off, cnt, _av) in enumerate(o.loops):
        loops.append((np.array([ev, fid, kept], dtype="<i8"), o.loop_he[off:off + cnt].astype("<i8"),
                      o.loop_pts[off:off + cnt].astype("<f8"), np.array([o.loop_len[i]], dtype="<f8")))
    return dict(
        steps=int(o.steps), status=int(o.status), n_events=int(o.n_events), n_handles=int(o.n_handles),
        T=np.where(o.T == _I64MAX, -1, o.T).astype("<i8"), rnd=o.rnd.astype("<i8"),
        parent=o.parent.astype("<i8"), rho=o.rho.astype("<f8"),
        events=o.events[:, :11].astype("<i8"),
        fronts=[np.concatenate([np.asarray(a, "<i8"), np.asarray(b, "<i8")]) for a, b in zip(o.event_in, o.event_out)],
        reeb_pos=np.asarray(o.event_pos, "<f8").reshape(-1, 3),
        reeb_edges=np.array([(int(o.front_birth[f]), int(o.front_death[f]), f) for f in range(o.front_birth.size)],
                            dtype="<i8").reshape(-1, 3),
        loops=loops, tunnels=[np.asarray(t, "<i8") for t in o.tunnel_loops()])


def canon_gpu(g) -> dict:
    s = g.summary
    loops = []
    for lp in g.loops:
        loops.append((np.array([lp["event"], lp["front_id"], int(lp["kept"])], dtype="<i8"),
                      np.asarray(lp["he"], "<i8"), np.asarray(lp["pts"], "<f8"),
                      np.array([lp["length"]], dtype="<f8")))
    step = g.step.astype(np.int64)
    return dict(
        steps=int(s["steps"]), status=int(s["run_status"]), n_events=int(s["n_events"]),
        n_handles=int(s["n_handles"]),
        T=np.where(step == _I32MAX, -1, step).astype("<i8"), rnd=g.round.astype("<i8"),
        parent=g.parent.astype("<i8"), rho=g.rho.astype("<f8"),
        events=g.events[:, :11].astype("<i8"),
        fronts=[np.concatenate([np.asarray(a, "<i8"), np.asarray(b, "<i8")]) for a, b in zip(g.event_in, g.event_out)],
        reeb_pos=np.array([n[6:9] for n in g.reeb_nodes[1:]], dtype="<f8").reshape(-1, 3),
        reeb_edges=np.array([tuple(e) for e in g.reeb_edges], dtype="<i8").reshape(-1, 3),
        loops=loops, tunnels=[np.asarray(t, "<i8") for t in g.tunnels])


def sample_index(nv: int, k: int = 2000, seed: int = 12345) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(nv, size=min(k, nv), replace=False))


def digests(c: dict) -> dict:
    """sha256 per output plus counts and per-vertex samples (rho as hex)."""
    idx = sample_index(c["T"].size)
    return dict(
        steps=c["steps"], status=c["status"], n_events=c["n_events"], n_handles=c["n_handles"],
        n_loops=len(c["loops"]), n_tunnels=len(c["tunnels"]),
        T=_h([c["T"]]), rnd=_h([c["rnd"]]), parent=_h([c["parent"]]), rho=_h([c["rho"]]),
        events=_h([c["events"]]), fronts=_h(c["fronts"]), reeb_pos=_h([c["reeb_pos"]]),
        reeb_edges=_h([c["reeb_edges"]]), loops=_h([x for lp in c["loops"] for x in lp]),
        tunnels=_h(c["tunnels"]),
        sample_idx=idx.tolist(), sample_T=c["T"][idx].tolist(), sample_parent=c["parent"][idx].tolist(),
        sample_rho=[float(x).hex() for x in c["rho"][idx]],
        loop_lengths=[float(lp[3][0]).hex() for lp in c["loops"]])
