"""Writes tests/golden/oracle_summaries.json from the CPU oracle only.

Run from the repository root:  python -m tests.golden.make_golden
or:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import meshgen as mg  # noqa: E402

CASES = {
    "torus64x32_s0": lambda: mg.torus_grid(rng_seed=0),
    "torus64x32_s1": lambda: mg.torus_grid(rng_seed=1),
    "torus64x32_s2": lambda: mg.torus_grid(rng_seed=2),
    "double_torus32_s0": lambda: mg.multi_torus(2, 32, rng_seed=0),
    "pretzel48_s0": lambda: mg.pretzel(48, rng_seed=0),
}


def summarize(r):
    ev = r.events
    return {
        "status": int(r.status),
        "steps": int(r.steps),
        "n_events": int(r.n_events),
        "n_handles": int(r.n_handles),
        "genus": int(r.genus),
        "event_types": [int(x) for x in ev[:, 2]] if r.n_events else [],
        "event_steps": [int(x) for x in ev[:, 0]] if r.n_events else [],
        "event_vertices": [int(x) for x in ev[:, 1]] if r.n_events else [],
        "handle_lengths": [round(float(h[4]), 12) for h in r.handle_loops()],
        "tunnel_sizes": [int(len(t)) for t in r.tunnel_loops()],
    }


# full-size workloads: digests of every output plus sampled values
FULL_CASES = {
    "pretzel256_s0": lambda: mg.pretzel(256, rng_seed=0),
}


def main(full: bool = True):
    import oracle
    oracle.build(force=False)
    out = {}
    for name, make in CASES.items():
        m = make()
        r = oracle.run(m.xyz, m.tri, seed_vertex=m.seed)
        out[name] = summarize(r)
    with open(os.path.join(HERE, "oracle_summaries.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    if not full:
        return
    sys.path.insert(0, os.path.dirname(HERE))
    from _digest import canon_oracle, digests
    full_out = {}
    for name, make in FULL_CASES.items():
        m = make()
        r = oracle.run(m.xyz, m.tri, seed_vertex=m.seed)
        d = digests(canon_oracle(r))
        d["nv"] = int(m.nv)
        d["seed_vertex"] = int(m.seed)
        full_out[name] = d
    with open(os.path.join(HERE, "oracle_full.json"), "w") as f:
        json.dump(full_out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(full="--no-full" not in sys.argv)
