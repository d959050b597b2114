"""Writes tests/golden/oracle_summaries.json and oracle_full.json from the
CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
  --no-full          small summaries only
  --full NAME ...    recompute only the named full-size cases and merge them
                     into oracle_full.json (the lattice cases take minutes to
                     hours of one core each)
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
    # the 10^3-cell strut lattice (genus 2300) on 256^3 and 512^3 grids
    "lattice10_256_s0": lambda: mg.lattice(10, 256, rng_seed=0),
    "lattice10_512_s0": lambda: mg.lattice(10, 512, rng_seed=0),
    # the full-size lattice (1024^3 grid, about 95M vertices)
    "lattice10_1024_s0": lambda: mg.lattice(10, 1024, rng_seed=0),
    # the finite-element operator variant on a relaxed 128^3 pretzel
    "pretzel128_relaxed_fem_s0": (lambda: mg.relaxed(mg.pretzel(128, rng_seed=0), mg.pretzel_sdf(), 10),
                                  {"fem": 1}),
    # the Reeb junction refinement's second pass (from the first kept handle
    # loop of the ordinary pass): digests of that second pass
    "pretzel256_refined_s0": (lambda: mg.pretzel(256, rng_seed=0), {"reeb_refine": 1}),
    "lattice10_256_refined_s0": (lambda: mg.lattice(10, 256, rng_seed=0), {"reeb_refine": 1}),
    "lattice10_512_refined_s0": (lambda: mg.lattice(10, 512, rng_seed=0), {"reeb_refine": 1}),
}


def xyz_digest(xyz) -> str:
    import hashlib
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(xyz, dtype=np.float64).tobytes()).hexdigest()


def main(full: bool = True, only=None):
    import gc
    import time
    import oracle
    oracle.build(force=False)
    if not only:
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
    path = os.path.join(HERE, "oracle_full.json")
    full_out = json.load(open(path)) if (only and os.path.exists(path)) else {}
    for name, case in FULL_CASES.items():
        if only and name not in only:
            continue
        make, kw = case if isinstance(case, tuple) else (case, {})
        t0 = time.time()
        m = make()
        t1 = time.time()
        if kw.get("reeb_refine"):
            _first, r = oracle.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed)
        else:
            r = oracle.run(m.xyz, m.tri, seed_vertex=m.seed, **kw)
        t2 = time.time()
        d = digests(canon_oracle(r))
        if kw.get("reeb_refine"):
            d["refined_seed_vertex"] = int(oracle.refinement_seed_set(_first)[0])
            d["run_kwargs"] = kw
        elif kw:
            d["run_kwargs"] = kw
            d["xyz_sha256"] = xyz_digest(m.xyz)
        d["nv"] = int(m.nv)
        d["nf"] = int(m.nf)
        d["seed_vertex"] = int(m.seed)
        d["oracle_seconds"] = round(t2 - t1, 1)
        full_out[name] = d
        print(f"{name}: nv={m.nv} steps={r.steps} events={r.n_events} handles={r.n_handles} "
              f"mesh {t1 - t0:.0f} s, oracle {t2 - t1:.0f} s", flush=True)
        del m, r
        gc.collect()
        # written after every case: a later case may take hours
        with open(path, "w") as f:
            json.dump(full_out, f, indent=1, sort_keys=True)


# the batched workload (1024 uneven meshes, base seed 0): one combined
# digest of every output per mesh
BATCH_FIELDS = ("steps", "status", "n_events", "n_handles", "n_loops", "n_tunnels", "T", "rnd", "parent", "rho",
                "events", "fronts", "reeb_pos", "reeb_edges", "loops", "tunnels")
_BATCH = None


def combined_digest(d: dict) -> str:
    import hashlib
    return hashlib.sha256(json.dumps([d[k] for k in BATCH_FIELDS]).encode()).hexdigest()


def _batch_one(i):
    import oracle
    sys.path.insert(0, os.path.dirname(HERE))
    from _digest import canon_oracle, digests
    m = _BATCH[i]
    r = oracle.run(m.xyz, m.tri, seed_vertex=m.seed)
    d = digests(canon_oracle(r))
    return {"nv": int(m.nv), "seed_vertex": int(m.seed), "steps": d["steps"], "n_events": d["n_events"],
            "n_handles": d["n_handles"], "digest": combined_digest(d)}


def main_batch(n=1024, workers=6):
    import multiprocessing as mp
    import time
    import oracle
    global _BATCH
    oracle.build(force=False)
    t0 = time.time()
    _BATCH = mg.batch_workload(n, base_seed=0)
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_batch_one, range(n), chunksize=4)
    with open(os.path.join(HERE, "oracle_batch1024.json"), "w") as f:
        json.dump({"base_seed": 0, "meshes": out}, f, indent=0)
    print(f"batch digests: {n} meshes, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    argv = sys.argv[1:]
    if "--batch" in argv:
        main_batch()
        sys.exit(0)
    only = argv[argv.index("--full") + 1:] if "--full" in argv else None
    main(full="--no-full" not in argv, only=only)
