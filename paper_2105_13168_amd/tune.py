"""Schedule tuner of the batched kernel.

A batch's schedule has two knobs:
- the pool shape: one workgroup per CU, with the 2048-candidate LDS topology
  path and two list entries per field thread; or two per CU, with half of
  each;
- the gang granularity: a mesh gets one workgroup per that many vertices.

``tune_batch`` times whole ``vls_batch_run`` calls (launch, kernels and
result handling, as a caller sees them) for every candidate on the meshes it
is given, typically a sample of the workload.  It returns the fastest, and
can cache the choice in a JSON file keyed by device and workload signature.
The results of every candidate are identical (the schedule changes no
arithmetic); only the time differs.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
import time

from . import (VLS_BATCH_TWO_PER_CU, VLS_DEFER_RESULTS, VLSError, default_params, vls_batch_run,
               vls_params, vls_result_destroy)

CANDIDATES = tuple((two, gv) for two in (False, True) for gv in (32768, 65536, 131072))


def signature(meshes, device_name: str = "") -> str:
    h = hashlib.sha256(device_name.encode())
    for m in sorted(int(x.nv) for x in meshes):
        h.update(m.to_bytes(8, "little"))
    return h.hexdigest()[:16]


def _run(ctx, meshes, seeds, two, gv):
    n = len(meshes)
    hm = (C.c_void_p * n)(*[m.h.value for m in meshes])
    ps = (vls_params * n)()
    for i in range(n):
        ps[i] = default_params(seed_vertex=int(seeds[i]),
                               flags=VLS_DEFER_RESULTS | (VLS_BATCH_TWO_PER_CU if two else 0),
                               gang_vertices=int(gv))
    outs = (C.c_void_p * n)()
    t0 = time.perf_counter()
    st = vls_batch_run(ctx.h, n, hm, ps, outs)
    dt = time.perf_counter() - t0
    for i in range(n):
        if outs[i]:
            vls_result_destroy(C.c_void_p(outs[i]))
    if st != 0:
        raise VLSError(st, ctx.last_error())
    return dt


def tune_batch(ctx, meshes, seeds, candidates=CANDIDATES, cache_path: str | None = None,
               device_name: str = "") -> dict:
    """Fastest (two_per_cu, gang_vertices) for this batch; uses and updates
    the cache at cache_path when given."""
    key = signature(meshes, device_name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    _run(ctx, meshes, seeds, False, 65536)            # warm-up: run buffers, first launch
    times = {}
    for two, gv in candidates:
        times[f"{'two' if two else 'one'}_per_cu/{gv}"] = _run(ctx, meshes, seeds, two, gv)
    best = min(times, key=times.get)
    shape, gv = best.split("/")
    out = {"two_per_cu": shape == "two_per_cu", "gang_vertices": int(gv), "seconds": times}
    if cache_path:
        cache[key] = out
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return out
