"""Benchmark of the initial pass of the variational loop-shrinking method on
one MI355X.

A "step" here is one complete initial pass over the workload: seed region,
every diffusion step until the front has swept the whole surface (field,
threshold + closure, lower-link classification, front tags, split / merge /
vanish events with handle loops), then the Reeb-position and tunnel
post-passes.  The default workload is the full-size strut lattice: 10^3
cells of unit struts of radius 0.15 (genus 2300), level-0 surface on a
1024^3 sample grid (95.3M vertices, 190.5M triangles), seed vertex from rng
seed 0, with its mesh uploaded to HBM before the timed region.  Bulk
results stay on the device (deferred), so the timed region holds no result
download.

Extra keys: the 256^3 pretzel pass, the dense field step on the same
lattice, the batch of 1024 uneven meshes, the serving trace.  They run only
while the run stays within --time-budget seconds.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1]

Prints one JSON line.
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import meshgen as mg
    if name == "pretzel256":
        m = mg.pretzel(256, rng_seed=0)
        desc = "genus-3 pretzel, level-0 surface of three tori SDFs on a 256^3 grid (marching tetrahedra)"
    elif name == "pretzel128_relaxed":
        m = mg.relaxed(mg.pretzel(128, rng_seed=0), mg.pretzel_sdf(), 10)
        desc = ("genus-3 pretzel on a 128^3 grid (marching tetrahedra), relaxed: ten rounds of moving each vertex "
                "halfway to its neighbours' mean and projecting back onto the surface")
    elif name == "torus64x32":
        m = mg.torus_grid(rng_seed=0)
        desc = "64x32 torus grid, R=1, r=0.4"
    elif name.startswith("lattice10_"):
        grid = int(name.split("_")[1])
        m = mg.lattice(10, grid, rng_seed=0, progress=log)
        desc = (f"strut lattice, 10^3 cells (3630 struts of radius 0.15, genus 2300), level-0 surface on a "
                f"{grid}^3 grid over [-0.5, 10.5]^3 (marching tetrahedra), random seed vertex")
    else:
        raise SystemExit(f"unknown workload {name}")
    return m, desc


def alg_bytes(updates, degsum):
    # per updated vertex: read rho(v) 8 + write rho(v) 8 + two row offsets 8
    # + update-list entry in/out 8, plus 4 bytes per neighbour id
    return 32 * updates + 4 * degsum


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("vls_kernels.hip", "vls_internal.h"):
        with open(os.path.join(ROOT, "paper_2105_13168_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_ms, workload, steps=None, grid=None):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    runs (FETCH_SIZE, WRITE_SIZE scaled by a copy of known size), as GB/s over
    the live kernel time; None when the counters were taken on another
    workload, another number of steps, another grid or other kernel
    sources.  `workload` names the record (k_steps_<workload>_traffic.json)."""
    path = os.path.join(ROOT, "profiles", f"k_steps_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if steps is not None and t.get("diffusion_steps") != steps:
        return None
    if grid is not None and t.get("grid") != grid:
        return None
    return t["hbm_bytes_per_launch"] / (kernel_ms * 1e-3) / 1e9


def copy_calibration(nbytes=1 << 30):
    """One plain device-to-device copy of nbytes (a kernel of known traffic
    for scaling the HBM counters)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes read and written")


def dense_alg_bytes(updates, degsum):
    # per vertex of a dense step: read rho(v) 8 + write rho(v) 8 + one row
    # offset 4 (consecutive vertices share their row bounds: a tile of n
    # vertices reads n+1 offsets), plus 4 bytes per neighbour id (no update
    # list)
    return 20 * updates + 4 * degsum


def dense_leg(ctx, workload, steps, mesh=None):
    """The dense field step (every vertex each step) on a mesh whose working
    set is far beyond the caches, run for a fixed number of diffusion steps
    with the topology beside it, against the band-stepped default for the
    same steps; HBM share from the algorithmic bytes of a dense step.
    mesh = (generator mesh, uploaded Mesh, description) reuses a mesh that is
    already on the device."""
    import ctypes as C
    import paper_2105_13168_amd as vls
    t0 = time.time()
    if mesh is None:
        m, desc = make_workload(workload)
        M = vls.Mesh(ctx, m.xyz, m.tri)
        own = True
    else:
        m, M, desc = mesh
        own = False
    log(f"dense leg: {workload} V={m.nv} ({time.time() - t0:.1f}s)")

    def run(flags, k):
        p = vls.default_params(seed_vertex=m.seed, flags=vls.VLS_DEFER_RESULTS | flags, max_steps=k)
        h = C.c_void_p()
        st = vls.vls_run(ctx.h, M.h, C.byref(p), C.byref(h))
        if st not in (0, vls.VLS_E_STALLED) or not h:
            raise vls.VLSError(st, ctx.last_error())
        s = vls.vls_summary()
        vls.vls_result_summary(h, C.byref(s))
        vls.vls_result_destroy(h)
        out = {f: getattr(s, f) for f, _ in vls.vls_summary._fields_}
        assert out["steps"] == k, (out["steps"], k)
        return out

    run(vls.VLS_DENSE_FIELD, min(steps, 20))
    d = run(vls.VLS_DENSE_FIELD, steps)
    b = run(0, steps)
    assert d["n_inside"] == b["n_inside"] and d["n_events"] == b["n_events"]
    ab = dense_alg_bytes(d["active_vertex_updates"], d["active_degree_sum"])
    achieved = ab / (d["kernel_ms"] * 1e-3) / 1e9
    res = {
        "workload": desc, "nv": m.nv, "nf": m.nf, "diffusion_steps": steps,
        "grid": d["grid"], "ms_per_dense_step": d["kernel_ms"] / steps,
        "vertex_steps_per_s": m.nv * steps / (d["kernel_ms"] * 1e-3),
        "algorithmic_bytes_per_step": ab / steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(d["kernel_ms"], f"dense_{workload}", steps, grid=d["grid"]),
                     "kernel": "k_steps_dec (dense field)"},
        "band_ms_per_step": b["kernel_ms"] / steps,
        "band_updates_per_step": b["active_vertex_updates"] / steps,
        "same_front": True,
    }
    if own:
        M.close()
    return res


def fem_alg_bytes(updates, degsum):
    # the update-list step's bytes plus, per updated vertex, its row offset
    # 4 and, per neighbour, the operator coefficient 8
    return 36 * updates + 12 * degsum


def pass_leg(ctx, workload, steps, fem=False):
    """Whole initial passes of another workload (timed passes after a
    warm-up), as the main line measures its own; fem: with the
    finite-element operator (prepared once, outside the timed passes)."""
    import ctypes as C
    import torch
    import paper_2105_13168_amd as vls
    m, desc = make_workload(workload)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    flags = vls.VLS_DEFER_RESULTS
    fem_info = None
    if fem:
        t0 = time.perf_counter()
        sigma, rowmax = M.prepare_fem()
        fem_info = {"prepare_s": time.perf_counter() - t0, "sigma": sigma, "row_sum_max": rowmax,
                    "max_degree": M.dmax}
        flags |= vls.VLS_FEM_LAPLACIAN
    p = vls.default_params(seed_vertex=m.seed, flags=flags)
    sums, ms = [], []
    for k in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = C.c_void_p()
        st = vls.vls_run(ctx.h, M.h, C.byref(p), C.byref(h))
        if st != 0:
            raise vls.VLSError(st, ctx.last_error())
        s = vls.vls_summary()
        vls.vls_result_summary(h, C.byref(s))
        vls.vls_result_destroy(h)
        torch.cuda.synchronize()
        if k:
            ms.append((time.perf_counter() - t0) * 1e3)
            sums.append({f: getattr(s, f) for f, _ in vls.vls_summary._fields_})
    M.close()
    last = sums[-1]
    kernel_ms = sum(x["kernel_ms"] for x in sums) / len(sums)
    ab = (fem_alg_bytes if fem else alg_bytes)(last["active_vertex_updates"], last["active_degree_sum"])
    assert last["n_handles"] == last["euler_genus"]
    extra = {}
    if fem:
        extra["operator"] = fem_info
        extra["field_operator"] = "cotangent finite elements (VLS_FEM_LAPLACIAN)"
        try:
            with open(os.path.join(ROOT, "tests", "golden", "oracle_full.json")) as f:
                extra["oracle_whole_pass_seconds_recorded"] = json.load(f)[workload + "_fem_s0"]["oracle_seconds"]
        except (OSError, KeyError, ValueError):
            pass
    return {**extra, "workload": desc, "nv": m.nv, "nf": m.nf, "diffusion_steps": last["steps"],
            "events": last["n_events"], "handles": last["n_handles"], "ms_per_pass": sum(ms) / len(ms),
            "step_kernel_ms": kernel_ms, "vertex_steps_per_s": m.nv * last["steps"] / (sum(ms) / len(ms) * 1e-3),
            "roofline": {"bound": "hbm", "achieved": ab / (kernel_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS,
                         "unit": "GB/s", "frac": ab / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                         "traffic": None if fem else measured_traffic(kernel_ms, workload, grid=last["grid"]),
                         "kernel": "k_steps_dec<0, true>" if fem else "k_steps_dec"}}


def refine_leg(ctx, workload):
    """The Reeb junction refinement (VLS_REEB_REFINE): the ordinary pass,
    then the initial pass again from its first kept handle loop; one
    warm-up run, one timed run.  Reports both passes' step kernels and the
    second pass's algorithmic bandwidth."""
    import ctypes as C
    import torch
    import paper_2105_13168_amd as vls
    m, desc = make_workload(workload)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    p = vls.default_params(seed_vertex=m.seed, flags=vls.VLS_REEB_REFINE)
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = C.c_void_p()
        st = vls.vls_run(ctx.h, M.h, C.byref(p), C.byref(h))
        if st != 0:
            raise vls.VLSError(st, ctx.last_error())
        wall = (time.perf_counter() - t0) * 1e3
        h2 = C.c_void_p()
        vls.vls_result_refined(h, C.byref(h2))
        s1, s2 = vls.vls_summary(), vls.vls_summary()
        vls.vls_result_summary(h, C.byref(s1))
        vls.vls_result_summary(h2, C.byref(s2))
        vls.vls_result_destroy(h)
    M.close()
    first = {f: getattr(s1, f) for f, _ in vls.vls_summary._fields_}
    second = {f: getattr(s2, f) for f, _ in vls.vls_summary._fields_}
    assert second["n_handles"] == second["euler_genus"] == first["n_handles"]
    ab = alg_bytes(second["active_vertex_updates"], second["active_degree_sum"])
    return {"workload": desc, "nv": m.nv, "ms_both_passes": wall,
            "first_pass": {"diffusion_steps": first["steps"], "events": first["n_events"],
                           "step_kernel_ms": first["kernel_ms"]},
            "second_pass": {"root_vertex": second["seed_vertex"], "diffusion_steps": second["steps"],
                            "events": second["n_events"], "handles": second["n_handles"],
                            "reeb_nodes": second["reeb_nodes"], "step_kernel_ms": second["kernel_ms"],
                            "roofline": {"bound": "hbm", "achieved": ab / (second["kernel_ms"] * 1e-3) / 1e9,
                                         "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                         "frac": ab / (second["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                         "traffic": None, "kernel": "k_steps_dec"}}}


def batch_leg(ctx, n, seq_sample, tune=False):
    """Batch of n uneven meshes in one launch (one workgroup per mesh)
    against the same meshes run one at a time (default launch) on a sample,
    as meshes per second."""
    import ctypes as C
    import meshgen as mg
    import paper_2105_13168_amd as vls
    import torch
    t0 = time.time()
    ms = mg.batch_workload(n, base_seed=0)
    log(f"batch workload: {n} meshes, sum V = {sum(m.nv for m in ms)} ({time.time() - t0:.1f}s)")
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in ms]
    genus = [x.euler_genus for x in M]

    def run_batch(idx, extra=0, gv=0):
        hm = (C.c_void_p * len(idx))(*[M[i].h.value for i in idx])
        ps = (vls.vls_params * len(idx))()
        for k, i in enumerate(idx):
            ps[k] = vls.default_params(seed_vertex=ms[i].seed, flags=vls.VLS_DEFER_RESULTS | extra,
                                       gang_vertices=gv)
        outs = (C.c_void_p * len(idx))()
        st = vls.vls_batch_run(ctx.h, len(idx), hm, ps, outs)
        sums = []
        for k in range(len(idx)):
            s = vls.vls_summary()
            vls.vls_result_summary(C.c_void_p(outs[k]), C.byref(s))
            sums.append({f: getattr(s, f) for f, _ in vls.vls_summary._fields_})
            vls.vls_result_destroy(C.c_void_p(outs[k]))
        if st != 0:
            raise vls.VLSError(st, ctx.last_error())
        return sums

    run_batch(list(range(n)))                     # warm-up: allocates every mesh's run buffers
    torch.cuda.synchronize()
    # schedule: the default; with tune, also the tuner's pick on a sample of
    # the workload (every 4th mesh), both timed on the whole batch
    tuned = {"two_per_cu": False, "gang_vertices": 0, "seconds": {}}
    variants = [("default", 0, 0)]
    if tune:
        from paper_2105_13168_amd.tune import tune_batch
        t0 = time.time()
        samp = list(range(0, n, 4))
        tuned = tune_batch(ctx, [M[i] for i in samp], [ms[i].seed for i in samp])
        log(f"batch schedule tuned on {len(samp)} meshes: {tuned} ({time.time() - t0:.1f}s)")
        variants.append(("tuned", vls.VLS_BATCH_TWO_PER_CU if tuned["two_per_cu"] else 0, tuned["gang_vertices"]))
    shapes = {}
    for name, extra, gv in variants:
        t1 = time.perf_counter()
        sm = run_batch(list(range(n)), extra, gv)
        torch.cuda.synchronize()
        shapes[name] = (time.perf_counter() - t1, sm)
    best = min(shapes, key=lambda k: shapes[k][0])
    tb, sums = shapes[best]
    ok = all(s["run_status"] == 0 and s["n_handles"] == g
             for _, sm in shapes.values() for s, g in zip(sm, genus))
    vsteps = sum(m.nv * s["steps"] for m, s in zip(ms, sums))
    ab = sum(alg_bytes(s["active_vertex_updates"], s["active_degree_sum"]) for s in sums)
    kernel_ms = sums[0]["kernel_ms"]
    # one at a time, on an evenly spaced sample of the same meshes
    sample = list(range(0, n, max(1, n // seq_sample)))[:seq_sample]
    t2 = time.perf_counter()
    seq_ms = 0.0
    for i in sample:
        p = vls.default_params(seed_vertex=ms[i].seed, flags=vls.VLS_DEFER_RESULTS)
        h = C.c_void_p()
        st = vls.vls_run(ctx.h, M[i].h, C.byref(p), C.byref(h))
        vls.vls_result_destroy(h)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t2
    for x in M:
        x.close()
    seq_rate = len(sample) / ts
    # the sample's share of the batch's vertex-steps, to compare like with like
    sample_vsteps = sum(ms[i].nv * sums[i]["steps"] for i in sample)
    slow = sorted(range(n), key=lambda i: -(sums[i]["topo_ms"] + sums[i]["wait0_ms"]))[:5]
    return {
        "slowest": [{"nv": int(ms[i].nv), "steps": int(sums[i]["steps"]), "events": int(sums[i]["n_events"]),
                     "ms": round(sums[i]["topo_ms"] + sums[i]["wait0_ms"], 1)} for i in slow],
        "schedule": best, "tuned_schedule": {k: tuned[k] for k in ("two_per_cu", "gang_vertices")},
        "tuning_seconds": tuned["seconds"],
        "seconds_by_shape": {k: round(v[0], 3) for k, v in shapes.items()},
        "kernel_ms_by_shape": {k: round(v[1][0]["kernel_ms"], 1) for k, v in shapes.items()},
        "meshes": n, "total_vertices": int(sum(m.nv for m in ms)), "all_handles_equal_genus": ok,
        "seconds": tb, "meshes_per_s": n / tb, "batch_kernel_ms": kernel_ms,
        "vertex_steps_per_s": vsteps / tb,
        "dense_equivalent_frac": (vsteps / tb) * 56.0 / (HBM_PEAK_GBPS * 1e9),
        "hbm_roofline_frac": ab / (kernel_ms * 1e-3) / (HBM_PEAK_GBPS * 1e9),
        "sequential_sample": len(sample), "sequential_seconds": ts,
        "sequential_meshes_per_s": seq_rate,
        "sequential_vertex_steps_per_s": sample_vsteps / ts,
        "speedup_vertex_steps": (vsteps / tb) / (sample_vsteps / ts),
    }


def serve_leg(ctx, n_req, rate, lattice_share, slice_us, seed=0, two_per_cu=False, gang_vertices=0):
    """Serving: Poisson arrivals at ``rate``/s, each request an initial pass
    of a mesh drawn from the uneven batch distribution or, with probability
    ``lattice_share``, from two strut lattices of 2-8M triangles; meshes are
    uploaded once beforehand (resident operators), run state is allocated per
    request under an HBM budget of half the free device memory.  Latency =
    submission to results on the host.  The one-at-a-time GPU path is timed
    on every distinct mesh (vls_run, default launch) and replayed on the
    same arrival trace as a first-come-first-served single queue."""
    import ctypes as C
    import numpy as np
    import meshgen as mg
    import paper_2105_13168_amd as vls
    import torch
    rng = np.random.default_rng(seed)
    t0 = time.time()
    pool = mg.batch_workload(256, base_seed=1000)
    lat = [mg.lattice(3, 240, rng_seed=1), mg.lattice(4, 256, rng_seed=2)]
    meshes = pool + lat
    log(f"serving pool: {len(pool)} batch-distribution meshes + lattices of "
        f"{[x.nf for x in lat]} triangles ({time.time() - t0:.1f}s)")
    M = [vls.Mesh(ctx, m.xyz, m.tri) for m in meshes]
    genus = [x.euler_genus for x in M]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    pick = np.where(rng.random(n_req) < lattice_share, len(pool) + rng.integers(0, len(lat), size=n_req),
                    rng.integers(0, len(pool), size=n_req))
    free, _total = torch.cuda.mem_get_info()
    srv = vls.Server(ctx, hbm_budget_bytes=free // 2, max_slots=1024, slice_us=slice_us,
                     flags=vls.VLS_BATCH_TWO_PER_CU if two_per_cu else 0)
    # warm-up request (first launch, allocations)
    t = srv.submit(M[0], seed_vertex=meshes[0].seed)
    while srv.poll(t) is None:
        time.sleep(0.001)
    lat_ms, queue_ms, lat_of, ok = [], [], [], True
    outstanding = {}
    start = time.perf_counter()
    nxt = 0
    last_done = start
    while nxt < n_req or outstanding:
        now = time.perf_counter() - start
        while nxt < n_req and arrivals[nxt] <= now:
            i = int(pick[nxt])
            p = vls.default_params(seed_vertex=meshes[i].seed)
            p.gang_vertices = gang_vertices
            tk = C.c_uint64()
            st = vls.vls_server_submit(srv.h, M[i].h, C.byref(p), C.byref(tk))
            if st != 0:
                raise vls.VLSError(st, "submit")
            outstanding[tk.value] = i
            nxt += 1
        for tk in list(outstanding):
            h = C.c_void_p()
            st = vls.vls_server_poll(srv.h, C.c_uint64(tk), C.byref(h))
            if st == vls.VLS_E_PENDING:
                continue
            i = outstanding.pop(tk)
            sm = vls.vls_summary()
            vls.vls_result_summary(h, C.byref(sm))
            ok = ok and st == 0 and sm.n_handles == genus[i]
            lat_ms.append(sm.server_latency_ms)
            queue_ms.append(sm.server_queue_ms)
            lat_of.append(i >= len(pool))
            vls.vls_result_destroy(h)
            last_done = time.perf_counter()
        time.sleep(0.0005)
    makespan = last_done - start
    stats = srv.stats()
    srv.close()
    # the one-at-a-time path: service time of every distinct mesh used
    service = {}
    for i in sorted(set(int(x) for x in pick)):
        p = vls.default_params(seed_vertex=meshes[i].seed, flags=vls.VLS_DEFER_RESULTS)
        h = C.c_void_p()
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = vls.vls_run(ctx.h, M[i].h, C.byref(p), C.byref(h))
        vls.vls_result_fetch(h)
        service[i] = time.perf_counter() - a
        vls.vls_result_destroy(h)
    free_at = 0.0
    seq_lat = []
    for k in range(n_req):
        begin = max(free_at, arrivals[k])
        free_at = begin + service[int(pick[k])]
        seq_lat.append((free_at - arrivals[k]) * 1e3)
    for x in M:
        x.close()
    lat_ms = np.array(lat_ms)
    seq_lat = np.array(seq_lat)
    is_lat = np.array(lat_of, dtype=bool)
    by_class = {}
    for name, sel in (("lattice", is_lat), ("pool", ~is_lat)):
        if sel.any():
            by_class[name] = {"requests": int(sel.sum()), "p50_ms": float(np.percentile(lat_ms[sel], 50)),
                              "p99_ms": float(np.percentile(lat_ms[sel], 99)), "max_ms": float(lat_ms[sel].max())}
    by_class["lattice_solo_service_ms"] = [round(1e3 * service[i], 1) for i in sorted(service) if i >= len(pool)]
    return {
        "requests": int(n_req), "rate_per_s": rate, "lattice_share": lattice_share,
        "lattice_requests": int((pick >= len(pool)).sum()), "slice_us": slice_us,
        "gang_vertices": int(gang_vertices) if gang_vertices > 0 else 65536,
        "all_handles_equal_genus": bool(ok),
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "mean_ms": float(lat_ms.mean()), "mean_queue_ms": float(np.mean(queue_ms)),
        "meshes_per_s": n_req / makespan, "makespan_s": makespan, "launches": stats["launches"],
        "scheduler_ms": {k: round(stats[k], 1) for k in ("admit_ms", "launch_ms", "complete_ms")},
        "by_class": by_class,
        "sequential": {"p50_ms": float(np.percentile(seq_lat, 50)), "p99_ms": float(np.percentile(seq_lat, 99)),
                       "meshes_per_s": n_req / (free_at - 0.0) if free_at > 0 else None,
                       "service_ms_mean": 1e3 * float(np.mean([service[int(i)] for i in pick]))},
    }


def passes_leg(ctx, workload):
    """The tunnel-loop pass of every handle loop and the refinement pass of
    every tunnel after one initial pass (vls_run with VLS_REFINE_PASS): pass
    launches timed on the device, loops found, and the passes' field steps
    against HBM (32 + 4 deg bytes per vertex update, deg the mean degree)."""
    import ctypes as C
    import paper_2105_13168_amd as vls
    m, desc = make_workload(workload)
    M = vls.Mesh(ctx, m.xyz, m.tri)
    p = vls.default_params(seed_vertex=m.seed, flags=vls.VLS_DEFER_RESULTS | vls.VLS_REFINE_PASS)
    h = C.c_void_p()
    st = vls.vls_run(ctx.h, M.h, C.byref(p), C.byref(h))
    if st != 0:
        raise vls.VLSError(st, ctx.last_error())
    s = vls.vls_summary()
    vls.vls_result_summary(h, C.byref(s))
    labels = {3: [0, 0], 4: [0, 0]}
    for kind, cnt in ((3, s.n_tunnel_passes), (4, s.n_refine_passes)):
        for i in range(cnt):
            lab = C.c_int32()
            vls.vls_result_pass_info(h, kind, i, None, None, None, C.byref(lab), None, None)
            if lab.value >= 0:
                labels[kind][lab.value] += 1
    vls.vls_result_destroy(h)
    M.close()
    ms = s.tunnel_pass_ms + s.refine_pass_ms
    deg = 3.0 * m.nf / m.nv                   # mean degree: 2E / V = 3F / V
    ab = s.pass_vertex_updates * (32.0 + 4.0 * deg)
    return {"workload": desc, "nv": m.nv, "handles": s.n_handles,
            "tunnel_passes": s.n_tunnel_passes, "tunnel_loops": s.n_tunnel_loops,
            "refine_passes": s.n_refine_passes, "refined_loops": s.n_refined_loops,
            "labels_tunnel_pass_handle_tunnel": labels[3], "labels_refine_pass_handle_tunnel": labels[4],
            "pass_slots": s.pass_slots, "tunnel_pass_ms": s.tunnel_pass_ms, "refine_pass_ms": s.refine_pass_ms,
            "passes_per_s": (s.n_tunnel_passes + s.n_refine_passes) / (ms * 1e-3) if ms > 0 else None,
            "pass_vertex_updates": s.pass_vertex_updates,
            "roofline": {"bound": "hbm", "achieved": ab / (ms * 1e-3) / 1e9 if ms > 0 else None,
                         "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS if ms > 0 else None,
                         "kernel": "k_passes"}}


def host_cpu():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(workload, max_steps, head=None):
    """The oracle (sequential C, one thread) on a bounded sample: the first
    max_steps diffusion steps of `workload`'s pass (0: the whole pass),
    timed without the oracle's own mesh setup (a one-step run measures it).
    value is in the main line's unit; when head = (nv, steps, updates) of
    the main line's workload is given, the oracle's update rate is scaled to
    that workload's vertex-steps per update."""
    import oracle
    oracle.build(force=False)
    m, desc = make_workload(workload)
    t0 = time.perf_counter()
    oracle.run(m.xyz, m.tri, seed_vertex=m.seed, max_steps=1)
    t_setup = time.perf_counter() - t0
    kw = {"max_steps": max_steps} if max_steps > 0 else {}
    t0 = time.perf_counter()
    r = oracle.run(m.xyz, m.tri, seed_vertex=m.seed, **kw)
    dt = time.perf_counter() - t0 - t_setup
    model, ncpu = host_cpu()
    what = "the whole pass" if max_steps <= 0 else f"the first {r.steps} diffusion steps of the pass"
    upd_rate = r.active_updates / dt
    out = {"unit": "vertex-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{what} on {desc} (V={m.nv}), one thread, {dt:.1f} s of stepping after {t_setup:.1f} s "
                     f"of the oracle's mesh setup",
           "seconds": round(dt, 3), "oracle_updates_per_s": upd_rate, "sample_vertex_steps_per_s": m.nv * r.steps / dt,
           "host_cpu": model, "host_nproc": ncpu,
           "threads_note": "the oracle is sequential C (no threads); nproc copies would not share one pass"}
    # the oracle's whole pass of the full workloads, timed when their digests
    # were recorded (build container, one core): context for the sample
    try:
        with open(os.path.join(ROOT, "tests", "golden", "oracle_full.json")) as f:
            gold = json.load(f)
        out["oracle_whole_pass_seconds_recorded"] = {k: v["oracle_seconds"] for k, v in gold.items()
                                                     if "oracle_seconds" in v}
    except (OSError, ValueError, KeyError):
        pass
    if head is not None:
        nv, steps, updates = head
        out["value"] = upd_rate * (nv * steps / updates)
        out["scaling"] = ("oracle update rate on the sample times the main workload's vertex-steps per "
                          "update (dense-equivalent, as the GPU value)")
    else:
        out["value"] = m.nv * r.steps / dt
    return out


def main():
    t_start = time.time()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lattice10_1024")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds: extra legs are skipped when they would end past it")
    ap.add_argument("--cpu-workload", default="lattice10_256", help="oracle sample workload")
    ap.add_argument("--cpu-steps", type=int, default=10000, help="oracle diffusion steps (0: whole pass)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--maps-out", default="",
                    help="write the process's memory map here at interpreter exit (places the addresses of "
                         "frames that later exit handlers print)")
    ap.add_argument("--pretzel-passes", type=int, default=3, help="timed passes of the 256^3 pretzel (0: skip)")
    ap.add_argument("--batch", type=int, default=1024, help="meshes in the batched leg (0: skip)")
    ap.add_argument("--batch-seq-sample", type=int, default=16)
    ap.add_argument("--tune", action="store_true", help="time the batch schedule tuner's pick too")
    ap.add_argument("--serve", type=int, default=1000, help="requests in the serving trace (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-lattice-share", type=float, default=0.05)
    ap.add_argument("--serve-slice-us", type=int, default=20000)
    ap.add_argument("--serve-two-per-cu", action="store_true", help="server step launches at two workgroups per CU")
    ap.add_argument("--serve-gang-vertices", type=int, default=0,
                    help="vertices per gang workgroup of a served request (0: the library's 65536)")
    ap.add_argument("--dense-workload", default="same",
                    help="mesh of the dense-step leg ('same': the main workload's mesh; 'none': skip)")
    ap.add_argument("--dense-steps", type=int, default=200)
    ap.add_argument("--dense", action="store_true", help="time the whole pass with the dense field step")
    ap.add_argument("--passes-workload", default="lattice10_256",
                    help="mesh of the tunnel-loop / refinement pass leg ('none': skip)")
    ap.add_argument("--refine-workload", default="pretzel256",
                    help="workload of the Reeb refinement leg (none: skip)")
    ap.add_argument("--fem-passes", type=int, default=2,
                    help="timed passes of the relaxed 128^3 pretzel with the finite-element operator (0: skip)")
    args = ap.parse_args()
    if args.maps_out:
        import atexit
        import shutil

        def _dump_maps(path=args.maps_out):
            with open("/proc/self/maps") as src, open(path, "w") as dst:
                shutil.copyfileobj(src, dst)
        atexit.register(_dump_maps)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(meshes shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    def left():
        return args.time_budget - (time.time() - t_start)

    t0 = time.time()
    m, desc = make_workload(args.workload)
    log(f"workload {args.workload}: V={m.nv} F={m.nf} seed={m.seed} ({time.time() - t0:.1f}s)")
    import torch
    import paper_2105_13168_amd as vls
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = vls.Context(0, stream=stream.cuda_stream)
    t1 = time.time()
    M = vls.Mesh(ctx, m.xyz, m.tri)
    log(f"mesh validated, adjacency built and uploaded ({time.time() - t1:.1f}s)")

    def one_pass():
        p = vls.default_params(seed_vertex=m.seed, grid=args.grid,
                               flags=vls.VLS_DEFER_RESULTS | (vls.VLS_DENSE_FIELD if args.dense else 0))
        h = C.c_void_p()
        st = vls.vls_run(ctx.h, M.h, C.byref(p), C.byref(h))
        if st != 0:
            raise vls.VLSError(st, ctx.last_error())
        s = vls.vls_summary()
        vls.vls_result_summary(h, C.byref(s))
        return h, {f: getattr(s, f) for f, _ in vls.vls_summary._fields_}

    for k in range(args.warmup):
        h, _s = one_pass()
        vls.vls_result_destroy(h)
        log(f"warm-up pass {k + 1}/{args.warmup}: {_s['kernel_ms']:.0f} ms step kernel")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sums = []
    handles = []
    ev0.record(stream)
    for k in range(args.steps):
        h, s = one_pass()
        sums.append(s)
        handles.append(h)
        log(f"timed pass {k + 1}/{args.steps}: {s['kernel_ms']:.0f} ms step kernel")
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    # validate the last pass outside the timed region
    last = sums[-1]
    for h in handles[:-1]:
        vls.vls_result_destroy(h)
    vls.vls_result_fetch(handles[-1])
    vls.vls_result_destroy(handles[-1])
    assert last["run_status"] == 0
    assert last["n_handles"] == M.euler_genus and last["n_tunnels"] == M.euler_genus
    steps = last["steps"]
    kernel_ms = sum(s["kernel_ms"] for s in sums) / len(sums)
    device_ms = sum(s["total_ms"] for s in sums) / len(sums)
    upd = last["active_vertex_updates"]
    deg = last["active_degree_sum"]
    ab = alg_bytes(upd, deg)
    achieved = ab / (kernel_ms * 1e-3) / 1e9
    value = m.nv * steps / (ms * 1e-3)
    dense_bytes = 20.0 + 4.0 * deg / upd          # per vertex of a dense step: 20 B + 4 B per neighbour id
    out = {
        "metric": "vertex-diffusion-steps/sec",
        "value": value,
        "unit": "vertex-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc, "nv": m.nv, "nf": m.nf, "seed_vertex": m.seed, "genus": M.euler_genus,
            "diffusion_steps": steps, "events": last["n_events"], "handles": last["n_handles"],
            "active_vertex_updates": upd, "grid": last["grid"], "block": last["block"],
            "device_ms_per_pass": device_ms, "step_kernel_ms": kernel_ms,
            "active_updates_per_s": upd / (ms * 1e-3),
            "phase_ms": {"topology": last["topo_ms"], "topology_wait": last["wait0_ms"],
                         "field": last["field_ms"], "field_wait": last["wait1_ms"],
                         "topology_global_path_steps": last["topo_global_steps"],
                         "topology_split": {k: v for k, v in zip(
                             ("candidates", "closure", "classification", "insert_events"), last["topo_split_ms"])},
                         "topology_event_steps_ms": last["topo_event_ms"],
                         "topology_rounds_ms": last["topo_rounds_ms"],
                         "event_split": {k: v for k, v in zip(
                             ("merge_walks", "split_walkers", "relabel", "rest"), last["event_split_ms"])},
                         "global_path_split": {k: v for k, v in zip(
                             ("candidates", "closure", "classification", "insert_events"),
                             last["topo_global_split_ms"])}},
            "event_steps": last["event_steps"],
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(kernel_ms, args.workload, grid=last["grid"]),
                     "kernel": "k_steps_dec", "algorithmic_bytes": ab,
                     # a dense step (every vertex, 20 + 4 deg bytes) at this
                     # vertex-steps/s would need this share of HBM peak
                     "dense_equivalent_frac": value * dense_bytes / (HBM_PEAK_GBPS * 1e9),
                     "kernel_source_hash": kernel_source_hash()},
    }
    if args.dense:
        ab = dense_alg_bytes(upd, deg)
        out["roofline"]["achieved"] = ab / (kernel_ms * 1e-3) / 1e9
        out["roofline"]["frac"] = out["roofline"]["achieved"] / HBM_PEAK_GBPS
        out["roofline"]["algorithmic_bytes"] = ab
        out["roofline"]["traffic"] = None
        out["config"]["field_step"] = "dense"
    skipped = []
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_workload, args.cpu_steps, head=(m.nv, steps, upd))
        log(f"cpu baseline done ({time.time() - t_start:.0f}s since start)")
    if args.dense_workload != "none" and args.dense_steps > 0:
        if args.dense_workload == "same":
            out["dense_step"] = dense_leg(ctx, args.workload, args.dense_steps, mesh=(m, M, desc))
        elif left() > 60:
            out["dense_step"] = dense_leg(ctx, args.dense_workload, args.dense_steps)
        else:
            skipped.append("dense_step")
    M.close()
    del m
    if args.pretzel_passes > 0 and args.workload != "pretzel256":
        if left() > 30:
            out["pretzel_pass"] = pass_leg(ctx, "pretzel256", args.pretzel_passes)
            log(f"pretzel leg done ({time.time() - t_start:.0f}s since start)")
        else:
            skipped.append("pretzel_pass")
    if args.batch > 0:
        if left() > 75:
            out["batched"] = batch_leg(ctx, args.batch, args.batch_seq_sample, tune=args.tune)
            log(f"batch leg done ({time.time() - t_start:.0f}s since start)")
        else:
            skipped.append("batched")
    if args.serve > 0:
        if left() > 80:
            out["serving"] = serve_leg(ctx, args.serve, args.serve_rate, args.serve_lattice_share,
                                       args.serve_slice_us, two_per_cu=args.serve_two_per_cu,
                                       gang_vertices=args.serve_gang_vertices)
            out["serving"]["workgroups_per_cu"] = 2 if args.serve_two_per_cu else 1
            log(f"serving leg done ({time.time() - t_start:.0f}s since start)")
        else:
            skipped.append("serving")
    if args.passes_workload != "none":
        if left() > 60:
            out["passes"] = passes_leg(ctx, args.passes_workload)
            log(f"passes leg done ({time.time() - t_start:.0f}s since start)")
        else:
            skipped.append("passes")
    if args.fem_passes > 0:
        if left() > 45:
            out["fem_pass"] = pass_leg(ctx, "pretzel128_relaxed", args.fem_passes, fem=True)
            log(f"finite-element leg done ({time.time() - t_start:.0f}s since start)")
        else:
            skipped.append("fem_pass")
    if args.refine_workload != "none":
        if left() > 30:
            out["reeb_refine"] = refine_leg(ctx, args.refine_workload)
            log(f"Reeb refinement leg done ({time.time() - t_start:.0f}s since start)")
        else:
            skipped.append("reeb_refine")
    if skipped:
        out["skipped_for_time_budget"] = skipped
    if args.copy_calibration:
        copy_calibration()
    ctx.close()
    out["bench_seconds"] = round(time.time() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
