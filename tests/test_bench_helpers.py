"""Host logic of bench.py: the algorithmic byte counts behind the roofline
figures, and the rule that a committed traffic record is used only for the
kernel sources, workload, step count and grid it was measured on."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402


def test_algorithmic_bytes_per_update():
    # update-set step: value in and out, row offsets, list entry in and out,
    # 4 B per neighbour id: 56 B at degree 6
    assert bench.alg_bytes(1, 6) == 56
    assert bench.alg_bytes(10, 60) == 560
    # dense step: no list entry, one row offset per vertex, 44 B at degree 6
    assert bench.dense_alg_bytes(1, 6) == 44
    assert bench.dense_alg_bytes(0, 0) == 0


def _record(tmp_path, name, **kw):
    rec = {"kernel_source_hash": bench.kernel_source_hash(), "hbm_bytes_per_launch": 2.0e9}
    rec.update(kw)
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    (prof / f"k_steps_{name}_traffic.json").write_text(json.dumps(rec))


def test_traffic_record_matching(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the source hash is read from the package next to ROOT
    pkg = tmp_path / "paper_2105_13168_amd" / "csrc"
    pkg.mkdir(parents=True)
    src = os.path.join(os.path.dirname(HERE), "paper_2105_13168_amd", "csrc")
    for f in ("vls_kernels.hip", "vls_internal.h"):
        (pkg / f).write_bytes(open(os.path.join(src, f), "rb").read())
    _record(tmp_path, "w1", grid=64)
    # 2 GB over 1 s = 2 GB/s
    assert abs(bench.measured_traffic(1000.0, "w1", grid=64) - 2.0) < 1e-12
    assert bench.measured_traffic(1000.0, "w1") is not None
    assert bench.measured_traffic(1000.0, "w1", grid=99) is None
    assert bench.measured_traffic(1000.0, "missing", grid=64) is None
    _record(tmp_path, "w2", grid=256, diffusion_steps=400)
    assert bench.measured_traffic(500.0, "w2", 400, grid=256) is not None
    assert bench.measured_traffic(500.0, "w2", 200, grid=256) is None
    # other kernel sources: the record no longer applies
    (pkg / "vls_internal.h").write_bytes(b"// changed\n")
    assert bench.measured_traffic(1000.0, "w1", grid=64) is None


def test_committed_records_name_their_grid():
    root = os.path.dirname(HERE)
    for name in ("lattice10_1024", "pretzel256", "dense_lattice10_1024"):
        rec = json.load(open(os.path.join(root, "profiles", f"k_steps_{name}_traffic.json")))
        assert isinstance(rec.get("grid"), int) and rec["hbm_bytes_per_launch"] > 0
        assert rec["fetch_factor"] > 0 and rec["write_factor"] > 0


def test_host_cpu_reports_model_and_count():
    model, n = bench.host_cpu()
    assert isinstance(model, str) and n >= 1
