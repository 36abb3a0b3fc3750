"""Host logic of bench.py (CPU): the one-GPU refusal and the rule that the
measured HBM traffic is reported only for the kernel sources it was taken on."""
import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""  # no JSON line


def _tree(tmp_path):
    for f in bench.KERNEL_SOURCES:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), dst)
    (tmp_path / "profiles").mkdir()
    return tmp_path


def test_source_hash_follows_every_kernel_source(tmp_path, monkeypatch):
    t = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(t))
    h0 = bench.source_hash()
    assert h0 == bench.source_hash()
    for f in bench.KERNEL_SOURCES:
        p = t / f
        orig = p.read_bytes()
        p.write_bytes(orig + b"\n")
        assert bench.source_hash() != h0, f
        p.write_bytes(orig)
    assert bench.source_hash() == h0


def test_traffic_only_for_the_recorded_sources(tmp_path, monkeypatch):
    t = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(t))
    w = "some-workload"
    assert bench.recorded_traffic(w, "coupling") is None  # no record
    rec = {"workload": w, "pass": "coupling", "source_sha": bench.source_hash(),
           "fetch_bytes": 1000.25, "write_bytes": 24.5}
    path = t / "profiles" / f"hbm_traffic_{w}.json"
    path.write_text(json.dumps(rec))
    assert bench.recorded_traffic(w, "coupling") == 1024.8  # rounded to 0.1 byte
    assert bench.recorded_traffic(w, "near") is None  # another pass
    p = t / bench.KERNEL_SOURCES[0]
    p.write_bytes(p.read_bytes() + b"// changed\n")
    assert bench.recorded_traffic(w, "coupling") is None  # sources changed since the counters


def test_default_workload_is_the_100k_matern_configuration():
    # the metric's configuration: 100,000 uniform cube points, Matern-3/2 with
    # l = 0.1 plus 1e-4 I, leaf 200, H^2 tolerance 1e-8, HSS tolerance 1e-2,
    # one N(0,1) right-hand side, PCG to 1e-8
    w = bench.workloads.MEDIUM
    assert (w.n, w.point_set, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, w.hss_tol, w.nrhs, w.pcg_tol) == \
        (100_000, "cube", "matern32", 0.1, 1e-4, 200, 1e-8, 1e-2, 1, 1e-8)
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--workload", default=workloads.MEDIUM.name' in src
