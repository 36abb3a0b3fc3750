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
    rec = {"workload": w, "source_sha": bench.source_hash(),
           "passes": {"coupling": {"fetch_bytes": 1000.25, "write_bytes": 24.5}}}
    path = t / "profiles" / f"hbm_traffic_{w}.json"
    path.write_text(json.dumps(rec))
    assert bench.recorded_traffic(w, "coupling") == 1024.8  # rounded to 0.1 byte
    assert bench.recorded_traffic(w, "near") is None  # another pass
    p = t / bench.KERNEL_SOURCES[0]
    p.write_bytes(p.read_bytes() + b"// changed\n")
    assert bench.recorded_traffic(w, "coupling") is None  # sources changed since the counters


def test_default_workload_is_the_1m_gaussian_configuration():
    # the metric's size: 1,000,000 uniform cube points, Gaussian with l = 0.2
    # plus 1e-3 I, leaf 400, 16 N(0,1) right-hand sides, PCG to 1e-8; with the
    # two stated changes eps_H 1e-6 -> 1e-8 and (tau, r) (1e-1, 100) -> (1e-2, 200)
    w = bench.workloads.HEADLINE
    assert (w.n, w.point_set, w.kernel, w.ell, w.shift, w.leaf, w.nrhs, w.pcg_tol) == \
        (1_000_000, "cube", "gaussian", 0.2, 1e-3, 400, 16, 1e-8)
    assert (w.h2_tol, w.hss_tol, w.max_rank, w.oversample) == (1e-8, 1e-2, 200, 10)
    L = bench.workloads.LARGE
    assert (L.n, L.kernel, L.ell, L.shift, L.leaf, L.h2_tol, L.hss_tol, L.nrhs) == \
        (1_000_000, "gaussian", 0.2, 1e-3, 400, 1e-6, 1e-1, 16)
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--workload", default=workloads.HEADLINE.name' in src


def test_oracle_small_configuration_end_to_end():
    """The unscaled oracle leg of the CPU baseline solves the small
    configuration to its tolerance."""
    r = bench.oracle_small_end_to_end()
    assert r["n"] == 2000 and r["seconds"] > 0
    assert r["relres_max"] <= 1e-8 and 1 <= r["pcg_iterations"] < 5000
