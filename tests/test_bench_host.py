"""Host-side logic of bench.py (no GPU): the one-GPU contract, the roofline
bound chosen from a kernel's algorithmic intensity, and the HBM traffic that is
reported only for the kernel source the counters were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in (res.stdout + res.stderr)


def _prof(**kernels):
    return {"kernels": {k: {"ms": ms, "launches": 10, "flops": fl, "bytes": by}
                        for k, (ms, fl, by) in kernels.items()}}


def test_roofline_bound_follows_intensity():
    # intensity 30 flop/B is above the FP32 ridge (157.3 TF / 8 TB/s = 19.7): MFMA
    name, r = bench.roofline(_prof(jacobi_gram=(40.0, 30e9, 1e9), jacobi_update=(10.0, 1e9, 1e9)),
                             "fp32")
    assert name == "jacobi_gram" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(30e9 / 40e-3 / 1e12)
    assert r["frac"] == pytest.approx(30e9 / 40e-3 / 157.3e12)
    # 16 flop/B is below the FP32 ridge: HBM, achieved in GB/s
    name, r = bench.roofline(_prof(jacobi_update=(40.0, 16e9, 1e9)), "fp32")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1e9 / 40e-3 / 1e9)
    assert r["frac"] == pytest.approx(1e9 / 40e-3 / 8e12)
    # the same 16 flop/B is above the FP64 ridge (9.8): MFMA against the FP64 peak
    _, r = bench.roofline(_prof(jacobi_update=(40.0, 16e9, 1e9)), "fp64")
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(78.6)
    # the pair eigen-solver is FP64 vector work in every mode
    _, r = bench.roofline(_prof(jacobi_eig64=(40.0, 1e9, 1e6)), "fp32")
    assert r["bound"] == "alu" and r["peak"] == pytest.approx(78.6)


def test_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    # a copy of the tree's layout: the kernel source and the counter record
    src = tmp_path / "paper_2003_13163_amd" / "csrc"
    src.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src / "jacobi.hip").write_text("kernel source A\n")
    import hashlib
    sha = hashlib.sha256(b"kernel source A\n").hexdigest()
    rec = {"source_sha256": {"paper_2003_13163_amd/csrc/jacobi.hip": sha}, "precision": "fp32",
           "kernels": {"jacobi_gram": {"bytes_per_launch": 1.25e8}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("jacobi_gram", "fp32") == pytest.approx(1.25e8)
    assert bench.measured_traffic("jacobi_gram", "fp64") is None       # other precision
    assert bench.measured_traffic("jacobi_update", "fp32") is None     # kernel not measured
    (src / "jacobi.hip").write_text("kernel source B\n")                # source changed
    assert bench.measured_traffic("jacobi_gram", "fp32") is None


def test_nominal_gate_work_and_per_gate_fraction():
    """Nominal work of a bulk gate at chi = 1024: about 1.15e12 real flops
    (about 1074 chi^3), FP64 roofline time about 14.6 ms, FP32 (contractions on
    FP32 MFMA, eigen core on FP64) about 10.5 ms; fused bytes 16 chi^2 values."""
    w64 = bench.nominal_gate_work(1024, "fp64")
    w32 = bench.nominal_gate_work(1024, "fp32")
    assert w64["nominal_flops"] == pytest.approx(1.154e12, rel=2e-3)
    assert w64["nominal_flops"] / 1024 ** 3 == pytest.approx(1074.7, rel=1e-3)
    assert w64["t_roof_ms"] == pytest.approx(14.68, rel=2e-3)
    assert w32["t_roof_ms"] == pytest.approx(10.54, rel=2e-3)
    assert w64["fused_min_bytes"] == 16 * 1024 ** 2 * 16
    assert w32["fused_min_bytes"] == 16 * 1024 ** 2 * 8
    prof = _prof(jacobi_gram=(40.0, 3e12, 1e11), gemm=(10.0, 1e11, 1e10))
    r = bench.per_gate_roofline(prof, "fp32", 1024, 500.0, 10)
    assert r["frac"] == pytest.approx(w32["t_roof_ms"] / 500.0)
    assert r["counted_flops_per_gate"] == pytest.approx(3.1e11)
    assert r["algorithmic_bytes_per_gate"] == pytest.approx(1.1e10)


def test_traffic_digest_follows_the_kernel_only(tmp_path, monkeypatch):
    """A record keyed by the kernel's own functions and constants stays valid
    when another function of the file changes and is dropped when the kernel,
    a helper it names or a constant it names changes."""
    src = tmp_path / "paper_2003_13163_amd" / "csrc"
    src.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    body = ("constexpr int kTile = 64;\n"
            "__device__ double helper(double v) { return v * 2.0; }\n"
            "__global__ void k_main(const double* x, double* y) {\n    y[0] = helper(x[0]) + kTile;\n}\n"
            "__global__ void k_other(double* y) { y[0] = 1.0; }\n")
    (src / "k.hip").write_text(body)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    spec = {"paper_2003_13163_amd/csrc/k.hip": ["k_main", "helper", "kTile"]}
    rec = {"source_digest": {"spec": spec, "sha256": bench.source_digest(spec)}, "precision": "fp32",
           "kernels": {"main": {"bytes_per_launch": 3.0e7}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("main", "fp32") == pytest.approx(3.0e7)
    (src / "k.hip").write_text(body.replace("y[0] = 1.0", "y[0] = 2.0"))       # another kernel
    assert bench.measured_traffic("main", "fp32") == pytest.approx(3.0e7)
    for old, new in (("v * 2.0", "v * 3.0"), ("kTile = 64", "kTile = 32"), ("+ kTile", "- kTile")):
        (src / "k.hip").write_text(body.replace(old, new))
        assert bench.measured_traffic("main", "fp32") is None
    (src / "k.hip").write_text(body.replace("k_main", "k_renamed"))            # the kernel is gone
    assert bench.measured_traffic("main", "fp32") is None
