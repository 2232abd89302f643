"""Host-side checks of bench.py: the single-GPU guard and the rule that a committed traffic
figure is reported only for the kernel source it was measured on."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_reported_only_for_the_counted_source(tmp_path, monkeypatch):
    import bench
    src_rel = bench.KERNEL_SOURCES["gemm_bf16_tn"]
    digest = hashlib.sha256(open(os.path.join(ROOT, src_rel), "rb").read()).hexdigest()
    fake_root = tmp_path
    os.makedirs(fake_root / "profiles")
    os.makedirs(fake_root / os.path.dirname(src_rel))
    (fake_root / src_rel).write_bytes(open(os.path.join(ROOT, src_rel), "rb").read())
    rec = {"kernels": {"gemm_bf16_tn": {"hbm_bytes_per_launch": 123.0, "source_sha256": digest}}}
    (fake_root / "profiles" / "hbm_traffic_n64.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    assert bench.measured_traffic("gemm_bf16_tn", 64) == 123.0
    # another size, another kernel, or a changed source: no figure
    assert bench.measured_traffic("gemm_bf16_tn", 128) is None
    assert bench.measured_traffic("split_bf16_ab", 64) is None
    (fake_root / src_rel).write_bytes(b"// changed\n")
    assert bench.measured_traffic("gemm_bf16_tn", 64) is None


@pytest.mark.parametrize("name", ["gemm_bf16_tn", "gemm_bf16x3_tn", "gemm_fp8r_tn", "gemm_f32_simt",
                                  "gemm_fp6x3_tn", "quant_fp8_ab", "quant_mx6_ab", "split_bf16_ab",
                                  "split_bf16_hilo_ab"])
def test_roofline_work_per_launch(name):
    import bench
    bound, work, peak, unit = bench.kernel_roofline(name, 256, 512, 128)
    mnk = 256 * 512 * 128
    expect = {"gemm_bf16_tn": 2 * mnk, "gemm_bf16x3_tn": 6 * mnk, "gemm_fp8r_tn": 8 * mnk,
              "gemm_f32_simt": 2 * mnk, "gemm_fp6x3_tn": 6 * mnk,
              "quant_fp8_ab": 4 * (256 * 128 + 128 * 512) + 2 * (256 + 512) * 128,
              "quant_mx6_ab": 4 * (256 * 128 + 128 * 512) + 1.5625 * (256 + 512) * 128,
              "split_bf16_ab": 4 * (256 * 128 + 128 * 512) + 2 * (256 + 512) * 128,
              "split_bf16_hilo_ab": 4 * (256 * 128 + 128 * 512) + 4 * (256 + 512) * 128}[name]
    assert work == expect
    assert (bound == "hbm") == (unit == "GB/s")
