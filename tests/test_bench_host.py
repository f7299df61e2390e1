"""Host-side logic of bench.py, on the CPU: the single-GPU guard, the
algorithmic byte count behind the product's roofline figure, and the rule
that ties a committed counter summary to the kernel sources it was taken on."""
import os
import subprocess
import sys

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_video_product_algorithmic_bytes():
    # one fused-product launch on the video-shaped operands (FP32): read P and
    # write Q once (8 B per entry), both Laplacians once in CSR (int32 index
    # and FP32 value per entry, int32 row pointers), the two byte masks; the
    # figure the roofline fraction and the traffic ratio are quoted against
    P = synth.cfg3_video(0)
    assert (P.p, P.n) == (20480, 4096)
    counted = (8 * P.p * P.n + 8 * P.Lr.nnz + 4 * (P.p + 1) + 8 * P.Lc.nnz + 4 * (P.n + 1)
               + P.p + P.n)
    assert bench.algorithmic_apply_bytes(P, 4) == counted == 673697688
    # FP64 operands: 16 B per entry and 12 B per operator entry
    assert bench.algorithmic_apply_bytes(P, 8) == (16 * P.p * P.n + 12 * (P.Lr.nnz + P.Lc.nnz)
                                                 + 4 * (P.p + P.n + 2) + P.p + P.n)


def test_counter_traffic_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    summary = tmp_path / "summary.md"
    summary.write_text("kernel source hash: `0123abcd`\n\n"
                       "HBM bytes per launch (fetch + write, calibrated): `929268807`\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123abcd")
    assert bench.measured_traffic("video", "fp32_ir") == 929268807
    # taken for the video workload in FP32 with residual replacement only
    assert bench.measured_traffic("face", "fp32_ir") is None
    assert bench.measured_traffic("video", "fp64") is None
    # kernel sources changed since: no traffic figure
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "89abcdef")
    assert bench.measured_traffic("video", "fp32_ir") is None
    # a summary without the figure
    summary.write_text("kernel source hash: `89abcdef`\n")
    assert bench.measured_traffic("video", "fp32_ir") is None


def test_kernel_source_hash_covers_the_product_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    for rel in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel
