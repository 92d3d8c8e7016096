"""Host logic of bench.py, no GPU: the algorithmic bytes per node of each
kernel (the figures its roofline divides by launch time), the launch
accounting over iteration counts, the choice between the HBM and MFMA roofs
and their arithmetic, the fingerprint that ties committed traffic counters to
the kernel code, and the refusal of more than one GPU."""
import json
import math
import os
import shutil
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bytes_per_node_matches_the_kernels_accesses():
    # headline: BF16 transforms, two-valued fields (one coefficient byte per
    # cell), the next direction formed in the last transform: the apply reads
    # p of both systems (2 x 4) and a; each 16-bit transform reads and writes
    # one 2-byte value, the last also reads p_k and writes p_{k+1} (4 + 4);
    # the update reads r (8), p (4), half of a's byte, writes r (8) and the
    # BF16 copy (2); the fold reads each direction once (4)
    b = bench.bytes_per_node("bf16", flexible=False, coef_bytes=1, pdirect=True)
    assert b == {"stencil": 9, "gemm1": 4, "gemm2": 4, "gemm3": 4, "gemm4": 10, "update_r": 22.5, "fold_x": 4}
    # the same with the directions stored in BF16: 2 bytes less in each of
    # the apply's reads (both systems), the last transform's write and read,
    # the update's read and the fold's read
    b = bench.bytes_per_node("bf16", flexible=False, coef_bytes=1, pdirect=True, dir_bytes=2)
    assert b == {"stencil": 5, "gemm1": 4, "gemm2": 4, "gemm3": 4, "gemm4": 6, "update_r": 20.5, "fold_x": 2}
    # three dimensions: one system per apply workgroup (a read per system),
    # six transforms (gemm3: the four plain ones), FP32 directions
    assert bench.bytes_per_node_3d("bf16") == {"stencil": 28, "gemm1": 4, "gemm2": 4, "gemm3": 16, "gemm4": 8,
                                               "update_r": 26, "fold_x": 4}
    # the apply fused with the direction step: reads z and p_old, writes p_new
    assert bench.bytes_per_node("bf16", False, 1)["stencil"] == 25
    assert bench.bytes_per_node("bf16", False, 8)["stencil"] == 32
    assert bench.bytes_per_node("fp64", False, 1)["stencil"] == 49
    assert bench.bytes_per_node("bf16", False, 8)["update_r"] == 26
    assert bench.bytes_per_node("fp64", False, 1)["update_r"] == 24.5
    assert bench.bytes_per_node("bf16", True, 1)["update_r"] == 26.5       # + z (flexible beta)
    # FP64 / FP32 transforms: the last writes z and re-reads r for r.z
    assert bench.bytes_per_node("fp64", False, 8)["gemm4"] == 24
    assert bench.bytes_per_node("fp32", False, 8)["gemm4"] == 12
    assert bench.bytes_per_node("fp64", False, 8)["gemm1"] == 16


def test_kernel_entries_count_realizations_systems_and_folds():
    from paper_1903_12227_amd import DIRECTION_RING
    n = 64
    N2 = n * n
    it = torch.tensor([[[3, 5], [8, 2]], [[1, 1], [12, 30]]])      # (steps, B, 2)
    tim = {k: (1.0, 10) for k in ("stencil", "gemm1", "gemm2", "gemm3", "gemm4", "update_r", "fold_x")}
    e = bench.kernel_entries(tim, it, n, "bf16", False, coef_bytes=1, pdirect=True)
    real_iters = 5 + 8 + 1 + 30          # the apply runs while either system of a realization iterates
    sys_iters = 3 + 5 + 8 + 2 + 1 + 1 + 12 + 30
    folds = sum(math.ceil(v / DIRECTION_RING) for v in (3, 5, 8, 2, 1, 1, 12, 30))
    assert e["stencil"]["bytes"] == real_iters * 9 * N2
    assert e["update_r"]["bytes"] == sys_iters * 22.5 * N2
    assert e["gemm4"]["bytes"] == sys_iters * 10 * N2
    assert e["gemm2"]["flops"] == sys_iters * 2.0 * n * N2
    assert e["fold_x"]["bytes"] == sys_iters * 4 * N2 + 16.0 * folds * N2
    assert "flops" not in e["update_r"]


def test_roofline_picks_the_roof_and_divides_by_launch_time():
    n, S = 512, 512
    N2 = n * n
    # 16-bit transform: 2n flops per 4 bytes = 256 flop/B, below the ridge of
    # 2500 TFLOP/s over 8 TB/s (312.5 flop/B): HBM-bound
    e = {"ms": 2.0, "launches": 10, "bytes": 4.0 * N2 * S * 10, "flops": 2.0 * n * N2 * S * 10}
    r = bench.roofline_for("gemm1", e, "bf16", n)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(e["bytes"] / 2e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_ms"] == pytest.approx(0.2)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(e["bytes"] / 10)
    # FP64 transform: 1024 flops per 24 bytes, far above the FP64 ridge
    # (78.6 TFLOP/s over 8 TB/s): MFMA-bound, against the FP64 peak
    e64 = {"ms": 2.0, "launches": 10, "bytes": 24.0 * N2 * S * 10, "flops": 2.0 * n * N2 * S * 10}
    r = bench.roofline_for("gemm1", e64, "fp64", n)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(e64["flops"] / 2e-3 / 1e12)
    # a kernel without flops is HBM-bound
    r = bench.roofline_for("update_r", {"ms": 1.0, "launches": 4, "bytes": 8e9}, "bf16", n)
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx(8000.0) and r["frac"] == pytest.approx(1.0)


def test_source_fingerprint_ignores_comments_but_not_code(tmp_path, monkeypatch):
    h_repo = bench.kernel_source_hash()
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h_repo
    f = tmp_path / bench.KERNEL_SOURCES[3]
    f.write_text(f.read_text() + "\n// a note\n/* a block\n   comment */\n\n")
    assert bench.kernel_source_hash() == h_repo
    f.write_text(f.read_text() + "\nstatic int rve_unused_value = 1;\n")
    assert bench.kernel_source_hash() != h_repo


def test_traffic_is_reported_only_for_the_kernel_code_it_was_measured_on(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("update_r") is None                     # no file
    path.write_text(json.dumps({"source_hash": bench.kernel_source_hash(),
                                "kernels": {"update_r": {"hbm_bytes_per_launch": 3.0e9}}}))
    assert bench.measured_traffic("update_r") == 3.0e9
    assert bench.measured_traffic("fold_x") is None                       # kernel not measured
    path.write_text(json.dumps({"source_hash": "0" * 16,
                                "kernels": {"update_r": {"hbm_bytes_per_launch": 3.0e9}}}))
    assert bench.measured_traffic("update_r") is None                     # other kernel code


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert res.returncode == 2
    assert "--gpus above 1 is not supported" in res.stderr
