"""The vector and transform kernels' gfx950 code has no store of more than 8
bytes whose data registers the next instruction overwrites.

Such a store (its row offset in a scalar register) reads its data a cycle
after issue; the compiler inserts no wait state for that form, so a value
written by the following instruction is what lands in memory. The stencil
passes once stored the residual scaled for its FP16 copy that way (the
solves then stalled). Their stores are now at most 8 bytes wide. The 16-bit
transforms store 16 bytes per lane with global stores, for which the
compiler does insert the wait. This test compiles both sources to gfx950
assembly (no GPU needed) and scans them.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "paper_1903_12227_amd", "csrc", f) for f in ("kernels_vec.hip", "kernels_gemm.hip")]


def _hipcc():
    cand = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return cand if os.path.exists(cand) else shutil.which("hipcc")


def _regs(op):
    m = re.match(r"v\[(\d+):(\d+)\]$", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", op)
    return {int(m.group(1))} if m else set()


def wide_store_hazards(asm_lines):
    """(store, next instruction) pairs where a store of 12 or 16 bytes is
    followed directly by an instruction writing one of its data VGPRs."""
    label = re.compile(r"^[A-Za-z_.$][\w.$]*:\s*(;.*)?$")
    code = [ln.strip() for ln in asm_lines
            if ln.strip() and not ln.strip().startswith((";", ".")) and not label.match(ln.strip())]
    out = []
    for cur, nxt in zip(code, code[1:]):
        m = re.match(r"(buffer|global|flat)_store_dwordx[34]\s+(.*)$", cur)
        if not m:
            continue
        ops = [o.strip() for o in m.group(2).split(",")]
        data = _regs(ops[0] if m.group(1) == "buffer" else ops[1])
        d = re.match(r"(v_\S+)\s+([^,\s]+)", nxt)
        if d and data & _regs(d.group(2)):
            out.append((cur, nxt))
    return out


def test_scanner_finds_the_pattern():
    # the pair the stencil pass once produced, and two harmless ones
    bad = ["buffer_store_dwordx4 v[2:5], v88, s[36:39], s74 offen nt", "v_mul_f64 v[2:3], s[18:19], v[2:3]"]
    ok1 = ["buffer_store_dwordx4 v[2:5], v88, s[36:39], s74 offen nt", "s_nop 0", "v_mul_f64 v[2:3], s[18:19], v[2:3]"]
    ok2 = ["buffer_store_dwordx2 v[2:3], v88, s[36:39], s74 offen nt", "v_mul_f64 v[2:3], s[18:19], v[2:3]"]
    assert len(wide_store_hazards(bad)) == 1
    assert wide_store_hazards(ok1) == [] and wide_store_hazards(ok2) == []


@pytest.mark.timeout(900)
def test_kernels_have_no_wide_store_data_hazard(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    jobs = []
    for src in SRCS:
        out = tmp_path / (os.path.basename(src) + ".s")
        cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out), src]
        jobs.append((src, out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    for src, out, proc in jobs:
        _, err = proc.communicate()
        assert proc.returncode == 0, (src, err[-2000:])
        with open(out) as f:
            hits = wide_store_hazards(f.readlines())
        assert hits == [], (src, hits[:5])
