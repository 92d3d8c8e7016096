"""Throughput of the RVE corrector path on one MI355X.

One step = the whole hot path over one batch of realizations already resident
in HBM: Galerkin right-hand sides, PCG solves of both correctors (matrix-free
Q1 stencil, Hartley-transform preconditioner on MFMA), A_hom in energy and
flux form, the per-cell gradient of A_11 and A_12 with the contrast
derivative, and the ensemble statistics of the batch.

Workload: L = 64, h = 1/8 (n = 512 nodes per axis), 256 realizations per
step, Poisson(ln 2 L^2) unit-square inclusions, contrast 10, tolerance 1e-10.
The headline value runs the preconditioner GEMMs in BF16 (FP32 accumulation)
with FP64 residuals, dots and A_hom; beside it: the same step with scaled
FP16 transforms, in FP64, at B = 64, with the inputs copied from pinned host
memory in the timed region, and the plain per-realization FP64 PCG.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
Prints one JSON line.

    python bench.py --survey
Times the other workloads of the study instead (one JSON line each): one
realization at L = 8; 256 at L = 32 with their mean and variance; 1024 of
mixed L in {8, 16, 32, 64} at contrast 100 with FP64 and FP32 operator
applies; 16 at L = 128, h = 1/16 with BF16, FP16 and FP32 transforms against
FP64; an FFT comparison point for the preconditioner; the gradient at L = 64
for 64 realizations and the quartic tensor of 4096 realizations at L = 16;
on-device sampling and ensembles; the paper's table of standard deviations;
the spectral density; and the three-dimensional workloads (also alone with
--survey3d).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RVE realizations/sec (2 corrector solves + A_hom) at L=64, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3, "fp64": 78.6}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_batches(model, count, B, config=1):
    from sampler import batch
    return [batch(model, config, B, start=k * B) for k in range(count)]


def run_step(rve, a, h, opts, G, contrast, L):
    res = rve.solve_batch(a, h, opts, want_phi=True, want_flux=True)
    g, gin, _ = rve.grad(a, res.phi, h, G, a_in=contrast)
    st = rve.stats(res.ahom, L)
    return res, g, gin, st


def timed_steps(rve, torch, batches_dev, h, opts, G, contrast, L, warmup, steps, ctx, timing=False):
    for k in range(warmup):
        run_step(rve, batches_dev[k % len(batches_dev)], h, opts, G, contrast, L)
    torch.cuda.synchronize()
    if timing:
        ctx.set_timing(True)
    iters, codes = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        res, _, _, _ = run_step(rve, batches_dev[(warmup + k) % len(batches_dev)], h, opts, G,
                                contrast, L)
        iters.append(res.iters)
        codes.append(res.code)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = ctx.timing() if timing else None
    if timing:
        ctx.set_timing(False)
    it = torch.stack(iters).to(torch.float64)
    return (t1 - t0), it, tim, codes


def bytes_per_node(prec_name, flexible, coef_bytes=8, pdirect=False, dir_bytes=None):
    """Algorithmic HBM bytes per node of each kernel, per corrector system
    (the operator apply: per realization, both systems).

    coef_bytes: bytes per cell of the coefficients the operator kernels read:
    8 (FP64), or 1 when every field of the batch is two-valued (the library
    then reads one byte per cell, decoded exactly).
    pdirect: the last transform forms the next direction (16-bit tile
    transforms with the standard beta): it reads p_old and writes p instead of
    z, and the apply reads p alone.
    dir_bytes: bytes per value of the directions p where they differ from
    s_p (2: stored in BF16 where the last transform forms them).

    FP64 path: every vector FP64. Mixed paths: the directions p and z are
    stored in FP32 (s_p = 4) and the residual has a copy in the GEMM
    precision (s_g bytes) that the first transform reads; x, r stay FP64.
    With the FP64 operator apply (all workloads timed here) q = A p is never
    stored: the residual update recomputes it from p_new and a.
      stencil   fused direction step + operator apply: read z, p_old;
                write p_new (per system), read a (once)
      gemm1     read the r copy (FP64 r on the FP64 path), write T1
      gemm2     read T1, write W = (Q R Q)./(a0 E)   (1/E: a shared table, or
                formed in the 16-bit kernels; those also take r.z here, as
                the sum of (Q R Q) .* W)
      gemm3     read W, write T3
      gemm4     read T3, write z; FP64 / FP32 transforms also re-read the
                residual the transforms started from (FP64 r, or the r copy)
                for r.z
      update_r  read r, p_new, a (shared by the two systems: 4 bytes each)
                [+ z for flexible beta]; write r [+ r copy]
      fold_x    x += sum alpha_j p_j over the direction ring: per fold,
                read and write x; per direction, read p once (handled in
                kernel_entries: 16 ceil(iters / ring) + s_p iters per system)
    """
    sg = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[prec_name]
    sp = 8 if prec_name == "fp64" else 4
    # the directions p (BF16 where the last transform forms them, unless
    # switched off; z, never stored then, does not appear)
    sd = sp if dir_bytes is None else dir_bytes
    lo = 0 if prec_name == "fp64" else sg
    first_in = 8 if prec_name == "fp64" else sg
    return {
        "stencil": (2 * sd if pdirect else 2 * (sp + sp + sp)) + coef_bytes,
        "gemm1": first_in + sg,
        "gemm2": 2 * sg,
        "gemm3": 2 * sg,
        "gemm4": sg + (2 * sd if pdirect else sp) + (0 if sg == 2 else first_in),
        "update_r": 8 + sd + coef_bytes / 2 + 8 + lo + (sp if flexible else 0),
        "fold_x": sd,
    }


def kernel_entries(tim, it_all, n, prec_name, flexible, coef_bytes=8, pdirect=False, dir_bytes=None):
    """Per-kernel algorithmic bytes (and flops) summed over the timed launches.

    it_all: (steps, B, 2) iteration counts. A realization takes part in the
    operator apply while either of its systems iterates (max over the two);
    a system takes part in each residual update and each preconditioner
    apply (one before the loop and one per continuing iteration) = iters;
    the iterate update folds each direction into x once and reads and writes
    x once per ring of directions, ceil(iters / DIRECTION_RING) times."""
    import math
    from paper_1903_12227_amd import DIRECTION_RING
    N2 = float(n * n)
    real_iters = float(it_all.max(dim=2).values.sum())
    sys_iters = float(it_all.sum())
    folds = float(sum(math.ceil(v / DIRECTION_RING) for v in it_all.flatten().tolist()))
    bpn = bytes_per_node(prec_name, flexible, coef_bytes, pdirect, dir_bytes)
    units = {"stencil": real_iters, "gemm1": sys_iters, "gemm2": sys_iters, "gemm3": sys_iters,
             "gemm4": sys_iters, "update_r": sys_iters, "fold_x": sys_iters}
    out = {}
    for k, u in units.items():
        ms, cnt = tim[k]
        e = {"ms": ms, "launches": cnt, "bytes_per_node": bpn[k], "bytes": u * bpn[k] * N2}
        if k == "fold_x":
            e["bytes"] += 16.0 * folds * N2
        if k.startswith("gemm"):
            e["flops"] = u * 2.0 * n * N2            # one n x n x n product per system
        out[k] = e
    return out


def roofline_for(name, e, prec_name, n):
    """Roofline of one kernel: HBM-bound unless its arithmetic intensity
    (flops per algorithmic byte) times the HBM peak exceeds the MFMA peak."""
    sec = e["ms"] * 1e-3
    avg = e["ms"] / max(e["launches"], 1)
    if "flops" in e:
        ai = e["flops"] / e["bytes"]
        peak_f = MFMA_PEAK_TFS[prec_name]
        if ai * HBM_PEAK_GBS / 1e3 > peak_f:
            ach = e["flops"] / sec / 1e12
            return {"kernel": name, "bound": "mfma", "achieved": ach, "peak": peak_f, "unit": "TFLOP/s",
                    "frac": ach / peak_f, "traffic": None, "avg_launch_ms": avg,
                    "intensity_flop_per_byte": ai}
    ach = e["bytes"] / sec / 1e9
    out = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ach / HBM_PEAK_GBS, "traffic": None, "avg_launch_ms": avg,
           "algorithmic_bytes_per_launch": e["bytes"] / max(e["launches"], 1)}
    if "flops" in e:
        out["intensity_flop_per_byte"] = e["flops"] / e["bytes"]
    return out


KERNEL_SOURCES = ("paper_1903_12227_amd/csrc/common.h", "paper_1903_12227_amd/csrc/launch.h",
                  "paper_1903_12227_amd/csrc/stencil2d.h",
                  "paper_1903_12227_amd/csrc/kernels_vec.hip", "paper_1903_12227_amd/csrc/kernels_gemm.hip",
                  "paper_1903_12227_amd/csrc/rve_api.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_L64_n512_b256.json")


def kernel_source_hash():
    """Fingerprint of the code of the kernel sources: comments and whitespace
    are left out, so an edit of a comment keeps the committed counters valid
    while any change of code invalidates them."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            t = f.read()
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(re.sub(r"\s+", " ", t).strip().encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if it is absent or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    k = data.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def copy_calibration(torch, dev):
    """One plain device copy of a known size (2^28 bytes read, 2^28 written),
    whose FETCH_SIZE / WRITE_SIZE counters calibrate the traffic figures."""
    src = torch.ones(2 ** 25, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--m0", type=int, default=8)
    ap.add_argument("--contrast", type=float, default=10.0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--plain", type=int, default=8, help="realizations for the per-realization FP64 leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines file of autotuned kernel choices to read and extend "
                         "(lets profiling runs replay the choices of a normal run)")
    ap.add_argument("--survey", action="store_true", help="time the other workloads instead")
    ap.add_argument("--survey3d", action="store_true", help="time only the three-dimensional workloads")
    ap.add_argument("--systematic", action="store_true",
                    help="the paper's systematic-error study: ensemble means at L = 16..128 (N realizations "
                         "each, checkpointed) under the fixed-count and Poisson-count laws")
    ap.add_argument("--systematic-n", type=int, default=100000)
    ap.add_argument("--checkpoint-dir", default=None)
    args = ap.parse_args()
    if args.tune_cache:
        os.environ["RVE_TUNE_CACHE"] = args.tune_cache

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the realizations are independent and the library runs "
              "on a single MI355X; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1903_12227_amd as rve
    from sampler import BooleanModel

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.survey:
        survey(rve, torch, dev)
        return
    if args.survey3d:
        survey_3d(rve, torch, dev, lambda name, **kw: print(json.dumps({"survey": name, **kw}), flush=True))
        return
    if args.systematic:
        systematic(rve, torch, dev, args.systematic_n, args.checkpoint_dir)
        return
    L, m0, B = args.L, args.m0, args.batch
    n, h = L * m0, 1.0 / m0
    model = BooleanModel(L=L, m0=m0, a_in=args.contrast, a_bg=1.0)
    nb = args.warmup + args.steps
    log(f"sampling {min(nb, 3)} batches of {B} realizations at n={n}")
    host = make_batches(model, min(nb, 3), B)
    batches = [torch.from_numpy(x).to(dev) for x in host]
    G = torch.zeros((B, 2, 2), dtype=torch.float64, device=dev)
    G[:, 0, 0] = 1.0      # d A_11 + d A_12
    G[:, 0, 1] = 1.0
    ctx = rve.context(0)
    copy_calibration(torch, dev)

    # headline: mixed precision (BF16 transform GEMMs), batched
    mixed = rve.Options(tol=args.tol, prec=rve.MIX_BF16)
    log("mixed-precision leg")
    t_mix, it_mix, tim_mix, codes = timed_steps(rve, torch, batches, h, mixed, G, args.contrast, L,
                                                args.warmup, args.steps, ctx, timing=False)
    if max(codes) != 0:
        raise SystemExit(f"mixed leg: non-converged or failed items (codes {codes})")
    # the same leg again with per-kernel event timing on the library's stream
    _, it_mix_t, tim_mix, _ = timed_steps(rve, torch, batches, h, mixed, G, args.contrast, L, 0,
                                          args.steps, ctx, timing=True)
    value = args.steps * B / t_mix

    log("FP64 batched leg")
    fp64 = rve.Options(tol=args.tol, prec=rve.FP64)
    t64, it64, tim64, codes64 = timed_steps(rve, torch, batches, h, fp64, G, args.contrast, L, 1,
                                            args.fp64_steps, ctx, timing=True)
    v64 = args.fp64_steps * B / t64

    log("FP16-transform leg")
    half = rve.Options(tol=args.tol, prec=rve.MIX_FP16)
    t16, it16, _, codes16 = timed_steps(rve, torch, batches, h, half, G, args.contrast, L, 1, args.steps, ctx)
    if max(codes16) != 0:
        raise SystemExit(f"FP16 leg: non-converged or failed items (codes {codes16})")
    v16 = args.steps * B / t16

    log("B = 64 and host-resident legs")
    b64 = [x[:64].contiguous() for x in batches]
    t_b64, _, _, _ = timed_steps(rve, torch, b64, h, mixed, G[:64].contiguous(), args.contrast, L, 1,
                                 args.steps, ctx)
    v_b64 = args.steps * 64 / t_b64
    # inputs resident in pinned host memory: each step first copies its batch
    # to the device (PCIe-inclusive rate; `value` keeps inputs in HBM)
    pinned = [torch.from_numpy(x).pin_memory() for x in host]
    a_buf = torch.empty_like(batches[0])
    a_buf.copy_(pinned[0], non_blocking=True)
    run_step(rve, a_buf, h, mixed, G, args.contrast, L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        a_buf.copy_(pinned[k % len(pinned)], non_blocking=True)
        run_step(rve, a_buf, h, mixed, G, args.contrast, L)
    torch.cuda.synchronize()
    v_h2d = args.steps * B / (time.perf_counter() - t0)
    del pinned, a_buf, b64

    log("plain per-realization FP64 leg")
    single = batches[0][: args.plain]
    rve.solve_batch(single[0:1].contiguous(), h, fp64, want_phi=True, want_flux=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(args.plain):
        rve.solve_batch(single[b:b + 1].contiguous(), h, fp64, want_phi=True, want_flux=True)
    torch.cuda.synchronize()
    v_plain = args.plain / (time.perf_counter() - t0)

    # flux form against energy form for each realization of the first timed
    # batch, headline options, outside every timed region: the gap is set by
    # the correctors' accuracy, and the flux form's asymmetry is what the
    # paper tabulates against the tolerance (Sec. 4.1, Table conv_Symmet_thresh)
    rf = rve.solve_batch(batches[0], h, mixed, want_phi=False, want_flux=True)
    Ae, Af = rf.ahom.cpu().numpy(), rf.ahom_flux.cpu().numpy()
    fscale = np.maximum(np.abs(Ae[:, 0, 0]), np.abs(Ae[:, 1, 1]))
    fgap = np.abs(Af - Ae).reshape(len(fscale), -1).max(axis=1) / fscale
    fasym = np.abs(Af[:, 0, 1] - Af[:, 1, 0]) / fscale
    flux_gap = {"realizations": int(len(fscale)), "tol": args.tol, "max_rel": float(fgap.max()),
                "median_rel": float(np.median(fgap)), "flux_asym_max_rel": float(fasym.max()),
                "flux_asym_median_rel": float(np.median(fasym))}
    del rf

    # roofline of the dominant kernel (largest total event time) of the headline leg
    # every field here takes two values only, so the operator kernels read
    # one byte per cell (the library's rule: each cell equals its field's
    # minimum or maximum)
    two_valued = all(bool(np.all((x == x.min(axis=(1, 2), keepdims=True)) | (x == x.max(axis=(1, 2), keepdims=True))))
                     for x in host)
    coef_bytes = 1 if two_valued else 8
    # the last transform forms the next direction with the 16-bit tile
    # variants (every one but 0 and the folded 2) and the standard beta
    tuned = ctx.tuned(n, rve.MIX_BF16, B)
    pdirect = tuned["gemm_variant"] not in (0, 2, -1)
    # ... and stores it in BF16 (the library's default)
    dir_bytes = 2 if pdirect else None
    ent = kernel_entries(tim_mix, it_mix_t, n, "bf16", flexible=False, coef_bytes=coef_bytes, pdirect=pdirect,
                         dir_bytes=dir_bytes)
    dom = max(ent, key=lambda k: ent[k]["ms"])
    roof = roofline_for(dom, ent[dom], "bf16", n)
    roof["traffic"] = measured_traffic(dom)
    kernels = {}
    for k, v in ent.items():
        r = roofline_for(k, v, "bf16", n)
        kernels[k] = {"ms_total": v["ms"], "launches": v["launches"], "bytes_per_node": v["bytes_per_node"],
                      "bound": r["bound"], "achieved": r["achieved"], "unit": r["unit"], "frac": r["frac"]}
    ent64 = kernel_entries(tim64, it64, n, "fp64", flexible=False, coef_bytes=coef_bytes)
    g64 = [ent64[k] for k in ("gemm1", "gemm2", "gemm3", "gemm4")]
    fp64_gemm_tfs = sum(e["flops"] for e in g64) / (sum(e["ms"] for e in g64) * 1e-3) / 1e12

    cpu, oracle_ahoms = None, []
    if not args.no_cpu:
        cpu, oracle_ahoms = cpu_baseline(host[0], args.cpu_seconds)

    # error of each leg against the oracle, on the items of the first timed
    # batch that the CPU-baseline leg solved (outside every timed region)
    oracle_err = None
    if oracle_ahoms:
        import numpy as np
        k = len(oracle_ahoms)
        ref = np.stack(oracle_ahoms)
        oracle_err = {"items": k, "oracle_tol": 1e-10}
        for name, o in (("bf16", mixed), ("fp16", half), ("fp64", fp64)):
            # the whole timed batch (same shape and kernel choices as timed)
            got = rve.solve_batch(batches[0], h, o, want_phi=False).ahom[:k].cpu().numpy()
            scale = np.maximum(np.abs(ref[:, 0, 0]), np.abs(ref[:, 1, 1]))
            oracle_err[name] = float(np.max(np.abs(got - ref).reshape(k, -1).max(axis=1) / scale))

    line = {
        "metric": METRIC, "value": value, "unit": "realizations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_mix / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+bf16", "data": "synthetic",
        "config": {"workload": f"L={L} h=1/{m0} (n={n}), {B} realizations per step, contrast "
                               f"{args.contrast:g}, tol {args.tol:g}, Poisson(ln2 L^2) unit squares; "
                               "BF16 transform GEMMs, FP64 residual/dots/A_hom",
                   "L": L, "n": n, "batch": B, "contrast": args.contrast, "tol": args.tol,
                   "precision": "mixed-bf16"},
        "iters_mean": float(it_mix.mean()),
        "tuned": tuned,
        "mixed_fp16_transforms": {"value": v16, "ms_per_step": 1e3 * t16 / args.steps,
                                  "iters_mean": float(it16.mean())},
        "fp64_batched": {"value": v64, "ms_per_step": 1e3 * t64 / args.fp64_steps,
                         "iters_mean": float(it64.mean()), "gemm_TFLOPs": fp64_gemm_tfs},
        "plain_fp64_per_realization": {"value": v_plain, "realizations": args.plain},
        "batch_64": {"value": v_b64, "ms_per_step": 1e3 * t_b64 / args.steps},
        "host_inputs_pcie_inclusive": {"value": v_h2d, "note": "each step copies its batch from pinned host "
                                                               "memory to the device inside the timed region"},
        "speedup_vs_plain_fp64": value / v_plain,
        "speedup_vs_fp64_batched": value / v64,
        "ahom_rel_err_vs_oracle": oracle_err,
        "flux_energy_gap": flux_gap,
        "roofline": roof,
        "kernels": kernels,
        "coefficient_bytes_per_cell": coef_bytes,
        "direction_in_last_transform": pdirect,
        "direction_bytes": dir_bytes or 4,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


STORED_ORACLE = os.path.join(ROOT, "tests", "golden", "config_sizes.json")


def stored_oracle_error(name, field, A):
    """Relative error (max |dA_ij| / max_i |A_ii|) of one result against the
    oracle's A_hom for the same input, stored by
    tests/golden/make_config_sizes.py (which calls only the oracle; about a
    minute of host time per item at these sizes). None when the stored input
    is not this field."""
    import hashlib

    import numpy as np
    with open(STORED_ORACLE) as f:
        g = json.load(f)[name]
    h = hashlib.sha256(np.ascontiguousarray(field, dtype=np.float64).tobytes()).hexdigest()[:16]
    if h != g["field_sha256_16"]:
        return None
    R, A = np.array(g["ahom"]), np.asarray(A)
    return float(np.max(np.abs(A - R)) / np.max(np.abs(np.diagonal(R))))


def survey(rve, torch, dev):
    """One JSON line per workload: wall time per call (after one warm-up call
    of the same shape, so tuning and graph capture are excluded), mean PCG
    iterations, and where a reference run exists the largest relative A_hom
    deviation from it (max |dA_ij| / max(|A_11|, |A_22|))."""
    import numpy as np

    from sampler import BooleanModel, batch, uneven_batch

    def timed(fn, reps=1):
        out = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    def dev_rel(A, R):
        A, R = A.cpu().numpy(), R.cpu().numpy()
        scale = np.maximum(np.abs(R[:, 0, 0]), np.abs(R[:, 1, 1]))
        return float(np.max(np.abs(A - R).reshape(len(A), -1).max(axis=1) / scale))

    def emit(name, **kw):
        print(json.dumps({"survey": name, **kw}), flush=True)

    def fields(L, m0, contrast, count, config):
        return torch.from_numpy(batch(BooleanModel(L=L, m0=m0, a_in=contrast), config, count)).to(dev)

    # one realization, L = 8 (n = 64), FP64: latency, with the
    # single-workgroup solver (the default at this size) and with the batched
    # iteration chunks (graph replay or launched one by one); then many
    # realizations at that size both ways
    a = fields(8, 8, 10.0, 1, 11)
    for small, graphs in ((True, True), (False, True), (False, False)):
        ctx = rve.Context(0)
        ctx.set_small_solver(small)
        ctx.set_graphs(graphs)
        dt, r = timed(lambda: rve.solve_batch(a, 1 / 8, rve.Options(prec=rve.FP64), ctx=ctx), reps=20)
        emit("L=8 n=64, 1 realization, FP64", single_workgroup_solver=small, graphs=graphs, ms=1e3 * dt,
             iters_mean=float(r.iters.double().mean()))
        ctx.close()
    a = fields(8, 8, 10.0, 1024, 18)
    for small in (True, False):
        ctx = rve.Context(0)
        ctx.set_small_solver(small)
        dt, r = timed(lambda: rve.solve_batch(a, 1 / 8, rve.Options(prec=rve.FP64), want_phi=False, ctx=ctx), reps=3)
        emit("L=8 n=64, 1024 realizations, FP64", single_workgroup_solver=small, ms=1e3 * dt,
             realizations_s=1024 / dt, iters_mean=float(r.iters.double().mean()))
        ctx.close()

    # 256 realizations at L = 32 (n = 256) with mean and variance
    a = fields(32, 8, 10.0, 256, 12)
    for prec, name in ((rve.FP64, "fp64"), (rve.MIX_BF16, "bf16")):
        def step():
            r = rve.solve_batch(a, 1 / 8, rve.Options(prec=prec), want_phi=False)
            return r, rve.stats(r.ahom, 32.0)
        dt, (r, st) = timed(step, reps=3)
        emit("L=32 n=256, 256 realizations + mean/variance", gemm=name, ms=1e3 * dt,
             realizations_s=256 / dt, iters_mean=float(r.iters.double().mean()))
        if prec == rve.FP64:
            ref = r.ahom

    # 1024 realizations of L in {8, 16, 32, 64}, contrast 100, FP64 vs FP32 operator apply;
    # the first L = 32 and L = 64 items are inputs whose oracle A_hom is stored
    mix = uneven_batch([8, 16, 32, 64], m0=8, a_in=100.0, a_bg=1.0, config=3, per_size=256)
    ft = [torch.from_numpy(f).to(dev) for _, f in mix]
    stored3 = [(f"c3_n{8 * L}_contrast100", next(k for k, (LL, _) in enumerate(mix) if LL == L)) for L in (32, 64)]
    ref = None
    for prec, pname in ((rve.FP64, "fp64"), (rve.MIX_BF16, "bf16"), (rve.MIX_FP16, "fp16")):
        for sprec, sname in ((0, "fp64"), (1, "fp32")):
            o = rve.Options(prec=prec, stencil_prec=sprec)
            dt, r = timed(lambda: rve.solve_uneven(ft, 1 / 8, o))
            if ref is None:
                ref = r.ahom
            Ah = r.ahom.cpu().numpy()
            errs = {nm: stored_oracle_error(nm, mix[k][1], Ah[k]) for nm, k in stored3}
            emit("1024 realizations, L in {8,16,32,64} (n 64..512), contrast 100", gemm=pname, stencil=sname,
                 ms=1e3 * dt, realizations_s=len(ft) / dt, iters_mean=float(r.iters.double().mean()),
                 ahom_rel_err_vs_oracle=errs, ahom_rel_dev_vs_fp64=dev_rel(r.ahom, ref), code=r.code)

    # 16 realizations at L = 128, h = 1/16 (n = 2048); the first is the input
    # whose oracle A_hom is stored
    a = fields(128, 16, 10.0, 16, 4)
    a0 = a[0].cpu().numpy()
    r64 = rve.solve_batch(a, 1 / 16, rve.Options(prec=rve.FP64), want_phi=False)
    ctx4 = rve.Context(0)
    for prec, pname in ((rve.MIX_BF16, "bf16"), (rve.MIX_FP16, "fp16"), (rve.MIX_FP32, "fp32"), (rve.FP64, "fp64")):
        dt, r = timed(lambda: rve.solve_batch(a, 1 / 16, rve.Options(prec=prec), want_phi=False, ctx=ctx4))
        # transform-GEMM utilisation from an event-timed solve: 2 n^3 flops per
        # system and transform, four transforms per apply, iters applies per system
        ctx4.set_timing(True)
        rt = rve.solve_batch(a, 1 / 16, rve.Options(prec=prec), want_phi=False, ctx=ctx4)
        torch.cuda.synchronize()
        tim = ctx4.timing()
        ctx4.set_timing(False)
        gms = sum(tim[k][0] for k in ("gemm1", "gemm2", "gemm3", "gemm4"))
        gfl = float(rt.iters.double().sum()) * 4 * 2.0 * 2048.0 ** 3
        tfs = gfl / (gms * 1e-3) / 1e12
        emit("L=128 h=1/16 n=2048, 16 realizations", gemm=pname, ms=1e3 * dt, realizations_s=16 / dt,
             iters_mean=float(r.iters.double().mean()),
             ahom_rel_err_vs_oracle={"c4_n2048": stored_oracle_error("c4_n2048", a0, r.ahom[0].cpu().numpy())},
             ahom_rel_dev_vs_fp64=dev_rel(r.ahom, r64.ahom), gemm_TFLOPs=tfs, gemm_peak_frac=tfs / MFMA_PEAK_TFS[pname])
    ctx4.close()
    del a, r64

    # comparison point: the same preconditioner apply by real FFTs (the
    # vendor FFT through torch, not part of the path), 512 systems of 512^2
    # (the headline batch), against the transform GEMMs' event time per apply
    a = fields(64, 8, 10.0, 256, 17)
    ctxp = rve.Context(0)
    rve.solve_batch(a, 1 / 8, rve.Options(prec=rve.MIX_BF16), want_phi=False, ctx=ctxp)
    ctxp.set_timing(True)
    rve.solve_batch(a, 1 / 8, rve.Options(prec=rve.MIX_BF16), want_phi=False, ctx=ctxp)
    torch.cuda.synchronize()
    tim = ctxp.timing()
    ctxp.set_timing(False)
    ctxp.close()
    per_apply = sum(tim[k][0] for k in ("gemm1", "gemm2", "gemm3", "gemm4")) / max(tim["gemm1"][1], 1)
    c = torch.cos(2 * torch.pi * torch.arange(512, dtype=torch.float64, device=dev) / 512)
    E = (8 - 2 * c[:, None] - 2 * c[None, :] - 4 * c[:, None] * c[None, :]) / 3
    inv = 1.0 / E
    inv[0, 0] = 0.0
    inv = inv[:, :257]
    for dt_, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
        r = torch.randn((512, 512, 512), dtype=dt_, device=dev)
        iv = inv.to(dt_)

        def fft_apply():
            return torch.fft.irfft2(torch.fft.rfft2(r) * iv, s=(512, 512))
        fft_apply()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fft_apply()
        e1.record()
        torch.cuda.synchronize()
        emit("comparison: preconditioner apply for 512 systems of 512^2 by real FFTs (vendor, via torch)",
             fft_dtype=name, fft_ms=e0.elapsed_time(e1) / 5, hartley_bf16_gemms_ms=per_apply)
        del r
    del a

    # gradient at L = 64 for 64 realizations; quartic tensor over 4096 at L = 16
    a = fields(64, 8, 10.0, 64, 15)
    G = torch.zeros((64, 2, 2), dtype=torch.float64, device=dev)
    G[:, 0, 0] = 1.0
    G[:, 0, 1] = 1.0

    def grad_step():
        r = rve.solve_batch(a, 1 / 8, rve.Options(prec=rve.MIX_BF16))
        return rve.grad(a, r.phi, 1 / 8, G, a_in=10.0)
    dt, _ = timed(grad_step, reps=2)
    emit("L=64 n=512, 64 realizations: solve + dA/da per cell + dA/dcontrast", gemm="bf16", ms=1e3 * dt)
    a = fields(16, 8, 10.0, 4096, 16)

    def quartic():
        r = rve.solve_batch(a, 1 / 8, rve.Options(prec=rve.MIX_BF16), want_phi=False)
        return rve.stats(r.ahom, 16.0)
    dt, st = timed(quartic)
    emit("L=16 n=128, 4096 realizations: A_hom and the quartic tensor", gemm="bf16", ms=1e3 * dt,
         realizations_s=4096 / dt)
    del a

    # on-device sampling: fields per second, and whole ensembles sampled and
    # solved on the device (the spread of A_hom should fall like 1/L)
    import math

    from paper_1903_12227_amd import ensemble
    for L, B in ((64, 256), (16, 4096)):
        thr = rve.occupancy_threshold(math.log(2.0) / 64)
        dt, _ = timed(lambda: rve.sample_lattice(B, 8 * L, 8, seed=1, occ_threshold=thr, a_in=10.0, device=dev),
                      reps=5)
        emit(f"on-device sampling, L={L} n={8 * L}", fields=B, ms=1e3 * dt, fields_s=B / dt)
    for L, Nn in ((8, 16384), (16, 16384), (32, 4096), (64, 1024)):
        t0 = time.perf_counter()
        out = ensemble.run_ensemble(L, 8, 10.0, Nn, batch=4096 if L <= 16 else 1024, seed=2, device=dev)
        dt = time.perf_counter() - t0
        st = out["stats"]
        emit(f"ensemble sampled and solved on the device, L={L} n={8 * L}", N=Nn, s=dt, realizations_s=Nn / dt,
             mean_a11=float(st["mean"][0, 0]), std_a12=float(st["std_a12"]),
             std_a11_minus_a22=float(st["std_a11_minus_a22"]), L_times_std_a12=L * float(st["std_a12"]),
             L_times_std_a11_minus_a22=L * float(st["std_a11_minus_a22"]))

    # the paper's ensemble (exactly L^2 squares of side 2 alpha = 1/2, a = 1 on
    # the covered set and 0.4 elsewhere, m0 = 4) with the lumped five-point
    # scheme: spread of A_hom against Sec. 5, Table a_stan_dev_L1 (N = 10^4)
    paper = {16: (0.000656, 0.001527), 32: (0.000337, 0.000778), 64: (0.000167, 0.000386)}
    from sampler import BooleanModel as BM
    for L in (16, 32, 64):
        model = BM(L=L, m0=4, a_in=1.0, a_bg=0.4, law="paper", alpha=0.25)
        Nn = 10000
        fields_host = [batch(model, 77, 2500, start=s0) for s0 in range(0, Nn, 2500)]
        for scheme, sname in ((rve.SCHEME_FD5, "fd5"), (rve.SCHEME_Q1, "q1")):
            A = []
            t0 = time.perf_counter()
            for fh in fields_host:
                r = rve.solve_batch(torch.from_numpy(fh).to(dev), 0.25,
                                    rve.Options(prec=rve.MIX_BF16, scheme=scheme), want_phi=False, want_flux=False)
                A.append(r.ahom.cpu().numpy())
            dt = time.perf_counter() - t0
            A = np.concatenate(A)
            s12 = float(np.sqrt(np.mean(A[:, 0, 1] ** 2)))
            sdd = float(np.sqrt(np.mean((A[:, 0, 0] - A[:, 1, 1]) ** 2)))
            emit(f"paper ensemble, L={L} n={4 * L} (m0=4, alpha=1/4, lambda=0.4)", scheme=sname, N=Nn, s=dt,
                 std_a12=s12, paper_std_a12=paper[L][0], ratio_a12=s12 / paper[L][0],
                 std_a11_minus_a22=sdd, paper_std_a11_minus_a22=paper[L][1], ratio_a11_minus_a22=sdd / paper[L][1],
                 mean_a11=float(A[:, 0, 0].mean()))

    # spectral density (Appendix): sample-average DOS of 20 realizations at
    # L = 8 and L = 16 (lambda = 0.5, alpha = 1/4, m0 = 8), the shapes the
    # appendix finds nearly independent of L (Remark DOS_Per_L)
    t = torch.linspace(0.0, 16.0 / 3.0, 200, dtype=torch.float64, device=dev)
    curves = {}
    for L in (8, 16):
        model = BM(L=L, m0=8, a_in=1.0, a_bg=0.5, law="paper", alpha=0.25)
        a = torch.from_numpy(batch(model, 78, 20)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi = rve.spectral_density(a, t, 0.02 * 16.0 / 3.0, probes=8, seed=L)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        curves[L] = phi.mean(dim=0).cpu().numpy()
        emit(f"spectral density, L={L} n={8 * L}, 20 realizations", probes=8, s=dt)
    d = float(np.abs(curves[8] - curves[16]).sum() / np.abs(curves[16]).sum())
    emit("spectral density: relative L1 distance of the mean curves at L=8 and L=16", distance=d)

    survey_3d(rve, torch, dev, emit)


def systematic(rve, torch, dev, N_total, ck_dir):
    """The systematic-error study of Sec. 5 (Table a_sys_er_L1, Fig.
    sys_a11_vsL): <a_11>_L - <a_11>_2L over N realizations per size, with the
    paper's ensemble (alpha = 1/4, lambda = 0.4 as a = 1 on the covered set
    and 0.4 elsewhere, m0 = 4, the lumped five-point scheme), under the
    fixed-count law (exactly L^2 squares) and its Poisson-count counterpart.
    One JSON line per (law, L) and per difference, with 95 % intervals."""
    import numpy as np

    from paper_1903_12227_amd import ensemble
    paper = {16: 0.000277, 32: 0.000067}    # Table a_sys_er_L1, N = 10^5 column
    for law in ("fixed", "poisson"):
        means = {}
        for L in (16, 32, 64, 128):
            ck = os.path.join(ck_dir, f"sys_{law}_L{L}.npz") if ck_dir else None
            t0 = time.perf_counter()
            out = ensemble.run_ensemble(L, 4, 1.0, N_total, batch=4096 if L <= 32 else 1024, seed=1903 + L,
                                        device=dev, law=law, alpha=0.25, a_bg=0.4, scheme=rve.SCHEME_FD5,
                                        checkpoint=ck)
            dt = time.perf_counter() - t0
            A = out["ahom"]
            a11, iso = A[:, 0, 0], 0.5 * (A[:, 0, 0] + A[:, 1, 1])
            means[L] = (float(a11.mean()), float(a11.std(ddof=1) / np.sqrt(len(a11))),
                        float(iso.mean()), float(iso.std(ddof=1) / np.sqrt(len(iso))))
            print(json.dumps({"systematic": law, "L": L, "n": 4 * L, "N": len(a11), "s": dt,
                              "mean_a11": means[L][0], "se_a11": means[L][1],
                              "mean_iso": means[L][2], "se_iso": means[L][3]}), flush=True)
        for L in (16, 32, 64):
            d = means[L][0] - means[2 * L][0]
            se = float(np.hypot(means[L][1], means[2 * L][1]))
            di = means[L][2] - means[2 * L][2]
            sei = float(np.hypot(means[L][3], means[2 * L][3]))
            print(json.dumps({"systematic_difference": law, "L": L, "a11_L_minus_a11_2L": d, "ci95": 1.96 * se,
                              "iso_L_minus_iso_2L": di, "iso_ci95": 1.96 * sei,
                              "paper_N1e5": paper.get(L)}), flush=True)


def bytes_per_node_3d(prec_name):
    """Algorithmic HBM bytes per node and corrector system of each kernel
    class of the three-dimensional path. As bytes_per_node, except that the
    operator apply runs one system per workgroup (it reads a for each
    system) and the preconditioner has six transforms: gemm1 the first (reads
    the residual copy), gemm2 the scaling one, gemm3 the four plain ones
    together, gemm4 the last (writes z, re-reads the residual copy)."""
    sg = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[prec_name]
    sp = 8 if prec_name == "fp64" else 4
    lo = 0 if prec_name == "fp64" else sg
    first_in = 8 if prec_name == "fp64" else sg
    return {"stencil": 3 * sp + 8 + 8, "gemm1": first_in + sg, "gemm2": 2 * sg, "gemm3": 4 * 2 * sg,
            "gemm4": sg + sp + first_in, "update_r": 8 + 8 + 8 + lo, "fold_x": sp}


def survey_3d(rve, torch, dev, emit):
    """Three-dimensional corrector problems (unit cubes, contrast 10, tol
    1e-10): wall time per batch, and per kernel class the event time, the
    algorithmic bandwidth and its fraction of the HBM peak (and the GEMMs'
    TFLOP/s)."""
    import math

    import numpy as np

    from paper_1903_12227_amd import DIRECTION_RING
    from sampler import BooleanModel3D, batch_3d

    ctx = rve.Context(0)
    for L, B in ((8, 64), (16, 8)):
        n = 8 * L
        N3 = float(n) ** 3
        # (L = 16: the first realization is the input whose oracle A_hom is stored)
        a = torch.from_numpy(batch_3d(BooleanModel3D(L=L, m0=8, a_in=10.0), 80 + L, B)).to(dev)
        a0 = a[0].cpu().numpy()
        ref = None
        for prec, pname in ((rve.FP64, "fp64"), (rve.MIX_BF16, "bf16"), (rve.MIX_FP16, "fp16")):
            opts = rve.Options(tol=1e-10, prec=prec)
            rve.solve_batch_3d(a, 0.125, opts, want_phi=False, ctx=ctx)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = rve.solve_batch_3d(a, 0.125, opts, want_phi=False, ctx=ctx)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            A = res.ahom.cpu().numpy()
            if ref is None:
                ref = A
            dev_rel = float(np.max(np.abs(A - ref)) / np.max(np.abs(np.diagonal(ref, axis1=1, axis2=2))))
            ctx.set_timing(True)
            r2 = rve.solve_batch_3d(a, 0.125, opts, want_phi=False, ctx=ctx)
            torch.cuda.synchronize()
            tim = ctx.timing()
            ctx.set_timing(False)
            its = r2.iters.cpu().numpy()
            sys_it = float(its.sum())
            folds = float(sum(math.ceil(v / DIRECTION_RING) for v in its.ravel().tolist()))
            bpn = bytes_per_node_3d(pname)
            kern = {}
            for k, (ms, cnt) in tim.items():
                if cnt == 0:
                    continue
                byts = sys_it * bpn[k] * N3 + (16.0 * folds * N3 if k == "fold_x" else 0.0)
                e = {"ms": round(ms, 3), "launches": cnt, "GBps": round(byts / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
                if k.startswith("gemm"):
                    per = 4 if k == "gemm3" else 1
                    e["TFLOPs"] = round(sys_it * per * 2.0 * n * N3 / (ms * 1e-3) / 1e12, 1)
                kern[k] = e
            oerr = {"3d_n128": stored_oracle_error("3d_n128", a0, A[0])} if n == 128 else None
            emit(f"3D L={L} n={n}, {B} realizations (3 correctors + 3x3 A_hom)", gemm=pname, ms=1e3 * dt,
                 realizations_s=B / dt, iters_mean=float(its.mean()), ahom_rel_err_vs_oracle=oerr,
                 ahom_rel_dev_vs_fp64=dev_rel,
                 code=int(res.code), mean_a11=float(A[:, 0, 0].mean()), kernels=kern)
    ctx.close()

def _oracle_one(field):
    """One realization by the oracle on one host thread (pool worker)."""
    from threadpoolctl import threadpool_limits

    from oracle import ahom as oracle_ahom
    with threadpool_limits(limits=1):
        return oracle_ahom.solve(field, tol=1e-10).ahom


def _host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))   # at most the host share of one GPU


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fields, seconds):
    """The oracle, as it is, on the host: (1) realizations of the same
    workload one after another on one host thread until about `seconds`
    have passed (at least two), and (2) one realization per worker process
    on every host core (up to 16) for about as long. Returns the baseline
    entry and the oracle's A_hom of the items the single-thread leg solved
    (items 0, 1, ... of the first timed batch)."""
    import multiprocessing as mp

    done, ahoms = 0, []
    t0 = time.perf_counter()
    while done < len(fields):
        ahoms.append(_oracle_one(fields[done]))
        done += 1
        if done >= 2 and time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    cores = _host_cores()
    all_core = None
    if cores > 1:
        # spawned workers: they import only the oracle, never the device; a
        # worker that dies breaks the pool with an error instead of a hang
        from concurrent.futures import ProcessPoolExecutor, as_completed
        try:
            with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
                list(ex.map(_oracle_one, [fields[k] for k in range(cores)]))   # worker start-up, untimed
                t1 = time.perf_counter()
                futs = [ex.submit(_oracle_one, fields[k % len(fields)]) for k in range(8 * cores)]
                got = 0
                for fu in as_completed(futs):
                    fu.result()
                    got += 1
                    if time.perf_counter() - t1 >= seconds and got >= cores:
                        break
                dt_all = time.perf_counter() - t1
                for fu in futs:
                    fu.cancel()
            all_core = {"value": got / dt_all, "cores": cores, "realizations": got}
        except Exception as e:   # the single-thread figure stands without it
            all_core = {"error": f"{type(e).__name__}: {e}"}
    entry = {"value": done / dt, "unit": "realizations/s", "cores": 1, "kind": "oracle",
             "sample": f"{done} realizations of the same workload (n={fields.shape[1]}, contrast and "
                       "tolerance as timed), solved one after another on one host thread; all_cores: "
                       "the same realizations, one per worker process on each host core",
             "cpu_model": _cpu_model(), "all_cores": all_core}
    return entry, ahoms


if __name__ == "__main__":
    main()
