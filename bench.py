"""Throughput of the RVE corrector path on one MI355X.

One step = the whole hot path over one batch of realizations already resident
in HBM: Galerkin right-hand sides, PCG solves of both correctors (matrix-free
Q1 stencil, Hartley-transform preconditioner on MFMA), A_hom in energy and
flux form, the per-cell gradient of A_11 and A_12 with the contrast
derivative, and the ensemble statistics of the batch.

Workload: L = 64, h = 1/8 (n = 512 nodes per axis), 256 realizations per
step, Poisson(ln 2 L^2) unit-square inclusions, contrast 10, tolerance 1e-10.
The headline value runs the preconditioner GEMMs in BF16 (FP32 accumulation)
with FP64 residuals, dots and A_hom; the same workload in FP64 and the plain
per-realization FP64 PCG are timed beside it.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
Prints one JSON line.
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
MFMA_PEAK_TFS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_batches(model, count, B, config=1):
    from sampler import batch
    return [batch(model, config, B, start=k * B) for k in range(count)]


def run_step(rve, a, h, opts, G, contrast, L):
    res = rve.solve_batch(a, h, opts, want_phi=True, want_flux=True)
    g, gin = rve.grad(a, res.phi, h, G, a_in=contrast)
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


def bytes_per_node(prec_name, flexible):
    """Algorithmic HBM bytes per node of each kernel class.

    FP64 path: every vector FP64. Mixed paths: the directions p and z are
    stored in FP32 (s_p = 4) and the residual has a copy in the GEMM
    precision (s_g bytes) that the first transform reads; x, r, q stay FP64.
      stencil   fused direction step + operator apply, per realization (both
                systems): read z, p_old, x; write p_new, x, q; read a
      update_r  per system: read r, q [+ z for flexible beta]; write r [+ r copy]
      precond   per system, four transforms: read the r copy (FP64 r on the
                FP64 path), write/read three intermediates, write z, re-read r
                (FP64) for r.z
      finalize  per system, once per solve: x += alpha p
    """
    sg = {"fp64": 8, "fp32": 4, "bf16": 2}[prec_name]
    sp = 8 if prec_name == "fp64" else 4
    lo = 0 if prec_name == "fp64" else sg
    first_in = 8 if prec_name == "fp64" else sg
    return {
        "stencil": 2 * (sp + sp + 16 + sp + 8) + 8,
        "update_r": 8 + 8 + 8 + lo + (sp if flexible else 0),
        "precond": first_in + 6 * sg + sp + 8,
        "finalize": 8 + sp + 8,
    }


def roofline_entries(tim, it_all, n, B, prec_name, flexible):
    """Achieved rates of the timed kernel classes from algorithmic bytes/flops.

    it_all: (steps, B, 2) iteration counts. Per realization-step, stencil
    applies = max over its two systems; per system, x/r and p updates = iters,
    preconditioner applies = iters (one before the loop, one per continuing
    iteration)."""
    N2 = n * n
    stencil_applies = float(it_all.max(dim=2).values.sum())       # realization-launch units
    sys_iters = float(it_all.sum())
    bpn = bytes_per_node(prec_name, flexible)
    out = {}
    ms, cnt = tim["stencil"]
    out["stencil"] = {"bound": "hbm", "bytes": stencil_applies * bpn["stencil"] * N2, "ms": ms,
                      "launches": cnt, "bytes_per_node": bpn["stencil"]}
    ms, cnt = tim["update_r"]
    out["update_r"] = {"bound": "hbm", "bytes": sys_iters * bpn["update_r"] * N2, "ms": ms,
                       "launches": cnt, "bytes_per_node": bpn["update_r"]}
    ms, cnt = tim["precond"]
    # four transforms of 2 n^3 flops each per system-apply
    out["precond"] = {"bound": "mfma", "flops": sys_iters * 8.0 * n * N2,
                      "bytes": sys_iters * bpn["precond"] * N2, "ms": ms, "launches": 4 * cnt,
                      "bytes_per_node": bpn["precond"]}
    return out


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
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the realizations are independent and this build runs "
              "on a single MI355X; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1903_12227_amd as rve
    from sampler import BooleanModel

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
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

    log("plain per-realization FP64 leg")
    single = batches[0][: args.plain]
    rve.solve_batch(single[0:1].contiguous(), h, fp64, want_phi=True, want_flux=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(args.plain):
        rve.solve_batch(single[b:b + 1].contiguous(), h, fp64, want_phi=True, want_flux=True)
    torch.cuda.synchronize()
    v_plain = args.plain / (time.perf_counter() - t0)

    # roofline of the dominant kernel class of the headline leg
    ent = roofline_entries(tim_mix, it_mix_t, n, B, "bf16", flexible=False)
    dom = max(ent, key=lambda k: ent[k]["ms"])
    e = ent[dom]
    if e["bound"] == "hbm" or dom != "precond":
        achieved = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_ms": e["ms"] / max(e["launches"], 1)}
    else:
        achieved = e["flops"] / (e["ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK_TFS["bf16"],
                "unit": "TFLOP/s", "frac": achieved / MFMA_PEAK_TFS["bf16"], "traffic": None,
                "avg_launch_ms": e["ms"] / max(e["launches"], 1)}
    kernels = {}
    for k, v in ent.items():
        rec = {"ms_total": v["ms"], "launches": v["launches"], "bytes_per_node": v["bytes_per_node"],
               "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None}
        if "flops" in v:
            rec["TFLOPs"] = v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else None
        kernels[k] = rec
    ent64 = roofline_entries(tim64, it64, n, B, "fp64", flexible=False)
    p64 = ent64["precond"]
    fp64_gemm_tfs = p64["flops"] / (p64["ms"] * 1e-3) / 1e12 if p64["ms"] > 0 else None

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(host[0], args.cpu_seconds)

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
        "tuned": ctx.tuned(n, rve.MIX_BF16, B),
        "fp64_batched": {"value": v64, "ms_per_step": 1e3 * t64 / args.fp64_steps,
                         "iters_mean": float(it64.mean()), "gemm_TFLOPs": fp64_gemm_tfs},
        "plain_fp64_per_realization": {"value": v_plain, "realizations": args.plain},
        "speedup_vs_plain_fp64": value / v_plain,
        "speedup_vs_fp64_batched": value / v64,
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(fields, seconds):
    """The oracle, as it is, on the host: sequential realizations of the same
    workload until about `seconds` have passed (at least one)."""
    from threadpoolctl import threadpool_limits

    from oracle import ahom as oracle_ahom
    done = 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        while done < len(fields):
            oracle_ahom.solve(fields[done], tol=1e-10)
            done += 1
            if time.perf_counter() - t0 >= seconds:
                break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "realizations/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} realizations of the same workload (n={fields.shape[1]}, contrast and "
                      "tolerance as timed), solved one after another on one host thread"}


if __name__ == "__main__":
    main()
