"""Ensemble runs with on-device sampling, checkpointed so that long runs
resume where they stopped.

The empirical averages of Sec. 4.2 (eqn. A_hom_Empir) and the variances and
quartic tensor of Sec. 4.3-4.4 are taken over N realizations; Sec. 5 uses up
to N = 10^5 per RVE size. Realization r is sampled on the device by
rve_sample_lattice from (seed, r) alone, so a run split over several calls,
batches or processes gives the same A_hom values as one uninterrupted run.
After every batch the A_hom values so far are written to the checkpoint file
(a NumPy .npz, replaced atomically); a later call with the same parameters
continues from it.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional

import numpy as np
import torch

from . import _native as N
from . import api


def _params(L, m0, contrast, a_bg, N_total, seed, prec, tol, thr, law="lattice", side=None, K=None, scheme=0):
    p = {"L": int(L), "m0": int(m0), "contrast": float(contrast), "a_bg": float(a_bg), "N": int(N_total),
         "seed": int(seed), "prec": int(prec), "tol": float(tol), "occ_threshold": int(thr)}
    if law != "lattice" or scheme:
        p.update({"law": law, "side": int(side), "K": int(K), "scheme": int(scheme)})
    return p


def _load(checkpoint: str, params: dict):
    with np.load(checkpoint, allow_pickle=False) as d:
        got = json.loads(str(d["params"]))
        if got != params:
            raise ValueError(f"checkpoint {checkpoint} belongs to another run: {got} != {params}")
        done = int(d["done"])
        return done, np.array(d["ahom"][:done]), np.array(d["iters"][:done])


def _save(checkpoint: str, params: dict, done: int, ahom: np.ndarray, iters: np.ndarray):
    tmp = checkpoint + ".tmp.npz"
    np.savez(tmp, params=np.array(json.dumps(params, sort_keys=True)), done=np.array(done),
             ahom=ahom[:done], iters=iters[:done])
    os.replace(tmp, checkpoint)


def run_ensemble(L: int, m0: int, contrast: float, N_total: int, *, batch: int = 256, seed: int = 1903,
                 prec: int = N.MIX_BF16, tol: float = 1e-10, a_bg: float = 1.0,
                 checkpoint: Optional[str] = None, max_batches: Optional[int] = None,
                 device=None, ctx: Optional[api.Context] = None, law: str = "lattice",
                 alpha: float = 0.25, scheme: int = 0) -> dict:
    """A_hom of realizations 0 .. N_total - 1 of the inclusion model on the
    n = m0 L torus, a_in = contrast, a_bg; and their statistics.

    law "lattice": unit squares (side m0 cells) with lattice Poisson centres
    of mean ln 2 / m0^2 per node, Poisson(ln 2 L^2) squares on average (half
    the torus covered). law "fixed": the paper's law, exactly L^2 squares of
    side 2 alpha (2 alpha m0 cells) at uniformly drawn nodes (Sec. 2, eqn.
    Stoch-decomp). law "poisson": the same squares with lattice Poisson
    centres of mean 1/m0^2 per node, i.e. Poisson(L^2) squares (the
    fixed count replaced by its Poisson counterpart). scheme: the
    discretisation (0 consistent Q1, 1 the lumped five-point scheme).

    max_batches bounds the batches done in this call (the run then stops
    with ``complete`` False and can be resumed from ``checkpoint``).
    Returns {"done", "complete", "ahom" (done, 2, 2) NumPy, "iters",
    "stats" (mean, var, std_a12, std_a11_minus_a22, quartic as NumPy; only
    when done >= 2)}."""
    n = int(L) * int(m0)
    if law == "lattice":
        side, K = int(m0), None
        mu = math.log(2.0) / float(m0) ** 2           # expected square centres per lattice site
        thr = api.occupancy_threshold(mu)
    elif law in ("fixed", "poisson"):
        side, K, thr = int(round(2.0 * alpha * m0)), int(L) * int(L), 0
        if side < 1 or abs(side - 2.0 * alpha * m0) > 1e-12:
            raise ValueError("2 alpha m0 must be a positive whole number of cells")
        if law == "poisson":
            thr = api.occupancy_threshold(1.0 / float(m0) ** 2)
    else:
        raise ValueError(f"unknown law {law!r}")
    params = _params(L, m0, contrast, a_bg, N_total, seed, prec, tol, thr, law, side, K, scheme)
    ahom = np.zeros((N_total, 2, 2))
    iters = np.zeros((N_total, 2), dtype=np.int32)
    done = 0
    if checkpoint and os.path.exists(checkpoint):
        done, ah, it = _load(checkpoint, params)
        ahom[:done], iters[:done] = ah, it
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ctx = ctx or api.context(dev.index)
    opts = api.Options(tol=tol, prec=prec, scheme=scheme)
    batches = 0
    while done < N_total and (max_batches is None or batches < max_batches):
        B = min(int(batch), N_total - done)
        if law in ("lattice", "poisson"):
            a = api.sample_lattice(B, n, side, seed=seed, first=done, occ_threshold=thr, a_in=contrast, a_bg=a_bg,
                                   device=dev, ctx=ctx)
        else:
            a = api.sample_fixed_count(B, n, side, K, seed=seed, first=done, a_in=contrast, a_bg=a_bg,
                                       device=dev, ctx=ctx)
        res = api.solve_batch(a, 1.0 / m0, opts, want_phi=False, want_flux=False, ctx=ctx)
        if res.code != N.OK:
            bad = [int(k) for k in torch.nonzero(res.status != 0).flatten().tolist()]
            raise RuntimeError(f"realizations {[done + k for k in bad]} did not converge (code {res.code})")
        ahom[done:done + B] = res.ahom.cpu().numpy()
        iters[done:done + B] = res.iters.cpu().numpy()
        done += B
        batches += 1
        if checkpoint:
            _save(checkpoint, params, done, ahom, iters)
    out = {"done": done, "complete": done == N_total, "ahom": ahom[:done], "iters": iters[:done]}
    if done >= 2:
        st = api.stats(torch.from_numpy(np.ascontiguousarray(ahom[:done])).to(dev), float(L), ctx=ctx)
        out["stats"] = {k: v.cpu().numpy() for k, v in st.items()}
    return out
