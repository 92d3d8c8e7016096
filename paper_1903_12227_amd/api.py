"""Python binding of librve: argument marshalling only.

Every step of the corrector path runs in librve's HIP kernels; this module
checks shapes/dtypes/devices of torch tensors, passes their device pointers
through the C ABI (include/rve.h) on torch's current HIP stream, and wraps
the results. PyTorch provides device memory and streams, nothing else.
"""
from __future__ import annotations

import ctypes
import warnings
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _native as N
from ._native import DIRECTION_RING, FP64, MIX_BF16, MIX_FP16, MIX_FP32  # noqa: F401


@dataclass
class Options:
    tol: float = 1e-10          # relative residual target ||r||/||f||
    maxit: int = 2000
    prec: int = FP64            # FP64, MIX_FP32, MIX_BF16 or MIX_FP16 (preconditioner GEMMs)
    flexible: int = -1          # -1 automatic, 0 standard beta, 1 flexible beta
    check_every: int = 0        # convergence poll period (0 = library default)
    stencil_prec: int = 0       # 0 FP64 operator apply, 1 FP32 (with FP64 residual replacement)
    scheme: int = 0             # 0 consistent Q1 (nine-point), 1 lumped five-point

    def to_c(self) -> N.RveOpts:
        return N.RveOpts(float(self.tol), int(self.maxit), int(self.prec), int(self.flexible),
                         int(self.check_every), int(self.stencil_prec), int(self.scheme))


@dataclass
class Result:
    ahom: torch.Tensor                  # (B, d, d) energy form (d = 2, or 3 for the 3D solver)
    ahom_flux: Optional[torch.Tensor]   # (B, d, d) flux form
    phi: Optional[torch.Tensor]         # (B, d, n, n[, n]) correctors x h, mean zero
    iters: torch.Tensor                 # (B, d) int32
    relres: torch.Tensor                # (B, d) float64
    status: torch.Tensor                # (B,) int32
    code: int                           # worst status of the call


class Context:
    """Owns one rve_ctx bound to a device; enqueues on torch's current stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("librve needs a HIP device; none is visible")
        self.device = int(device)
        self._lib = N.lib()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            N.check(self._lib.rve_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream)),
                    "rve_create")
        self.handle = h

    def bind_stream(self):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        N.check(self._lib.rve_set_stream(self.handle, ctypes.c_void_p(stream)), "rve_set_stream")
        return self.handle

    def set_timing(self, enable: bool):
        N.check(self._lib.rve_set_timing(self.handle, int(bool(enable))), "rve_set_timing")

    def timing(self):
        """Accumulated event timing since set_timing(True): kernel ->
        (total ms, launches) for 'stencil' (fused direction step and operator
        apply), 'gemm1'..'gemm4' (the preconditioner's transforms),
        'update_r', 'fold_x' (x += sum alpha_j p_j, once per
        DIRECTION_RING iterations and once at the end of a solve)."""
        ms = (ctypes.c_double * 7)()
        cnt = (ctypes.c_longlong * 7)()
        N.check(self._lib.rve_last_timing(self.handle, ms, cnt), "rve_last_timing")
        names = ("stencil", "gemm1", "gemm2", "gemm3", "gemm4", "update_r", "fold_x")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(names)}

    def set_autotune(self, enable: bool):
        N.check(self._lib.rve_set_autotune(self.handle, int(bool(enable))), "rve_set_autotune")

    def force_variants(self, stencil: int = -1, gemm: int = -1, update: int = -1):
        """Use these kernel variants instead of the autotuner's (-1: no
        override): an operator-apply shape code (see tuned()), a
        transform-GEMM variant (0: 64 x 64, 1: 128 x 128 16-bit, 2: even/odd
        folded 128 x 128 BF16, 3: 128 x 128 16-bit with the operands loaded
        straight into LDS, 4: 256 x 128 16-bit, 5: 256 x 256 16-bit, 6: 256 x 256
        16-bit from 8 waves, 7: as 6 through a four-stage LDS ring), and a
        shape code for the residual update that recomputes A p (-1 with a
        stencil shape given: that shape)."""
        N.check(self._lib.rve_force_variants(self.handle, int(stencil), int(gemm), int(update)),
                "rve_force_variants")

    def set_small_solver(self, enable: bool):
        """Single-workgroup PCG for n = 64 FP64 solves (on by default)."""
        N.check(self._lib.rve_set_small_solver(self.handle, int(bool(enable))), "rve_set_small_solver")

    def set_direction_update(self, in_transform: bool):
        """Form the next search direction in the last transform's epilogue
        where possible (the default) or always in the operator apply; the
        results are identical (with BF16 directions off)."""
        N.check(self._lib.rve_set_direction_update(self.handle, int(bool(in_transform))),
                "rve_set_direction_update")

    def set_direction_bf16(self, enable: bool):
        """Store the directions the last transform forms in BF16 (the
        default) or FP32 (16-bit transforms, n <= 512 and contrast <= 20
        only)."""
        N.check(self._lib.rve_set_direction_bf16(self.handle, int(bool(enable))), "rve_set_direction_bf16")

    def set_graphs(self, enable: bool):
        """Replay each chunk of PCG iterations from a captured HIP graph (the
        default) or launch its kernels one by one; results are identical."""
        N.check(self._lib.rve_set_graphs(self.handle, int(bool(enable))), "rve_set_graphs")

    def tuned(self, n: int, prec: int, B: int, stencil_prec: int = 0) -> dict:
        """The autotuner's choices for a shape: columns per lane, rows per
        wave strip and rows of loads in flight per wave of the operator
        apply, and the transform-GEMM tile variant (-1: not tuned)."""
        got = []
        for kind in (2 if stencil_prec else 0, 1, 4):
            c = ctypes.c_int(-1)
            self._lib.rve_get_tuned(self.handle, kind, int(n), int(prec), int(B), ctypes.byref(c))
            got.append(c.value)
        out = {}
        for name, st in (("stencil", got[0]), ("update", got[2])):
            out[f"{name}_columns_per_lane"] = st & 7 if st >= 0 else -1
            out[f"{name}_rows_per_strip"] = 16 * ((st >> 3) & 7) if st >= 0 else -1
            out[f"{name}_prefetch_rows"] = (4 if st & 128 else 1 + ((st >> 6) & 1)) if st >= 0 else -1
        out["gemm_variant"] = got[1]
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.rve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict = {}


def context(device: Optional[int] = None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    ctx = _contexts.get(dev)
    if ctx is None:
        ctx = Context(dev)
        _contexts[dev] = ctx
    return ctx


_UNSET = 127   # status sentinel: items the library never reached


def _check_batch(code: int, status: torch.Tensor, what: str) -> int:
    """Errors raise unless they are per-item outcomes written into `status`
    (a coefficient <= 0 or NaN found on the device); warnings pass through."""
    if code >= 0:
        return code
    if code == N.EINVAL and not bool(torch.any(status == _UNSET)):
        return code
    return N.check(code, what)


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t: torch.Tensor, name: str, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a HIP device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class SingleResult:
    ahom: torch.Tensor                  # (2, 2) energy form, host
    ahom_flux: torch.Tensor             # (2, 2) flux form, host
    phi: Optional[torch.Tensor]         # (2, n, n) correctors x h (device), mean zero
    iters: tuple                        # PCG iterations per direction
    relres: tuple                       # final recursive relative residuals
    code: int                           # RVE_OK, or the warning RVE_NOT_CONVERGED / RVE_BREAKDOWN


def solve(a: torch.Tensor, h: float = 1.0, opts: Optional[Options] = None, *, want_phi: bool = True,
          ctx: Optional[Context] = None) -> SingleResult:
    """One realization a (n, n) FP64 on the device, synchronously (see
    rve_solve): A_hom and the iteration data come back on the host. Errors,
    including a coefficient <= 0 or NaN, raise RveError."""
    _need(a, "a")
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must have shape (n, n)")
    n = a.shape[0]
    opts = opts or Options()
    ctx = ctx or context(a.device.index)
    phi = torch.empty((2, n, n), dtype=torch.float64, device=a.device) if want_phi else None
    A = (ctypes.c_double * 4)()
    F = (ctypes.c_double * 4)()
    its = (ctypes.c_int * 2)()
    rr = (ctypes.c_double * 2)()
    c_opts = opts.to_c()
    code = N.check(ctx._lib.rve_solve(ctx.bind_stream(), n, float(h), _p(a), ctypes.byref(c_opts), _p(phi), A, F,
                                      its, rr), "rve_solve")
    return SingleResult(torch.tensor(list(A), dtype=torch.float64).view(2, 2),
                        torch.tensor(list(F), dtype=torch.float64).view(2, 2), phi, (its[0], its[1]),
                        (rr[0], rr[1]), code)


def _warn_bf16_large(opts, n: int) -> None:
    """BF16 transforms need far more PCG iterations than the scaled FP16 ones
    on large grids (about 100 against 41 at n = 2048); say so once."""
    if opts.prec == MIX_BF16 and n >= 1024:
        warnings.warn(f"BF16 transform GEMMs at n = {n}: the scaled FP16 transforms (MIX_FP16) run at the "
                      "same rate with far fewer iterations on grids this large", RuntimeWarning, stacklevel=3)


def solve_batch(a: torch.Tensor, h: float = 1.0, opts: Optional[Options] = None, *,
                want_phi: bool = True, want_flux: bool = True,
                ctx: Optional[Context] = None) -> Result:
    """Correctors and A_hom of B equal-size realizations a (B, n, n) FP64."""
    _need(a, "a")
    if a.dim() == 2:
        a = a.unsqueeze(0)
    if a.dim() != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("a must have shape (B, n, n)")
    B, n = a.shape[0], a.shape[1]
    opts = opts or Options()
    _warn_bf16_large(opts, n)
    ctx = ctx or context(a.device.index)
    dev = a.device
    ahom = torch.empty((B, 2, 2), dtype=torch.float64, device=dev)
    flux = torch.empty((B, 2, 2), dtype=torch.float64, device=dev) if want_flux else None
    phi = torch.empty((B, 2, n, n), dtype=torch.float64, device=dev) if want_phi else None
    iters = torch.empty((B, 2), dtype=torch.int32, device=dev)
    relres = torch.empty((B, 2), dtype=torch.float64, device=dev)
    status = torch.full((B,), _UNSET, dtype=torch.int32, device=dev)
    c_opts = opts.to_c()
    code = ctx._lib.rve_solve_batch(ctx.bind_stream(), B, n, float(h), _p(a), ctypes.byref(c_opts),
                                    _p(phi), _p(ahom), _p(flux), _p(iters), _p(relres), _p(status))
    _check_batch(code, status, "rve_solve_batch")
    return Result(ahom, flux, phi, iters, relres, status, code)


def solve_batch_3d(a: torch.Tensor, h: float = 1.0, opts: Optional[Options] = None, *,
                   want_phi: bool = True, want_flux: bool = True,
                   ctx: Optional[Context] = None) -> Result:
    """Correctors and the 3 x 3 A_hom of B equal-size three-dimensional
    realizations a (B, n, n, n) FP64 (see rve_solve_batch_3d)."""
    _need(a, "a")
    if a.dim() == 3:
        a = a.unsqueeze(0)
    if a.dim() != 4 or not (a.shape[1] == a.shape[2] == a.shape[3]):
        raise ValueError("a must have shape (B, n, n, n)")
    B, n = a.shape[0], a.shape[1]
    opts = opts or Options()
    ctx = ctx or context(a.device.index)
    dev = a.device
    ahom = torch.empty((B, 3, 3), dtype=torch.float64, device=dev)
    flux = torch.empty((B, 3, 3), dtype=torch.float64, device=dev) if want_flux else None
    phi = torch.empty((B, 3, n, n, n), dtype=torch.float64, device=dev) if want_phi else None
    iters = torch.empty((B, 3), dtype=torch.int32, device=dev)
    relres = torch.empty((B, 3), dtype=torch.float64, device=dev)
    status = torch.full((B,), _UNSET, dtype=torch.int32, device=dev)
    c_opts = opts.to_c()
    code = ctx._lib.rve_solve_batch_3d(ctx.bind_stream(), B, n, float(h), _p(a), ctypes.byref(c_opts),
                                       _p(phi), _p(ahom), _p(flux), _p(iters), _p(relres), _p(status))
    _check_batch(code, status, "rve_solve_batch_3d")
    return Result(ahom, flux, phi, iters, relres, status, code)


def apply_operator_3d(a: torch.Tensor, u: torch.Tensor, ctx: Optional[Context] = None) -> torch.Tensor:
    """A u for the trilinear Q1 operator of each field: a and u (B, n, n, n)."""
    _need(a, "a")
    _need(u, "u")
    if a.dim() != 4 or u.shape != a.shape:
        raise ValueError("a and u must be (B, n, n, n)")
    B, n = a.shape[0], a.shape[1]
    ctx = ctx or context(a.device.index)
    out = torch.empty_like(u)
    N.check(ctx._lib.rve_apply_operator_3d(ctx.bind_stream(), B, n, _p(a), _p(u), _p(out)), "rve_apply_operator_3d")
    return out


def apply_precond_3d(a: torch.Tensor, r: torch.Tensor, prec: int = FP64,
                     ctx: Optional[Context] = None) -> torch.Tensor:
    """(a0 A_Delta)^+ r in three dimensions: a (B, n, n, n), r (B, 3, n, n, n)."""
    _need(a, "a")
    _need(r, "r")
    if a.dim() != 4:
        raise ValueError("a must be (B, n, n, n)")
    B, n = a.shape[0], a.shape[1]
    if r.shape != (B, 3, n, n, n):
        raise ValueError("r must be (B, 3, n, n, n)")
    ctx = ctx or context(a.device.index)
    z = torch.empty_like(r)
    N.check(ctx._lib.rve_apply_precond_3d(ctx.bind_stream(), B, n, _p(a), _p(r), _p(z), int(prec)),
            "rve_apply_precond_3d")
    return z


def solve_uneven(fields: Sequence[torch.Tensor], h: float = 1.0, opts: Optional[Options] = None, *,
                 want_phi: bool = False, want_flux: bool = True,
                 ctx: Optional[Context] = None):
    """Realizations of different sizes in one call. Returns a Result whose
    ahom/flux/iters/relres/status are stacked per item and whose phi (if
    requested) is a list of (2, n_b, n_b) tensors."""
    if len(fields) == 0:
        raise ValueError("no realizations")
    dev = fields[0].device
    for k, f in enumerate(fields):
        _need(f, f"fields[{k}]")
        if f.dim() != 2 or f.shape[0] != f.shape[1] or f.device != dev:
            raise ValueError("each field must be (n, n) on one device")
    B = len(fields)
    ns = [int(f.shape[0]) for f in fields]
    offs = [0]
    for n in ns:
        offs.append(offs[-1] + n * n)
    packed = torch.cat([f.reshape(-1) for f in fields])
    opts = opts or Options()
    _warn_bf16_large(opts, max(ns))
    ctx = ctx or context(dev.index)
    ahom = torch.empty((B, 2, 2), dtype=torch.float64, device=dev)
    flux = torch.empty((B, 2, 2), dtype=torch.float64, device=dev) if want_flux else None
    phi = torch.empty(2 * offs[-1], dtype=torch.float64, device=dev) if want_phi else None
    iters = torch.empty((B, 2), dtype=torch.int32, device=dev)
    relres = torch.empty((B, 2), dtype=torch.float64, device=dev)
    status = torch.full((B,), _UNSET, dtype=torch.int32, device=dev)
    n_c = (ctypes.c_int * B)(*ns)
    off_c = (ctypes.c_int64 * (B + 1))(*offs)
    c_opts = opts.to_c()
    code = ctx._lib.rve_solve_uneven(ctx.bind_stream(), B, n_c, off_c, float(h), _p(packed),
                                     ctypes.byref(c_opts), _p(phi), _p(ahom), _p(flux), _p(iters),
                                     _p(relres), _p(status))
    _check_batch(code, status, "rve_solve_uneven")
    phis = None
    if want_phi:
        phis = [phi[2 * offs[b]: 2 * offs[b + 1]].view(2, ns[b], ns[b]) for b in range(B)]
    return Result(ahom, flux, phis, iters, relres, status, code)


def _mask_bytes(mask: torch.Tensor, shape, dev) -> torch.Tensor:
    if not isinstance(mask, torch.Tensor) or mask.device != dev:
        raise ValueError("mask must be a tensor on the fields' device")
    if mask.dtype not in (torch.bool, torch.uint8):
        raise ValueError("mask must have dtype bool or uint8")
    if tuple(mask.shape) != tuple(shape):
        raise ValueError(f"mask must have shape {tuple(shape)}")
    return mask.contiguous()


def grad(a: torch.Tensor, phi: torch.Tensor, h: float, G: torch.Tensor,
         a_in: Optional[float] = None, *, mask: Optional[torch.Tensor] = None, want_sum: bool = False,
         ctx: Optional[Context] = None, scheme: int = 0, noalloc: bool = False):
    """sum_ij G_ij dA_ij/da per cell, (B, n, n); and, if a covered set is
    given (mask (B, n, n) bool/uint8, or else the cells equal to a_in), the
    derivative with respect to the inclusion value per realization (B,),
    and with want_sum its sum over the batch (a 1-element tensor).
    noalloc: use rve_grad_noalloc (the library allocates no device memory;
    outputs are still allocated here).
    Returns (grad_a, grad_in or None, grad_in_sum or None)."""
    _need(a, "a")
    _need(phi, "phi")
    _need(G, "G")
    if a.dim() != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("a must have shape (B, n, n)")
    B, n = a.shape[0], a.shape[1]
    if phi.shape != (B, 2, n, n) or G.shape != (B, 2, 2):
        raise ValueError("phi must be (B, 2, n, n) and G (B, 2, 2)")
    if mask is not None:
        mask = _mask_bytes(mask, (B, n, n), a.device)
    want_in = mask is not None or a_in is not None
    if want_sum and not want_in:
        raise ValueError("want_sum needs a covered set (mask or a_in)")
    ctx = ctx or context(a.device.index)
    out = torch.empty_like(a)
    gin = torch.empty((B,), dtype=torch.float64, device=a.device) if want_in else None
    gsum = torch.empty((1,), dtype=torch.float64, device=a.device) if want_sum else None
    fn = ctx._lib.rve_grad_noalloc if noalloc else ctx._lib.rve_grad
    N.check(fn(ctx.bind_stream(), B, n, _p(a), _p(phi), float(h), _p(G), _p(out), _p(mask),
               float(a_in if a_in is not None else 0.0), _p(gin), _p(gsum), int(scheme)),
            "rve_grad_noalloc" if noalloc else "rve_grad")
    return out, gin, gsum


def field_from_mask(mask: torch.Tensor, a_in, a_bg: float = 1.0, ctx: Optional[Context] = None) -> torch.Tensor:
    """Fields (B, ...) FP64 with a_in[b] on the cells where mask[b] is set and
    a_bg elsewhere (see rve_field_from_mask); a_in a float or a (B,) FP64
    device tensor."""
    if not isinstance(mask, torch.Tensor) or not mask.is_cuda or mask.dim() < 2:
        raise ValueError("mask must be a (B, ...) device tensor")
    B = mask.shape[0]
    mask = _mask_bytes(mask, mask.shape, mask.device)
    if isinstance(a_in, torch.Tensor):
        _need(a_in, "a_in")
        if a_in.shape != (B,):
            raise ValueError("a_in must have shape (B,)")
        ain = a_in
    else:
        ain = torch.full((B,), float(a_in), dtype=torch.float64, device=mask.device)
    ctx = ctx or context(mask.device.index)
    out = torch.empty(mask.shape, dtype=torch.float64, device=mask.device)
    N.check(ctx._lib.rve_field_from_mask(ctx.bind_stream(), B, mask[0].numel(), _p(mask), _p(ain), float(a_bg),
                                         _p(out)), "rve_field_from_mask")
    return out


def stats(ahom: torch.Tensor, L: float, ctx: Optional[Context] = None) -> dict:
    """Mean, centred variance, Var1/Var2 standard deviations and the 4x4
    quartic tensor of N homogenized matrices (N, 2, 2)."""
    _need(ahom, "ahom")
    Nn = ahom.shape[0]
    ctx = ctx or context(ahom.device.index)
    out = torch.empty(26, dtype=torch.float64, device=ahom.device)
    N.check(ctx._lib.rve_stats(ctx.bind_stream(), Nn, float(L), _p(ahom), _p(out)), "rve_stats")
    return {"mean": out[0:4].view(2, 2), "var": out[4:8].view(2, 2), "std_a12": out[8],
            "std_a11_minus_a22": out[9], "quartic": out[10:26].view(4, 4)}


def apply_operator(a: torch.Tensor, u: torch.Tensor, ctx: Optional[Context] = None,
                   scheme: int = 0) -> torch.Tensor:
    """A u for the Q1 operator of each field: a (B, n, n), u (B, 2, n, n)."""
    _need(a, "a")
    _need(u, "u")
    B, n = a.shape[0], a.shape[1]
    if u.shape != (B, 2, n, n):
        raise ValueError("u must be (B, 2, n, n)")
    ctx = ctx or context(a.device.index)
    out = torch.empty_like(u)
    N.check(ctx._lib.rve_apply_operator(ctx.bind_stream(), B, n, _p(a), _p(u), _p(out), int(scheme)),
            "rve_apply_operator")
    return out


def dos_moments(a: torch.Tensor, v: torch.Tensor, lmax: float, K: int, scheme: int = 0,
                ctx: Optional[Context] = None) -> torch.Tensor:
    """Chebyshev moments (B, nv, K) of the stiffness matrix of each field a
    (B, n, n) with probes v (B, nv, n, n), nv even (see rve_dos_moments)."""
    _need(a, "a")
    _need(v, "v")
    B, n = a.shape[0], a.shape[1]
    if v.dim() != 4 or v.shape[0] != B or v.shape[2:] != (n, n):
        raise ValueError("v must be (B, nv, n, n)")
    nv = v.shape[1]
    ctx = ctx or context(a.device.index)
    mu = torch.empty((B, nv, int(K)), dtype=torch.float64, device=a.device)
    N.check(ctx._lib.rve_dos_moments(ctx.bind_stream(), B, n, int(scheme), _p(a), nv, _p(v), float(lmax), int(K),
                                     _p(mu)), "rve_dos_moments")
    return mu


def dos_eval(mu: torch.Tensor, t: torch.Tensor, lmax: float, eta: float, Q: Optional[int] = None,
             ctx: Optional[Context] = None) -> torch.Tensor:
    """Gaussian-broadened spectral density (B, nt) at the points t (nt,)
    from moments mu (B, nv, K), averaged over the probes (Q quadrature
    nodes; None: the library's default)."""
    _need(mu, "mu")
    _need(t, "t")
    B, nv, K = mu.shape
    Q = int(Q) if Q is not None else 0
    ctx = ctx or context(mu.device.index)
    phi = torch.empty((B, t.numel()), dtype=torch.float64, device=mu.device)
    N.check(ctx._lib.rve_dos_eval(ctx.bind_stream(), B, nv, K, _p(mu), float(lmax), float(eta), Q, t.numel(),
                                  _p(t), _p(phi)), "rve_dos_eval")
    return phi


def dos_plan(a: torch.Tensor, eta: float, scheme: int = 0, ctx: Optional[Context] = None):
    """(lmax, K): the Gershgorin bound of the spectrum of the fields a
    (B, n, n) and the moment count that resolves width eta (rve_dos_plan)."""
    _need(a, "a")
    if a.dim() != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("a must have shape (B, n, n)")
    ctx = ctx or context(a.device.index)
    lmax = ctypes.c_double()
    K = ctypes.c_int()
    N.check(ctx._lib.rve_dos_plan(ctx.bind_stream(), a.shape[0], a.shape[1], int(scheme), _p(a), float(eta),
                                  ctypes.byref(lmax), ctypes.byref(K)), "rve_dos_plan")
    return lmax.value, K.value


def dos_probes(B: int, nv: int, n: int, seed: int, device=None, ctx: Optional[Context] = None) -> torch.Tensor:
    """+-1 probe vectors (B, nv, n, n) drawn on the device (rve_dos_probes)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ctx = ctx or context(dev.index)
    v = torch.empty((int(B), int(nv), int(n), int(n)), dtype=torch.float64, device=dev)
    N.check(ctx._lib.rve_dos_probes(ctx.bind_stream(), int(B), int(nv), int(n), int(seed) & (2**64 - 1), _p(v)),
            "rve_dos_probes")
    return v


def spectral_density(a: torch.Tensor, t: torch.Tensor, eta: float, *, probes: int = 8, K: Optional[int] = None,
                     scheme: int = 0, seed: int = 0, ctx: Optional[Context] = None) -> torch.Tensor:
    """Spectral density (B, nt) of the stiffness matrix of each field, with
    `probes` +-1 probe vectors drawn on the device from `seed`, and (K None)
    enough moments to resolve the width eta."""
    lmax, K_auto = dos_plan(a, eta, scheme, ctx)
    v = dos_probes(a.shape[0], probes, a.shape[1], seed, a.device, ctx)
    return dos_eval(dos_moments(a, v, lmax, K_auto if K is None else int(K), scheme, ctx), t, lmax, eta, ctx=ctx)


def occupancy_threshold(mu: float) -> int:
    """Integer site-occupancy threshold of rve_sample_lattice for Poisson
    centres with mean mu per lattice site (rve_occupancy_threshold)."""
    return int(N.lib().rve_occupancy_threshold(float(mu)))


def sample_lattice(B: int, n: int, side: int, *, seed: int, first: int = 0, occ_threshold: int,
                   a_in: float, a_bg: float = 1.0, device=None, ctx: Optional[Context] = None) -> torch.Tensor:
    """B fields (B, n, n) FP64 of the inclusion model sampled on the device
    for realizations first .. first + B - 1 (see rve_sample_lattice)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ctx = ctx or context(dev.index)
    a = torch.empty((int(B), int(n), int(n)), dtype=torch.float64, device=dev)
    N.check(ctx._lib.rve_sample_lattice(ctx.bind_stream(), int(B), int(n), int(side), int(seed) & (2**64 - 1),
                                        int(first), int(occ_threshold), float(a_in), float(a_bg), _p(a)),
            "rve_sample_lattice")
    return a


def sample_fixed_count(B: int, n: int, side: int, K: int, *, seed: int, first: int = 0, a_in: float,
                       a_bg: float = 1.0, device=None, ctx: Optional[Context] = None) -> torch.Tensor:
    """B fields (B, n, n) FP64 of the paper's fixed-count law (exactly K
    squares of side `side` cells at uniform grid nodes) for realizations
    first .. first + B - 1 (see rve_sample_fixed_count)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ctx = ctx or context(dev.index)
    a = torch.empty((int(B), int(n), int(n)), dtype=torch.float64, device=dev)
    N.check(ctx._lib.rve_sample_fixed_count(ctx.bind_stream(), int(B), int(n), int(side), int(seed) & (2**64 - 1),
                                            int(first), int(K), float(a_in), float(a_bg), _p(a)),
            "rve_sample_fixed_count")
    return a


def apply_precond(a: torch.Tensor, r: torch.Tensor, prec: int = FP64,
                  ctx: Optional[Context] = None, scheme: int = 0) -> torch.Tensor:
    """(a0 A_Delta)^+ r with a0 from each field a: a (B, n, n), r (B, 2, n, n)."""
    _need(a, "a")
    _need(r, "r")
    B, n = a.shape[0], a.shape[1]
    if r.shape != (B, 2, n, n):
        raise ValueError("r must be (B, 2, n, n)")
    ctx = ctx or context(a.device.index)
    z = torch.empty_like(r)
    N.check(ctx._lib.rve_apply_precond(ctx.bind_stream(), B, n, _p(a), _p(r), _p(z), int(prec), int(scheme)),
            "rve_apply_precond")
    return z
