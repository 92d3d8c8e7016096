"""The C ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rve.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rve_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1903_12227_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("librve.so is not built (run __graft_entry__.build())")
    return _native.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    from paper_1903_12227_amd import _native
    assert set(_native.EXPORTS) == set(names)


def test_host_argument_validation_3d(lib):
    from paper_1903_12227_amd import _native as N
    o = N.RveOpts()
    lib.rve_default_opts(ctypes.byref(o))
    fake = ctypes.c_void_p(1)
    other = ctypes.c_void_p(2)
    assert lib.rve_solve_batch_3d(None, 1, 64, 0.125, fake, ctypes.byref(o), None, fake, None, None, None,
                                  None) == N.EINVAL
    # n must be a multiple of 64 in [64, 256]
    for n in (0, 32, 96, 320, 512):
        assert lib.rve_solve_batch_3d(fake, 1, n, 0.125, fake, ctypes.byref(o), None, fake, None, None,
                                      None, None) == N.EINVAL
        assert lib.rve_apply_operator_3d(fake, 1, n, fake, fake, other) == N.EINVAL
        assert lib.rve_apply_precond_3d(fake, 1, n, fake, fake, other, 0) == N.EINVAL
    # the FP32 apply and the five-point scheme are two-dimensional only
    for bad in (N.RveOpts(1e-10, 10, 0, -1, 0, 1, 0), N.RveOpts(1e-10, 10, 0, -1, 0, 0, 1)):
        assert lib.rve_solve_batch_3d(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                                      None, None) == N.EINVAL
    assert lib.rve_solve_batch_3d(fake, 0, 64, 0.125, fake, ctypes.byref(o), None, fake, None, None, None,
                                  None) == N.EINVAL
    assert lib.rve_solve_batch_3d(fake, 1, 64, 0.125, fake, ctypes.byref(o), None, None, None, None, None,
                                  None) == N.EINVAL
    # in-place operands and unknown precisions
    assert lib.rve_apply_operator_3d(fake, 1, 64, fake, fake, fake) == N.EINVAL
    assert lib.rve_apply_precond_3d(fake, 1, 64, fake, fake, fake, 0) == N.EINVAL
    assert lib.rve_apply_precond_3d(fake, 1, 64, fake, fake, other, 5) == N.EINVAL
    # launch-size bound: B so large that a grid would pass 2^31 workgroups
    assert lib.rve_solve_batch_3d(fake, 1 << 22, 256, 0.125, fake, ctypes.byref(o), None, fake, None, None,
                                  None, None) == N.EINVAL


def test_status_strings_and_defaults(lib):
    from paper_1903_12227_amd import _native as N
    for code in (N.OK, N.NOT_CONVERGED, N.BREAKDOWN, N.EINVAL, N.EHIP, N.ENOMEM):
        assert N.status_string(code).startswith("RVE_")
    o = N.RveOpts()
    lib.rve_default_opts(ctypes.byref(o))
    assert o.tol == 1e-10 and o.maxit == 2000 and o.prec == N.FP64 and o.flexible == -1
    assert o.stencil_prec == N.STENCIL_FP64 and o.scheme == N.SCHEME_Q1


def test_host_argument_validation(lib):
    from paper_1903_12227_amd import _native as N
    o = N.RveOpts()
    lib.rve_default_opts(ctypes.byref(o))
    fake = ctypes.c_void_p(1)
    # null context, bad n (not a multiple of 64 / too small), bad h, bad opts
    assert lib.rve_solve_batch(None, 1, 64, 0.125, fake, ctypes.byref(o), None, fake, None, None, None,
                               None) == N.EINVAL
    for n in (0, 32, 96, 4160, 8192):         # 4096 is the largest grid
        assert lib.rve_solve_batch(fake, 1, n, 0.125, fake, ctypes.byref(o), None, fake, None, None,
                                   None, None) == N.EINVAL
    # an empty or negative batch is an error, not a no-op
    other = ctypes.c_void_p(2)
    for B in (0, -1):
        assert lib.rve_solve_batch(fake, B, 64, 0.125, fake, ctypes.byref(o), None, fake, None, None,
                                   None, None) == N.EINVAL
        assert lib.rve_apply_operator(fake, B, 64, fake, fake, other, 0) == N.EINVAL
        assert lib.rve_apply_precond(fake, B, 64, fake, fake, other, 0, 0) == N.EINVAL
        assert lib.rve_stats(fake, B, 8.0, fake, other) == N.EINVAL
    assert lib.rve_solve_batch(fake, 1, 64, -1.0, fake, ctypes.byref(o), None, fake, None, None, None,
                               None) == N.EINVAL
    bad = N.RveOpts(-1.0, 10, 0, -1, 0)
    assert lib.rve_solve_batch(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                               None, None) == N.EINVAL
    bad = N.RveOpts(1e-10, 0, 0, -1, 0)
    assert lib.rve_solve_batch(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                               None, None) == N.EINVAL
    # variant overrides: GEMM variant out of range, malformed operator-apply shape
    assert lib.rve_force_variants(fake, -1, 8, -1) == N.EINVAL
    assert lib.rve_force_variants(fake, 5, -1, -1) == N.EINVAL
    assert lib.rve_force_variants(fake, -1, -1, 5) == N.EINVAL
    assert lib.rve_force_variants(fake, 9 + 64 + 128, -1, -1) == N.EINVAL   # two prefetch depths at once
    assert lib.rve_force_variants(None, -1, -1, -1) == N.EINVAL
    assert lib.rve_set_small_solver(None, 1) == N.EINVAL
    assert lib.rve_set_small_solver(fake, 2) == N.EINVAL
    assert lib.rve_set_direction_bf16(None, 1) == N.EINVAL
    assert lib.rve_set_direction_bf16(fake, 2) == N.EINVAL
    assert lib.rve_set_direction_bf16(fake, -1) == N.EINVAL
    for bad in (N.RveOpts(1e-10, 10, 0, -1, 0, 0, 2), N.RveOpts(1e-10, 10, 0, -1, 0, 1, 1)):
        # unknown scheme; five-point with the FP32 apply
        assert lib.rve_solve_batch(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                                   None, None) == N.EINVAL
    bad = N.RveOpts(1e-10, 10, 0, -1, 0, 2)
    assert lib.rve_solve_batch(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                               None, None) == N.EINVAL
    bad = N.RveOpts(1e-10, 10, 4, -1, 0)
    assert lib.rve_solve_batch(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                               None, None) == N.EINVAL
    bad = N.RveOpts(1e-10, 10, 7, -1, 0)
    assert lib.rve_solve_batch(fake, 1, 64, 0.125, fake, ctypes.byref(bad), None, fake, None, None,
                               None, None) == N.EINVAL
    # uneven: overlapping offsets and extents beyond the total are rejected
    ns = (ctypes.c_int * 2)(64, 64)
    offs = (ctypes.c_int64 * 3)(0, 100, 8192)
    assert lib.rve_solve_uneven(fake, 2, ns, offs, 0.125, fake, ctypes.byref(o), None, fake, None, None,
                                None, None) == N.EINVAL
    offs = (ctypes.c_int64 * 3)(0, 4096, 4096)
    assert lib.rve_solve_uneven(fake, 2, ns, offs, 0.125, fake, ctypes.byref(o), None, fake, None, None,
                                None, None) == N.EINVAL
    assert lib.rve_stats(fake, 1, 16.0, fake, fake) == N.EINVAL
    assert lib.rve_grad(fake, 1, 48, fake, fake, 0.125, fake, fake, None, 10.0, None, None, 0) == N.EINVAL
    # an inclusion derivative by value needs a finite inclusion value
    assert lib.rve_grad(fake, 1, 64, fake, fake, 0.125, fake, fake, None, float("nan"), fake, None, 0) == N.EINVAL
    # rve_solve: unsupported n, missing host output, bad h
    A = (ctypes.c_double * 4)()
    assert lib.rve_solve(fake, 48, 0.125, fake, ctypes.byref(o), None, A, None, None, None) == N.EINVAL
    assert lib.rve_solve(fake, 64, 0.125, fake, ctypes.byref(o), None, None, None, None, None) == N.EINVAL
    assert lib.rve_solve(fake, 64, 0.0, fake, ctypes.byref(o), None, A, None, None, None) == N.EINVAL
    assert lib.rve_field_from_mask(fake, 1, 4096, fake, fake, 0.0, fake) == N.EINVAL
    assert lib.rve_field_from_mask(fake, 0, 4096, fake, fake, 1.0, fake) == N.EINVAL
    lmax, K = ctypes.c_double(), ctypes.c_int()
    assert lib.rve_dos_plan(fake, 1, 64, 0, fake, 0.0, ctypes.byref(lmax), ctypes.byref(K)) == N.EINVAL
    assert lib.rve_dos_plan(fake, 1, 64, 2, fake, 0.1, ctypes.byref(lmax), ctypes.byref(K)) == N.EINVAL
    assert lib.rve_dos_probes(fake, 1, 1, 48, 0, fake) == N.EINVAL
    assert lib.rve_apply_operator(fake, 1, 64, fake, fake, fake, 0) == N.EINVAL   # u aliases out
    assert lib.rve_apply_precond(fake, 1, 64, fake, fake, fake, 0, 0) == N.EINVAL
    # unknown scheme
    other = ctypes.c_void_p(2)
    assert lib.rve_grad(fake, 1, 64, fake, fake, 0.125, fake, other, None, 10.0, None, None, 2) == N.EINVAL
    assert lib.rve_apply_operator(fake, 1, 64, fake, fake, other, 2) == N.EINVAL
    assert lib.rve_apply_precond(fake, 1, 64, fake, fake, other, 0, 2) == N.EINVAL


def test_header_constants_match_binding():
    from paper_1903_12227_amd import _native as N
    src = open(HEADER).read()
    m = re.search(r"#define\s+RVE_DIRECTION_RING\s+(\d+)", src)
    assert m and int(m.group(1)) == N.DIRECTION_RING
    for name, val in (("RVE_OK", N.OK), ("RVE_NOT_CONVERGED", N.NOT_CONVERGED), ("RVE_BREAKDOWN", N.BREAKDOWN),
                      ("RVE_EINVAL", N.EINVAL), ("RVE_EHIP", N.EHIP), ("RVE_ENOMEM", N.ENOMEM),
                      ("RVE_FP64", N.FP64), ("RVE_MIX_FP32", N.MIX_FP32), ("RVE_MIX_BF16", N.MIX_BF16),
                      ("RVE_MIX_FP16", N.MIX_FP16), ("RVE_STENCIL_FP64", N.STENCIL_FP64), ("RVE_STENCIL_FP32", N.STENCIL_FP32),
                      ("RVE_SCHEME_Q1", N.SCHEME_Q1), ("RVE_SCHEME_FD5", N.SCHEME_FD5)):
        m = re.search(r"\b%s\s*=\s*(-?\d+)" % name, src)
        assert m and int(m.group(1)) == val, name


def test_occupancy_threshold_host_rule(lib):
    # Poisson centres with mean mu per site: a site is a centre with
    # probability 1 - exp(-mu), scaled to the 32-bit comparison threshold
    import math
    for mu in (1e-6, math.log(2.0) / 64, math.log(2.0) / 4, 0.5, 3.0):
        want = round(4294967296.0 * -math.expm1(-mu))
        assert lib.rve_occupancy_threshold(mu) == min(want, 0xFFFFFFFF)
    assert lib.rve_occupancy_threshold(0.0) == 0
    assert lib.rve_occupancy_threshold(-1.0) == 0
    assert lib.rve_occupancy_threshold(float("nan")) == 0
    assert lib.rve_occupancy_threshold(800.0) == 0xFFFFFFFF
