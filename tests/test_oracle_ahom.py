"""Pins of the oracle's homogenized matrix (CPU only)."""
import os

import numpy as np
import pytest

from brute import direct_ahom
from oracle import ahom as oa
from sampler import BooleanModel, realization

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _two_valued(n, seed, lo=1.0, hi=10.0):
    m = np.random.default_rng(seed).random((n, n)) < 0.5
    return np.where(m, hi, lo)


def test_constant_field_is_exactly_a_identity():
    r = oa.solve(np.full((8, 8), 3.25))
    assert r.iters == (0, 0)
    assert np.array_equal(r.ahom, 3.25 * np.eye(2))
    assert np.array_equal(r.ahom_flux, 3.25 * np.eye(2))


@pytest.mark.parametrize("n", [8, 16])
def test_laminate_harmonic_and_arithmetic_means(n):
    # a depends on x1 only: the exact corrector is piecewise linear in x1, so
    # it lies in the Q1 space and the discrete A_hom is exact.
    c = np.random.default_rng(n).uniform(1.0, 10.0, n)
    a = np.repeat(c[:, None], n, axis=1)
    r = oa.solve(a)
    harm = 1.0 / np.mean(1.0 / c)
    arit = np.mean(c)
    assert abs(r.ahom[0, 0] - harm) <= 1e-12 * harm
    assert abs(r.ahom[1, 1] - arit) <= 1e-12 * arit
    assert abs(r.ahom[0, 1]) <= 1e-12 and abs(r.ahom[1, 0]) <= 1e-12
    rt = oa.solve(a.T.copy())
    assert abs(rt.ahom[1, 1] - harm) <= 1e-12 * harm
    assert abs(rt.ahom[0, 0] - arit) <= 1e-12 * arit


@pytest.mark.parametrize("n", [4, 6, 10])
def test_matches_dense_direct_solve(n):
    a = _two_valued(n, 100 + n)
    ref, _ = direct_ahom(a)
    r = oa.solve(a)
    assert np.max(np.abs(r.ahom - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_homogeneity_bounds_symmetry_flux():
    a = realization(BooleanModel(L=4, m0=8, a_in=10.0), 5, 3)
    r = oa.solve(a)
    r2 = oa.solve(2.5 * a)
    assert np.allclose(r2.ahom, 2.5 * r.ahom, rtol=1e-12, atol=1e-13)
    ev = np.linalg.eigvalsh(r.ahom)
    reuss, voigt = 1.0 / np.mean(1.0 / a), np.mean(a)
    assert reuss - 1e-12 <= ev[0] and ev[1] <= voigt + 1e-12
    assert r.ahom[0, 1] == r.ahom[1, 0]
    assert np.max(np.abs(r.ahom_flux - r.ahom)) <= 1e-11


def test_monotone_in_coefficient():
    a = realization(BooleanModel(L=4, m0=4, a_in=10.0), 6, 0)
    b = a.copy()
    b[3, 5] += 4.0
    d = oa.solve(b).ahom - oa.solve(a).ahom
    assert np.linalg.eigvalsh(d)[0] >= -1e-12


def test_cube_group_covariance_per_realization():
    # Q1 on a square grid is invariant under the symmetries of the square
    # (argument for wg19): transposing the field swaps A11 and A22, reflecting
    # x1 negates A12, integer translations change nothing.
    a = realization(BooleanModel(L=4, m0=4, a_in=10.0), 7, 1)
    A = oa.solve(a).ahom
    At = oa.solve(a.T.copy()).ahom
    Ar = oa.solve(a[::-1, :].copy()).ahom
    As = oa.solve(np.roll(np.roll(a, 3, axis=0), 5, axis=1)).ahom
    tol = 1e-11
    assert abs(At[0, 0] - A[1, 1]) <= tol and abs(At[1, 1] - A[0, 0]) <= tol
    assert abs(At[0, 1] - A[0, 1]) <= tol
    assert abs(Ar[0, 1] + A[0, 1]) <= tol and abs(Ar[0, 0] - A[0, 0]) <= tol
    assert np.max(np.abs(As - A)) <= tol


def test_flux_asymmetry_tracks_tolerance():
    # Table conv_Symmet_thresh: the flux form is symmetric only to the solver
    # tolerance; the paper's values (its own realization) shrink with tol.
    data = np.loadtxt(os.path.join(GOLDEN, "symmetry_vs_tol.txt"))
    assert np.all(np.diff(data[:, 1]) <= 0)       # the printed trend itself
    a = realization(BooleanModel(L=4, m0=8, a_in=1.0, a_bg=0.2, law="paper", alpha=0.5), 11, 0)
    asym = []
    for tol in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11):
        F = oa.solve(a, tol=tol).ahom_flux
        asym.append(abs(F[0, 1] - F[1, 0]))
    assert asym[-1] <= 1e-11
    assert asym[-1] < asym[0]
    for tol, v in zip((1e-3, 1e-5, 1e-7, 1e-9, 1e-11), asym):
        assert v <= 10 * tol


def test_preconditioner_scale_is_the_minimax_shift():
    # Proof of Lemma Cond_Number: with a(x) between a_min and a_max, the
    # constant-coefficient preconditioner is scaled by the midpoint (the
    # paper's (1 + lambda)/2 for a in [lambda, 1]); that midpoint is the
    # scale s that minimises max_x |1 - a(x)/s|, the contraction factor of
    # the preconditioned Richardson step. Pinned by the paper's value, by
    # brute-force minimisation over s, and by its order-free definition.
    lam = 0.1
    a = np.where(np.random.default_rng(4).random((8, 8)) < 0.5, 1.0, lam)
    assert abs(oa.preconditioner_scale(a) - (1.0 + lam) / 2.0) <= 1e-15
    b = np.where(np.random.default_rng(5).random((8, 8)) < 0.5, 10.0, 1.0)
    assert oa.preconditioner_scale(b) == 5.5
    rng = np.random.default_rng(6)
    c = rng.uniform(0.3, 7.0, (6, 6))
    s = np.linspace(0.3, 7.0, 200001)
    worst = np.max(np.abs(1.0 - c.ravel()[None, :] / s[:, None]), axis=1)
    best = s[np.argmin(worst)]
    assert abs(oa.preconditioner_scale(c) - best) <= 2 * (s[1] - s[0])
    assert oa.preconditioner_scale(c) == oa.preconditioner_scale(np.flip(c.T))


def test_pcg_iterates_do_not_depend_on_the_preconditioner_scale():
    # Sec. 3.5: B = a0 A_Delta enters PCG only through directions and step
    # lengths, which a positive factor on B leaves unchanged (alpha scales by
    # 1/s, z by s); the iterate after k steps is the same for any a0.
    from oracle import q1
    from oracle.pcg import pcg
    a = _two_valued(16, 21)
    A = q1.assemble(a)
    f = q1.rhs(a)[0]
    f = f - f.mean()
    for k in (1, 3, 7):
        x1, _, _ = pcg(A, f, 1.0, 0.0, k)
        x2, _, _ = pcg(A, f, 37.5, 0.0, k)
        assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x1))
