"""Pins of the oracle's derivative and ensemble statistics (CPU only)."""
import numpy as np
import pytest

from oracle import ahom as oa
from oracle import stats as ost
from sampler import BooleanModel, realization


def test_gradient_matches_central_differences():
    n = 4
    a = np.random.default_rng(3).uniform(1.0, 6.0, (n, n))
    r = oa.solve(a, tol=1e-14)
    g = oa.dahom_da(a, r.phi)
    step = 1e-5
    for (x, y) in [(0, 0), (1, 3), (3, 2)]:
        ap = a.copy(); ap[x, y] += step
        am = a.copy(); am[x, y] -= step
        fd = (oa.solve(ap, tol=1e-14).ahom - oa.solve(am, tol=1e-14).ahom) / (2 * step)
        assert np.max(np.abs(fd - g[:, :, x, y])) <= 1e-8


def test_gradient_euler_identity():
    # A_hom is homogeneous of degree one in a
    a = realization(BooleanModel(L=4, m0=8, a_in=10.0), 21, 0)
    r = oa.solve(a)
    g = oa.dahom_da(a, r.phi)
    assert np.allclose(np.einsum("ijxy,xy->ij", g, a), r.ahom, rtol=1e-11, atol=1e-12)


def test_gradient_laminate_closed_form():
    n = 8
    c = np.random.default_rng(4).uniform(1.0, 10.0, n)
    a = np.repeat(c[:, None], n, axis=1)
    r = oa.solve(a)
    g = oa.dahom_da(a, r.phi)
    A11 = r.ahom[0, 0]
    # d/da_e of the harmonic mean of rows, spread over the n cells of a row
    expect11 = np.repeat(((A11 / c) ** 2 / (n * n))[:, None], n, axis=1)
    assert np.allclose(g[0, 0], expect11, rtol=1e-10, atol=1e-14)
    assert np.allclose(g[1, 1], 1.0 / (n * n), rtol=1e-10)
    assert np.max(np.abs(g[0, 1])) <= 1e-12


def test_contrast_derivative_matches_fd():
    model = BooleanModel(L=2, m0=4, a_in=10.0)
    from sampler.boolean_model import covered_mask
    mask = covered_mask(model, 31, 0)
    field = lambda c: np.where(mask, c, 1.0)
    r = oa.solve(field(10.0), tol=1e-14)
    d = oa.dahom_dcontrast(oa.dahom_da(field(10.0), r.phi), mask)
    s = 1e-5
    fd = (oa.solve(field(10.0 + s), tol=1e-14).ahom - oa.solve(field(10.0 - s), tol=1e-14).ahom) / (2 * s)
    assert np.max(np.abs(fd - d)) <= 1e-8


def test_stats_against_numpy():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((50, 2, 2)) * 0.01 + np.array([[2.0, 0.0], [0.0, 2.1]])
    A = 0.5 * (A + A.transpose(0, 2, 1))               # homogenized matrices are symmetric
    flat = A.reshape(50, 4)
    assert np.allclose(ost.empirical_mean(A).ravel(), flat.mean(0))
    assert np.allclose(ost.centred_variance(A).ravel(), flat.var(0, ddof=1))
    Q = ost.quartic(A, L=16)
    C = 256 * np.cov(flat, rowvar=False, ddof=1)      # C[(i,j),(k,l)] = L^2 cov(A_ij, A_kl)
    # Kronecker layout of the tensor square: Q[(i,k),(j,l)] = L^2 cov(A_ij, A_kl)
    for i, j, k, l in np.ndindex(2, 2, 2, 2):
        assert np.isclose(Q[2 * i + k, 2 * j + l], C[2 * i + j, 2 * k + l], rtol=1e-12, atol=1e-18)
    # symmetric A makes the Kronecker layout symmetric; the covariance layout is PSD
    assert np.allclose(Q, Q.T, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(C)[0] >= -1e-15
    # uncentred standard deviations reduce to np.std for mean-zero data
    B = A - A.mean(0)
    s12, sdd = ost.std_uncentred(B)
    assert np.isclose(s12, np.std(B[:, 0, 1])) and np.isclose(sdd, np.std(B[:, 0, 0] - B[:, 1, 1]))


def _orbit(a):
    """The 8 images of a cell field under the symmetries of the square."""
    out = []
    for k in range(4):
        r = np.rot90(a, k)
        out.append(r.copy())
        out.append(r.T.copy())
    return out


def test_quartic_zero_and_equality_pattern_on_orbit_closed_sample():
    # eqns. wg14-wg18: on a sample closed under the cube group the pattern is exact
    fields = []
    for idx in range(3):
        fields += _orbit(realization(BooleanModel(L=2, m0=4, a_in=10.0), 41, idx))
    A = np.stack([oa.solve(f, tol=1e-14).ahom for f in fields])
    Q = ost.quartic(A, L=2)
    q = lambda i, j, k, l: Q[2 * i + k, 2 * j + l]   # q[(i,k),(j,l)] = L^2 cov(A_ij, A_kl)
    tol = 1e-12 * np.max(np.abs(Q))
    zeros = [(0, 0, 0, 1), (0, 0, 1, 0), (0, 1, 0, 0), (1, 0, 0, 0),
             (0, 1, 1, 1), (1, 0, 1, 1), (1, 1, 0, 1), (1, 1, 1, 0)]
    for z in zeros:                                    # wg16, wg17
        assert abs(q(*z)) <= tol
    v = q(0, 1, 0, 1)                                  # wg14
    for z in [(0, 1, 1, 0), (1, 0, 0, 1), (1, 0, 1, 0)]:
        assert abs(q(*z) - v) <= tol
    assert abs(q(0, 0, 1, 1) - q(1, 1, 0, 0)) <= tol   # wg15
    assert abs(q(0, 0, 0, 0) - q(1, 1, 1, 1)) <= tol   # wg18
    m = ost.empirical_mean(A)                          # wg04 (exact on the orbit)
    assert abs(m[0, 0] - m[1, 1]) <= 1e-12 and abs(m[0, 1]) <= 1e-12
