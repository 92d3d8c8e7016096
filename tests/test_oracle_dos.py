"""Pins of the oracle's spectral density (oracle/dos.py)."""
import numpy as np

from oracle import dos, fd5, q1


def _field(n, seed):
    return np.where(np.random.default_rng(seed).random((n, n)) < 0.5, 10.0, 1.0)


def test_constant_coefficient_spectrum_is_the_symbol():
    n = 8
    for A, E in ((q1.assemble(np.full((n, n), 2.0)), 2.0 * q1.symbol(n)),
                 (fd5.assemble(np.full((n, n), 2.0)), 2.0 * fd5.symbol(n))):
        assert np.allclose(np.sort(np.linalg.eigvalsh(A.toarray())), np.sort(E.ravel()), atol=1e-12)


def test_moments_against_dense_eigendecomposition():
    n = 8
    a = _field(n, 1)
    A = q1.assemble(a)
    lam, U = np.linalg.eigh(A.toarray())
    lmax = 16.0 / 3.0 * a.max()          # Gershgorin bound of the Q1 operator
    v = np.random.default_rng(2).choice([-1.0, 1.0], size=n * n)
    mu = dos.chebyshev_moments(A, v, lmax, 40)
    x = lam / (0.5 * lmax) - 1.0
    w2 = (U.T @ v) ** 2
    want = np.array([np.sum(w2 * np.cos(k * np.arccos(np.clip(x, -1, 1)))) for k in range(40)]) / (n * n)
    assert np.allclose(mu, want, rtol=0, atol=1e-12)


def test_estimate_with_all_unit_probes_is_the_exact_density():
    # probes e_1 .. e_m give the trace exactly, so the estimate differs from
    # eqn. DOS_gauss only by the truncated Chebyshev expansion
    n = 6
    a = _field(n, 3)
    for A, lmax in ((q1.assemble(a), 16.0 / 3.0 * a.max()), (fd5.assemble(a), 8.0 * a.max())):
        m = n * n
        mu = np.zeros(300)
        for j in range(m):
            e = np.zeros(m)
            e[j] = 1.0
            mu += dos.chebyshev_moments(A, e, lmax, 300)
        lam = np.linalg.eigvalsh(A.toarray())
        t = np.linspace(0.0, lam.max(), 41)
        eta = 0.05 * lmax
        exact = dos.dos_exact(lam, t, eta)
        est = dos.dos_from_moments(mu, t, lmax, eta, 1200)
        assert np.max(np.abs(est - exact)) <= 1e-8 * np.max(exact)


def test_gershgorin_bounds_hold():
    n = 8
    a = _field(n, 5)
    assert np.linalg.eigvalsh(q1.assemble(a).toarray()).max() <= 16.0 / 3.0 * a.max()
    assert np.linalg.eigvalsh(fd5.assemble(a).toarray()).max() <= 8.0 * a.max()
