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


def test_gaussian_is_the_normal_density_of_width_eta():
    # eqn. DOS_gauss: g_eta is the centred normal density with standard
    # deviation eta. Pinned by quadrature (unit mass, second moment eta^2,
    # zero first moment), its peak 1 / (sqrt(2 pi) eta), the ratio
    # exp(-1/2) one width out, and the library's normal density.
    from scipy import integrate, stats
    for eta in (0.05, 0.3, 2.0):
        mass = integrate.quad(lambda t: dos.gaussian(t, eta), -np.inf, np.inf)[0]
        first = integrate.quad(lambda t: t * dos.gaussian(t, eta), -np.inf, np.inf)[0]
        second = integrate.quad(lambda t: t * t * dos.gaussian(t, eta), -np.inf, np.inf)[0]
        assert abs(mass - 1.0) <= 1e-10
        assert abs(first) <= 1e-10 * eta
        assert abs(second - eta * eta) <= 1e-10 * eta * eta
        assert abs(dos.gaussian(0.0, eta) - 1.0 / (np.sqrt(2.0 * np.pi) * eta)) <= 1e-15 / eta
        assert abs(dos.gaussian(eta, eta) / dos.gaussian(0.0, eta) - np.exp(-0.5)) <= 1e-15
        t = np.linspace(-5 * eta, 5 * eta, 101)
        assert np.allclose(dos.gaussian(t, eta), stats.norm.pdf(t, loc=0.0, scale=eta), rtol=1e-13, atol=0)


def test_exact_density_integrates_to_one_and_peaks_at_eigenvalues():
    # eqn. DOS: (1/m) sum_j delta(t - lambda_j) broadened by g_eta has unit
    # mass; for well separated eigenvalues and a small width it is a sum of
    # bumps of mass 1/m (weights counted with multiplicity)
    from scipy import integrate
    lam = np.array([0.0, 1.0, 1.0, 3.0])
    eta = 0.01
    mass = integrate.quad(lambda t: dos.dos_exact(lam, np.array([t]), eta)[0], -1.0, 4.0,
                          points=[0.0, 1.0, 3.0], limit=200)[0]
    assert abs(mass - 1.0) <= 1e-9
    peaks = dos.dos_exact(lam, np.array([0.0, 1.0, 3.0]), eta)
    g0 = 1.0 / (np.sqrt(2.0 * np.pi) * eta)
    assert np.allclose(peaks, np.array([0.25, 0.5, 0.25]) * g0, rtol=1e-12)


def test_philox_probes_bit_rule_by_brute_force():
    # the probe rule evaluated entry by entry with Python integers, on the
    # generator pinned by its known-answer vectors (test_oracle_sample)
    from oracle.lattice_sample import philox4x32_10
    seed = (7 << 32) | 12345
    count = 300
    v = dos.philox_probes(count, seed)
    assert set(np.unique(v)) <= {-1.0, 1.0}
    for i in range(count):
        t = i // 128
        w = philox4x32_10([t & 0xFFFFFFFF], [t >> 32], [0], [0x50524F42], seed & 0xFFFFFFFF, seed >> 32)
        word = int(w[(i % 128) // 32][0])
        assert v[i] == (-1.0 if (word >> (i % 32)) & 1 else 1.0), i
    big = dos.philox_probes(1 << 16, 99)
    assert abs(big.mean()) <= 5.0 / np.sqrt(big.size)       # fair signs
    assert not np.array_equal(big[:1000], dos.philox_probes(1000, 98))
