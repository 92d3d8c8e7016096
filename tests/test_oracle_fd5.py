"""Pins of the oracle's lumped five-point discretisation (oracle/fd5.py)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fd5, q1


def _two_valued(n, seed, lo=1.0, hi=10.0):
    m = np.random.default_rng(seed).random((n, n)) < 0.5
    return np.where(m, hi, lo)


def _edge_loop_dense(a):
    """Independent construction: for every edge, w (u_p - u_q) into both end
    nodes, the weight being the mean of the two cells that share the edge."""
    n = a.shape[0]
    A = np.zeros((n * n, n * n))
    idx = lambda p, q: (p % n) * n + (q % n)
    for p in range(n):
        for q in range(n):
            for (dp, dq, w) in ((1, 0, 0.5 * (a[p, (q - 1) % n] + a[p, q])),
                                (0, 1, 0.5 * (a[(p - 1) % n, q] + a[p, q]))):
                i, j = idx(p, q), idx(p + dp, q + dq)
                A[i, i] += w
                A[j, j] += w
                A[i, j] -= w
                A[j, i] -= w
    return A


@pytest.mark.parametrize("n", [4, 6, 8])
def test_kronecker_assembly_matches_edge_loop(n):
    a = _two_valued(n, n)
    assert np.allclose(fd5.assemble(a).toarray(), _edge_loop_dense(a), rtol=0, atol=1e-13)


def test_constant_coefficient_is_the_fd_laplacian():
    n = 8
    A = fd5.assemble(np.full((n, n), 2.0)).toarray()
    assert np.allclose(A, 2.0 * fd5.laplacian_fd(n).toarray())
    row = A[3 * n + 4].reshape(n, n)
    assert row[3, 4] == 8.0
    for p, q in ((2, 4), (4, 4), (3, 3), (3, 5)):
        assert row[p, q] == -2.0
    assert np.count_nonzero(row) == 5


def test_laplacian_matches_paper_kronecker_form():
    # Delta_1 (x) I + I (x) Delta_2 with -Delta = tridiag(1, -2, 1) + periodic corners (eqn. Lap_Kron)
    n = 7
    D = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    D[0, -1] = D[-1, 0] = -1
    want = np.kron(D, np.eye(n)) + np.kron(np.eye(n), D)
    assert np.array_equal(fd5.laplacian_fd(n).toarray(), want)


def test_operator_symmetric_psd_one_dim_kernel():
    a = _two_valued(6, 3)
    A = fd5.assemble(a).toarray()
    assert np.allclose(A, A.T)
    assert np.allclose(A.sum(axis=1), 0.0)
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12 and ev[1] > 1e-6


def test_symbol_matches_dense_eigenvalues():
    n = 6
    ev = np.sort(np.linalg.eigvalsh(fd5.laplacian_fd(n).toarray()))
    assert np.allclose(ev, np.sort(fd5.symbol(n).ravel()), atol=1e-12)


def test_rhs_is_minus_A_times_affine_coordinate():
    # f_i = -A x_i with x_i the affine coordinate (brute force on the dense
    # operator with the wrap-around edges carrying a unit jump), and it equals
    # the Galerkin right-hand side of the Q1 scheme
    n = 6
    a = _two_valued(n, 9)
    A = _edge_loop_dense(a)
    f1, f2 = fd5.rhs(a)
    for f, axis in ((f1, 0), (f2, 1)):
        want = np.zeros((n, n))
        for p in range(n):
            for q in range(n):
                for (dp, dq, w) in ((1, 0, 0.5 * (a[p, (q - 1) % n] + a[p, q])),
                                    (0, 1, 0.5 * (a[(p - 1) % n, q] + a[p, q]))):
                    if (dp, dq)[axis] == 0:
                        continue
                    # x_i increases by 1 from (p, q) to its neighbour along axis
                    want[p, q] += w
                    want[(p + dp) % n, (q + dq) % n] -= w
        assert np.allclose(f, want, atol=1e-14)
    g1, g2 = q1.rhs(a)
    assert np.allclose(f1, g1, atol=1e-14) and np.allclose(f2, g2, atol=1e-14)


def test_constant_field_and_laminates_exact():
    r = fd5.solve(np.full((8, 8), 3.25))
    assert r.iters == (0, 0) and np.array_equal(r.ahom, 3.25 * np.eye(2))
    n = 12
    c = np.random.default_rng(1).uniform(1.0, 10.0, n)
    lam = np.repeat(c[:, None], n, axis=1)
    harm, arit = 1.0 / np.mean(1.0 / c), np.mean(c)
    r = fd5.solve(lam)
    assert abs(r.ahom[0, 0] - harm) <= 1e-12 * harm and abs(r.ahom[1, 1] - arit) <= 1e-12 * arit
    assert abs(r.ahom[0, 1]) <= 1e-12
    rt = fd5.solve(lam.T.copy())
    assert abs(rt.ahom[1, 1] - harm) <= 1e-12 * harm and abs(rt.ahom[0, 0] - arit) <= 1e-12 * arit


@pytest.mark.parametrize("n", [4, 6])
def test_matches_dense_direct_solve(n):
    a = _two_valued(n, 20 + n)
    A = _edge_loop_dense(a)
    Ap = np.linalg.pinv(A)
    r = fd5.solve(a)
    for i, f in enumerate(fd5.rhs(a)):
        f = f - f.mean()
        u = (Ap @ f.ravel()).reshape(n, n)
        u -= u.mean()
        assert np.allclose(r.phi[i], u, atol=1e-10)


def test_energy_equals_flux_symmetric_and_voigt_bound():
    a = _two_valued(16, 4)
    r = fd5.solve(a)
    assert np.allclose(r.ahom, r.ahom.T, atol=1e-15)
    assert np.allclose(r.ahom, r.ahom_flux, atol=1e-10)
    ev = np.linalg.eigvalsh(r.ahom)
    assert ev[1] <= np.mean(a) + 1e-12 and ev[0] > 0


def test_cube_group_covariance():
    a = _two_valued(12, 6)
    r = fd5.solve(a).ahom
    rt = fd5.solve(a.T.copy()).ahom
    assert np.allclose(rt, r[::-1, ::-1], atol=1e-10)
    rr = fd5.solve(np.roll(a, (3, 5), axis=(0, 1))).ahom
    assert np.allclose(rr, r, atol=1e-10)
    # reflecting x1 maps cell (p, q) to (n-1-p, q) and flips the sign of a12
    rf = fd5.solve(a[::-1, :].copy()).ahom
    assert np.allclose(rf, [[r[0, 0], -r[0, 1]], [-r[1, 0], r[1, 1]]], atol=1e-10)


def test_gradient_euler_identity_and_central_differences():
    n = 6
    a = _two_valued(n, 8, 1.0, 4.0)
    r = fd5.solve(a)
    g = fd5.dahom_da(a, r.phi)
    for i in range(2):
        for j in range(2):
            assert abs(np.sum(a * g[i, j]) - r.ahom[i, j]) <= 1e-12 * abs(r.ahom).max()
    eps = 1e-6
    for (p, q) in ((0, 0), (2, 3), (5, 1)):
        ap, am = a.copy(), a.copy()
        ap[p, q] += eps
        am[p, q] -= eps
        fdq = (fd5.solve(ap).ahom - fd5.solve(am).ahom) / (2 * eps)
        assert np.allclose(fdq, g[:, :, p, q], atol=1e-8)
