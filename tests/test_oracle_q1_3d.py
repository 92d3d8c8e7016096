"""Pins of the three-dimensional oracle (oracle/q1_3d.py) against facts that
do not come from its own code: the rank-3 Kronecker form of the element and
of the constant-coefficient operator (Sec. 3.2, eqn. As_Kron_d), entries of
the trilinear element derived by hand, the two-dimensional oracle for fields
constant along x3, closed forms for laminates, the Voigt/Reuss bounds and the
cube symmetries."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ahom as ahom2
from oracle import q1_3d as q3

K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])           # 1D element stiffness on [0, 1]
M1 = np.array([[1.0, 0.5], [0.5, 1.0]]) / 3.0        # 1D element mass


def rng(seed):
    return np.random.default_rng([3, 1903, seed])


def field(n, seed, contrast=10.0):
    return np.where(rng(seed).random((n, n, n)) < 0.5, contrast, 1.0)


def test_element_matrix_is_the_rank3_kronecker_form():
    K = q3.element_matrix()
    ref = np.kron(np.kron(K1, M1), M1) + np.kron(np.kron(M1, K1), M1) + np.kron(np.kron(M1, M1), K1)
    np.testing.assert_allclose(K, ref, atol=1e-15)


def test_element_matrix_entries_by_hand():
    # same corner 1/3; corners differing in one coordinate 0, in two or three -1/12
    K = q3.element_matrix()
    for m in range(8):
        for mp in range(8):
            d = bin(m ^ mp).count("1")
            want = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}[d]
            assert abs(K[m, mp] - want) < 1e-15


def test_element_grad_integrals():
    # int over the cube of d(phi)/dx_i = +-1/4 (the other two hats integrate to 1/2 each)
    g = q3.element_grad_integrals()
    for m in range(8):
        s = ((m >> 2) & 1, (m >> 1) & 1, m & 1)
        for i in range(3):
            assert abs(g[m, i] - (0.25 if s[i] else -0.25)) < 1e-15


def periodic_1d(n, k_or_m):
    """Assembled periodic 1D stiffness circ(-1, 2, -1) or mass circ(1, 4, 1)/6."""
    I = np.eye(n)
    S = np.roll(I, 1, axis=1)
    if k_or_m == "k":
        return 2 * I - S - S.T
    return (4 * I + S + S.T) / 6.0


@pytest.mark.parametrize("n", [3, 4])
def test_constant_coefficient_assembly_is_global_kronecker_sum(n):
    K, M = periodic_1d(n, "k"), periodic_1d(n, "m")
    ref = np.kron(np.kron(K, M), M) + np.kron(np.kron(M, K), M) + np.kron(np.kron(M, M), K)
    A = q3.assemble(np.full((n, n, n), 2.5)).toarray()
    np.testing.assert_allclose(A, 2.5 * ref, atol=1e-13)


@pytest.mark.parametrize("n", [4, 6])
def test_symbol_is_the_spectrum_of_the_constant_operator(n):
    A = q3.assemble(np.ones((n, n, n)))
    e0 = np.zeros(n ** 3)
    e0[0] = 1.0
    col = (A @ e0).reshape(n, n, n)           # circulant column: eigenvalues = its DFT
    lam = np.fft.fftn(col)
    np.testing.assert_allclose(lam.imag, 0.0, atol=1e-13)
    np.testing.assert_allclose(lam.real, q3.symbol(n), atol=1e-13)


def test_assembly_symmetric_psd_constant_kernel():
    a = field(4, 1)
    A = q3.assemble(a).toarray()
    np.testing.assert_allclose(A, A.T, atol=1e-14)
    np.testing.assert_allclose(A @ np.ones(64), 0.0, atol=1e-13)
    w = np.linalg.eigvalsh(A)
    assert w[0] > -1e-12 and w[1] > 1e-3          # one-dimensional kernel (constants)


def test_energy_of_random_fields_by_independent_quadrature():
    # u^T A v = sum_e a_e int_e grad u . grad v, with the gradient of the
    # trilinear interpolant written out through its edge differences
    n = 3
    a = field(n, 2)
    g = rng(3)
    u, v = g.standard_normal((n, n, n)), g.standard_normal((n, n, n))
    A = q3.assemble(a)
    lhs = u.ravel() @ (A @ v.ravel())
    tot = 0.0
    gp = [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)]
    for i in range(n):
        for j in range(n):
            for k in range(n):
                def corner(w, s1, s2, s3):
                    return w[(i + s1) % n, (j + s2) % n, (k + s3) % n]

                def grad(w, x, y, z):
                    c = lambda s1, s2, s3: corner(w, s1, s2, s3)
                    dx = ((c(1, 0, 0) - c(0, 0, 0)) * (1 - y) * (1 - z) + (c(1, 1, 0) - c(0, 1, 0)) * y * (1 - z)
                          + (c(1, 0, 1) - c(0, 0, 1)) * (1 - y) * z + (c(1, 1, 1) - c(0, 1, 1)) * y * z)
                    dy = ((c(0, 1, 0) - c(0, 0, 0)) * (1 - x) * (1 - z) + (c(1, 1, 0) - c(1, 0, 0)) * x * (1 - z)
                          + (c(0, 1, 1) - c(0, 0, 1)) * (1 - x) * z + (c(1, 1, 1) - c(1, 0, 1)) * x * z)
                    dz = ((c(0, 0, 1) - c(0, 0, 0)) * (1 - x) * (1 - y) + (c(1, 0, 1) - c(1, 0, 0)) * x * (1 - y)
                          + (c(0, 1, 1) - c(0, 1, 0)) * (1 - x) * y + (c(1, 1, 1) - c(1, 1, 0)) * x * y)
                    return np.array([dx, dy, dz])

                cell = 0.0
                for x in gp:
                    for y in gp:
                        for z in gp:
                            cell += 0.125 * grad(u, x, y, z) @ grad(v, x, y, z)
                tot += a[i, j, k] * cell
    assert abs(lhs - tot) <= 1e-12 * abs(tot) + 1e-12


def test_rhs_is_minus_operator_on_the_affine_coordinate():
    # f_i = -A xi_i for xi_i(x) = x_i (interior nodes, where the stencil does not wrap)
    n = 6
    a = field(n, 4)
    A = q3.assemble(a)
    f = q3.rhs(a)
    idx = np.arange(n)
    for i in range(3):
        xi = np.broadcast_to(idx.reshape([n if d == i else 1 for d in range(3)]), (n, n, n)).astype(float)
        Ax = (A @ xi.ravel()).reshape(n, n, n)
        sl = tuple(slice(1, n - 1) for _ in range(3))
        np.testing.assert_allclose(f[i][sl], -Ax[sl], atol=1e-12)
    np.testing.assert_allclose(f.sum(axis=(1, 2, 3)), 0.0, atol=1e-12)


def test_precond_exact_for_constant_coefficient():
    n = 8
    a = np.full((n, n, n), 3.0)
    A = q3.assemble(a)
    r = rng(5).standard_normal((n, n, n))
    r -= r.mean()
    z = q3.precond_apply(r, 3.0, q3.symbol(n))
    np.testing.assert_allclose((A @ z.ravel()).reshape(n, n, n), r, atol=1e-12)
    assert abs(z.mean()) < 1e-14


def test_constant_field_gives_identity_scaled():
    E, F, phi, its = q3.homogenize(np.full((4, 4, 4), 2.0))
    np.testing.assert_allclose(E, 2.0 * np.eye(3), atol=1e-14)
    np.testing.assert_allclose(F, 2.0 * np.eye(3), atol=1e-14)
    assert its == [0, 0, 0] and np.all(phi == 0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_closed_form(axis):
    # layers normal to x_axis: A_hom = harmonic mean along the normal,
    # arithmetic mean along the layers (exact for the Q1 discretisation: the
    # corrector is piecewise linear along the normal)
    n = 8
    c = np.array([1.0, 5.0, 5.0, 2.0, 9.0, 1.0, 3.0, 4.0])
    a = np.broadcast_to(c.reshape([n if d == axis else 1 for d in range(3)]), (n, n, n)).copy()
    E, F, _phi, _its = q3.homogenize(a)
    want = np.eye(3) * c.mean()
    want[axis, axis] = 1.0 / np.mean(1.0 / c)
    np.testing.assert_allclose(E, want, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(F, want, rtol=1e-10, atol=1e-12)


def test_field_constant_along_x3_matches_the_2d_oracle():
    n = 8
    a2 = np.where(rng(6).random((n, n)) < 0.5, 10.0, 1.0)
    a = np.repeat(a2[:, :, None], n, axis=2)
    E3, F3, x3, _ = q3.homogenize(a)
    r2 = ahom2.solve(a2, tol=1e-12)
    np.testing.assert_allclose(E3[:2, :2], r2.ahom, rtol=1e-10)
    np.testing.assert_allclose(E3[2, 2], a2.mean(), rtol=1e-12)
    np.testing.assert_allclose(E3[:2, 2], 0.0, atol=1e-12)
    np.testing.assert_allclose(F3, E3, rtol=1e-9, atol=1e-12)
    # the correctors are the 2D ones, constant along x3; the third one vanishes
    assert np.max(np.abs(x3[2])) < 1e-12
    for i in range(2):
        for k in range(n):
            np.testing.assert_allclose(x3[i][:, :, k], r2.phi[i], atol=1e-9)


def test_bounds_symmetry_and_forms_agree():
    n = 8
    a = field(n, 7)
    E, F, _phi, _ = q3.homogenize(a)
    np.testing.assert_allclose(E, E.T, atol=1e-13)
    np.testing.assert_allclose(F, E, rtol=1e-9, atol=1e-11)
    w = np.linalg.eigvalsh(E)
    assert w[0] >= 1.0 / np.mean(1.0 / a) - 1e-12
    assert w[-1] <= a.mean() + 1e-12


def test_axis_permutation_and_reflection():
    n = 8
    a = field(n, 8)
    E, _F, _phi, _ = q3.homogenize(a)
    perm = (2, 0, 1)
    Ep, _, _, _ = q3.homogenize(np.transpose(a, perm))
    # new axis d is old axis perm[d]
    np.testing.assert_allclose(Ep, E[np.ix_(perm, perm)], rtol=1e-10, atol=1e-12)
    # reflecting x1 (cells i -> n-1-i) flips the sign of the (1, j) entries
    Er, _, _, _ = q3.homogenize(a[::-1, :, :].copy())
    S = np.diag([-1.0, 1.0, 1.0])
    np.testing.assert_allclose(Er, S @ E @ S, rtol=1e-10, atol=1e-12)


def test_energy_form_matches_matrix_expansion():
    # n^3 A_ij = delta_ij sum a - f_i.x_j - f_j.x_i + x_i^T A x_j at any x
    n = 4
    a = field(n, 9)
    x = rng(10).standard_normal((3, n, n, n))
    A = q3.assemble(a)
    f = q3.rhs(a)
    E, F = q3.ahom(a, x)
    for i in range(3):
        for j in range(3):
            want = ((i == j) * a.sum() - f[i].ravel() @ x[j].ravel() - f[j].ravel() @ x[i].ravel()
                    + x[i].ravel() @ (A @ x[j].ravel())) / n ** 3
            assert abs(E[i, j] - want) < 1e-11
            want_f = ((i == j) * a.sum() - f[j].ravel() @ x[i].ravel()) / n ** 3
            assert abs(F[i, j] - want_f) < 1e-11


def test_pcg_true_residual():
    n = 8
    a = field(n, 11)
    A = q3.assemble(a)
    f = q3.rhs(a)[0]
    f = f - f.mean()
    x, it, rel = q3.pcg(A, f, 5.5, 1e-10, 500)
    assert rel < 2e-10 and 5 < it < 100
    assert isinstance(A, sp.csr_matrix)


def test_matches_dense_pseudoinverse_solve():
    # n = 4 (64 unknowns): the correctors against the dense pseudo-inverse
    n = 4
    a = field(n, 12)
    A = q3.assemble(a).toarray()
    f = q3.rhs(a)
    Ap = np.linalg.pinv(A)
    x, its = q3.correctors(a, tol=1e-13)
    for i in range(3):
        xd = Ap @ (f[i] - f[i].mean()).ravel()
        xd -= xd.mean()
        np.testing.assert_allclose(x[i].ravel(), xd, atol=1e-11)
    E, _F = q3.ahom(a, x)
    Ed, _ = q3.ahom(a, np.array([(Ap @ (f[i] - f[i].mean()).ravel()).reshape(n, n, n) for i in range(3)]))
    np.testing.assert_allclose(E, Ed, rtol=1e-11)


def test_homogeneity():
    n = 4
    a = field(n, 13)
    E1, _, _, _ = q3.homogenize(a)
    E2, _, _, _ = q3.homogenize(2.5 * a)
    np.testing.assert_allclose(E2, 2.5 * E1, rtol=1e-11)
