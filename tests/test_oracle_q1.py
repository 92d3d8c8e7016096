"""Pins of the oracle's discretisation and solver (CPU only)."""
import numpy as np
import pytest

from brute import dense_system
from oracle import q1
from oracle.pcg import pcg, precond_apply
from sampler import BooleanModel, realization


def _rand_field(n, seed, lo=0.5, hi=5.0):
    return np.random.default_rng(seed).uniform(lo, hi, (n, n))


@pytest.mark.parametrize("n", [2, 3, 4, 7, 8])
def test_kronecker_assembly_matches_element_loop(n):
    # Kronecker sums of 1D matrices (Sec. 3.2) vs a dense loop over cells with
    # Gauss quadrature of the bilinear basis gradients.
    a = _rand_field(n, n)
    A_kron = q1.assemble(a).toarray()
    A_dense, _ = dense_system(a)
    assert np.max(np.abs(A_kron - A_dense)) <= 1e-13 * np.max(np.abs(A_dense))


@pytest.mark.parametrize("n", [3, 6])
def test_rhs_matches_element_loop(n):
    a = _rand_field(n, 10 + n)
    f1, f2 = q1.rhs(a)
    _, f = dense_system(a)
    assert np.allclose(f1.ravel(), f[0], atol=1e-13, rtol=0)
    assert np.allclose(f2.ravel(), f[1], atol=1e-13, rtol=0)


def test_rhs_sums_to_zero():
    a = _rand_field(16, 3)
    for f in q1.rhs(a):
        assert abs(f.sum()) <= 1e-12 * np.abs(f).sum()


def test_operator_symmetric_zero_rowsum_psd_one_dim_kernel():
    a = _rand_field(6, 5)
    A = q1.assemble(a).toarray()
    assert np.max(np.abs(A - A.T)) <= 1e-15 * np.max(np.abs(A))
    assert np.max(np.abs(A.sum(axis=1))) <= 1e-13
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12
    assert abs(ev[0]) <= 1e-12 and ev[1] > 1e-3   # exactly one zero eigenvalue


def test_constant_coefficient_weights():
    # textbook Q1 Laplacian stencil: 8/3 at the centre, -1/3 at all 8 neighbours
    n = 5
    A = q1.assemble(np.ones((n, n))).toarray()
    row = A[2 * n + 2].reshape(n, n)
    expect = np.zeros((n, n))
    expect[1:4, 1:4] = -1.0 / 3.0
    expect[2, 2] = 8.0 / 3.0
    assert np.allclose(row, expect, atol=1e-15)


def test_symbol_matches_dense_eigenvalues():
    n = 8
    E = q1.symbol(n)
    ev = np.linalg.eigvalsh(q1.laplacian_q1(n).toarray())
    assert np.allclose(np.sort(E.ravel()), ev, atol=1e-12)
    # closed form of the symbol: (8 - 2c_k - 2c_l - 4 c_k c_l)/3
    c = np.cos(2 * np.pi * np.arange(n) / n)
    closed = (8 - 2 * c[:, None] - 2 * c[None, :] - 4 * np.outer(c, c)) / 3
    assert np.allclose(E, closed, atol=1e-13)


def test_preconditioner_matches_dense_pseudoinverse():
    n = 8
    a0 = 2.75
    rng = np.random.default_rng(1)
    r = rng.standard_normal((n, n))
    r -= r.mean()
    P = np.linalg.pinv(a0 * q1.laplacian_q1(n).toarray(), hermitian=True)
    z = precond_apply(r, a0, q1.symbol(n))
    assert np.allclose(z.ravel(), P @ r.ravel(), atol=1e-12)


@pytest.mark.parametrize("n", [6, 12])
def test_pcg_matches_direct_solve(n):
    a = _rand_field(n, 7)
    A = q1.assemble(a)
    f1, _ = q1.rhs(a)
    f1 = f1 - f1.mean()
    u, it, res = pcg(A, f1, 0.5 * (a.max() + a.min()), 1e-14, 500)
    ud = np.linalg.pinv(A.toarray(), hermitian=True) @ f1.ravel()
    u = u.ravel() - u.mean()
    assert res <= 1e-12
    assert np.max(np.abs(u - ud)) <= 1e-10 * np.max(np.abs(ud))


def test_pcg_constant_field_converges_in_one_iteration():
    # exact preconditioner: a constant field makes B = a0 A_Delta the operator itself
    n = 16
    a = np.full((n, n), 3.5)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((n, n))
    f -= f.mean()
    u, it, res = pcg(q1.assemble(a), f, 3.5, 1e-12, 50)
    assert it == 1 and res <= 1e-12


def test_pcg_iterations_bounded_in_n():
    # cond(B^-1 A) is bounded independently of the grid (Lemma Cond_Number)
    its = []
    for L in (4, 8, 16):
        a = realization(BooleanModel(L=L, m0=8, a_in=10.0), 99, 0)
        A = q1.assemble(a)
        f1, _ = q1.rhs(a)
        _, it, _ = pcg(A, f1 - f1.mean(), 5.5, 1e-10, 500)
        its.append(it)
    assert max(its) <= 1.4 * min(its) + 2, its
