"""Q1 Galerkin discretisation on the periodic grid, in FP64 (oracle).

Grid units throughout (h = 1): in 2D the Q1 stiffness matrix does not depend
on h, the Galerkin right-hand side scales like h and so the corrector scales
like h, while its gradient and the homogenized matrix are h-free.

Index conventions: n periodic nodes per axis; node (p, q) has linear index
p*n + q (x1 slow, x2 fast: the big-endian map of Sec. 3.2); cell (i, j) spans
nodes i..i+1 along x1 and j..j+1 along x2, mod n. Kronecker factors are
ordered x1 (left) then x2 (right), matching Definition Kron.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _periodic_tridiag(n: int, diag: np.ndarray, upper: np.ndarray) -> sp.csr_matrix:
    """Symmetric periodic tridiagonal matrix with the given diagonal and
    (p, p+1 mod n) entries; duplicate positions (n = 2) are summed."""
    p = np.arange(n)
    rows = np.concatenate([p, p, (p + 1) % n])
    cols = np.concatenate([p, (p + 1) % n, p])
    vals = np.concatenate([diag, upper, upper])
    out = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    out.eliminate_zeros()
    return out


def weighted_stiffness_1d(c: np.ndarray) -> sp.csr_matrix:
    """Periodic 1D stiffness with piecewise-constant coefficient (Sec. 3.2,
    eqn. stiff_matrix_1point): c[j] is the value on interval [j, j+1]; row p
    has diagonal c[p-1] + c[p] and off-diagonals -c[p] to p+1, -c[p-1] to p-1."""
    c = np.asarray(c, dtype=np.float64)
    return _periodic_tridiag(c.size, np.roll(c, 1) + c, -c)


def weighted_mass_1d(c: np.ndarray) -> sp.csr_matrix:
    """Periodic 1D mass matrix int c psi_p psi_q with the same piecewise
    constant coefficient: each interval contributes c[j]*[[2,1],[1,2]]/6."""
    c = np.asarray(c, dtype=np.float64)
    return _periodic_tridiag(c.size, (np.roll(c, 1) + c) * (2.0 / 6.0), c / 6.0)


def interval_indicator(n: int, i: int) -> np.ndarray:
    """Coefficient vector of the indicator of interval [i, i+1]."""
    e = np.zeros(n)
    e[i] = 1.0
    return e


def assemble(a: np.ndarray) -> sp.csr_matrix:
    """Stiffness matrix a_{mu nu} = int a grad psi_mu . grad psi_nu (eqn.
    FEM_discr) by Kronecker sums (Sec. 3.2).

    The per-cell field is written as a sum of separable terms, one per strip
    of cells along x1: a(x1, x2) = sum_i 1_[i,i+1](x1) c_i(x2) with
    c_i = a[i, :]. For each separable term the rank-2 Kronecker form
    A1 (x) S2 + S1 (x) A2 holds (stiffness (x) weighted mass plus weighted mass
    (x) stiffness), so A is the sum of n such pairs.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("coefficient field must be square")
    rows, cols, vals = [], [], []
    for i in range(n):
        ind = interval_indicator(n, i)
        k1 = weighted_stiffness_1d(ind)
        m1 = weighted_mass_1d(ind)
        s2 = weighted_mass_1d(a[i])
        a2 = weighted_stiffness_1d(a[i])
        for term in (sp.kron(k1, s2, format="coo"), sp.kron(m1, a2, format="coo")):
            rows.append(term.row)
            cols.append(term.col)
            vals.append(term.data)
    # COO -> CSR sums the contributions that land on the same entry.
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * n, n * n)).tocsr()


def laplacian_q1(n: int) -> sp.csr_matrix:
    """Constant-coefficient periodic Q1 operator A_Delta = K (x) M + M (x) K
    (the coefficient-one member of :func:`assemble`)."""
    one = np.ones(n)
    K = weighted_stiffness_1d(one)
    M = weighted_mass_1d(one)
    return (sp.kron(K, M) + sp.kron(M, K)).tocsr()


def _cell_to_node_1d(n: int):
    """1D cell-to-node integrals: D[p, j] = int_j^{j+1} psi_p' and
    W[p, j] = int_j^{j+1} psi_p, for hat functions psi_p."""
    j = np.arange(n)
    D = np.zeros((n, n))
    W = np.zeros((n, n))
    np.add.at(D, ((j + 1) % n, j), 1.0)
    np.add.at(D, (j, j), -1.0)
    np.add.at(W, ((j + 1) % n, j), 0.5)
    np.add.at(W, (j, j), 0.5)
    return D, W


def rhs(a: np.ndarray):
    """Galerkin right-hand sides f_i with entries -int a d(psi_alpha)/dx_i
    (eqn. FEM_discr_RHS, and the flux form before eqn. wg01), integrated
    exactly per cell. Separability of psi and of each cell indicator turns the
    cell sum into two 1D matrix products: f_1 = -D a W^T, f_2 = -W a D^T."""
    a = np.asarray(a, dtype=np.float64)
    D, W = _cell_to_node_1d(a.shape[0])
    f1 = -(D @ a @ W.T)
    f2 = -(W @ a @ D.T)
    return f1, f2


def circulant_eigenvalues(first_column: np.ndarray) -> np.ndarray:
    """Eigenvalues of a real symmetric circulant matrix, in Fourier order."""
    return np.fft.fft(first_column).real


def symbol(n: int) -> np.ndarray:
    """Eigenvalues E[k, l] of A_Delta = K (x) M + M (x) K on the Fourier mode
    (k, l): lamK[k]*lamM[l] + lamM[k]*lamK[l]. E[0, 0] = 0 (constants)."""
    one = np.ones(n)
    lamK = circulant_eigenvalues(weighted_stiffness_1d(one)[:, 0].toarray().ravel())
    lamM = circulant_eigenvalues(weighted_mass_1d(one)[:, 0].toarray().ravel())
    return np.outer(lamK, lamM) + np.outer(lamM, lamK)


def element_matrices():
    """Unit-coefficient Q1 element data on one cell, local node order
    (0,0), (0,1), (1,0), (1,1) (x1 slow). Returns (k_e, b_1, b_2): the 4x4
    element stiffness k (x) m + m (x) k from the 1D element stiffness
    k = [[1,-1],[-1,1]] and mass m = [[2,1],[1,2]]/6, and the element
    right-hand-side vectors b_i = -int grad psi . e_i."""
    k = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    d = np.array([-1.0, 1.0])   # int psi' over the cell
    w = np.array([0.5, 0.5])    # int psi over the cell
    ke = np.kron(k, m) + np.kron(m, k)
    b1 = -np.kron(d, w)
    b2 = -np.kron(w, d)
    return ke, b1, b2


def cell_corners(u: np.ndarray) -> np.ndarray:
    """Corner values of a nodal field on every cell, shape (n, n, 4) in the
    local order of :func:`element_matrices`."""
    return np.stack([u, np.roll(u, -1, axis=1), np.roll(u, -1, axis=0),
                     np.roll(np.roll(u, -1, axis=0), -1, axis=1)], axis=-1)
