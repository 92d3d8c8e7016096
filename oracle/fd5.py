"""The lumped (five-point) discretisation of Sec. 3.2, FP64 (oracle) -- TEST
INFRASTRUCTURE ONLY.

Lumping the mass matrices turns the Q1 stiffness into the Kronecker form
A = A_1 (x) D_2 + D_1 (x) A_2 with diagonal D (eqn. Lapl_Kron_D); cell by cell
(eqn. As_Kron with the smallest blocks, m0bar = 2) each cell e contributes
a_e (k_e (x) d_e + d_e (x) k_e), where k_e = [[1, -1], [-1, 1]] is the 1D
element stiffness and d_e = diag(1/2, 1/2) the lumped element mass
(Ihat = diag(1/2, ..., 1/2) of eqn. As_Kron). The result is a five-point
operator: the edge between nodes (p, q) and (p+1, q) carries the mean of the
two cells beside it, (a[p][q-1] + a[p][q]) / 2, and likewise in x2.
Its constant-coefficient member is the finite-difference Laplacian
Delta_1 (x) I + I (x) Delta_2 of eqn. Lap_Kron, the preconditioner of this
scheme, with symbol (2 - 2 c_k) + (2 - 2 c_l).

Grid units and index conventions as in q1.py. The right-hand sides are
f_i = -A x_i for the affine coordinate x_i (each edge along x_i increments
it by one, the wrap-around edge included); the homogenized matrix is the
edge-quadrature average < (e_i + grad phi_i) . a (e_j + grad phi_j) > with
the edge weights above, and its derivative in a_e is, by stationarity in the
correctors, the cell's share of that sum (half of each of its four edges).

Pins: tests/test_oracle_fd5.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import q1
from .ahom import Realization, preconditioner_scale
from .pcg import pcg


def lumped_mass_1d(c: np.ndarray) -> sp.csr_matrix:
    """Lumped periodic 1D mass of a piecewise constant coefficient: each
    interval [j, j+1] puts c[j]/2 on both its end nodes."""
    c = np.asarray(c, dtype=np.float64)
    return sp.diags(0.5 * (np.roll(c, 1) + c)).tocsr()


def assemble(a: np.ndarray) -> sp.csr_matrix:
    """A = sum over strips of cells along x1 of K_i (x) D(a[i, :]) +
    D_i (x) K(a[i, :]) (eqns. Lapl_Kron_D, As_Kron): K_i and D_i are the
    stiffness and lumped mass of the interval [i, i+1], K(c) and D(c) the
    weighted ones of the strip's coefficients."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("coefficient field must be square")
    rows, cols, vals = [], [], []
    for i in range(n):
        ind = q1.interval_indicator(n, i)
        k1 = q1.weighted_stiffness_1d(ind)
        d1 = lumped_mass_1d(ind)
        for term in (sp.kron(k1, lumped_mass_1d(a[i]), format="coo"),
                     sp.kron(d1, q1.weighted_stiffness_1d(a[i]), format="coo")):
            rows.append(term.row)
            cols.append(term.col)
            vals.append(term.data)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * n, n * n)).tocsr()


def laplacian_fd(n: int) -> sp.csr_matrix:
    """Delta_1 (x) I + I (x) Delta_2 with the periodic tridiag(-1, 2, -1)
    (eqn. Lap_Kron, sign as a positive semidefinite operator)."""
    one = np.ones(n)
    K = q1.weighted_stiffness_1d(one)
    I = sp.identity(n, format="csr")
    return (sp.kron(K, I) + sp.kron(I, K)).tocsr()


def symbol(n: int) -> np.ndarray:
    """Eigenvalues of laplacian_fd on the Fourier mode (k, l):
    (2 - 2 cos(2 pi k / n)) + (2 - 2 cos(2 pi l / n))."""
    lam = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)
    return lam[:, None] + lam[None, :]


def edge_weights(a: np.ndarray):
    """W1[p][q]: edge (p, q)-(p+1, q), mean of cells (p, q-1) and (p, q);
    W2[p][q]: edge (p, q)-(p, q+1), mean of cells (p-1, q) and (p, q)."""
    a = np.asarray(a, dtype=np.float64)
    W1 = 0.5 * (np.roll(a, 1, axis=1) + a)
    W2 = 0.5 * (np.roll(a, 1, axis=0) + a)
    return W1, W2


def rhs(a: np.ndarray):
    """f_i = -A x_i: with the x1-edge weights, f_1[p][q] = W1[p][q] -
    W1[p-1][q]; likewise f_2 with W2 along x2."""
    W1, W2 = edge_weights(a)
    return W1 - np.roll(W1, 1, axis=0), W2 - np.roll(W2, 1, axis=1)


def _edge_grads(phi: np.ndarray):
    """Differences of a nodal field along the x1 and x2 edges."""
    return np.roll(phi, -1, axis=0) - phi, np.roll(phi, -1, axis=1) - phi


def ahom_energy(a, phis) -> np.ndarray:
    """< (e_i + grad phi_i) . a (e_j + grad phi_j) > by edge quadrature."""
    W1, W2 = edge_weights(a)
    g = [_edge_grads(p) for p in phis]
    n2 = a.size
    out = np.empty((2, 2))
    for i in range(2):
        for j in range(2):
            t1 = ((i == 0) + g[i][0]) * ((j == 0) + g[j][0])
            t2 = ((i == 1) + g[i][1]) * ((j == 1) + g[j][1])
            out[i, j] = (np.sum(W1 * t1) + np.sum(W2 * t2)) / n2
    return out


def ahom_flux(a, phis, fs) -> np.ndarray:
    n2 = a.size
    abar = float(np.sum(a)) / n2
    return np.array([[abar * (i == j) - np.vdot(phis[i], fs[j]) / n2 for j in range(2)] for i in range(2)])


def solve(a: np.ndarray, tol: float = 1e-13, maxit: int = 2000) -> Realization:
    a = np.asarray(a, dtype=np.float64)
    A = assemble(a)
    E = symbol(a.shape[0])
    a0 = preconditioner_scale(a)
    fs, phis, its, res = [], [], [], []
    for f in rhs(a):
        f = f - f.mean()
        u, it, rr = pcg(A, f, a0, tol, maxit, E)
        fs.append(f)
        phis.append(u - u.mean())
        its.append(it)
        res.append(rr)
    return Realization(phi=np.stack(phis), ahom=ahom_energy(a, phis), ahom_flux=ahom_flux(a, phis, fs),
                       iters=tuple(its), relres=tuple(res), f=np.stack(fs))


def dahom_da(a: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """(2, 2, n, n): d abar_ij / d a_e for every cell e = (p, q), the cell's
    share of the edge sum: its two x1-edges (p, q)-(p+1, q), (p, q+1)-(p+1, q+1)
    and its two x2-edges (p, q)-(p, q+1), (p+1, q)-(p+1, q+1), each with weight
    1/2, divided by n^2."""
    n2 = a.size
    g = [_edge_grads(p) for p in phi]
    out = np.empty((2, 2) + a.shape)
    for i in range(2):
        for j in range(2):
            t1 = ((i == 0) + g[i][0]) * ((j == 0) + g[j][0])     # at x1-edges, indexed by start node
            t2 = ((i == 1) + g[i][1]) * ((j == 1) + g[j][1])
            # cell (p, q): x1-edges start at (p, q) and (p, q+1); x2-edges at (p, q) and (p+1, q)
            out[i, j] = 0.5 * (t1 + np.roll(t1, -1, axis=1) + t2 + np.roll(t2, -1, axis=0)) / n2
    return out
