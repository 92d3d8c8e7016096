"""Three-dimensional corrector problems (d = 3) with the Q1 (trilinear)
Galerkin discretisation on the periodic grid, FP64 -- TEST INFRASTRUCTURE ONLY.

The problem setting is unchanged for d > 2 (Sec. 2: the coefficient matrix is
a(x) times the d x d identity, one corrector per unit vector e_i), and the
Kronecker construction of Sec. 3.2 extends to d-factor products (eqn.
As_Kron_d and the rank-3 periodic Laplacian of Sec. 3.2). Here, in grid units
(h = 1):

  element matrix    K_e = int grad phi_m . grad phi_m' over the unit cube,
                    phi_m the eight trilinear corner functions, by 2-point
                    Gauss quadrature per axis (exact: the integrands have
                    degree <= 2 in each variable);
  stiffness         A = sum_e a_e K_e (node indices mod n);
  right-hand sides  f_i[node] = - sum_e a_e int_e d(psi_node)/dx_i;
  preconditioner    B = a0 A_Delta with A_Delta the constant-coefficient
                    stiffness, applied as its pseudo-inverse by a 3D FFT with
                    the symbol  kappa_k mu_l mu_m + mu_k kappa_l mu_m +
                    mu_k mu_l kappa_m  (kappa = 2 - 2 cos, mu = (4 + 2 cos)/6);
  A_hom             energy form <a (e_i + grad phi_i).(e_j + grad phi_j)> and
                    flux form <a (delta_ij + d_j phi_i)>, both by the same
                    cell quadrature.

In physical units the stiffness scales like h and the right-hand side like
h^2, so phi = h x with x the grid-unit solution, and A_hom is h-free.

Index conventions: node (p, q, r) has linear index (p n + q) n + r (x3
fastest); cell (i, j, k) spans nodes i..i+1, j..j+1, k..k+1 (mod n); corner
(s1, s2, s3) in {0,1}^3 of a cell is local index 4 s1 + 2 s2 + s3.

Pins: tests/test_oracle_q1_3d.py (element matrix against the Kronecker form
and hand-derived entries, assembly against global Kronecker products, the
symbol against the FFT of the assembled operator, laminates, fields constant
along x3 against the two-dimensional oracle, bounds and symmetries).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))   # 2-point rule on [0, 1], weights 1/2


def _corners():
    return [(s1, s2, s3) for s1 in (0, 1) for s2 in (0, 1) for s3 in (0, 1)]


def _hat(s: int, t: float) -> float:
    return t if s == 1 else 1.0 - t


def _dhat(s: int) -> float:
    return 1.0 if s == 1 else -1.0


def _grad_phi(corner, x):
    """Gradient of the trilinear corner function at the point x of the unit cube."""
    s = corner
    return np.array([
        _dhat(s[0]) * _hat(s[1], x[1]) * _hat(s[2], x[2]),
        _hat(s[0], x[0]) * _dhat(s[1]) * _hat(s[2], x[2]),
        _hat(s[0], x[0]) * _hat(s[1], x[1]) * _dhat(s[2]),
    ])


def _quad_points():
    return [((g1, g2, g3), 0.125) for g1 in _GAUSS for g2 in _GAUSS for g3 in _GAUSS]


def element_matrix() -> np.ndarray:
    """8 x 8 unit-cube stiffness int grad phi_m . grad phi_m'."""
    C = _corners()
    K = np.zeros((8, 8))
    for x, w in _quad_points():
        G = np.array([_grad_phi(c, x) for c in C])   # (8, 3)
        K += w * (G @ G.T)
    return K


def element_grad_integrals() -> np.ndarray:
    """(8, 3): int over the unit cube of d(phi_m)/dx_i."""
    C = _corners()
    out = np.zeros((8, 3))
    for x, w in _quad_points():
        out += w * np.array([_grad_phi(c, x) for c in C])
    return out


def _corner_nodes(n: int) -> np.ndarray:
    """(8, n^3): linear node index of each corner of every cell (cells in
    linear order (i n + j) n + k)."""
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    out = []
    for s1, s2, s3 in _corners():
        out.append(((((i + s1) % n) * n + (j + s2) % n) * n + (k + s3) % n).ravel())
    return np.array(out)


def assemble(a: np.ndarray) -> sp.csr_matrix:
    """Stiffness matrix sum_e a_e K_e of the field a (n, n, n) (cells)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    K = element_matrix()
    nodes = _corner_nodes(n)
    av = a.ravel()
    rows, cols, vals = [], [], []
    for m in range(8):
        for mp in range(8):
            rows.append(nodes[m])
            cols.append(nodes[mp])
            vals.append(av * K[m, mp])
    N = n ** 3
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def rhs(a: np.ndarray) -> np.ndarray:
    """(3, n, n, n): f_i[node] = - sum_e a_e int_e d(psi_node)/dx_i."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    gi = element_grad_integrals()
    nodes = _corner_nodes(n)
    av = a.ravel()
    f = np.zeros((3, n ** 3))
    for m in range(8):
        for i in range(3):
            np.add.at(f[i], nodes[m], -av * gi[m, i])
    return f.reshape(3, n, n, n)


def symbol(n: int) -> np.ndarray:
    """(n, n, n): eigenvalues of the constant-coefficient operator A_Delta
    (a = 1) on the Fourier modes (k, l, m)."""
    c = np.cos(2.0 * np.pi * np.arange(n) / n)
    kap = 2.0 - 2.0 * c
    mu = (4.0 + 2.0 * c) / 6.0
    return (kap[:, None, None] * mu[None, :, None] * mu[None, None, :]
            + mu[:, None, None] * kap[None, :, None] * mu[None, None, :]
            + mu[:, None, None] * mu[None, :, None] * kap[None, None, :])


def precond_apply(r: np.ndarray, a0: float, E: np.ndarray) -> np.ndarray:
    """z = (a0 A_Delta)^+ r by a 3D FFT; the constant mode is set to zero."""
    R = np.fft.fftn(r)
    with np.errstate(divide="ignore"):
        inv = 1.0 / (a0 * E)
    inv[0, 0, 0] = 0.0
    return np.fft.ifftn(R * inv).real


def pcg(A, f: np.ndarray, a0: float, tol: float, maxit: int):
    """Standard PCG (x0 = 0) on A x = f with z = B^+ r, stopping when the
    recursive ||r|| / ||f|| <= tol. Returns (x, iterations, true relative
    residual). A zero right-hand side returns x = 0 after 0 iterations."""
    n = f.shape[0]
    E = symbol(n)
    fv = f.ravel()
    fnorm = np.linalg.norm(fv)
    x = np.zeros_like(fv)
    if fnorm == 0.0:
        return x.reshape(f.shape), 0, 0.0
    r = fv.copy()
    z = precond_apply(r.reshape(f.shape), a0, E).ravel()
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) / fnorm <= tol:
            break
        z = precond_apply(r.reshape(f.shape), a0, E).ravel()
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x.reshape(f.shape), it, np.linalg.norm(fv - A @ x) / fnorm


def cell_gradients(x: np.ndarray) -> np.ndarray:
    """(8 quadrature points, 3 components, n^3 cells): grad x of the trilinear
    interpolant of the nodal field x (n, n, n) at the Gauss points of every cell."""
    n = x.shape[0]
    nodes = _corner_nodes(n)
    xv = np.asarray(x, dtype=np.float64).ravel()
    C = _corners()
    out = []
    for pt, _w in _quad_points():
        g = np.zeros((3, n ** 3))
        for m, c in enumerate(C):
            g += np.outer(_grad_phi(c, pt), xv[nodes[m]])
        out.append(g)
    return np.array(out)


def ahom(a: np.ndarray, x: np.ndarray):
    """Energy and flux forms of A_hom from the grid-unit correctors x
    (3, n, n, n) by cell quadrature:
      energy[i][j] = mean_e a_e int_e (e_i + grad x_i).(e_j + grad x_j),
      flux[i][j]   = mean_e a_e int_e (delta_ij + d_j x_i)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    av = a.ravel()
    G = [cell_gradients(x[i]) for i in range(3)]   # each (8, 3, n^3)
    w = np.array([wq for _p, wq in _quad_points()])
    energy = np.zeros((3, 3))
    flux = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            gi = G[i] + np.eye(3)[i][None, :, None]
            gj = G[j] + np.eye(3)[j][None, :, None]
            cell = np.einsum("q,qcn,qcn->n", w, gi, gj)
            energy[i, j] = np.sum(av * cell) / n ** 3
            fl = np.einsum("q,qn->n", w, G[i][:, j, :]) + (1.0 if i == j else 0.0)
            flux[i, j] = np.sum(av * fl) / n ** 3
    return energy, flux


def correctors(a: np.ndarray, tol: float = 1e-12, maxit: int = 5000):
    """Grid-unit correctors x (3, n, n, n), mean zero, with their PCG
    iteration counts (a0 = (max a + min a) / 2, Sec. 3.5)."""
    a = np.asarray(a, dtype=np.float64)
    A = assemble(a)
    f = rhs(a)
    a0 = 0.5 * (a.max() + a.min())
    xs, its = [], []
    for i in range(3):
        fi = f[i] - f[i].mean()
        x, it, _rel = pcg(A, fi, a0, tol, maxit)
        xs.append(x - x.mean())
        its.append(it)
    return np.array(xs), its


def homogenize(a: np.ndarray, h: float = 1.0, tol: float = 1e-12):
    """One realization end to end: (energy A_hom, flux A_hom, phi = h x,
    iterations)."""
    x, its = correctors(a, tol)
    energy, flux = ahom(a, x)
    return energy, flux, h * x, its
