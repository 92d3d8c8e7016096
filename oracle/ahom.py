"""One realization end to end, FP64 (oracle): correctors, homogenized matrix
and its derivative with respect to the per-cell coefficient.

Corrector problem (Sec. 2, eqns. RHS_grad1 and scaled_setting; Sec. 4.3,
eqn. wg03): find phi_i in the Q1 space with
int grad psi . a (e_i + grad phi_i) = 0 for every test function psi, i.e.
A phi_i = f_i with the Galerkin stiffness A and right-hand side f_i.

Homogenized matrix (Sec. 4.1, eqns. A_hom_m and Ahom_m_entry; Sec. 4.3,
eqn. wg01), as an average over the torus:

* flux form   abar_ij = < a (delta_ij + d_j phi_i) >
                      = <a> delta_ij - phi_i . f_j / n^2
  because phi_i . f_j = -int a grad phi_i . e_j by the definition of f_j;
* energy form abar_ij = < (e_j + grad phi_j) . a (e_i + grad phi_i) >
                      = <a> delta_ij - (phi_i . f_j + phi_j . f_i) / n^2
                        + phi_j^T A phi_i / n^2,
  the symmetric expression used in the argument for wg02. Both equal the
  exact discrete value once the correctors solve their systems; the energy
  form's error is quadratic in the solver error.

Derivative (form of wg03 + wg01): the energy form is stationary in phi_i, so
d abar_ij / d a_e is its partial derivative at fixed phi, the cell integral
(1/n^2) int_e (e_i + grad phi_i) . (e_j + grad phi_j).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import q1
from .pcg import pcg


@dataclass
class Realization:
    phi: np.ndarray          # (2, n, n) correctors in grid units, mean zero
    ahom: np.ndarray         # (2, 2) energy form
    ahom_flux: np.ndarray    # (2, 2) flux form
    iters: tuple             # PCG iterations per direction
    relres: tuple            # true relative residuals per direction
    f: np.ndarray            # (2, n, n) right-hand sides


def preconditioner_scale(a: np.ndarray) -> float:
    """a0 = (a_max + a_min)/2: the mean of the coefficient's majorant and
    minorant (proof of Lemma Cond_Number)."""
    return 0.5 * (float(np.max(a)) + float(np.min(a)))


def ahom_flux(a, phis, fs) -> np.ndarray:
    n2 = a.size
    out = np.empty((2, 2))
    abar = float(np.sum(a)) / n2
    for i in range(2):
        for j in range(2):
            out[i, j] = abar * (i == j) - np.vdot(phis[i], fs[j]) / n2
    return out


def ahom_energy(A, a, phis, fs) -> np.ndarray:
    n2 = a.size
    Aphi = [A @ phis[i].ravel() for i in range(2)]
    out = np.empty((2, 2))
    abar = float(np.sum(a)) / n2
    for i in range(2):
        for j in range(i, 2):   # the expression is symmetric in (i, j)
            out[i, j] = (abar * (i == j)
                         - (np.vdot(phis[i], fs[j]) + np.vdot(phis[j], fs[i])) / n2
                         + np.vdot(phis[j].ravel(), Aphi[i]) / n2)
            out[j, i] = out[i, j]
    return out


def solve(a: np.ndarray, tol: float = 1e-13, maxit: int = 2000) -> Realization:
    """Correctors and homogenized matrix of one realization."""
    a = np.asarray(a, dtype=np.float64)
    A = q1.assemble(a)
    f1, f2 = q1.rhs(a)
    fs = []
    for f in (f1, f2):
        fs.append(f - f.mean())           # the systems are solvable on mean-zero data
    a0 = preconditioner_scale(a)
    phis, its, res = [], [], []
    for f in fs:
        u, it, rr = pcg(A, f, a0, tol, maxit)
        phis.append(u - u.mean())
        its.append(it)
        res.append(rr)
    phi = np.stack(phis)
    f = np.stack(fs)
    return Realization(phi=phi, ahom=ahom_energy(A, a, phis, fs),
                       ahom_flux=ahom_flux(a, phis, fs),
                       iters=tuple(its), relres=tuple(res), f=f)


def dahom_da(a: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """d abar_ij / d a_e for every cell e, shape (2, 2, n, n).

    A = sum_e a_e k_e and f_j = sum_e a_e b_j (element stiffness k_e and
    element right-hand-side vectors b_j from q1.element_matrices, embedded at
    the cell's four nodes). Differentiating the energy form at fixed phi, with
    corner values phi_{i,e}:
    n^2 d abar_ij/d a_e = delta_ij - (phi_{i,e}.b_j + phi_{j,e}.b_i)
                          + phi_{j,e}^T k_e phi_{i,e}.
    """
    a = np.asarray(a, dtype=np.float64)
    n2 = a.size
    ke, b1, b2 = q1.element_matrices()
    bs = (b1, b2)
    corners = [q1.cell_corners(phi[i]) for i in range(2)]   # (n, n, 4)
    out = np.empty((2, 2) + a.shape)
    for i in range(2):
        for j in range(2):
            quad = np.einsum("xyk,kl,xyl->xy", corners[j], ke, corners[i])
            lin = corners[i] @ bs[j] + corners[j] @ bs[i]
            out[i, j] = ((i == j) - lin + quad) / n2
    return out


def dahom_dcontrast(grad_a: np.ndarray, inclusion: np.ndarray) -> np.ndarray:
    """d abar_ij / d(contrast) when the inclusion cells carry a = contrast:
    the sum of d abar_ij/d a_e over those cells."""
    return np.einsum("ijxy,xy->ij", grad_a, inclusion.astype(np.float64))
