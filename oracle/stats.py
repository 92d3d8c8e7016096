"""Ensemble statistics of the per-realization homogenized matrices (oracle).

Input: an (N, 2, 2) array of abar^(n), n = 1..N, all at the same RVE size L.
"""
from __future__ import annotations

import numpy as np


def empirical_mean(A: np.ndarray) -> np.ndarray:
    """Empirical average (1/N) sum_n abar^(n) (Sec. 4.2, eqn. A_hom_Empir)."""
    return np.asarray(A, dtype=np.float64).mean(axis=0)


def centred_variance(A: np.ndarray) -> np.ndarray:
    """Per-entry variance with the 1/(N-1) normalisation used for the
    covariances in Sec. 4.3."""
    A = np.asarray(A, dtype=np.float64)
    d = A - A.mean(axis=0)
    return (d * d).sum(axis=0) / (A.shape[0] - 1)


def std_uncentred(A: np.ndarray):
    """The two monitored standard deviations (Sec. 5, eqns. Var1 and Var2),
    exactly as written there: uncentred, normalised by 1/N.
    Returns ((1/N) sum a12^2)^(1/2) and ((1/N) sum (a11 - a22)^2)^(1/2)."""
    A = np.asarray(A, dtype=np.float64)
    s12 = np.sqrt(np.mean(A[:, 0, 1] ** 2))
    sdd = np.sqrt(np.mean((A[:, 0, 0] - A[:, 1, 1]) ** 2))
    return s12, sdd


def quartic(A: np.ndarray, L: float, d: int = 2) -> np.ndarray:
    """Computable quartic tensor (Sec. 5.3, eqn. quartic):
    Q = L^d/(N-1) sum_n (abar^(n) - mean)^{(x)2}, with the tensor square taken
    as the Kronecker product of 2x2 matrices (Definition Kron), giving a 4x4
    matrix q with q[(i,k),(j,l)] = L^d cov(abar_ij, abar_kl)."""
    A = np.asarray(A, dtype=np.float64)
    D = A - A.mean(axis=0)
    Q = np.zeros((4, 4))
    for Dn in D:
        Q += np.kron(Dn, Dn)
    return (float(L) ** d) * Q / (A.shape[0] - 1)
