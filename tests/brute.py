"""Brute-force reference constructions used only by the tests to pin the
oracle: dense element-loop assembly with Gauss quadrature of the bilinear
basis, written independently of the oracle's Kronecker-sum assembly."""
from __future__ import annotations

import numpy as np

_G = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])   # 2-point Gauss on [0, 1]


def _basis_grads(s, t):
    """Gradients of the 4 bilinear shape functions at (s, t) of the unit cell,
    local node (alpha, beta) -> index 2*alpha + beta, alpha along x1."""
    out = np.zeros((4, 2))
    for al in (0, 1):
        for be in (0, 1):
            fs = s if al else 1 - s
            ft = t if be else 1 - t
            ds = 1.0 if al else -1.0
            dt = 1.0 if be else -1.0
            out[2 * al + be] = (ds * ft, fs * dt)
    return out


def element_data():
    K = np.zeros((4, 4))
    b = np.zeros((2, 4))
    for s in _G:
        for t in _G:
            g = _basis_grads(s, t)
            K += 0.25 * g @ g.T
            b[0] -= 0.25 * g[:, 0]
            b[1] -= 0.25 * g[:, 1]
    return K, b


def dense_system(a):
    """Dense stiffness matrix and right-hand sides by looping over cells."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    K, b = element_data()
    A = np.zeros((n * n, n * n))
    f = np.zeros((2, n * n))
    for i in range(n):
        for j in range(n):
            nodes = [((i + al) % n) * n + (j + be) % n for al in (0, 1) for be in (0, 1)]
            for x in range(4):
                f[0, nodes[x]] += a[i, j] * b[0, x]
                f[1, nodes[x]] += a[i, j] * b[1, x]
                for y in range(4):
                    A[nodes[x], nodes[y]] += a[i, j] * K[x, y]
    return A, f


def direct_ahom(a):
    """A_hom (energy form) from a dense pseudo-inverse solve."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    A, f = dense_system(a)
    Ap = np.linalg.pinv(A, rcond=1e-12, hermitian=True)
    phis = [Ap @ f[i] for i in range(2)]
    out = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            out[i, j] = (a.sum() * (i == j) - phis[i] @ f[j] - phis[j] @ f[i]
                         + phis[j] @ A @ phis[i]) / (n * n)
    return out, phis
