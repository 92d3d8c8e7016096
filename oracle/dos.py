"""Spectral density of the stochastic stiffness matrix (Appendix, eqns. DOS
and DOS_gauss), FP64 -- TEST INFRASTRUCTURE ONLY.

phi_eta(t) = (1/m) sum_j g_eta(t - lambda_j), g_eta the Gaussian of width
eta, lambda_j the m = n^2 eigenvalues of the stiffness matrix A. For large m
the trace is estimated with probe vectors v: (1/m) tr g(t - A) ~ mean over
probes of v^T g(t - A) v / m, and g(t - A) is expanded in Chebyshev
polynomials of the scaled operator Ahat = (A - c I)/c, c = lmax/2, with
lmax >= lambda_max: v^T g(t - A) v = sum_k a_k(t) v^T T_k(Ahat) v, where
a_k(t) are the Chebyshev coefficients of x -> g_eta(t - c (1 + x)).

Here: the exact density from dense eigenvalues (small n), the Chebyshev
moments by the plain three-term recurrence, the coefficients a_k(t) by a
Chebyshev-Gauss rule, and the estimate from moments. Pins:
tests/test_oracle_dos.py (moments against dense eigendecompositions, the
estimate with all unit vectors as probes against the exact density, the
constant-coefficient spectrum against the symbols).
"""
from __future__ import annotations

import numpy as np


def gaussian(t, eta):
    return np.exp(-0.5 * (np.asarray(t) / eta) ** 2) / (np.sqrt(2.0 * np.pi) * eta)


def dos_exact(eigenvalues: np.ndarray, t: np.ndarray, eta: float) -> np.ndarray:
    """eqn. DOS_gauss from the eigenvalues."""
    lam = np.asarray(eigenvalues, dtype=np.float64)
    return gaussian(np.asarray(t)[:, None] - lam[None, :], eta).mean(axis=1)


def chebyshev_moments(A, v: np.ndarray, lmax: float, K: int) -> np.ndarray:
    """mu_k = v^T T_k(Ahat) v / m, k = 0 .. K-1, by w_0 = v, w_1 = Ahat v,
    w_{k+1} = 2 Ahat w_k - w_{k-1}."""
    c = 0.5 * lmax
    v = np.asarray(v, dtype=np.float64).ravel()
    m = v.size
    ahat = lambda w: (A @ w) / c - w
    mu = np.empty(K)
    w_prev, w = v, ahat(v)
    mu[0] = v @ v / m
    if K > 1:
        mu[1] = v @ w / m
    for k in range(2, K):
        w_prev, w = w, 2.0 * ahat(w) - w_prev
        mu[k] = v @ w / m
    return mu


def chebyshev_coefficients(t: np.ndarray, lmax: float, eta: float, K: int, Q: int) -> np.ndarray:
    """a_k(t), k < K, of x -> g_eta(t - c (1 + x)) on [-1, 1] by the
    Chebyshev-Gauss rule with Q nodes: a_k = (2 - [k == 0]) / Q *
    sum_q f(cos theta_q) cos(k theta_q), theta_q = pi (q + 1/2) / Q."""
    c = 0.5 * lmax
    th = np.pi * (np.arange(Q) + 0.5) / Q
    f = gaussian(np.asarray(t)[:, None] - c * (1.0 + np.cos(th))[None, :], eta)    # (nt, Q)
    cosk = np.cos(np.arange(K)[:, None] * th[None, :])                               # (K, Q)
    a = f @ cosk.T / Q
    a[:, 1:] *= 2.0
    return a                                                                         # (nt, K)


def dos_from_moments(mu: np.ndarray, t: np.ndarray, lmax: float, eta: float, Q: int) -> np.ndarray:
    """phi_eta(t) ~ sum_k a_k(t) mu_k (mu averaged over probes)."""
    mu = np.asarray(mu, dtype=np.float64)
    return chebyshev_coefficients(t, lmax, eta, mu.size, Q) @ mu


def philox_probes(count: int, seed: int) -> np.ndarray:
    """Probe vectors with entries +-1 drawn from Philox4x32-10 (Salmon et
    al., SC'11; the generator of lattice_sample), flat: entry i is -1 iff
    bit i mod 32 of word (i div 32) mod 4 of Philox4x32-10 with counter
    (i div 128 mod 2^32, i div 2^39, 0, 0x50524F42) and key (seed mod 2^32,
    seed div 2^32) is set. Reshape to (B, nv, n, n) as needed."""
    from .lattice_sample import philox4x32_10
    i = np.arange(int(count), dtype=np.uint64)
    t = i // np.uint64(128)
    words = np.stack(philox4x32_10(t & np.uint64(0xFFFFFFFF), t >> np.uint64(32), np.zeros_like(t),
                                   np.full_like(t, 0x50524F42), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    k = (i % np.uint64(128)).astype(np.int64)
    w = words[k // 32, np.arange(int(count))]
    bit = (w >> (k % 32).astype(np.uint32)) & np.uint32(1)
    return np.where(bit == 1, -1.0, 1.0)
