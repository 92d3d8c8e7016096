"""Plain preconditioned conjugate gradients, FP64 (oracle).

Sec. 3.5 (eqn. DD_Eqn, Lemma Cond_Number): the corrector systems are solved
by PCG with a constant-coefficient periodic Laplacian as preconditioner,
B = a0 * A_Delta, scaled by the mean of the coefficient's majorant and
minorant. The paper adds a small shift delta*I for stability; here delta -> 0
on the mean-zero subspace where the solution lives: B is applied as its
pseudo-inverse, which drops the constant Fourier mode (the right-hand sides
have zero mean).

This oracle applies B^+ by a 2D FFT, which diagonalises every periodic
circulant-of-circulants operator; the GPU path uses a different route.
"""
from __future__ import annotations

import numpy as np

from . import q1


def precond_apply(r: np.ndarray, a0: float, E: np.ndarray) -> np.ndarray:
    """z = (a0 * A_Delta)^+ r via FFT; the (0, 0) mode is set to zero."""
    R = np.fft.fft2(r)
    with np.errstate(divide="ignore"):
        inv = 1.0 / (a0 * E)
    inv[0, 0] = 0.0
    return np.fft.ifft2(R * inv).real


def pcg(A, f: np.ndarray, a0: float, tol: float, maxit: int, E: np.ndarray = None):
    """Standard PCG (x0 = 0) on A u = f with z = B^+ r.

    Stops when ||r||_2 / ||f||_2 <= tol (r is the recursively updated
    residual). An iteration is one product with A. Returns (u, iterations,
    true relative residual ||f - A u|| / ||f||). A zero right-hand side
    returns u = 0 after 0 iterations. E is the symbol of the constant
    coefficient operator B / a0 (default: the Q1 one).
    """
    n = f.shape[0]
    if E is None:
        E = q1.symbol(n)
    fv = f.ravel()
    fnorm = np.linalg.norm(fv)
    x = np.zeros_like(fv)
    if fnorm == 0.0:
        return x.reshape(n, n), 0, 0.0
    r = fv.copy()
    z = precond_apply(r.reshape(n, n), a0, E).ravel()
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
        z = precond_apply(r.reshape(n, n), a0, E).ravel()
        rz_new = r @ z
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    relres = np.linalg.norm(fv - A @ x) / fnorm
    return x.reshape(n, n), it, relres
