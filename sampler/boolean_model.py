"""Boolean model of overlapping axis-parallel square inclusions on a periodic grid.

The paper's ensemble (Sec. 2, eqns. Stoch-decomp, ahm_coef, Am_coef and
coef_diag; grid alignment in Sec. 3.1) places square cells with uniformly
random centres on the torus, wraps them periodically, and sets a two-valued
coefficient: one value on the covered set, another elsewhere. Centres sit on
grid points, so every square is a union of whole grid cells.

Two laws are provided:

* ``"poisson"`` -- a Poisson(ln 2 * L^2) number of squares of side ``side``
  grid cells (default ``m0``: unit squares). Each cell is then covered by a
  Poisson(ln 2) number of squares, so half the torus is covered on average.
* ``"paper"`` -- exactly L^2 squares of side 2*alpha*m0 cells (the paper's
  overlap factor alpha; alpha = 1/4 in most of its runs, Sec. 5).

Grid: ``n = m0 * L`` periodic nodes (and cells) per axis, h = 1/m0. Cell
(i, j) spans nodes i..i+1 along x1 and j..j+1 along x2 (mod n). Arrays are
indexed ``[i][j]`` with x2 contiguous (the paper's big-endian index map,
Sec. 3.2).

Every realization is keyed by (config, index) through
``SeedSequence([1903, 12227, config, index])`` so any subset of a batch can be
regenerated independently.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_ROOT = (1903, 12227)
_ORDER_KEY = 2**31 - 1


@dataclass(frozen=True)
class BooleanModel:
    L: int                 # RVE size (torus [0, L)^2)
    m0: int                # grid cells per unit length, h = 1/m0
    a_in: float = 10.0     # coefficient on the covered set
    a_bg: float = 1.0      # coefficient elsewhere
    law: str = "poisson"   # "poisson" or "paper"
    side: int | None = None  # square side in cells ("poisson" law); default m0
    alpha: float = 0.25    # overlap factor ("paper" law): side = 2*alpha*m0 cells

    @property
    def n(self) -> int:
        return self.m0 * self.L

    def square_side(self) -> int:
        if self.law == "paper":
            s = 2.0 * self.alpha * self.m0
            if abs(s - round(s)) > 1e-12 or round(s) < 1:
                raise ValueError("2*alpha*m0 must be a positive integer number of cells")
            return int(round(s))
        return self.m0 if self.side is None else int(self.side)


def _rng(config: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [SEED_ROOT[0], SEED_ROOT[1], int(config), int(index)])))


def covered_mask(model: BooleanModel, config: int, index: int) -> np.ndarray:
    """Boolean (n, n) mask of cells covered by at least one square."""
    n = model.n
    rng = _rng(config, index)
    if model.law == "poisson":
        k = int(rng.poisson(np.log(2.0) * model.L * model.L))
    elif model.law == "paper":
        k = model.L * model.L
    else:
        raise ValueError(f"unknown law {model.law!r}")
    side = model.square_side()
    centres = rng.integers(0, n, size=(k, 2))
    if k == 0:
        return np.zeros((n, n), dtype=bool)
    off = np.arange(side) - side // 2
    rows = (centres[:, 0, None] + off[None, :]) % n          # (k, side)
    cols = (centres[:, 1, None] + off[None, :]) % n          # (k, side)
    rr = np.broadcast_to(rows[:, :, None], (k, side, side)).ravel()
    cc = np.broadcast_to(cols[:, None, :], (k, side, side)).ravel()
    mask = np.zeros(n * n, dtype=bool)
    mask[rr * n + cc] = True
    return mask.reshape(n, n)


def realization(model: BooleanModel, config: int, index: int) -> np.ndarray:
    """Per-cell coefficient field, float64 (n, n), C-contiguous."""
    mask = covered_mask(model, config, index)
    return np.where(mask, float(model.a_in), float(model.a_bg)).astype(np.float64)


def batch(model: BooleanModel, config: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` realizations with indices start..start+count-1, shape (count, n, n)."""
    n = model.n
    out = np.empty((count, n, n), dtype=np.float64)
    for b in range(count):
        out[b] = realization(model, config, start + b)
    return out


def uneven_sizes(sizes, config: int, per_size: int) -> np.ndarray:
    """RVE size L of each realization of :func:`uneven_batch` (equal shares
    of ``sizes`` in a seeded random order)."""
    Ls = np.repeat(np.asarray(sizes, dtype=np.int64), per_size)
    order = _rng(config, _ORDER_KEY).permutation(len(Ls))
    return Ls[order]


def uneven_batch(sizes, m0: int, a_in: float, a_bg: float, config: int,
                 per_size: int):
    """Equal shares of several RVE sizes in a seeded random order.

    Returns a list of (L, field) pairs; realization ``r`` of the shuffled list
    uses key (config, r) whatever its size.
    """
    Ls = uneven_sizes(sizes, config, per_size)
    out = []
    for r, L in enumerate(Ls):
        model = BooleanModel(L=int(L), m0=m0, a_in=a_in, a_bg=a_bg)
        out.append((int(L), realization(model, config, r)))
    return out


@dataclass(frozen=True)
class BooleanModel3D:
    """The same model on the three-dimensional torus [0, L)^3 (the setting of
    Sec. 2 carries over unchanged to d = 3): a Poisson(ln 2 * L^3) number of
    cubes of side ``side`` cells (default m0: unit cubes) with centres uniform
    on the node lattice, so each cell is covered by a Poisson(ln 2) number of
    cubes and half the torus is covered on average. Cell (i, j, k) spans
    nodes i..i+1, j..j+1, k..k+1; arrays are [i][j][k] with x3 contiguous."""
    L: int
    m0: int
    a_in: float = 10.0
    a_bg: float = 1.0
    side: int | None = None

    @property
    def n(self) -> int:
        return self.m0 * self.L


_KEY_3D = 3


def covered_mask_3d(model: BooleanModel3D, config: int, index: int) -> np.ndarray:
    """Boolean (n, n, n) mask of cells covered by at least one cube."""
    n = model.n
    rng = _rng(config, index + (_KEY_3D << 40))
    k = int(rng.poisson(np.log(2.0) * model.L ** 3))
    side = model.m0 if model.side is None else int(model.side)
    centres = rng.integers(0, n, size=(k, 3))
    mask = np.zeros((n, n, n), dtype=bool)
    off = np.arange(side) - side // 2
    for c in centres:
        ii = (c[0] + off) % n
        jj = (c[1] + off) % n
        kk = (c[2] + off) % n
        mask[np.ix_(ii, jj, kk)] = True
    return mask


def realization_3d(model: BooleanModel3D, config: int, index: int) -> np.ndarray:
    """Per-cell coefficient field, float64 (n, n, n), C-contiguous."""
    return np.where(covered_mask_3d(model, config, index), float(model.a_in), float(model.a_bg)).astype(np.float64)


def batch_3d(model: BooleanModel3D, config: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` realizations with indices start..start+count-1, shape (count, n, n, n)."""
    n = model.n
    out = np.empty((count, n, n, n), dtype=np.float64)
    for b in range(count):
        out[b] = realization_3d(model, config, start + b)
    return out
