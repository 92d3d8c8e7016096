"""Seeded input generator: determinism, values and the coverage law."""
import numpy as np

from sampler import BooleanModel, batch, realization, uneven_batch
from sampler.boolean_model import covered_mask


def test_deterministic_and_keyed():
    m = BooleanModel(L=8, m0=8, a_in=10.0)
    a = realization(m, 1, 5)
    assert a.shape == (64, 64) and a.dtype == np.float64 and a.flags.c_contiguous
    assert np.array_equal(a, realization(m, 1, 5))
    assert not np.array_equal(a, realization(m, 1, 6))
    assert not np.array_equal(a, realization(m, 2, 5))
    b = batch(m, 1, 3, start=4)
    assert np.array_equal(b[1], a)


def test_two_values_and_half_coverage():
    # Poisson(ln 2 L^2) unit squares cover each cell with probability 1/2
    m = BooleanModel(L=16, m0=4, a_in=7.0, a_bg=1.5)
    fr = []
    for k in range(20):
        a = realization(m, 3, k)
        assert set(np.unique(a)) <= {1.5, 7.0}
        fr.append(np.mean(a == 7.0))
    assert abs(np.mean(fr) - 0.5) < 0.03


def test_paper_law_square_size():
    m = BooleanModel(L=4, m0=4, law="paper", alpha=0.25)   # squares of 2x2 cells
    assert m.square_side() == 2
    mask = covered_mask(m, 0, 0)
    assert mask.shape == (16, 16) and 0 < mask.sum() <= 16 * 4


def test_uneven_batch_shares():
    items = uneven_batch([8, 16], m0=4, a_in=10.0, a_bg=1.0, config=2, per_size=3)
    Ls = [L for L, _ in items]
    assert sorted(Ls) == [8, 8, 8, 16, 16, 16]
    for L, a in items:
        assert a.shape == (4 * L, 4 * L)


def test_3d_model_deterministic_half_coverage_and_cube_size():
    from sampler import BooleanModel3D, batch_3d, realization_3d
    m = BooleanModel3D(L=4, m0=8, a_in=7.0)
    a = batch_3d(m, 5, 3)
    assert a.shape == (3, 32, 32, 32) and a.dtype == np.float64 and a.flags.c_contiguous
    np.testing.assert_array_equal(a[1], realization_3d(m, 5, 1))
    assert set(np.unique(a)) <= {1.0, 7.0}
    # each cell covered by Poisson(ln 2) cubes: half the torus on average
    cover = np.mean([(realization_3d(BooleanModel3D(L=4, m0=2), 6, r) == 10.0).mean() for r in range(40)])
    assert abs(cover - 0.5) < 0.04
    # a realization with a single cube of side 3 covers a 3 x 3 x 3 block
    one = [realization_3d(BooleanModel3D(L=1, m0=8, side=3), 7, r) for r in range(20)]
    counts = sorted({int((f == 10.0).sum()) for f in one} - {0})
    assert counts[0] == 27
    f = next(f for f in one if (f == 10.0).sum() == 27)
    idx = np.argwhere(f == 10.0)
    assert all(len(np.unique(idx[:, d])) == 3 for d in range(3))
