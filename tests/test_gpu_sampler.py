"""The on-device sampler and the checkpointed ensemble runner against the
oracle (through the C ABI)."""
import math

import numpy as np
import pytest
import torch

from oracle import ahom as oa
from oracle import lattice_sample as ls

pytestmark = pytest.mark.gpu


def _rve():
    import paper_1903_12227_amd as rve
    return rve


def _thr(side):
    return int(round(2**32 * -math.expm1(-math.log(2.0) / side ** 2)))


@pytest.mark.parametrize("n,side,seed,first,B,thr", [
    (64, 8, 1903, 0, 3, None),
    (128, 16, 2**40 + 5, 2**32 - 1, 2, None),     # realization index crosses 2^32
    (192, 6, 7, 12345, 2, None),
    (64, 8, 3, 0, 1, 0),                           # no centres: background only
    (64, 4, 3, 0, 1, 2**32 - 1),                   # almost every site a centre
])
def test_device_fields_equal_oracle(dev, n, side, seed, first, B, thr):
    rve = _rve()
    thr = _thr(side) if thr is None else thr
    a = rve.sample_lattice(B, n, side, seed=seed, first=first, occ_threshold=thr, a_in=10.0, a_bg=1.0,
                           device=dev).cpu().numpy()
    for b in range(B):
        want = ls.field(n, side, seed, first + b, thr, 10.0, 1.0)
        assert np.array_equal(a[b], want), (b, int((a[b] != want).sum()))


def test_sampled_fields_solve_to_oracle(dev):
    rve = _rve()
    n, side, B = 128, 8, 2
    a = rve.sample_lattice(B, n, side, seed=99, first=40, occ_threshold=_thr(side), a_in=10.0, device=dev)
    res = rve.solve_batch(a, 1.0 / 8, rve.Options(tol=1e-10, prec=2), want_phi=False)
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    for b in range(B):
        ref = oa.solve(ls.field(n, side, 99, 40 + b, _thr(side), 10.0, 1.0), tol=1e-13).ahom
        assert np.max(np.abs(A[b] - ref)) <= 1e-8 * max(abs(ref[0, 0]), abs(ref[1, 1]))


def test_ensemble_resume_equals_one_run(dev, tmp_path):
    from paper_1903_12227_amd import ensemble
    kw = dict(batch=16, seed=5, device=dev)
    full = ensemble.run_ensemble(8, 8, 10.0, 40, **kw)
    ck = str(tmp_path / "ens.npz")
    part = ensemble.run_ensemble(8, 8, 10.0, 40, checkpoint=ck, max_batches=1, **kw)
    assert part["done"] == 16 and not part["complete"]
    rest = ensemble.run_ensemble(8, 8, 10.0, 40, checkpoint=ck, **kw)
    assert rest["complete"] and np.array_equal(rest["ahom"], full["ahom"])
    for k in ("mean", "var", "quartic"):
        assert np.array_equal(rest["stats"][k], full["stats"][k])
    # a different batch size samples the same realizations
    other = ensemble.run_ensemble(8, 8, 10.0, 40, batch=7, seed=5, device=dev)
    assert np.max(np.abs(other["ahom"] - full["ahom"])) <= 1e-9


@pytest.mark.parametrize("n,side,K,seed,first,B", [
    (64, 2, 256, 1903, 0, 3),            # L = 16 at m0 = 4: the paper's alpha = 1/4
    (128, 2, 1024, 2**40 + 7, 2**32 - 1, 2),   # realization index crosses 2^32
    (192, 6, 50, 5, 77, 2),
    (64, 2, 0, 3, 0, 1),                 # no squares: background only
])
def test_device_fixed_count_fields_equal_oracle(dev, n, side, K, seed, first, B):
    rve = _rve()
    a = rve.sample_fixed_count(B, n, side, K, seed=seed, first=first, a_in=1.0, a_bg=0.4, device=dev).cpu().numpy()
    for b in range(B):
        want = ls.fixed_count_field(n, side, K, seed, first + b, 1.0, 0.4)
        assert np.array_equal(a[b], want), (b, int((a[b] != want).sum()))


def test_fixed_count_ensemble_with_the_five_point_scheme(dev, tmp_path):
    # the paper's ensemble (exactly L^2 squares, alpha = 1/4, lambda = 0.4,
    # m0 = 4) with the lumped scheme, resumed from a checkpoint: the same
    # A_hom as one run, and sampled items against the oracle's five-point solve
    from oracle import fd5
    from paper_1903_12227_amd import ensemble
    kw = dict(batch=32, seed=11, device=dev, law="fixed", alpha=0.25, a_bg=0.4, scheme=1, tol=1e-10)
    full = ensemble.run_ensemble(16, 4, 1.0, 80, **kw)
    ck = str(tmp_path / "ensf.npz")
    ensemble.run_ensemble(16, 4, 1.0, 80, checkpoint=ck, max_batches=1, **kw)
    rest = ensemble.run_ensemble(16, 4, 1.0, 80, checkpoint=ck, **kw)
    assert rest["complete"] and np.array_equal(rest["ahom"], full["ahom"])
    for r in (0, 79):
        f = ls.fixed_count_field(64, 2, 256, 11, r, 1.0, 0.4)
        ref = fd5.solve(f, tol=1e-13).ahom
        assert np.max(np.abs(full["ahom"][r] - ref)) <= 1e-8 * max(abs(ref[0, 0]), abs(ref[1, 1]))
