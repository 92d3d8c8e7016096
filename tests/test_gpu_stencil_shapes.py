"""Every operator-apply shape of the fused PCG step (V columns per lane,
H rows per wave strip, D rows of loads in flight), forced through the C ABI
for the apply and the residual update that recomputes A p, against the
oracles: the Q1 operator with FP64 and FP32 directions and with the FP32
apply, and the five-point operator; and apply and update in different
shapes.

n = 256 admits all eighteen shapes (the 64V x 4H tile divides the grid); two
realizations per solve, in FP64, BF16, scaled FP16 and FP32 transforms. Bars: A_hom within 1e-10 (FP64 transforms) or 1e-8
(BF16 transforms) of the oracle's, relative to max(|A_11|, |A_22|), and the
true residual of every corrector within twice the tolerance (the stopping
test is on the recursive residual, which tracks f - A x to FP64 rounding;
the FP32 apply replaces it by f - A x at each chunk start).
"""
import functools

import numpy as np
import pytest
import torch

from oracle import ahom as oa
from oracle import fd5
from oracle import q1
from sampler import BooleanModel, batch

pytestmark = pytest.mark.gpu

N, B, H_GRID, TOL = 256, 2, 1.0 / 8, 1e-10


def _code(v, hs, d):
    return v + 8 * (hs // 16) + (128 if d == 4 else 64 * (d - 1))


def _shapes():
    out = []
    for v in (1, 2, 4):
        for hs in (16, 64):
            for d in (1, 2, 4):
                out.append((_code(v, hs, d), f"V{v}-H{hs}-D{d}"))
    return out


@functools.lru_cache(maxsize=None)
def _case():
    a = batch(BooleanModel(L=N // 8, m0=8, a_in=10.0), 71, B)
    ref_q1 = [oa.solve(a[b], tol=1e-13).ahom for b in range(B)]
    ref_fd5 = [fd5.solve(a[b], tol=1e-13).ahom for b in range(B)]
    return a, ref_q1, ref_fd5


def _rel2(A, R):
    return float(np.max(np.abs(A - R)) / max(abs(R[0, 0]), abs(R[1, 1])))


# (transform precision, operator apply precision, scheme, A_hom bar); the
# scaled FP16 and the FP32 transforms give the residual update other
# instantiations (GEMM-copy types), so every shape runs with each
CONFIGS = [(0, 0, 0, 1e-10), (2, 0, 0, 1e-8), (3, 0, 0, 1e-8), (1, 0, 0, 1e-8), (2, 1, 0, 1e-8),
           (0, 0, 1, 1e-10)]


def _check(dev, a, ref_q1, ref_fd5, name, stencil, update, configs):
    import paper_1903_12227_amd as rve
    ad = torch.from_numpy(a).to(dev)
    for prec, sprec, scheme, bar in configs:
        ctx = rve.Context(0)
        ctx.set_autotune(False)
        ctx.force_variants(stencil=stencil, update=update)
        res = rve.solve_batch(ad, H_GRID, rve.Options(tol=TOL, prec=prec, stencil_prec=sprec, scheme=scheme),
                              ctx=ctx)
        ctx.close()
        assert res.code == 0, (name, prec, sprec, scheme)
        A = res.ahom.cpu().numpy()
        x = res.phi.cpu().numpy() / H_GRID
        ref = ref_fd5 if scheme else ref_q1
        mod = fd5 if scheme else q1
        for b in range(B):
            assert _rel2(A[b], ref[b]) <= bar, (name, prec, sprec, scheme, b)
            K = mod.assemble(a[b])
            for i, f in enumerate(mod.rhs(a[b])):
                f = f - f.mean()
                rr = np.linalg.norm(f.ravel() - K @ x[b, i].ravel()) / np.linalg.norm(f)
                assert rr <= 2 * TOL, (name, prec, sprec, scheme, b, i, rr)


@pytest.mark.parametrize("code,name", _shapes(), ids=[s[1] for s in _shapes()])
def test_every_shape_matches_oracle(dev, code, name):
    a, ref_q1, ref_fd5 = _case()
    _check(dev, a, ref_q1, ref_fd5, name, code, -1, CONFIGS)


# apply and residual update in different shapes (the update's r.r partials
# then number its own tiles); the FP32 apply has no recomputing update
MIXED = [((4, 64, 4), (1, 16, 2)), ((1, 16, 2), (4, 64, 4)), ((2, 16, 1), (1, 64, 4))]


@pytest.mark.parametrize("pair", MIXED, ids=[f"apply{p[0]}-update{p[1]}" for p in MIXED])
def test_apply_and_update_in_different_shapes(dev, pair):
    a, ref_q1, ref_fd5 = _case()
    _check(dev, a, ref_q1, ref_fd5, str(pair), _code(*pair[0]), _code(*pair[1]),
           [c for c in CONFIGS if c[1] == 0])
