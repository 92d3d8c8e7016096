"""Every operator-apply shape of the fused PCG step (V columns per lane,
H rows per wave strip, D rows of loads in flight), forced through the C ABI,
against the oracles: the Q1 operator with FP64 and FP32 directions and with
the FP32 apply, and the five-point operator.

n = 256 admits all twelve shapes (the 64V x 4H tile divides the grid); two
realizations per solve. Bars: A_hom within 1e-10 (FP64 transforms) or 1e-8
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


def _shapes():
    out = []
    for v in (1, 2, 4):
        for hs in (16, 64):
            for d in (1, 2):
                out.append((v + 8 * (hs // 16) + 64 * (d - 1), f"V{v}-H{hs}-D{d}"))
    return out


@functools.lru_cache(maxsize=None)
def _case():
    a = batch(BooleanModel(L=N // 8, m0=8, a_in=10.0), 71, B)
    ref_q1 = [oa.solve(a[b], tol=1e-13).ahom for b in range(B)]
    ref_fd5 = [fd5.solve(a[b], tol=1e-13).ahom for b in range(B)]
    return a, ref_q1, ref_fd5


def _rel2(A, R):
    return float(np.max(np.abs(A - R)) / max(abs(R[0, 0]), abs(R[1, 1])))


# (transform precision, operator apply precision, scheme, A_hom bar)
CONFIGS = [(0, 0, 0, 1e-10), (2, 0, 0, 1e-8), (2, 1, 0, 1e-8), (0, 0, 1, 1e-10)]


@pytest.mark.parametrize("code,name", _shapes(), ids=[s[1] for s in _shapes()])
def test_every_shape_matches_oracle(dev, code, name):
    import paper_1903_12227_amd as rve
    a, ref_q1, ref_fd5 = _case()
    ad = torch.from_numpy(a).to(dev)
    for prec, sprec, scheme, bar in CONFIGS:
        ctx = rve.Context(0)
        ctx.set_autotune(False)
        ctx.force_variants(stencil=code)
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
