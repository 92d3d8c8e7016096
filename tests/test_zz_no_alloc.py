"""rve_grad_noalloc (the gradient call that allocates no device memory)
against rve_grad, through the C ABI: two calls in a row, the second with a
smaller input, each bit for bit equal to rve_grad's output (same kernels,
same summation order); and the size limit of its fixed scratch."""
import ctypes

import numpy as np
import pytest
import torch

from sampler import BooleanModel, covered_mask

pytestmark = pytest.mark.gpu


def _case(rve, dev, B, n, config):
    model = BooleanModel(L=n // 8, m0=8, a_in=10.0)
    masks = np.stack([covered_mask(model, config, b) for b in range(B)])
    a = torch.from_numpy(np.where(masks, 10.0, 1.0)).to(dev)
    res = rve.solve_batch(a, 0.125, rve.Options(tol=1e-10, prec=rve.MIX_BF16), want_flux=False)
    assert res.code == 0
    G = torch.from_numpy(np.random.default_rng(config).standard_normal((B, 2, 2))).to(dev)
    return a, res.phi, G, torch.from_numpy(masks).to(dev)


def test_noalloc_gradient_matches_workspace_gradient(dev):
    import paper_1903_12227_amd as rve
    ctx = rve.Context(0)
    for B, n, config in ((24, 256, 80), (5, 128, 81)):   # second call smaller
        a, phi, G, mask = _case(rve, dev, B, n, config)
        for kw in ({"mask": mask, "want_sum": True}, {"a_in": 10.0}):
            ref = rve.grad(a, phi, 0.125, G, ctx=ctx, **kw)
            got = rve.grad(a, phi, 0.125, G, ctx=ctx, noalloc=True, **kw)
            torch.cuda.synchronize()
            for x, y in zip(ref, got):
                assert (x is None) == (y is None)
                if x is not None:
                    assert torch.equal(x, y), (B, n, kw.keys())
    # beyond the fixed scratch: rejected on the host, nothing enqueued
    lib = ctx._lib
    fake = ctypes.c_void_p(1)
    out = ctypes.c_void_p(2)
    big_B = 4096   # 4096 realizations at n = 4096 need 128 MiB of partials
    rc = lib.rve_grad_noalloc(ctx.bind_stream(), big_B, 4096, fake, fake, 0.125, fake, out, fake, 10.0, fake, None, 0)
    assert rc == rve._native.EINVAL
    ctx.close()
