"""The lumped five-point scheme on the device against the oracle (through
the C ABI): operator, preconditioner, solves, gradient."""
import numpy as np
import pytest
import torch

from oracle import fd5
from oracle.pcg import precond_apply
from oracle import ahom as oa
from sampler import BooleanModel, batch

pytestmark = pytest.mark.gpu


def _rve():
    import paper_1903_12227_amd as rve
    return rve


def _fields(n, count, config, contrast=10.0):
    return batch(BooleanModel(L=n // 8, m0=8, a_in=contrast), config, count)


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def rel2(A, B):
    return float(np.max(np.abs(A - B)) / max(abs(B[0, 0]), abs(B[1, 1])))


@pytest.mark.parametrize("n", [64, 192])
def test_fd5_operator_matches_oracle(dev, n):
    rve = _rve()
    rng = np.random.default_rng(n + 1)
    a = np.stack([_fields(n, 1, 60)[0], rng.uniform(0.5, 3.0, (n, n))])
    u = rng.standard_normal((2, 2, n, n))
    out = rve.apply_operator(_to(a, dev), _to(u, dev), scheme=1).cpu().numpy()
    for b in range(2):
        A = fd5.assemble(a[b])
        for i in range(2):
            ref = (A @ u[b, i].ravel()).reshape(n, n)
            assert np.max(np.abs(out[b, i] - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-2)])
def test_fd5_preconditioner_matches_fft(dev, prec, tol):
    rve = _rve()
    n = 128
    rng = np.random.default_rng(prec)
    a = _fields(n, 2, 61)
    r = rng.standard_normal((2, 2, n, n))
    r -= r.mean(axis=(2, 3), keepdims=True)
    z = rve.apply_precond(_to(a, dev), _to(r, dev), prec, scheme=1).cpu().numpy()
    E = fd5.symbol(n)
    for b in range(2):
        a0 = oa.preconditioner_scale(a[b])
        for i in range(2):
            ref = precond_apply(r[b, i], a0, E)
            zc = z[b, i] - z[b, i].mean()
            assert np.linalg.norm(zc - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("prec,bound", [(0, 1e-10), (2, 1e-8)])
def test_fd5_solve_matches_oracle(dev, prec, bound):
    rve = _rve()
    n, B, tol, h = 128, 2, 1e-10, 1.0 / 8
    a = _fields(n, B, 62)
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=tol, prec=prec, scheme=1))
    assert res.code == 0
    A, F = res.ahom.cpu().numpy(), res.ahom_flux.cpu().numpy()
    x = res.phi.cpu().numpy() / h
    for b in range(B):
        ref = fd5.solve(a[b], tol=1e-13)
        assert rel2(A[b], ref.ahom) <= bound
        assert rel2(F[b], ref.ahom_flux) <= 1e-7
        K = fd5.assemble(a[b])
        for i, f in enumerate(fd5.rhs(a[b])):
            f = f - f.mean()
            assert np.linalg.norm(f.ravel() - K @ x[b, i].ravel()) / np.linalg.norm(f) <= 2 * tol


def test_fd5_constant_and_laminate(dev):
    rve = _rve()
    n = 64
    c = np.random.default_rng(3).uniform(1.0, 10.0, n)
    lam = np.repeat(c[:, None], n, axis=1)
    a = np.stack([np.full((n, n), 2.5), lam, lam.T.copy()])
    res = rve.solve_batch(_to(a, dev), 0.125, rve.Options(tol=1e-12, scheme=1))
    A = res.ahom.cpu().numpy()
    assert np.array_equal(A[0], 2.5 * np.eye(2))
    harm, arit = 1.0 / np.mean(1.0 / c), np.mean(c)
    assert abs(A[1, 0, 0] - harm) <= 1e-11 * harm and abs(A[1, 1, 1] - arit) <= 1e-11 * arit
    assert abs(A[2, 1, 1] - harm) <= 1e-11 * harm and abs(A[2, 0, 0] - arit) <= 1e-11 * arit


def test_fd5_gradient_matches_oracle(dev):
    rve = _rve()
    n, B, h = 64, 2, 1.0 / 8
    a = _fields(n, B, 63)
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=1e-12, scheme=1))
    G = np.random.default_rng(4).standard_normal((B, 2, 2))
    g, gin, _ = rve.grad(_to(a, dev), res.phi, h, _to(G, dev), a_in=10.0, scheme=1)
    g, gin = g.cpu().numpy(), gin.cpu().numpy()
    for b in range(B):
        ref = fd5.solve(a[b], tol=1e-13)
        d = fd5.dahom_da(a[b], ref.phi)
        gref = np.einsum("ij,ijxy->xy", G[b], d)
        assert np.max(np.abs(g[b] - gref)) <= 1e-9 * np.max(np.abs(gref))
        cref = float(np.sum(gref[a[b] == 10.0]))
        assert abs(gin[b] - cref) <= 1e-9 * abs(cref)
        assert abs(np.sum(a[b] * g[b]) - np.sum(G[b] * res.ahom.cpu().numpy()[b])) <= 1e-10
    # autograd carries the scheme to the backward pass
    at = _to(a, dev).requires_grad_(True)
    out = rve.ahom(at, h, rve.Options(tol=1e-12, scheme=1))
    out[:, 0, 1].sum().backward()
    G01 = np.zeros((B, 2, 2))
    G01[:, 0, 1] = 1.0
    for b in range(B):
        ref = fd5.solve(a[b], tol=1e-13)
        want = np.einsum("ij,ijxy->xy", G01[b], fd5.dahom_da(a[b], ref.phi))
        assert np.max(np.abs(at.grad[b].cpu().numpy() - want)) <= 1e-9 * np.max(np.abs(want))
