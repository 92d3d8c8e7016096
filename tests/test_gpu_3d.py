"""Parity of the three-dimensional HIP path (through the C ABI) with the
three-dimensional oracle (oracle/q1_3d.py).

Tolerances: A_hom (relative to max |A_ii|) 1e-10 with FP64 transforms and
1e-8 with FP32 / BF16 transforms; the operator apply element by element at
1e-13 of its largest value (FP64 sums of 21 terms); the preconditioner at
the input rounding of its transform precision. n is a multiple of 64, so
every grid spans whole tiles (64 x3-columns, 4 x2-rows, 16 x1-planes); a
ragged tail cannot occur.
"""
import numpy as np
import pytest
import torch

from oracle import ahom as oa2
from oracle import q1_3d as q3
from sampler import BooleanModel, BooleanModel3D, batch, batch_3d

pytestmark = pytest.mark.gpu


def _rve():
    import paper_1903_12227_amd as rve
    return rve


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def rel3(A, B):
    return float(np.max(np.abs(A - B)) / np.max(np.abs(np.diag(B))))


def _fields(n, count, config, contrast=10.0):
    return batch_3d(BooleanModel3D(L=n // 8, m0=8, a_in=contrast), config, count)


def test_operator_matches_oracle_spmv(dev):
    rve = _rve()
    n = 64
    rng = np.random.default_rng(3064)
    a = np.stack([_fields(n, 1, 300)[0], rng.uniform(0.5, 3.0, (n, n, n))])
    u = rng.standard_normal((2, n, n, n))
    out = rve.apply_operator_3d(_to(a, dev), _to(u, dev)).cpu().numpy()
    for b in range(2):
        ref = (q3.assemble(a[b]) @ u[b].ravel()).reshape(n, n, n)
        assert np.max(np.abs(out[b] - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5), (2, 3e-2), (3, 4e-3)])
def test_preconditioner_matches_oracle_fft(dev, prec, tol):
    rve = _rve()
    n = 64
    rng = np.random.default_rng(3100 + prec)
    a = _fields(n, 2, 301)
    r = rng.standard_normal((2, 3, n, n, n))
    r -= r.mean(axis=(2, 3, 4), keepdims=True)
    z = rve.apply_precond_3d(_to(a, dev), _to(r, dev), prec).cpu().numpy()
    E = q3.symbol(n)
    for b in range(2):
        a0 = 0.5 * (a[b].max() + a[b].min())
        for i in range(3):
            ref = q3.precond_apply(r[b, i], a0, E)
            zc = z[b, i] - z[b, i].mean()        # a constant is in the operator's kernel
            assert np.linalg.norm(zc - ref) <= tol * np.linalg.norm(ref)


def test_preconditioner_on_a_single_mode(dev):
    # r = one real Fourier mode: z = r / (a0 E(k, l, m)) exactly (FP64)
    rve = _rve()
    n = 64
    a = np.full((1, n, n, n), 2.0)
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    kk = (3, 5, 1)
    r = np.cos(2 * np.pi * (kk[0] * i + kk[1] * j + kk[2] * k) / n)
    c = np.cos(2 * np.pi * np.array(kk) / n)
    kap, mu = 2 - 2 * c, (4 + 2 * c) / 6
    E = kap[0] * mu[1] * mu[2] + mu[0] * kap[1] * mu[2] + mu[0] * mu[1] * kap[2]
    rr = np.stack([r, 2 * r, -r])[None]
    z = rve.apply_precond_3d(_to(a, dev), _to(rr, dev), 0).cpu().numpy()
    np.testing.assert_allclose(z[0], rr[0] / (2.0 * E), atol=1e-13)


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 1e-8), (3, 1e-8)])
def test_solve_matches_oracle(dev, prec, tol):
    rve = _rve()
    n = 64
    a = _fields(n, 2, 302)
    res = rve.solve_batch_3d(_to(a, dev), h=0.125, opts=rve.Options(tol=1e-10, prec=prec))
    E = res.ahom.cpu().numpy()
    F = res.ahom_flux.cpu().numpy()
    phi = res.phi.cpu().numpy()
    its = res.iters.cpu().numpy()
    assert (res.status.cpu().numpy() == 0).all()
    for b in range(2):
        Eo, Fo, phio, itso = q3.homogenize(a[b], h=0.125, tol=1e-12)
        assert rel3(E[b], Eo) <= tol
        assert rel3(F[b], Fo) <= 1e-6          # the flux form's error is linear in the solver error
        assert np.max(np.abs(phi[b] - phio)) <= 1e-6 * np.max(np.abs(phio))
    if prec == 0:
        # same stopping test as the oracle's PCG at the same tolerance
        _x, itso = q3.correctors(a[0], tol=1e-10)
        assert np.all(np.abs(its[0] - np.array(itso)) <= 1)


def test_true_residual_meets_tolerance(dev):
    rve = _rve()
    n = 64
    a = _fields(n, 1, 303)
    for prec in (0, 1, 2, 3):
        res = rve.solve_batch_3d(_to(a, dev), h=1.0, opts=rve.Options(tol=1e-10, prec=prec))
        x = res.phi.cpu().numpy()[0]
        A = q3.assemble(a[0])
        f = q3.rhs(a[0])
        for i in range(3):
            fi = (f[i] - f[i].mean()).ravel()
            assert np.linalg.norm(fi - A @ x[i].ravel()) <= 2e-10 * np.linalg.norm(fi)


def test_constant_field_and_laminate(dev):
    rve = _rve()
    n = 64
    c = np.where(np.arange(n) % 8 < 4, 1.0, 10.0) * (1.0 + 0.1 * (np.arange(n) % 3))
    lam = np.broadcast_to(c[None, :, None], (n, n, n))      # layers normal to x2
    a = np.stack([np.full((n, n, n), 3.0), lam])
    res = rve.solve_batch_3d(_to(a, dev), opts=rve.Options(tol=1e-12))
    E = res.ahom.cpu().numpy()
    np.testing.assert_allclose(E[0], 3.0 * np.eye(3), atol=1e-14)
    assert (res.iters.cpu().numpy()[0] == 0).all()
    want = np.eye(3) * c.mean()
    want[1, 1] = 1.0 / np.mean(1.0 / c)
    np.testing.assert_allclose(E[1], want, rtol=1e-10, atol=1e-12)


def test_field_constant_along_x3_matches_the_2d_path(dev):
    # a 3D field constant along x3: the 2 x 2 block is the 2D A_hom of the
    # same cross-section (2D GPU path and 2D oracle), A_33 = <a>
    rve = _rve()
    n = 64
    a2 = batch(BooleanModel(L=8, m0=8, a_in=10.0), 304, 1)
    a3 = np.repeat(a2[:, :, :, None], n, axis=3)
    E3 = rve.solve_batch_3d(_to(a3, dev), opts=rve.Options(tol=1e-11)).ahom.cpu().numpy()[0]
    E2 = rve.solve_batch(_to(a2, dev), opts=rve.Options(tol=1e-11)).ahom.cpu().numpy()[0]
    Eo = oa2.solve(a2[0], tol=1e-12).ahom
    assert rel3(E3[:2, :2], Eo) <= 1e-10 and rel3(E2, Eo) <= 1e-10
    assert abs(E3[2, 2] - a2.mean()) <= 1e-12 * a2.mean()
    assert np.max(np.abs(E3[:2, 2])) <= 1e-12


def test_axis_permutation(dev):
    rve = _rve()
    n = 64
    a = _fields(n, 1, 305)
    perm = (1, 2, 0)
    both = np.stack([a[0], np.transpose(a[0], perm)])
    E = rve.solve_batch_3d(_to(both, dev), opts=rve.Options(tol=1e-11)).ahom.cpu().numpy()
    assert rel3(E[1], E[0][np.ix_(perm, perm)]) <= 1e-9


def test_graph_replay_matches_eager_and_is_reproducible(dev):
    rve = _rve()
    n = 64
    a = _to(_fields(n, 3, 306), dev)
    ctx = rve.Context(0)
    out = []
    for graphs in (True, False, True):
        ctx.set_graphs(graphs)
        r = rve.solve_batch_3d(a, opts=rve.Options(prec=2), ctx=ctx)
        out.append((r.ahom.cpu().numpy(), r.iters.cpu().numpy(), r.phi.cpu().numpy()))
    for o in out[1:]:
        assert np.array_equal(o[0], out[0][0]) and np.array_equal(o[1], out[0][1])
        assert np.array_equal(o[2], out[0][2])
    ctx.close()


def test_status_codes(dev):
    rve = _rve()
    n = 64
    a = _fields(n, 3, 307)
    a[1, 3, 4, 5] = -1.0                       # invalid cell
    res = rve.solve_batch_3d(_to(a, dev), opts=rve.Options(maxit=5), want_phi=False)
    st = res.status.cpu().numpy()
    assert st[1] == rve._native.EINVAL and res.code == rve._native.EINVAL
    assert st[0] == rve._native.NOT_CONVERGED and st[2] == rve._native.NOT_CONVERGED


@pytest.mark.parametrize("prec", [0, 2])
def test_larger_grid_properties(dev, prec):
    # n = 128 (L = 16, 2.1 M nodes per system), two realizations: symmetric,
    # energy = flux to solver accuracy, Voigt / Reuss bounds, true residual
    rve = _rve()
    n = 128
    a = _fields(n, 2, 308)
    res = rve.solve_batch_3d(_to(a, dev), opts=rve.Options(tol=1e-10, prec=prec))
    E = res.ahom.cpu().numpy()
    F = res.ahom_flux.cpu().numpy()
    assert (res.status.cpu().numpy() == 0).all()
    for b in range(2):
        assert np.max(np.abs(E[b] - E[b].T)) == 0.0
        assert rel3(F[b], E[b]) <= 1e-6
        w = np.linalg.eigvalsh(E[b])
        assert w[0] >= 1.0 / np.mean(1.0 / a[b]) and w[-1] <= a[b].mean()
    # the true residual of one system, with the device operator (checked
    # against the oracle above) and the oracle's right-hand side
    x = res.phi[0, 0:1].contiguous()
    Ax = rve.apply_operator_3d(_to(a[0:1], dev), x).cpu().numpy()[0]
    f = q3.rhs(a[0])[0]
    f -= f.mean()
    assert np.linalg.norm(f - Ax) <= 2e-10 * np.linalg.norm(f)
