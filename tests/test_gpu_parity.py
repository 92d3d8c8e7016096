"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (relative error of a 2x2 result = max |dA_ij| / max(|A11|, |A22|)):
FP64 path 1e-10 and mixed-precision path 1e-8 on the energy-form A_hom; the
linear maps alone are compared element by element (stencil: FP64 rounding of
a 9-term sum; transform GEMMs: the input rounding of their precision).
"""
import numpy as np
import pytest
import torch

from oracle import ahom as oa
from oracle import q1
from oracle import stats as ost
from oracle.pcg import precond_apply
from sampler import BooleanModel, batch, realization

pytestmark = pytest.mark.gpu


def _rve():
    import paper_1903_12227_amd as rve
    return rve


def rel2(A, B):
    return float(np.max(np.abs(A - B)) / max(abs(B[0, 0]), abs(B[1, 1])))


def _fields(n, count, config, contrast=10.0):
    return batch(BooleanModel(L=n // 8, m0=8, a_in=contrast), config, count)


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("n", [64, 192])
def test_operator_matches_oracle_spmv(dev, n):
    rve = _rve()
    rng = np.random.default_rng(n)
    a = np.stack([_fields(n, 1, 50)[0], rng.uniform(0.5, 3.0, (n, n))])
    u = rng.standard_normal((2, 2, n, n))
    out = rve.apply_operator(_to(a, dev), _to(u, dev)).cpu().numpy()
    for b in range(2):
        A = q1.assemble(a[b])
        for i in range(2):
            ref = (A @ u[b, i].ravel()).reshape(n, n)
            assert np.max(np.abs(out[b, i] - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-2), (3, 3e-3)])
@pytest.mark.parametrize("n", [64, 128])
def test_preconditioner_matches_oracle_fft(dev, n, prec, tol):
    rve = _rve()
    rng = np.random.default_rng(n + prec)
    a = _fields(n, 2, 51)
    r = rng.standard_normal((2, 2, n, n))
    r -= r.mean(axis=(2, 3), keepdims=True)
    z = rve.apply_precond(_to(a, dev), _to(r, dev), prec).cpu().numpy()
    E = q1.symbol(n)
    for b in range(2):
        a0 = oa.preconditioner_scale(a[b])
        for i in range(2):
            ref = precond_apply(r[b, i], a0, E)
            zc = z[b, i] - z[b, i].mean()        # a constant is in the operator's kernel
            assert np.linalg.norm(zc - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("n", [256, 512])
def test_bf16_transform_variants_match_oracle_fft(dev, n, variant):
    # 128-row tiles (1; 3 with the operands loaded straight into LDS; 4 with
    # 256 x 128 tiles for three of the four transforms, 5 with 256 x 256 for
    # all four, 6 the same from 8 waves) and the even/odd-folded
    # tiles (2, half the MFMA work, one more BF16 rounding of the folded
    # input) against the FFT apply
    rve = _rve()
    rng = np.random.default_rng(n + variant)
    a = _fields(n, 2, 52)
    r = rng.standard_normal((2, 2, n, n))
    r -= r.mean(axis=(2, 3), keepdims=True)
    ctx = rve.Context(0)
    ctx.force_variants(gemm=variant)
    z = rve.apply_precond(_to(a, dev), _to(r, dev), 2, ctx=ctx).cpu().numpy()
    E = q1.symbol(n)
    for b in range(2):
        a0 = oa.preconditioner_scale(a[b])
        for i in range(2):
            ref = precond_apply(r[b, i], a0, E)
            zc = z[b, i] - z[b, i].mean()
            assert np.linalg.norm(zc - ref) <= 3e-2 * np.linalg.norm(ref)


def test_folded_transform_solve_matches_oracle(dev):
    rve = _rve()
    n, B, tol, h = 256, 2, 1e-10, 1.0 / 8
    a = _fields(n, B, 53)
    ctx = rve.Context(0)
    ctx.force_variants(gemm=2)
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=tol, prec=2), ctx=ctx)
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    x = res.phi.cpu().numpy() / h
    for b in range(B):
        assert rel2(A[b], oa.solve(a[b], tol=1e-13).ahom) <= 1e-8
        K = q1.assemble(a[b])
        for i, f in enumerate(q1.rhs(a[b])):
            f = f - f.mean()
            assert np.linalg.norm(f.ravel() - K @ x[b, i].ravel()) / np.linalg.norm(f) <= 2.0 * tol


@pytest.mark.parametrize("n,B", [(64, 4), (128, 3)])
def test_solve_fp64_matches_oracle(dev, n, B):
    rve = _rve()
    a = _fields(n, B, 1)
    h = 1.0 / 8
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=1e-10))
    assert res.code == 0 and bool(torch.all(res.status == 0))
    A = res.ahom.cpu().numpy()
    F = res.ahom_flux.cpu().numpy()
    phi = res.phi.cpu().numpy() / h
    its = res.iters.cpu().numpy()
    for b in range(B):
        ref = oa.solve(a[b], tol=1e-13)
        assert rel2(A[b], ref.ahom) <= 1e-10
        assert rel2(F[b], ref.ahom_flux) <= 1e-8
        assert A[b, 0, 1] == A[b, 1, 0]
        for i in range(2):
            assert np.max(np.abs(phi[b, i] - ref.phi[i])) <= 1e-7 * np.max(np.abs(ref.phi[i]))
            assert abs(phi[b, i].mean()) <= 1e-12 * np.max(np.abs(phi[b, i]))
        ref10 = oa.solve(a[b], tol=1e-10)
        for i in range(2):
            assert abs(int(its[b, i]) - ref10.iters[i]) <= 1


def test_constant_field_and_laminate(dev):
    rve = _rve()
    n = 64
    c = np.random.default_rng(9).uniform(1.0, 10.0, n)
    lam = np.repeat(c[:, None], n, axis=1)
    a = np.stack([np.full((n, n), 3.25), lam, lam.T.copy()])
    res = rve.solve_batch(_to(a, dev), 0.125, rve.Options(tol=1e-12))
    A = res.ahom.cpu().numpy()
    assert np.array_equal(A[0], 3.25 * np.eye(2))
    assert res.iters.cpu().numpy()[0].tolist() == [0, 0]
    harm, arit = 1.0 / np.mean(1.0 / c), np.mean(c)
    assert abs(A[1, 0, 0] - harm) <= 1e-11 * harm and abs(A[1, 1, 1] - arit) <= 1e-11 * arit
    assert abs(A[2, 1, 1] - harm) <= 1e-11 * harm and abs(A[2, 0, 0] - arit) <= 1e-11 * arit
    assert abs(A[1, 0, 1]) <= 1e-12 and abs(A[2, 0, 1]) <= 1e-12


@pytest.mark.parametrize("n", [128, 192])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_mixed_precision_matches_oracle(dev, prec, n):
    rve = _rve()
    B = 3
    a = _fields(n, B, 4)
    res = rve.solve_batch(_to(a, dev), 1.0 / 8, rve.Options(tol=1e-10, prec=prec))
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    for b in range(B):
        assert rel2(A[b], oa.solve(a[b], tol=1e-13).ahom) <= 1e-8


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_true_residual_meets_tolerance(dev, prec):
    # The stopping test reads the recursively updated residual; it must stay
    # the true residual f - A x (to FP64 rounding) in every precision, since
    # x, r and q = A p are all updated with the same stored direction p.
    rve = _rve()
    n, B, tol = 128, 2, 1e-10
    a = _fields(n, B, 14)
    h = 1.0 / 8
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=tol, prec=prec))
    assert res.code == 0
    x = res.phi.cpu().numpy() / h
    for b in range(B):
        A = q1.assemble(a[b])
        for i, f in enumerate(q1.rhs(a[b])):
            f = f - f.mean()
            true = np.linalg.norm(f.ravel() - A @ x[b, i].ravel()) / np.linalg.norm(f)
            assert true <= 2.0 * tol, (b, i, true)


@pytest.mark.parametrize("prec", [0, 2, 3])
def test_fp32_stencil_matches_oracle(dev, prec):
    # FP32 operator apply with FP64 partial sums and the residual recomputed
    # as f - A x every 8 iterations: A_hom to the mixed-precision bound and
    # the true residual at the tolerance
    rve = _rve()
    n, B, tol = 128, 2, 1e-10
    a = _fields(n, B, 17)
    h = 1.0 / 8
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=tol, prec=prec, stencil_prec=1))
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    x = res.phi.cpu().numpy() / h
    for b in range(B):
        assert rel2(A[b], oa.solve(a[b], tol=1e-13).ahom) <= 1e-8
        K = q1.assemble(a[b])
        for i, f in enumerate(q1.rhs(a[b])):
            f = f - f.mean()
            true = np.linalg.norm(f.ravel() - K @ x[b, i].ravel()) / np.linalg.norm(f)
            assert true <= 2.0 * tol, (b, i, true)


def test_fp32_stencil_uneven_contrast_100(dev):
    rve = _rve()
    items = []
    for k, L in enumerate((8, 16, 8, 24)):
        items.append(realization(BooleanModel(L=L, m0=8, a_in=100.0), 5, k))
    opts = rve.Options(tol=1e-10, prec=2, stencil_prec=1)
    res = rve.solve_uneven([torch.from_numpy(f).to(dev) for f in items], 0.125, opts)
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    for b, f in enumerate(items):
        assert rel2(A[b], oa.solve(f, tol=1e-13).ahom) <= 1e-8


def test_uneven_batch_matches_oracle(dev):
    rve = _rve()
    items = []
    for k, L in enumerate([8, 16, 8, 24, 16]):
        items.append(realization(BooleanModel(L=L, m0=8, a_in=100.0), 3, k))
    res = rve.solve_uneven([_to(f, dev) for f in items], 1.0 / 8, rve.Options(tol=1e-10),
                           want_phi=True)
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    for b, f in enumerate(items):
        ref = oa.solve(f, tol=1e-13)
        assert rel2(A[b], ref.ahom) <= 1e-10
        phi = res.phi[b].cpu().numpy() * 8
        assert np.max(np.abs(phi - ref.phi)) <= 1e-6 * np.max(np.abs(ref.phi))


def test_gradient_matches_oracle(dev):
    rve = _rve()
    n, B = 64, 2
    a = _fields(n, B, 6)
    h = 1.0 / 8
    res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=1e-12))
    G = np.random.default_rng(2).standard_normal((B, 2, 2))
    g, gin, _ = rve.grad(_to(a, dev), res.phi, h, _to(G, dev), a_in=10.0)
    g = g.cpu().numpy()
    gin = gin.cpu().numpy()
    for b in range(B):
        ref = oa.solve(a[b], tol=1e-13)
        d = oa.dahom_da(a[b], ref.phi)
        gref = np.einsum("ij,ijxy->xy", G[b], d)
        assert np.max(np.abs(g[b] - gref)) <= 1e-9 * np.max(np.abs(gref))
        cref = np.einsum("ij,ij->", G[b], oa.dahom_dcontrast(d, a[b] == 10.0))
        assert abs(gin[b] - cref) <= 1e-9 * abs(cref)
        # Euler identity: sum_e a_e dA/da_e = A
        assert abs(np.sum(a[b] * g[b]) - np.sum(G[b] * res.ahom.cpu().numpy()[b])) <= 1e-10


def test_autograd_and_directional_fd(dev):
    rve = _rve()
    n = 64
    a = _to(_fields(n, 1, 7), dev).requires_grad_(True)
    opts = rve.Options(tol=1e-12)
    A = rve.ahom(a, 0.125, opts)
    (A[0, 0, 0] + A[0, 0, 1]).backward()
    v = torch.from_numpy(np.random.default_rng(3).choice([-1.0, 1.0], (1, n, n))).to(dev)
    s = 1e-4
    Ap = rve.solve_batch((a.detach() + s * v).contiguous(), 0.125, opts).ahom
    Am = rve.solve_batch((a.detach() - s * v).contiguous(), 0.125, opts).ahom
    fd = ((Ap - Am)[0, 0, 0] + (Ap - Am)[0, 0, 1]).item() / (2 * s)
    an = float(torch.sum(a.grad * v))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
    # contrast derivative through the autograd wrapper vs central FD in the contrast
    mask = (a.detach() == 10.0)
    cval = torch.tensor(10.0, dtype=torch.float64, device=dev, requires_grad=True)
    Ac = rve.RveAhomContrast.apply(cval, mask, 1.0, 0.125, opts)
    assert torch.equal(Ac, A.detach())      # the same field, built on the device from the mask
    Ac[0, 0, 0].backward()
    def f(c):
        field = torch.where(mask, torch.full_like(a.detach(), c), torch.ones_like(a.detach()))
        return rve.solve_batch(field.contiguous(), 0.125, opts).ahom[0, 0, 0].item()
    fdc = (f(10.0 + 1e-5) - f(10.0 - 1e-5)) / 2e-5
    assert abs(cval.grad.item() - fdc) <= 1e-6 * abs(fdc)


def test_stats_match_oracle(dev):
    rve = _rve()
    rng = np.random.default_rng(5)
    A = rng.standard_normal((300, 2, 2)) * 0.02 + np.array([[3.0, 0.0], [0.0, 3.0]])
    A = 0.5 * (A + A.transpose(0, 2, 1))
    out = rve.stats(_to(A, dev), L=16.0)
    assert np.allclose(out["mean"].cpu().numpy(), ost.empirical_mean(A), rtol=1e-14, atol=1e-15)
    assert np.allclose(out["var"].cpu().numpy(), ost.centred_variance(A), rtol=1e-12, atol=1e-18)
    s12, sdd = ost.std_uncentred(A)
    assert np.isclose(out["std_a12"].item(), s12, rtol=1e-12)
    assert np.isclose(out["std_a11_minus_a22"].item(), sdd, rtol=1e-12)
    assert np.allclose(out["quartic"].cpu().numpy(), ost.quartic(A, 16.0), rtol=1e-11, atol=1e-16)


def test_status_codes(dev):
    rve = _rve()
    n = 64
    a = _fields(n, 3, 8)
    a[1, 5, 7] = 0.0          # invalid coefficient
    a[2, 0, 0] = np.nan
    res = rve.solve_batch(_to(a, dev), 0.125, rve.Options(tol=1e-10))
    st = res.status.cpu().numpy().tolist()
    assert st == [0, -1, -1] and res.code == -1
    b = _fields(n, 2, 8)
    res = rve.solve_batch(_to(b, dev), 0.125, rve.Options(tol=1e-10, maxit=2))
    assert res.code == 1 and res.status.cpu().numpy().tolist() == [1, 1]
    assert bool(torch.all(res.iters == 2)) and bool(torch.all(res.relres > 1e-10))


@pytest.mark.parametrize("k", [1, 7, 8, 9, 16, 17])
def test_iterate_after_k_iterations(dev, k):
    # the iterate is folded in from the ring of directions every 8 iterations
    # and at the end: stopping after k iterations must still give the PCG
    # iterate x_k (here against the oracle's PCG stopped after k iterations)
    # (batched path), and the single-workgroup solver must too
    rve = _rve()
    n, B = 64, 2
    a = _fields(n, B, 13)
    h = 1.0 / 8
    for small in (False, True):
        ctx = rve.Context(0)
        ctx.set_small_solver(small)
        res = rve.solve_batch(_to(a, dev), h, rve.Options(tol=1e-300, maxit=k), ctx=ctx)
        ctx.close()
        assert res.code == 1 and bool(torch.all(res.iters == k))
        phi = res.phi.cpu().numpy() / h
        for b in range(B):
            ref = oa.solve(a[b], tol=1e-300, maxit=k)
            assert ref.iters == (k, k)
            for i in range(2):
                assert np.max(np.abs(phi[b, i] - ref.phi[i])) <= 1e-10 * np.max(np.abs(ref.phi[i]))


def _fixed_ctx(rve, graphs):
    ctx = rve.Context(0)
    ctx.set_autotune(False)      # same kernel variants in every context
    ctx.set_graphs(graphs)
    return ctx


def _same(r1, r2):
    return all(torch.equal(getattr(r1, k), getattr(r2, k)) for k in ("ahom", "ahom_flux", "phi", "iters", "relres",
                                                                     "status"))


@pytest.mark.parametrize("prec", [0, 2])
def test_graph_replay_matches_eager(dev, prec):
    # the captured chunk is replayed several times per solve, and the cached
    # graph again by later solves, with eager launches and host polls in
    # between; every result must equal the eager launches' to the last bit
    rve = _rve()
    a = _to(_fields(128, 3, 15), dev)
    opts = rve.Options(tol=1e-10, prec=prec)
    ref = rve.solve_batch(a, 0.125, opts, ctx=_fixed_ctx(rve, False))
    g = _fixed_ctx(rve, True)
    for _ in range(3):
        assert _same(rve.solve_batch(a, 0.125, opts, ctx=g), ref)
    # a poll every 24 iterations runs the same kernels
    opts24 = rve.Options(tol=1e-10, prec=prec, check_every=24)
    assert _same(rve.solve_batch(a, 0.125, opts24, ctx=g), ref)


def test_uneven_graph_matches_eager(dev):
    rve = _rve()
    fields = [_fields(n, 1, 16 + n)[0] for n in (64, 192, 64, 128, 192)]
    opts = rve.Options(tol=1e-10, prec=1)
    ref = rve.solve_uneven([torch.from_numpy(f).to(dev) for f in fields], 0.125, opts, want_phi=True,
                           ctx=_fixed_ctx(rve, False))
    g = _fixed_ctx(rve, True)
    for _ in range(2):
        got = rve.solve_uneven([torch.from_numpy(f).to(dev) for f in fields], 0.125, opts, want_phi=True, ctx=g)
        assert torch.equal(got.ahom, ref.ahom) and torch.equal(got.iters, ref.iters)
        assert all(torch.equal(x, y) for x, y in zip(got.phi, ref.phi))


def test_bitwise_reproducible(dev):
    rve = _rve()
    a = _to(_fields(128, 3, 9), dev)
    r1 = rve.solve_batch(a, 0.125, rve.Options(tol=1e-10, prec=2))
    r2 = rve.solve_batch(a, 0.125, rve.Options(tol=1e-10, prec=2))
    assert torch.equal(r1.ahom, r2.ahom) and torch.equal(r1.phi, r2.phi)


@pytest.mark.parametrize("prec", [0, 2])
def test_bench_workload_sampled(dev, prec):
    # L = 64, h = 1/8 (n = 512), 256 realizations, contrast 10, in one launch
    # sequence exactly as timed; the oracle checks two sampled items.
    rve = _rve()
    B, n = 256, 512
    model = BooleanModel(L=64, m0=8, a_in=10.0)
    a = batch(model, 1, B)
    res = rve.solve_batch(_to(a, dev), 1.0 / 8, rve.Options(tol=1e-10, prec=prec), want_phi=False)
    assert res.code == 0
    A = res.ahom.cpu().numpy()
    bound = 1e-10 if prec == 0 else 1e-8
    for b in (0, B - 1):
        assert rel2(A[b], oa.solve(a[b], tol=1e-13).ahom) <= bound
    # every item: symmetric, within the Voigt/Reuss bounds
    for b in range(B):
        ev = np.linalg.eigvalsh(A[b])
        assert 1.0 / np.mean(1.0 / a[b]) - 1e-9 <= ev[0] and ev[1] <= np.mean(a[b]) + 1e-9


def test_autotuner_choices_and_cache(dev, tmp_path, monkeypatch):
    rve = _rve()
    n, B = 256, 4
    a = _to(_fields(n, B, 12), dev)
    opts = rve.Options(tol=1e-10, prec=2)
    fixed = rve.Context(0)
    fixed.set_autotune(False)
    ref = rve.solve_batch(a, 0.125, opts, ctx=fixed).ahom.cpu().numpy()
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("RVE_TUNE_CACHE", str(cache))
    tuned_ctx = rve.Context(0)
    got = rve.solve_batch(a, 0.125, opts, ctx=tuned_ctx).ahom.cpu().numpy()
    for b in range(B):
        assert rel2(got[b], ref[b]) <= 1e-12
    ch = tuned_ctx.tuned(n, 2, B)
    assert ch["stencil_columns_per_lane"] in (1, 2, 4) and ch["stencil_rows_per_strip"] in (16, 64)
    assert ch["stencil_prefetch_rows"] in (1, 2, 4)
    assert ch["update_columns_per_lane"] in (1, 2, 4) and ch["update_rows_per_strip"] in (16, 64)
    assert ch["update_prefetch_rows"] in (1, 2, 4)
    assert ch["gemm_variant"] in (0, 1, 4, 5, 6)
    lines = cache.read_text().strip().splitlines()
    # operator apply, transform GEMM and residual update
    assert len(lines) == 3 and all(line.startswith('{"kind"') for line in lines)
    reload_ctx = rve.Context(0)          # reads the cache at creation
    assert reload_ctx.tuned(n, 2, B) == ch


@pytest.mark.parametrize("n", [256, 512])
def test_fp16_transforms_128_tiles_and_fewer_iterations(dev, n):
    # FP16 transforms in both tile variants against the FFT apply, and a
    # solve at contrast 100 where the scaled FP16 copies take fewer
    # iterations than BF16 (and no more than a few beyond FP64)
    rve = _rve()
    rng = np.random.default_rng(n + 33)
    a = _fields(n, 2, 54)
    r = rng.standard_normal((2, 2, n, n))
    r -= r.mean(axis=(2, 3), keepdims=True)
    E = q1.symbol(n)
    for variant in (0, 1, 3, 4, 5, 6, 7):
        ctx = rve.Context(0)
        ctx.force_variants(gemm=variant)
        z = rve.apply_precond(_to(a, dev), _to(r, dev), 3, ctx=ctx).cpu().numpy()
        ctx.close()
        for b in range(2):
            a0 = oa.preconditioner_scale(a[b])
            for i in range(2):
                ref = precond_apply(r[b, i], a0, E)
                zc = z[b, i] - z[b, i].mean()
                assert np.linalg.norm(zc - ref) <= 3e-3 * np.linalg.norm(ref)
    a = _fields(n, 2, 55, contrast=100.0)
    its = {}
    for prec in (0, 2, 3):
        res = rve.solve_batch(_to(a, dev), 1.0 / 8, rve.Options(tol=1e-10, prec=prec), want_phi=False)
        assert res.code == 0
        its[prec] = res.iters.cpu().numpy().astype(float).mean()
        if prec == 0:
            A64 = res.ahom.cpu().numpy()
        else:
            A = res.ahom.cpu().numpy()
            for b in range(2):
                assert rel2(A[b], A64[b]) <= 1e-8
    assert its[3] < its[2] and its[3] <= its[0] + 0.15 * its[0], its


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("n", [384, 512, 1024])
def test_lds_loaded_transforms_identical_to_register_staged(dev, prec, n):
    # the 16-bit transform variants (1: 128 x 128 register-staged, 3: LDS
    # loaded, 4: 256 x 128 for three of the four transforms, 5: 256 x 256
    # for all four, 6: the same from 8 waves; 4, 5 and 6 need n % 256 == 0)
    # accumulate every output and every r.z partial in the same order, so
    # the preconditioner and whole solves agree bit for bit (n = 384: three
    # tiles per axis, twelve K slices, no XCD remap of the tile order; n =
    # 1024: four 256 x 256 tiles per axis, 96 tiles remapped over the XCDs)
    rve = _rve()
    rng = np.random.default_rng(n + 7 * prec)
    a = _fields(n, 3, 56)
    r = rng.standard_normal((3, 2, n, n))
    r -= r.mean(axis=(2, 3), keepdims=True)
    out = {}
    variants = (1, 3, 4, 5, 6, 7) if n % 256 == 0 else (1, 3)
    for variant in variants:
        ctx = rve.Context(0)
        ctx.set_autotune(False)
        ctx.force_variants(gemm=variant)
        z = rve.apply_precond(_to(a, dev), _to(r, dev), prec, ctx=ctx).cpu().numpy()
        res = rve.solve_batch(_to(a, dev), 1.0 / 8, rve.Options(tol=1e-10, prec=prec), ctx=ctx)
        assert res.code == 0
        out[variant] = (z, res.ahom.cpu().numpy(), res.ahom_flux.cpu().numpy(), res.iters.cpu().numpy(),
                        res.phi.cpu().numpy())
        ctx.close()
    # every tile variant: z, and whole solves (their r.z partials are taken
    # per 64 x 64 output block in one order), bit for bit
    for v in variants[1:]:
        for x1, xv in zip(out[1], out[v]):
            assert np.array_equal(x1, xv), v
    E = q1.symbol(n)
    z = out[3][0]
    for b in range(3):
        a0 = oa.preconditioner_scale(a[b])
        ref = precond_apply(r[b, 1], a0, E)
        zc = z[b, 1] - z[b, 1].mean()
        assert np.linalg.norm(zc - ref) <= (3e-2 if prec == 2 else 3e-3) * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", [2, 3])
def test_persistent_256_tiles_match_per_tile_grid(dev, prec):
    # with at least four 256 x 256 tiles per CU (here 160 realizations, 320
    # systems, 1280 tiles at n = 512) the plain transforms of variants 5 and 6 run
    # one workgroup per CU over a range of tiles, loading each next tile's
    # first slice early; z and whole solves must still equal variant 1's bit
    # for bit, also where systems converge at different iterations (skipped
    # tiles: half the realizations at contrast 2, half at 10)
    rve = _rve()
    n, B = 512, 160
    rng = np.random.default_rng(11 + prec)
    a = np.concatenate([_fields(n, B // 2, 57), _fields(n, B // 2, 58, contrast=2.0)])
    r = rng.standard_normal((B, 2, n, n))
    r -= r.mean(axis=(2, 3), keepdims=True)
    ad, rd = _to(a, dev), _to(r, dev)
    out = {}
    for variant in (1, 5, 6, 7):
        ctx = rve.Context(0)
        ctx.set_autotune(False)
        ctx.force_variants(gemm=variant)
        z = rve.apply_precond(ad, rd, prec, ctx=ctx).cpu().numpy()
        res = rve.solve_batch(ad, 1.0 / 8, rve.Options(tol=1e-10, prec=prec), want_phi=False, ctx=ctx)
        assert res.code == 0
        out[variant] = (z, res.ahom.cpu().numpy(), res.iters.cpu().numpy())
        ctx.close()
    for v in (5, 6, 7):
        for x1, xv in zip(out[1], out[v]):
            assert np.array_equal(x1, xv), v
    assert out[5][2].min() < out[5][2].max()   # systems did converge at different iterations
    # sampled systems against the oracle's preconditioner
    E = q1.symbol(n)
    z = out[5][0]
    for b, c in ((0, 0), (77, 1), (159, 1)):
        ref = precond_apply(r[b, c], oa.preconditioner_scale(a[b]), E)
        zc = z[b, c] - z[b, c].mean()
        assert np.linalg.norm(zc - ref) <= (3e-2 if prec == 2 else 3e-3) * np.linalg.norm(ref)


@pytest.mark.parametrize("prec,variant,n", [(2, 1, 256), (3, 5, 256), (2, 6, 512), (3, 6, 512), (2, 7, 256)])
def test_bf16_directions_against_fp32_and_oracle(dev, prec, variant, n):
    # directions formed in the last transform and stored in BF16 (the
    # default) or FP32: A_hom of both agree with the oracle to 1e-8 and
    # with each other to 1e-10, the true residual ||f - A phi|| stays within
    # 2 tol (x and A p see the same rounded direction), and the rounding
    # costs at most a few iterations; a solve holding a field of contrast
    # above 20 keeps FP32 directions (the same bits either way)
    rve = _rve()
    a = _fields(n, 3, 67)
    res = {}
    for bf in (True, False):
        ctx = rve.Context(0)
        ctx.set_autotune(False)
        ctx.force_variants(gemm=variant)
        ctx.set_direction_bf16(bf)
        res[bf] = rve.solve_batch(_to(a, dev), 0.125, rve.Options(tol=1e-10, prec=prec), ctx=ctx)
        ctx.close()
        assert res[bf].code == 0
    A16, A32 = res[True].ahom.cpu().numpy(), res[False].ahom.cpu().numpy()
    it16, it32 = res[True].iters.cpu().numpy(), res[False].iters.cpu().numpy()
    assert np.all(it16 <= it32 + np.maximum(3, np.ceil(0.1 * it32))), (it16, it32)
    for b in range(3):
        assert rel2(A16[b], A32[b]) <= 1e-10
    phi = res[True].phi.cpu().numpy()
    for b in (0, 2) if n == 256 else (0,):
        ref = oa.solve(a[b], tol=1e-13)
        assert rel2(A16[b], ref.ahom) <= 1e-8
        A = q1.assemble(a[b])
        f1, f2 = q1.rhs(a[b])
        for i, f in enumerate((f1, f2)):
            f = (f - f.mean()).ravel()
            # phi is the corrector in physical units (grid units times h)
            u = phi[b, i].ravel() / 0.125
            assert np.linalg.norm(f - A @ u) <= 2e-10 * np.linalg.norm(f)
    if n == 256:
        hi = np.concatenate([a[:1], _fields(n, 1, 68, contrast=100.0)])
        out = []
        for bf in (True, False):
            ctx = rve.Context(0)
            ctx.set_autotune(False)
            ctx.force_variants(gemm=variant)
            ctx.set_direction_bf16(bf)
            out.append(rve.solve_batch(_to(hi, dev), 0.125, rve.Options(tol=1e-10, prec=prec), ctx=ctx))
            ctx.close()
        assert out[0].code == 0 and _same(out[0], out[1])


def test_bf16_direction_limits(dev):
    # BF16 directions are used up to contrast 20 on grids up to n = 512:
    # there the switch changes the iterates; above either limit the solve
    # keeps FP32 directions and the switch changes nothing
    rve = _rve()

    def both(a, h):
        # (default kernel shapes: the autotuner's timing-based pick of the
        # operator-apply shape sets how p.Ap is split into partial sums)
        out = []
        for bf in (True, False):
            ctx = rve.Context(0)
            ctx.set_autotune(False)
            ctx.set_direction_bf16(bf)
            out.append(rve.solve_batch(_to(a, dev), h, rve.Options(tol=1e-10, prec=rve.MIX_BF16), ctx=ctx))
            ctx.close()
            assert out[-1].code == 0
        return out

    r16, r32 = both(_fields(256, 1, 69, contrast=20.0), 0.125)
    assert not torch.equal(r16.phi, r32.phi)
    assert rel2(r16.ahom.cpu().numpy()[0], r32.ahom.cpu().numpy()[0]) <= 1e-10
    r16, r32 = both(_fields(256, 1, 69, contrast=21.0), 0.125)
    assert _same(r16, r32)
    r16, r32 = both(_fields(1024, 1, 70), 0.125)
    assert _same(r16, r32)


@pytest.mark.parametrize("scheme", [0, 1])
def test_small_solver_matches_batched_path_and_oracle(dev, scheme):
    # n = 64, FP64: the single-workgroup solver (default) against the batched
    # iteration chunks and the oracle; same iteration counts
    rve = _rve()
    n, B = 64, 5
    a = _fields(n, B, 60)
    a[3] = 2.0                                   # constant field: f = 0, no iteration
    ctx = rve.Context(0)
    opts = rve.Options(tol=1e-10, scheme=scheme)
    r1 = rve.solve_batch(_to(a, dev), 0.125, opts, ctx=ctx)
    ctx.set_small_solver(False)
    r2 = rve.solve_batch(_to(a, dev), 0.125, opts, ctx=ctx)
    ctx.close()
    assert r1.code == 0 and r2.code == 0
    A1, A2 = r1.ahom.cpu().numpy(), r2.ahom.cpu().numpy()
    it1, it2 = r1.iters.cpu().numpy(), r2.iters.cpu().numpy()
    assert np.all(np.abs(it1 - it2) <= 1)
    assert it1[3].tolist() == [0, 0] and np.array_equal(A1[3], 2.0 * np.eye(2))
    for b in range(B):
        assert rel2(A1[b], A2[b]) <= 1e-12
        if scheme == 0:
            assert rel2(A1[b], oa.solve(a[b], tol=1e-13).ahom) <= 1e-10
    # the true residual of the returned correctors
    x = r1.phi.cpu().numpy() / 0.125
    if scheme == 0:
        K = q1.assemble(a[0])
        for i, f in enumerate(q1.rhs(a[0])):
            f = f - f.mean()
            assert np.linalg.norm(f.ravel() - K @ x[0, i].ravel()) <= 2e-10 * np.linalg.norm(f)


def test_small_solver_status_codes(dev):
    rve = _rve()
    n = 64
    a = _fields(n, 3, 61)
    a[1, 5, 7] = -1.0
    res = rve.solve_batch(_to(a, dev), 0.125, rve.Options(tol=1e-10, maxit=3))
    st = res.status.cpu().numpy().tolist()
    assert st == [1, -1, 1] and res.code == -1
    its = res.iters.cpu().numpy()
    assert its[0].tolist() == [3, 3] and its[1].tolist() == [0, 0]


def test_autograd_raises_on_failed_forward_and_takes_one_field(dev):
    # the stationarity identity behind the backward pass needs converged
    # correctors: an invalid coefficient or a solve stopped by maxit raises
    rve = _rve()
    n = 64
    a = _fields(n, 2, 62)
    bad = a.copy()
    bad[1, 5, 7] = 0.0
    with pytest.raises(rve.RveError):
        rve.ahom(_to(bad, dev).requires_grad_(True), 0.125, rve.Options(tol=1e-10))
    with pytest.raises(rve.RveError):
        rve.ahom(_to(a, dev).requires_grad_(True), 0.125, rve.Options(tol=1e-10, maxit=2))
    with pytest.raises(rve.RveError):
        mask = torch.ones((2, n, n), dtype=torch.bool, device=dev)
        rve.ahom_contrast(torch.tensor(-1.0, dtype=torch.float64, device=dev), mask, 1.0, 0.125)
    # a single (n, n) field: A (2, 2), gradient (n, n), equal to the batched one
    opts = rve.Options(tol=1e-12)
    one = _to(a[0], dev).requires_grad_(True)
    A1 = rve.ahom(one, 0.125, opts)
    assert A1.shape == (2, 2)
    (A1[0, 0] + 2.0 * A1[0, 1]).backward()
    two = _to(a[:1], dev).requires_grad_(True)
    A2 = rve.ahom(two, 0.125, opts)
    (A2[0, 0, 0] + 2.0 * A2[0, 0, 1]).backward()
    assert one.grad.shape == (n, n)
    assert torch.equal(one.grad, two.grad[0]) and torch.equal(A1, A2[0])


@pytest.mark.parametrize("prec", [0, 2])
def test_single_realization_call_matches_batch(dev, prec):
    # rve_solve: the synchronous one-realization call with host outputs runs
    # the batched path for B = 1
    rve = _rve()
    n = 128
    a = _fields(n, 1, 63)
    opts = rve.Options(tol=1e-10, prec=prec)
    ctx = rve.Context(0)
    ctx.set_autotune(False)
    one = rve.solve(_to(a[0], dev), 0.125, opts, ctx=ctx)
    bat = rve.solve_batch(_to(a, dev), 0.125, opts, ctx=ctx)
    assert one.code == 0
    assert torch.equal(one.ahom, bat.ahom.cpu()[0]) and torch.equal(one.ahom_flux, bat.ahom_flux.cpu()[0])
    assert list(one.iters) == bat.iters.cpu()[0].tolist()
    assert torch.equal(one.phi, bat.phi[0])
    assert rel2(one.ahom.numpy(), oa.solve(a[0], tol=1e-13).ahom) <= (1e-10 if prec == 0 else 1e-8)
    bad = a[0].copy()
    bad[3, 3] = float("nan")
    with pytest.raises(rve.RveError):
        rve.solve(_to(bad, dev), 0.125, opts, ctx=ctx)
    short = rve.solve(_to(a[0], dev), 0.125, rve.Options(tol=1e-10, maxit=3), ctx=ctx)
    assert short.code == 1 and list(short.iters) == [3, 3]


@pytest.mark.parametrize("prec", [0, 2])
def test_two_valued_byte_coefficients_exact(dev, prec):
    # A batch of two-valued fields runs the operator on one byte per cell
    # (decoded to each field's two values); one three-valued field sends the
    # whole batch through the FP64 coefficients. Decoding is exact, so the
    # two-valued items come out bit for bit the same either way.
    rve = _rve()
    n = 256
    a = _fields(n, 3, 64)
    b = a.copy()
    b[2, 7, 9] = 0.5 * (b[2].min() + b[2].max())
    opts = rve.Options(tol=1e-10, prec=prec)
    ctx = rve.Context(0)
    ctx.set_autotune(False)
    ra = rve.solve_batch(_to(a, dev), 0.125, opts, ctx=ctx)
    rb = rve.solve_batch(_to(b, dev), 0.125, opts, ctx=ctx)
    ctx.close()
    assert ra.code == 0 and rb.code == 0
    for k in ("ahom", "ahom_flux", "phi", "iters", "relres"):
        assert torch.equal(getattr(ra, k)[:2], getattr(rb, k)[:2]), k
    bound = 1e-10 if prec == 0 else 1e-8
    assert rel2(rb.ahom.cpu().numpy()[2], oa.solve(b[2], tol=1e-13).ahom) <= bound


@pytest.mark.parametrize("prec,variant", [(2, 1), (2, 5), (3, 6), (2, 7)])
def test_direction_in_last_transform_identical(dev, prec, variant):
    # the next search direction formed in the last transform's epilogue (with
    # a ring of one more slot) or in the operator apply: the same arithmetic,
    # so solves agree to the last bit, also when systems stop at different
    # iterations, and across a chunk boundary and a poll every 24 iterations
    rve = _rve()
    n = 256
    a = np.concatenate([_fields(n, 2, 65), _fields(n, 2, 66, contrast=2.0)])
    out = []
    for mode in (True, False):
        ctx = rve.Context(0)
        ctx.set_autotune(False)
        ctx.force_variants(gemm=variant)
        ctx.set_direction_update(mode)
        ctx.set_direction_bf16(False)   # the apply forms FP32 directions
        for opts in (rve.Options(tol=1e-10, prec=prec), rve.Options(tol=1e-10, prec=prec, check_every=24)):
            out.append(rve.solve_batch(_to(a, dev), 0.125, opts, ctx=ctx))
        ctx.close()
    for r1, r0 in ((out[0], out[2]), (out[1], out[3])):
        assert r1.code == 0 and r0.code == 0
        assert _same(r1, r0)
    its = out[0].iters.cpu().numpy()
    assert its.min() < its.max()
    for b in (0, 3):
        assert rel2(out[0].ahom.cpu().numpy()[b], oa.solve(a[b], tol=1e-13).ahom) <= 1e-8
