"""The flux form of A_hom on the device (Sec. 4.1, eqn. Ahom_m_entry) against
the oracle's, and its asymmetry against the solver tolerance: the analogue of
Table conv_Symmet_thresh. The flux form is symmetric only to the accuracy of
the correctors, the energy form by construction.

One realization of the paper's fixed-count law (alpha = 0.5, a in {0.2, 1}),
L = 8 and m0 = 8 (n = 64, the smallest grid the device path takes; the
paper's table is at L = 4, h = 1/8, and does not print its realization, so
only the bound and the trend are compared), FP64 transforms.
"""
import numpy as np
import pytest
import torch

from oracle import ahom as oa
from sampler import BooleanModel, realization

pytestmark = pytest.mark.gpu

TOLS = (1e-3, 1e-5, 1e-7, 1e-9, 1e-11)
H = 1.0 / 8


def _field():
    return realization(BooleanModel(L=8, m0=8, a_in=1.0, a_bg=0.2, law="paper", alpha=0.5), 11, 0)


def _solve(rve, a, dev, tol):
    res = rve.solve_batch(torch.from_numpy(a[None]).to(dev), H, rve.Options(tol=tol, prec=rve.FP64),
                          want_flux=True)
    assert res.code == 0
    return res.ahom[0].cpu().numpy(), res.ahom_flux[0].cpu().numpy()


def test_flux_form_matches_oracle_and_energy_form(dev):
    import paper_1903_12227_amd as rve
    a = _field()
    ref = oa.solve(a, tol=1e-12)
    A, F = _solve(rve, a, dev, 1e-12)
    scale = max(abs(ref.ahom[0, 0]), abs(ref.ahom[1, 1]))
    assert np.max(np.abs(F - ref.ahom_flux)) <= 1e-9 * scale
    assert np.max(np.abs(F - A)) <= 1e-9 * scale
    assert A[0, 1] == A[1, 0]


def test_flux_asymmetry_tracks_tolerance(dev):
    import paper_1903_12227_amd as rve
    a = _field()
    asym = []
    for tol in TOLS:
        A, F = _solve(rve, a, dev, tol)
        asym.append(abs(F[0, 1] - F[1, 0]))
        assert A[0, 1] == A[1, 0]
    for tol, v in zip(TOLS, asym):
        assert v <= 10 * tol, (tol, v)
    assert asym[-1] <= 1e-11
    assert asym[-1] < asym[0]
