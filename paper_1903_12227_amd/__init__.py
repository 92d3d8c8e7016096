"""MI355X-native RVE corrector path for stochastic homogenization.

Hot path of Khoromskaia, Khoromskij, Otto, "Numerical study in stochastic
homogenization for elliptic PDEs: convergence rate in the size of
representative volume elements": for each realization of a two-valued
periodic coefficient field, solve the two corrector problems of the periodic
Q1 discretisation by preconditioned CG and reduce them to the homogenized
2x2 matrix A_hom; over many realizations, form the ensemble statistics.

All arithmetic runs in librve (hand-written HIP kernels for gfx950, C ABI in
include/rve.h); this package only marshals torch tensors into it.
"""
from ._native import (  # noqa: F401
    FP64, MIX_FP32, MIX_BF16, MIX_FP16, STENCIL_FP64, STENCIL_FP32, SCHEME_Q1, SCHEME_FD5, DIRECTION_RING, LIB_PATH,
    RveError,
)
from .api import (  # noqa: F401
    Context, Options, Result, SingleResult, context, solve, solve_batch, solve_uneven, grad, stats,
    field_from_mask, apply_operator, apply_precond, occupancy_threshold, sample_lattice, sample_fixed_count, dos_moments, dos_eval,
    dos_plan, dos_probes, spectral_density, solve_batch_3d, apply_operator_3d, apply_precond_3d,
)
from .autograd import RveAhom, RveAhomContrast, ahom, ahom_contrast  # noqa: F401
