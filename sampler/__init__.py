"""Seeded synthetic coefficient fields for the RVE corrector problem.

This module only draws random inputs. It holds none of the method's
arithmetic (no operator, right-hand side, solver or homogenized matrix), so
both the CPU oracle and the GPU path may take their inputs from it.
"""
from .boolean_model import (  # noqa: F401
    SEED_ROOT,
    BooleanModel,
    covered_mask,
    realization,
    batch,
    uneven_batch,
    uneven_sizes,
    BooleanModel3D,
    realization_3d,
    batch_3d,
)
