"""Plain, slow, CPU FP64 oracle for compressed patch-based relaxation.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU path never calls
it and shares no code with it: the two meet only through the seeded input
generators in ``gen``.

Every function follows a passage of Harper & Tuminaro, "Compression and
Reduced Representation Techniques for Patch-Based Relaxation" (arXiv
2306.10025), cited in its docstring by section, equation or algorithm.  Where
the paper is silent or ambiguous the reading taken is stated at the function.

Pins: each function is checked in ``tests/test_oracle_*.py`` against closed
forms, brute force on tiny inputs, library routines used as a different route,
and invariants the paper states.  Functions without such a pin say
"parity unpinned" in their docstring.
"""
from .patch import (OracleError, cover_weights, patch_tiles, patch_tiles_csr, batch_inverse, boundary_mask,
                    factor_inverse, apply_patch, apply_operator_dense, storage_bytes,
                    objective)
from .criterion import crit_spectral, crit_spectral_x, crit_l1, crit_fro, criterion
from .database import (alg1_tolerance, alg1_closest, alg1_reuse, compressibility, kmeans, partition_groups,
                       apportion, SplitMix64, alg1_invariants_hold, alg1_with_predictions)
from . import mlp
from .krylov import gmres, make_preconditioner
from .twolevel import linear_interpolation, coarse_operator, combo_preconditioner
from .lowprec import round_fp32, round_bf16, round_fp16, apply_lowprec, fp16_scale_exp

__all__ = [
    "OracleError", "cover_weights", "patch_tiles", "patch_tiles_csr", "batch_inverse", "boundary_mask", "factor_inverse",
    "apply_patch", "apply_operator_dense", "storage_bytes", "objective",
    "crit_spectral", "crit_spectral_x", "crit_l1", "crit_fro", "criterion",
    "alg1_tolerance", "alg1_closest", "alg1_reuse", "compressibility", "kmeans", "partition_groups", "apportion", "SplitMix64",
    "alg1_invariants_hold", "alg1_with_predictions", "mlp", "gmres", "make_preconditioner",
    "linear_interpolation", "coarse_operator", "combo_preconditioner",
    "round_fp32", "round_bf16", "round_fp16", "apply_lowprec", "fp16_scale_exp",
]
