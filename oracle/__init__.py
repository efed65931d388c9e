"""FP64 CPU oracle for the multigrid two-point-correlation descriptor.

TEST INFRASTRUCTURE ONLY.  The product path (the HIP library and its Python
binding) must never import, link or call anything in this package; only the
test suite, the smoke check and the benchmark's CPU-baseline leg do.
Parity of functions listed as "parity unpinned" in their docstrings is not
claimed.
"""
from . import _native
from .s2 import (DESCRIPTORS, Spec, adam_step, adjoint, adjoint_at_single_level, all_pairs, box,
                 correct_s3, correct_s3_adjoint, correct_sbar, correct_sbar_adjoint, descriptor, descriptor_at, error_Z, half_box,
                 in_half, lbfgs_direction, level_disp, level_slice, level_weights_per_entry, level_spec, loss, loss_grad, penalised_loss_grad, penalty, pool,
                 pool_adjoint, pyramid, reconstruct_adam, reconstruct_coarse_to_fine, reconstruct_lbfgs_projected, reconstruct_lbfgsb, soft_threshold,
                 soft_threshold_constants, upsample)

build = _native.build
