"""MI355X-native global registration of surface fragments (LoopSmart, Sec. IV).

Thin Python binding of the C ABI in ``include/lsr.h`` (``liblsr.so``, HIP for
gfx950).  Argument marshalling only: every step of the path runs in the HIP
kernels.  PyTorch provides device memory and the current stream.

A cloud is a float32 CUDA tensor of shape (6, N): rows x, y, z, nx, ny, nz.
"""
from ._lib import (  # noqa: F401
    ACCEPTED, REJECTED, DEGENERATE, FP32, BF16_SCREEN,
    Params, Result, LsrError, lib, default_params, Context, get_context,
    voxel_downsample, register_pair, register_batch, autotune, get_tune, set_tune, align_loss, align_loss_backward, set_timing, get_timing,
    stage_normals, stage_spfh, stage_fpfh, stage_match, stage_consistency, stage_gnc, stage_verify,
    ransac_pair, stage_ransac, stage_gnc_noalloc, surfel_correct, loop_params, edge_info, loop_solve, loop_verify,
    se3_retract, se3_retract_grad,
)
from .autograd import AlignLoss  # noqa: F401
