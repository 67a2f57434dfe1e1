"""MI355X-native map/reduce BLAS hot path of arXiv 1502.02389.

scal, asum, dot and gemv (and BlackScholes, a map over stock prices, and MD,
a map over particles of a reduce over neighbour lists) as hand-written gfx950
HIP kernels behind the C ABI declared in
``include/lift.h``; ``lift`` is the ctypes binding.
"""
from .lift import (  # noqa: F401
    ACC, LIFT_ACC_F32, LIFT_ACC_F32_COMP, LIFT_ACC_F32_F64COMBINE, LIFT_BF16, LIFT_EHIP,
    LIFT_EINVAL, LIFT_EUNSUPPORTED, LIFT_EWORKSPACE, LIFT_F16, LIFT_F32, LIFT_F64, LIFT_OK,
    LIFT_INTERLEAVE_CHUNK, LIFT_INTERLEAVE_DEFAULT, LIFT_INTERLEAVE_STRIDE,
    LIFT_LANES_TREE, LIFT_LANES_SEQ, LIFT_LANES_RUNS_TREE, LIFT_LANES_RUNS_SEQ,
    LiftError, asum, dot, gemv, knobs, library, lift_asum, lift_asum_ex, lift_dot, lift_dot_ex,
    lift_gemv, lift_gemv_ex, lift_knobs, lift_last_hip_error, lift_max_workgroups, lift_scal,
    lift_scal_ex, lift_status_string, lift_time_next_launch, lift_version, lift_workspace_bytes, scal,
    workspace, HipEvents, Batch, GraphRun, lift_problem, lift_batch_create, lift_batch_run,
    lift_batch_capture, lift_batch_info, lift_batch_destroy, LIFT_KIND_ASUM, LIFT_KIND_DOT, LIFT_KIND_GEMV,
    blackscholes, lift_blackscholes, lift_blackscholes_ex, md, lift_md, lift_md_ex,
    lift_stream_read, lift_stream_copy, lift_default_knobs, lift_dot_ex_noalloc,
    lift_stamp_next_launch,
)
