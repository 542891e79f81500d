"""LSMS tau00 hot path on MI355X: Python binding of liblsms_tau (C ABI).

Every step of the path runs in the library's HIP kernels; this package only
marshals arguments.  PyTorch provides device memory and the current stream.
"""

from .lsms import (  # noqa: F401
    GRAPH,
    INFO_FP64_FALLBACK,
    INFO_LU_FALLBACK,
    INFO_PIVOT_MASK,
    MLP_ACT,
    MLP_PARAMS,
    PERSISTENT,
    PREC_FP32_IR,
    PREC_FP64,
    Handle,
    Opts,
    Problem,
    BATCHED_WORK_PER_INST,
    autotune,
    autotune_load,
    autotune_save,
    build_kkr,
    build_liz,
    get_tuned_nb,
    gmres_workspace_size,
    lib,
    mlp_adamw,
    mlp_backward,
    mlp_cast,
    mlp_features,
    mlp_forward,
    mlp_mse,
    mlp_norm_stats,
    mlp_seed,
    mlp_targets,
    problem_for_workload,
    set_tuned_nb,
    tau00_batched,
    tau00_gmres,
    tau00_solve,
    workspace_size,
)
