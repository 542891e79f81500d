"""LSMS tau00 hot path on MI355X: Python binding of liblsms_tau (C ABI).

Every step of the path runs in the library's HIP kernels; this package only
marshals arguments.  PyTorch provides device memory and the current stream.
"""

from .lsms import (  # noqa: F401
    GRAPH,
    INFO_FP64_FALLBACK,
    PERSISTENT,
    PREC_FP32_IR,
    PREC_FP64,
    Handle,
    Opts,
    Problem,
    autotune,
    build_kkr,
    build_liz,
    lib,
    problem_for_workload,
    set_tuned_nb,
    tau00_batched,
    tau00_solve,
    workspace_size,
)
