"""MI355X-native piecewise-constant SIR particle filter (gfx950 HIP kernels behind a C ABI).

The filter step (propagate, bin, dummy, likelihood, weight copy, normalise,
resample) runs entirely in ``libpcsir.so``. This package is argument
marshalling only: torch supplies device memory and the stream.
"""
from ._lib import (  # noqa: F401
    DUMP, Config, Filter, LibraryMissing, MLPTrainer, PcsirError, SurrogateNet, Tuning, gemm_bf16, lib,
    lib_path, mlp_param_count,
)
