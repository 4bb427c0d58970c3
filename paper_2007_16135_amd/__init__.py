"""MI355X-native Time Warp Edit Distance (arXiv 2007.16135).

The distance kernels live in the HIP library libtwed.so (C ABI in
include/twed.h); this package is its thin binding plus seeded input
generators.  Nothing here computes distances on the CPU.
"""
from .binding import (  # noqa: F401
    TwedError, TwedParams, load_library, make_params, twed_pair, twed_pair_noalloc, twed_pair_matrix,
    twed_pair_workspace_size, twed_batch, twed_batch_workspace_size, twed_stream_check,
    twed_version, twed_host, twed_pair_tune, twed_tune_clear, twed_pair_tile, twed_pair_path,
    twed_dp, twed_dp_path, BatchPlan, twed_tune_save, twed_tune_load, twed_pair_config,
)
