"""MI355X-native PDE dehazing: HIP kernels behind a C ABI (include/dehaze.h).

The package holds the HIP sources (csrc/), the build script and a thin ctypes
binding.  Import fails if the library has not been built.
"""
from .binding import (  # noqa: F401
    CHW, EXPORTED, HWC, JACOBI, PAPER_EXPLICIT, PICARD_KRYLOV, U8, F32, Context, DehazeError, Params,
    Stats, Image, batch_workspace_bytes, cnn_workspace, dehaze_cnn_forward, dehaze_cnn_get_weights,
    dehaze_cnn_grad, dehaze_cnn_param_count, dehaze_cnn_set_weights, dehaze_cnn_train_step, dehaze_batch, dehaze_params_default, dehaze_prior, dehaze_residual, dehaze_residual_noalloc, dehaze_solve, dehaze_sweep_shape, solve_workspace,
)
