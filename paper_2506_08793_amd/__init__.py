"""MI355X-native PDE dehazing: HIP kernels behind a C ABI (include/dehaze.h).

The package holds the HIP sources (csrc/), the build script and a thin ctypes
binding.  Import fails if the library has not been built.
"""
from .binding import (  # noqa: F401
    CHW, EXPORTED, F32, HWC, JACOBI, PAPER_EXPLICIT, PICARD_KRYLOV, U8, U_F32, U_F64, Context, DehazeError,
    Image, Params, Stats, batch_workspace_bytes, cnn_workspace, dehaze_batch, dehaze_batch_strip_rows,
    dehaze_cnn_forward, dehaze_cnn_get_weights, dehaze_cnn_grad, dehaze_cnn_param_count, dehaze_cnn_set_weights,
    dehaze_cnn_train_step, dehaze_params_default, dehaze_prior, dehaze_residual, dehaze_residual_noalloc,
    dehaze_solve, dehaze_sweep_shape, solve_workspace,
)
