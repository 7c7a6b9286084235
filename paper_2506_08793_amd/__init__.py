"""MI355X-native PDE dehazing: HIP kernels behind a C ABI (include/dehaze.h).

The package holds the HIP sources (csrc/), the build script and a thin ctypes
binding.  Import fails if the library has not been built.
"""
from .binding import (  # noqa: F401
    CHW, EXPORTED, HWC, JACOBI, PAPER_EXPLICIT, PICARD_KRYLOV, U8, F32, Context, DehazeError, Params,
    Stats, Image, batch_workspace_bytes, dehaze_batch, dehaze_params_default, dehaze_prior, dehaze_residual, dehaze_solve, solve_workspace,
)
