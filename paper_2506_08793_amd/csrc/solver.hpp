// One-image solve orchestration (front-end reuse, scheme dispatch, stopping).
#pragma once

#include "internal.hpp"

namespace dz {

struct SolveArgs {
  const void* I;
  int dtype, layout, H, W, pitch;
  const float* t;   // H x W, pitch W
  const float* A;   // 3 device floats
  const float* u0;  // planar, pitch W, nullable
  float* u;         // planar, pitch W
  void* ws;
  size_t ws_bytes;
};

size_t solver_workspace_bytes(int H, int W, const dehaze_params& p);
int solve_one(Ctx& ctx, const SolveArgs& a, const dehaze_params& p, dehaze_stats* stats, hipStream_t s);
void solver_release(Ctx& ctx);
int sweep_shape(const Ctx& ctx, int H, int W, int scheme, int* K, int* S, int* C);
size_t batch_workspace_bytes(int n, const dehaze_image* imgs, const dehaze_params& p);
// Strip height of the BiCGSTAB kernels for each image of a batch (0: the tile
// kernels); *tuned = 1 when the context has timed this batch composition.
int batch_strip_rows(const Ctx* ctx, int n, const dehaze_image* imgs, const dehaze_params& p, int* rows, int* tuned);
int solve_batch(Ctx& ctx, int n, const dehaze_image* imgs, int dtype, int layout, const dehaze_params& p, void* ws,
                dehaze_stats* st, hipStream_t s);

}  // namespace dz
