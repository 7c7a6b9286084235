// Warm-start network (see cnn.hip).
#pragma once

#include "internal.hpp"

namespace dz {

constexpr int kCnnLayers = 6;
// The network predicts u / kCnnOutScale: converged solutions of the PDE lie
// in roughly [0, 40], so the raw outputs stay of order one.
constexpr float kCnnOutScale = 8.0f;

struct CnnState;
void cnn_release(CnnState* st);
size_t cnn_param_count();
size_t cnn_param_offset(int layer);
bool cnn_ready(const Ctx& ctx);
int cnn_set_weights(Ctx& ctx, const float* host_w, size_t count, hipStream_t s);
int cnn_get_weights(Ctx& ctx, float* host_w, size_t count, hipStream_t s);

// Inference on n images of H x W: I planar float (row pitch ip, plane stride
// iplane, image stride iimg), t (pitch tp, image stride timg), A (3 floats
// per image); out planar float (row pitch out_pitch, image stride).
size_t cnn_forward_bytes(int n, int H, int W);
int cnn_forward(Ctx& ctx, int n, int H, int W, const float* I, int ip, size_t iplane, size_t iimg, const float* t,
                int tp, size_t timg, const float* A, float* out, int out_pitch, size_t out_img_stride, void* ws,
                hipStream_t s);

// Training on n dense images (I: n x 3 x H x W, t: n x H x W, A: n x 3,
// target: n x 3 x H x W): mean squared error against target.
size_t cnn_train_bytes(int n, int H, int W);
int cnn_grad(Ctx& ctx, int n, int H, int W, const float* I, const float* t, const float* A, const float* target,
             float* grad_out, double* loss, void* ws, hipStream_t s);
int cnn_train_step(Ctx& ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                   const float* target, float lr, double* loss, void* ws, hipStream_t s);

}  // namespace dz
