// Warm-start network: six 3x3 convolutions (7 -> 32 -> 32 -> 32 -> 32 -> 32
// -> 3), ReLU after the first five, zero "same" padding, fed with the hazy
// image, the transmission and the broadcast atmospheric light.  The paper
// only points at hybrids of its PDE with learned models (end of Section I);
// the network gives the lagged-diffusivity solve a starting iterate, and the
// solve always finishes from it and judges convergence by its own residual.
//
// Arithmetic: bfloat16 activations and weights, float32 accumulation on the
// matrix cores (v_mfma_f32_32x32x8bf16_1k).  Each convolution is an implicit
// GEMM: M = 32 pixels of an output row, N = 32 output channels, K = 9 taps x
// input channels.  Activations are stored pixel-major with the channels
// contiguous (NHWC), so every lane's four K values are one 8-byte LDS read.
// The input-gradient pass is the same kernel with flipped, transposed
// weights and a ReLU-mask epilogue; the weight gradient is a GEMM over pixels
// whose per-workgroup partial sums are added in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cnn.hpp"

namespace dz {

namespace {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// float32 -> bfloat16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

constexpr int CTX = 32;  // output tile: 32 columns
constexpr int CTY = 8;   // x 8 rows; 4 waves, 2 rows each
constexpr int NT = 256;

enum ConvMode { kReluBf16 = 0, kMaskBf16 = 1, kOutF32 = 2 };

// out[p][co] = bias[co] + sum_{tap, ci} in[p + off(tap)][ci] * W[tap][ci][co]
// in: NHWC bf16 with CIN channels; wpk: packed [tap][CIN/8][2][32][4] bf16.
template <int CIN, int MODE>
__global__ __launch_bounds__(NT) void k_conv(const uint16_t* __restrict__ in, int H, int W,
                                              const uint16_t* __restrict__ wpk, const float* __restrict__ bias,
                                              uint16_t* __restrict__ out_bf, const uint16_t* __restrict__ mask,
                                              float* __restrict__ out_f, float out_scale, int out_ch,
                                              int out_pitch, size_t out_img_stride) {
  constexpr int PS = CIN + 4;  // LDS pixel stride (bf16): 8-byte aligned, staggers banks
  constexpr int LX = CTX + 2, LY = CTY + 2;
  __shared__ __attribute__((aligned(16))) uint16_t sin[LY * LX * PS];
  __shared__ __attribute__((aligned(16))) uint16_t sw[9 * CIN * 32];
  const int n = blockIdx.z;
  const size_t img = static_cast<size_t>(n) * H * W;
  const int x0 = blockIdx.x * CTX, y0 = blockIdx.y * CTY;
  const int tid = threadIdx.x;
  for (int i = tid; i < 9 * CIN * 32 / 4; i += NT)
    reinterpret_cast<uint2*>(sw)[i] = reinterpret_cast<const uint2*>(wpk)[i];
  for (int i = tid; i < LY * LX * (CIN / 4); i += NT) {
    const int pix = i / (CIN / 4), q = i - pix * (CIN / 4);
    const int ly = pix / LX, lx = pix - ly * LX;
    const int y = y0 - 1 + ly, x = x0 - 1 + lx;
    uint2 v = make_uint2(0u, 0u);
    if (y >= 0 && y < H && x >= 0 && x < W)
      v = reinterpret_cast<const uint2*>(in + (img + static_cast<size_t>(y) * W + x) * CIN)[q];
    *reinterpret_cast<uint2*>(&sin[pix * PS + q * 4]) = v;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int m = lane & 31, kh = lane >> 5;
  f16v acc0 = {}, acc1 = {};
  for (int dy = 0; dy < 3; ++dy)
    for (int dx = 0; dx < 3; ++dx) {
      const int tap = dy * 3 + dx;
#pragma unroll
      for (int kc = 0; kc < CIN / 8; ++kc) {
        const s4v b = *reinterpret_cast<const s4v*>(&sw[(((tap * (CIN / 8) + kc) * 2 + kh) * 32 + m) * 4]);
        const s4v a0 = *reinterpret_cast<const s4v*>(&sin[((2 * wave + dy) * LX + m + dx) * PS + kc * 8 + kh * 4]);
        const s4v a1 =
            *reinterpret_cast<const s4v*>(&sin[((2 * wave + 1 + dy) * LX + m + dx) * PS + kc * 8 + kh * 4]);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a0, b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b, acc1, 0, 0, 0);
      }
    }
  // D layout: lane holds column m (output channel) of rows (i/4)*8 + kh*4 + i%4 (pixels)
  const int co = m;
  const float bco = bias ? bias[co] : 0.0f;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const f16v acc = r ? acc1 : acc0;
    const int y = y0 + 2 * wave + r;
    if (y >= H) continue;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int x = x0 + (i / 4) * 8 + kh * 4 + (i % 4);
      if (x >= W) continue;
      const float v = acc[i] + bco;
      const size_t p = img + static_cast<size_t>(y) * W + x;
      if (MODE == kReluBf16) {
        out_bf[p * 32 + co] = f2bf(v > 0.0f ? v : 0.0f);
      } else if (MODE == kMaskBf16) {
        out_bf[p * 32 + co] = bf2f(mask[p * 32 + co]) > 0.0f ? f2bf(v) : static_cast<uint16_t>(0);
      } else if (co < out_ch) {
        out_f[static_cast<size_t>(n) * out_img_stride + static_cast<size_t>(co) * H * out_pitch +
              static_cast<size_t>(y) * out_pitch + x] = out_scale * v;
      }
    }
  }
}

// Network input [I^R, I^G, I^B, t, A^R, A^G, A^B, 0] per pixel, bf16.
__global__ __launch_bounds__(NT) void k_features(const float* __restrict__ I, int ip, size_t iplane,
                                                  size_t iimg, const float* __restrict__ t, int tp, size_t timg,
                                                  const float* __restrict__ A, int H, int W,
                                                  uint16_t* __restrict__ x8) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int n = blockIdx.z;
  if (x >= W) return;
  const float* In = I + n * iimg;
  uint16_t v[8];
  for (int c = 0; c < 3; ++c) v[c] = f2bf(In[c * iplane + static_cast<size_t>(y) * ip + x]);
  v[3] = f2bf(t[n * timg + static_cast<size_t>(y) * tp + x]);
  for (int c = 0; c < 3; ++c) v[4 + c] = f2bf(A[3 * n + c]);
  v[7] = 0;
  uint4 pk;
  pk.x = v[0] | (static_cast<uint32_t>(v[1]) << 16);
  pk.y = v[2] | (static_cast<uint32_t>(v[3]) << 16);
  pk.z = v[4] | (static_cast<uint32_t>(v[5]) << 16);
  pk.w = v[6] | (static_cast<uint32_t>(v[7]) << 16);
  reinterpret_cast<uint4*>(x8)[(static_cast<size_t>(n) * H + y) * W + x] = pk;
}

// Packs float32 weights W[co][ci][3][3] (cin x cout real channels) into the
// MFMA B layout [tap][CIN/8][2][32][4] with zero padding.  flip != 0 builds
// the input-gradient weights: W'[tap'][ci'=co][co'=ci] = W[co][ci][8 - tap'].
__global__ __launch_bounds__(NT) void k_pack(const float* __restrict__ w, int cin, int cout, int CINP, int flip,
                                              uint16_t* __restrict__ out) {
  const int total = 9 * CINP * 32;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int j = i & 3;
    const int o = (i >> 2) & 31;            // GEMM column (output channel of this conv)
    const int kh = (i >> 7) & 1;
    const int rest = i >> 8;                 // tap * (CINP/8) + kc
    const int kc = rest % (CINP / 8), tap = rest / (CINP / 8);
    const int k = kc * 8 + kh * 4 + j;       // GEMM row within the tap (input channel of this conv)
    float v = 0.0f;
    if (!flip) {
      if (k < cin && o < cout) v = w[(static_cast<size_t>(o) * cin + k) * 9 + tap];
    } else {
      // this conv maps the original output channels (k < cout) to the original inputs (o < cin)
      if (k < cout && o < cin) v = w[(static_cast<size_t>(k) * cin + o) * 9 + (8 - tap)];
    }
    out[i] = f2bf(v);
  }
}

// Loss: y (planar float, out_scale applied) against the target; writes
// dL/dz6 = 2 (y - target) out_scale / count as bf16 NHWC with 8 channels and
// per-block partial sums of the squared error.
__global__ __launch_bounds__(NT) void k_loss(const float* __restrict__ y, const float* __restrict__ tgt, int H,
                                              int W, int nimg, float gscale, uint16_t* __restrict__ g8,
                                              double* __restrict__ part) {
  __shared__ double red[NT / 64];
  const size_t npix = static_cast<size_t>(nimg) * H * W;
  double acc = 0.0;
  for (size_t q = static_cast<size_t>(blockIdx.x) * NT + threadIdx.x; q < npix;
       q += static_cast<size_t>(gridDim.x) * NT) {
    const size_t n = q / (static_cast<size_t>(H) * W);
    const size_t pix = q - n * H * W;
    uint16_t gv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      const size_t e = (n * 3 + c) * H * W + pix;
      const float d = y[e] - tgt[e];
      acc += static_cast<double>(d) * d;
      gv[c] = f2bf(gscale * d);
    }
    uint4 pk;
    pk.x = gv[0] | (static_cast<uint32_t>(gv[1]) << 16);
    pk.y = gv[2] | (static_cast<uint32_t>(gv[3]) << 16);
    pk.z = 0u;
    pk.w = 0u;
    reinterpret_cast<uint4*>(g8)[q] = pk;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

// Weight gradient dW[tap][co][ci] = sum_p g[p][co] h[p + off(tap)][ci] and
// bias gradient sum_p g[p][co], over 8 x 32 pixel tiles; each workgroup walks
// tiles with a fixed stride and writes one partial (9*1024 + 32 floats).
template <int CIN, int COUT>
__global__ __launch_bounds__(NT) void k_wgrad(const uint16_t* __restrict__ h, const uint16_t* __restrict__ g,
                                               int H, int W, int nimg, float* __restrict__ part) {
  constexpr int KP = CTY * CTX;  // 256 pixels per tile
  __shared__ __attribute__((aligned(16))) uint16_t gT[32][KP];
  __shared__ __attribute__((aligned(16))) uint16_t hT[3][32][CTY + 2][CTX];
  const int tiles_x = (W + CTX - 1) / CTX, tiles_y = (H + CTY - 1) / CTY;
  const int ntile = tiles_x * tiles_y * nimg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 31, kh = lane >> 5;
  f16v acc[3] = {{}, {}, {}};
  float bsum = 0.0f;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int n = tile / (tiles_x * tiles_y);
    const int rem = tile - n * tiles_x * tiles_y;
    const int y0 = (rem / tiles_x) * CTY, x0 = (rem % tiles_x) * CTX;
    const size_t img = static_cast<size_t>(n) * H * W;
    __syncthreads();
    for (int i = tid; i < 32 * KP; i += NT) {
      const int co = i / KP, px = i - co * KP;
      const int y = y0 + px / CTX, x = x0 + px % CTX;
      gT[co][px] = (co < COUT && y < H && x < W) ? g[(img + static_cast<size_t>(y) * W + x) * COUT + co]
                                                   : static_cast<uint16_t>(0);
    }
    for (int i = tid; i < 3 * 32 * (CTY + 2) * CTX; i += NT) {
      const int col = i % CTX;
      const int row = (i / CTX) % (CTY + 2);
      const int ci = (i / (CTX * (CTY + 2))) % 32;
      const int sx = i / (CTX * (CTY + 2) * 32);
      const int y = y0 - 1 + row, x = x0 - 1 + col + sx;
      hT[sx][ci][row][col] = (ci < CIN && y >= 0 && y < H && x >= 0 && x < W)
                                 ? h[(img + static_cast<size_t>(y) * W + x) * CIN + ci]
                                 : static_cast<uint16_t>(0);
    }
    __syncthreads();
    if (tid < 32)
      for (int px = 0; px < KP; ++px) bsum += bf2f(gT[tid][px]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int tap = wave + 4 * j;
      if (tap >= 9) break;
      const int dy = tap / 3, dx = tap % 3;
      for (int row = 0; row < CTY; ++row)
#pragma unroll
        for (int c0 = 0; c0 < CTX; c0 += 8) {
          const s4v a = *reinterpret_cast<const s4v*>(&gT[m][row * CTX + c0 + kh * 4]);
          const s4v b = *reinterpret_cast<const s4v*>(&hT[dx][m][row + dy][c0 + kh * 4]);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[j], 0, 0, 0);
        }
    }
  }
  // D: row = output channel co ((i/4)*8 + kh*4 + i%4), column = input channel m
  float* out = part + static_cast<size_t>(blockIdx.x) * (9 * 1024 + 32);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int tap = wave + 4 * j;
    if (tap >= 9) break;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int co = (i / 4) * 8 + kh * 4 + (i % 4);
      out[tap * 1024 + co * 32 + m] = acc[j][i];
    }
  }
  if (tid < 32) out[9 * 1024 + tid] = bsum;
}

// Sums the partials of nblk workgroups in block order and scatters them into
// the float32 gradient of one layer: dW[co][ci][3][3] then db[co].
__global__ __launch_bounds__(NT) void k_wgrad_reduce(const float* __restrict__ part, int nblk, int cin, int cout,
                                                      float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * 1024 + 32) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += part[static_cast<size_t>(b) * (9 * 1024 + 32) + i];
  if (i < 9 * 1024) {
    const int tap = i / 1024, co = (i / 32) % 32, ci = i % 32;
    if (co < cout && ci < cin) grad[(static_cast<size_t>(co) * cin + ci) * 9 + tap] = s;
  } else {
    const int co = i - 9 * 1024;
    if (co < cout) grad[static_cast<size_t>(cout) * cin * 9 + co] = s;
  }
}

__global__ __launch_bounds__(NT) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_bias32(const float* __restrict__ b, int cout, float* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < 32) out[i] = i < cout ? b[i] : 0.0f;
}

__global__ void k_zero(float* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

__global__ __launch_bounds__(NT) void k_sum_doubles(const double* __restrict__ in, int n, double* out) {
  __shared__ double s[NT];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) a += in[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

constexpr int kCin[kCnnLayers] = {7, 32, 32, 32, 32, 32};
constexpr int kCout[kCnnLayers] = {32, 32, 32, 32, 32, 3};

int cinp(int l) { return l == 0 ? 8 : 32; }

dim3 conv_grid(int H, int W, int n) { return dim3((W + CTX - 1) / CTX, (H + CTY - 1) / CTY, n); }

template <int CIN, int MODE>
int launch_conv(const uint16_t* in, int H, int W, int n, const uint16_t* wpk, const float* bias, uint16_t* out_bf,
                const uint16_t* mask, float* out_f, float scale, int out_ch, int out_pitch, size_t out_img_stride,
                hipStream_t s) {
  hipLaunchKernelGGL((k_conv<CIN, MODE>), conv_grid(H, W, n), dim3(NT), 0, s, in, H, W, wpk, bias, out_bf, mask,
                     out_f, scale, out_ch, out_pitch, out_img_stride);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int wgrad_blocks(int H, int W, int n) {
  const long long tiles = static_cast<long long>((W + CTX - 1) / CTX) * ((H + CTY - 1) / CTY) * n;
  return static_cast<int>(std::min<long long>(tiles, 1024));
}

}  // namespace

size_t cnn_param_offset(int l) {
  size_t off = 0;
  for (int k = 0; k < l; ++k) off += static_cast<size_t>(kCout[k]) * kCin[k] * 9 + kCout[k];
  return off;
}

size_t cnn_param_count() { return cnn_param_offset(kCnnLayers); }

struct CnnState {
  float* master = nullptr;   // float32 parameters, layer by layer: W[co][ci][3][3], b[co]
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* bias32[kCnnLayers] = {};  // per-layer bias padded to 32
  uint16_t* wf[kCnnLayers] = {};   // forward packing
  uint16_t* wd[kCnnLayers] = {};   // input-gradient packing
  int step = 0;
  bool ready = false;
};

void cnn_release(CnnState* st) {
  if (!st) return;
  (void)hipFree(st->master);
  delete st;
}

namespace {

int ensure_state(Ctx& ctx) {
  if (ctx.cnn) return DEHAZE_OK;
  CnnState* st = new CnnState();
  const size_t np = cnn_param_count();
  size_t bytes = align_up(4 * np * sizeof(float), 256);
  size_t packed = 0;
  for (int l = 0; l < kCnnLayers; ++l) packed += 2 * align_up(9 * 32 * 32 * sizeof(uint16_t), 256);
  bytes += packed + kCnnLayers * 256;
  char* base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    delete st;
    set_error("cannot allocate network weights");
    return DEHAZE_EHIP;
  }
  Carver cv(base, bytes);
  st->master = cv.take<float>(np);
  st->grad = cv.take<float>(np);
  st->m = cv.take<float>(np);
  st->v = cv.take<float>(np);
  for (int l = 0; l < kCnnLayers; ++l) {
    st->wf[l] = cv.take<uint16_t>(9 * 32 * 32);
    st->wd[l] = cv.take<uint16_t>(9 * 32 * 32);
    st->bias32[l] = cv.take<float>(32);
  }
  ctx.cnn = st;
  return DEHAZE_OK;
}

// Rebuilds the bf16 packings and the padded biases from the float32 master.
int repack(CnnState* st, hipStream_t s) {
  for (int l = 0; l < kCnnLayers; ++l) {
    const float* w = st->master + cnn_param_offset(l);
    hipLaunchKernelGGL(k_pack, dim3(36), dim3(NT), 0, s, w, kCin[l], kCout[l], cinp(l), 0, st->wf[l]);
    DZ_CHECK_LAUNCH();
    if (l > 0) {
      // input-gradient conv of layer l reads the gradient of its kCout[l] outputs
      const int cinp_d = kCout[l] <= 8 ? 8 : 32;
      hipLaunchKernelGGL(k_pack, dim3(36), dim3(NT), 0, s, w, kCin[l], kCout[l], cinp_d, 1, st->wd[l]);
      DZ_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_bias32, dim3(1), dim3(32), 0, s, w + static_cast<size_t>(kCout[l]) * kCin[l] * 9, kCout[l],
                       st->bias32[l]);
    DZ_CHECK_LAUNCH();
  }
  return DEHAZE_OK;
}

struct FwdBufs {
  uint16_t* x8;       // n*H*W*8
  uint16_t* h[5];     // n*H*W*32 each (training keeps all five; inference ping-pongs two)
};

size_t fwd_bytes(int n, int H, int W, bool keep_all) {
  const size_t px = static_cast<size_t>(n) * H * W;
  return align_up(px * 8 * 2, 256) + (keep_all ? 5 : 2) * align_up(px * 32 * 2, 256);
}

FwdBufs carve_fwd(Carver& cv, int n, int H, int W, bool keep_all) {
  const size_t px = static_cast<size_t>(n) * H * W;
  FwdBufs b{};
  b.x8 = cv.take<uint16_t>(px * 8);
  if (keep_all) {
    for (int l = 0; l < 5; ++l) b.h[l] = cv.take<uint16_t>(px * 32);
  } else {
    uint16_t* a = cv.take<uint16_t>(px * 32);
    uint16_t* c = cv.take<uint16_t>(px * 32);
    for (int l = 0; l < 5; ++l) b.h[l] = (l % 2 == 0) ? a : c;
  }
  return b;
}

// Runs the six layers; the output y = scale * z6 goes to out (planar float).
int forward(CnnState* st, const FwdBufs& b, int n, int H, int W, float* out, int out_pitch, size_t out_img_stride,
            hipStream_t s) {
  int rc;
  if ((rc = launch_conv<8, kReluBf16>(b.x8, H, W, n, st->wf[0], st->bias32[0], b.h[0], nullptr, nullptr, 0.f, 0, 0,
                                      0, s)))
    return rc;
  for (int l = 1; l < 5; ++l)
    if ((rc = launch_conv<32, kReluBf16>(b.h[l - 1], H, W, n, st->wf[l], st->bias32[l], b.h[l], nullptr, nullptr,
                                         0.f, 0, 0, 0, s)))
      return rc;
  return launch_conv<32, kOutF32>(b.h[4], H, W, n, st->wf[5], st->bias32[5], nullptr, nullptr, out, kCnnOutScale, 3,
                                  out_pitch, out_img_stride, s);
}

int features(const float* I, int ip, size_t iplane, size_t iimg, const float* t, int tp, size_t timg, const float* A,
             int n, int H, int W, uint16_t* x8, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3((W + NT - 1) / NT, H, n), dim3(NT), 0, s, I, ip, iplane, iimg, t, tp, timg, A,
                     H, W, x8);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

struct TrainBufs {
  FwdBufs f;
  float* y;          // n*3*H*W
  uint16_t* g8;      // n*H*W*8 : gradient of the last layer's output
  uint16_t* ga;      // n*H*W*32
  uint16_t* gb;      // n*H*W*32
  float* part;       // wgrad partials
  double* lpart;     // loss partials
  double* loss;      // 1
};

constexpr int kLossBlocks = 512;

size_t train_bytes(int n, int H, int W) {
  Carver cv(nullptr, ~size_t(0));
  const size_t px = static_cast<size_t>(n) * H * W;
  carve_fwd(cv, n, H, W, true);
  cv.take<float>(3 * px);
  cv.take<uint16_t>(px * 8);
  cv.take<uint16_t>(px * 32);
  cv.take<uint16_t>(px * 32);
  cv.take<float>(static_cast<size_t>(wgrad_blocks(H, W, n)) * (9 * 1024 + 32));
  cv.take<double>(kLossBlocks);
  cv.take<double>(1);
  return cv.used();
}

TrainBufs carve_train(void* ws, int n, int H, int W) {
  Carver cv(ws, ~size_t(0));
  const size_t px = static_cast<size_t>(n) * H * W;
  TrainBufs b{};
  b.f = carve_fwd(cv, n, H, W, true);
  b.y = cv.take<float>(3 * px);
  b.g8 = cv.take<uint16_t>(px * 8);
  b.ga = cv.take<uint16_t>(px * 32);
  b.gb = cv.take<uint16_t>(px * 32);
  b.part = cv.take<float>(static_cast<size_t>(wgrad_blocks(H, W, n)) * (9 * 1024 + 32));
  b.lpart = cv.take<double>(kLossBlocks);
  b.loss = cv.take<double>(1);
  return b;
}

template <int CIN, int COUT>
int wgrad_layer(const uint16_t* h, const uint16_t* g, int n, int H, int W, float* part, int cin, int cout,
                float* grad, hipStream_t s) {
  const int nb = wgrad_blocks(H, W, n);
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(nb), dim3(NT), 0, s, h, g, H, W, n, part);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((9 * 1024 + 32 + NT - 1) / NT), dim3(NT), 0, s, part, nb, cin, cout, grad);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

// Forward, loss and backward: fills st->grad and b.loss (sum of squares).
int forward_backward(CnnState* st, const TrainBufs& b, int n, int H, int W, const float* I, const float* t,
                     const float* A, const float* target, hipStream_t s) {
  int rc;
  const size_t plane = static_cast<size_t>(H) * W;
  if ((rc = features(I, W, plane, 3 * plane, t, W, plane, A, n, H, W, b.f.x8, s))) return rc;
  if ((rc = forward(st, b.f, n, H, W, b.y, W, 3 * plane, s))) return rc;
  const double count = 3.0 * static_cast<double>(n) * plane;
  const float gscale = static_cast<float>(2.0 * kCnnOutScale / count);
  hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(NT), 0, s, b.y, target, H, W, n, gscale, b.g8, b.lpart);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(NT), 0, s, b.lpart, kLossBlocks, b.loss);
  DZ_CHECK_LAUNCH();
  // layer 6: gradient wrt its weights, then wrt h5 (masked by h5 > 0)
  if ((rc = wgrad_layer<32, 8>(b.f.h[4], b.g8, n, H, W, b.part, 32, 3, st->grad + cnn_param_offset(5), s))) return rc;
  if ((rc = launch_conv<8, kMaskBf16>(b.g8, H, W, n, st->wd[5], nullptr, b.ga, b.f.h[4], nullptr, 0.f, 0, 0, 0, s)))
    return rc;
  uint16_t* gcur = b.ga;
  uint16_t* gnext = b.gb;
  for (int l = 4; l >= 1; --l) {
    if ((rc = wgrad_layer<32, 32>(b.f.h[l - 1], gcur, n, H, W, b.part, 32, 32, st->grad + cnn_param_offset(l), s)))
      return rc;
    if ((rc = launch_conv<32, kMaskBf16>(gcur, H, W, n, st->wd[l], nullptr, gnext, b.f.h[l - 1], nullptr, 0.f, 0, 0,
                                         0, s)))
      return rc;
    std::swap(gcur, gnext);
  }
  return wgrad_layer<8, 32>(b.f.x8, gcur, n, H, W, b.part, 7, 32, st->grad + cnn_param_offset(0), s);
}

}  // namespace

int cnn_set_weights(Ctx& ctx, const float* host_w, size_t count, hipStream_t s) {
  if (count != cnn_param_count()) {
    set_error("expected %zu network parameters, got %zu", cnn_param_count(), count);
    return DEHAZE_EINVAL;
  }
  int rc;
  if ((rc = ensure_state(ctx))) return rc;
  CnnState* st = ctx.cnn;
  DZ_HIP(hipMemcpyAsync(st->master, host_w, count * sizeof(float), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero, dim3((count + NT - 1) / NT), dim3(NT), 0, s, st->m, static_cast<int>(count));
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_zero, dim3((count + NT - 1) / NT), dim3(NT), 0, s, st->v, static_cast<int>(count));
  DZ_CHECK_LAUNCH();
  st->step = 0;
  if ((rc = repack(st, s))) return rc;
  DZ_HIP(hipStreamSynchronize(s));
  st->ready = true;
  return DEHAZE_OK;
}

int cnn_get_weights(Ctx& ctx, float* host_w, size_t count, hipStream_t s) {
  if (!ctx.cnn || !ctx.cnn->ready) { set_error("no network weights loaded"); return DEHAZE_EINVAL; }
  if (count != cnn_param_count()) { set_error("expected %zu parameters", cnn_param_count()); return DEHAZE_EINVAL; }
  DZ_HIP(hipMemcpyAsync(host_w, ctx.cnn->master, count * sizeof(float), hipMemcpyDeviceToHost, s));
  DZ_HIP(hipStreamSynchronize(s));
  return DEHAZE_OK;
}

bool cnn_ready(const Ctx& ctx) { return ctx.cnn && ctx.cnn->ready; }

size_t cnn_forward_bytes(int n, int H, int W) { return fwd_bytes(n, H, W, false); }

int cnn_forward(Ctx& ctx, int n, int H, int W, const float* I, int ip, size_t iplane, size_t iimg, const float* t,
                int tp, size_t timg, const float* A, float* out, int out_pitch, size_t out_img_stride, void* ws,
                hipStream_t s) {
  if (!cnn_ready(ctx)) { set_error("no network weights loaded"); return DEHAZE_EINVAL; }
  Carver cv(ws, ~size_t(0));
  FwdBufs b = carve_fwd(cv, n, H, W, false);
  int rc;
  if ((rc = features(I, ip, iplane, iimg, t, tp, timg, A, n, H, W, b.x8, s))) return rc;
  return forward(ctx.cnn, b, n, H, W, out, out_pitch, out_img_stride, s);
}

size_t cnn_train_bytes(int n, int H, int W) { return train_bytes(n, H, W); }

int cnn_grad(Ctx& ctx, int n, int H, int W, const float* I, const float* t, const float* A, const float* target,
             float* grad_out, double* loss, void* ws, hipStream_t s) {
  if (!cnn_ready(ctx)) { set_error("no network weights loaded"); return DEHAZE_EINVAL; }
  TrainBufs b = carve_train(ws, n, H, W);
  int rc;
  if ((rc = forward_backward(ctx.cnn, b, n, H, W, I, t, A, target, s))) return rc;
  if (grad_out)
    DZ_HIP(hipMemcpyAsync(grad_out, ctx.cnn->grad, cnn_param_count() * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (loss) {
    double h = 0.0;
    DZ_HIP(hipMemcpyAsync(&h, b.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    DZ_HIP(hipStreamSynchronize(s));
    *loss = h / (3.0 * static_cast<double>(n) * H * W);
  }
  return DEHAZE_OK;
}

int cnn_train_step(Ctx& ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                   const float* target, float lr, double* loss, void* ws, hipStream_t s) {
  int rc;
  if ((rc = cnn_grad(ctx, n, H, W, I, t, A, target, nullptr, nullptr, ws, s))) return rc;
  CnnState* st = ctx.cnn;
  st->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, static_cast<float>(st->step));
  const float c2 = 1.0f - std::pow(b2, static_cast<float>(st->step));
  const int np = static_cast<int>(cnn_param_count());
  hipLaunchKernelGGL(k_adam, dim3((np + NT - 1) / NT), dim3(NT), 0, s, st->master, st->grad, st->m, st->v, np, lr, b1,
                     b2, 1e-8f, c1, c2);
  DZ_CHECK_LAUNCH();
  if ((rc = repack(st, s))) return rc;
  if (loss) {
    TrainBufs b = carve_train(ws, n, H, W);
    double h = 0.0;
    DZ_HIP(hipMemcpyAsync(&h, b.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    DZ_HIP(hipStreamSynchronize(s));
    *loss = h / (3.0 * static_cast<double>(n) * H * W);
  }
  return DEHAZE_OK;
}

}  // namespace dz
