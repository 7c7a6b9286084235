// The sweep: one application of the discrete operator of the main PDE,
//
//   L_{D(u)} u = -div(D(grad u) grad u) + lambda G(u),
//
// fused with the update of Appendix A-1 (explicit relaxation u += tau r) or
// its diagonally scaled form (u += theta r / d), where r = Phi - L_{D(u)} u.
// Face coefficients follow Appendix A-2: on the face between cell (i, j) and
// its right neighbour, D = 1 / (sqrt(gn^2 + gt^2) + eps) with the forward
// normal difference gn and the central tangential difference gt at the
// lower-index cell; u is zero outside the image (H0^1).  G is the (2R+1)^2
// Gaussian applied separably, zero outside the image (Section II-C).
//
// Layout: planar float32 planes with a row pitch of P elements.  One
// workgroup owns a 64 x 16 output tile of all three channels; for each
// channel it stages the tile plus a halo of max(R, 1) in LDS, computes the
// horizontal Gaussian pass and every face flux of the tile once, then forms
// the update.  The workload is bound by HBM traffic (40 bytes per RGB pixel:
// read u, Phi, lambda, write u); the operator itself never touches HBM.
#include <cmath>

#include "internal.hpp"

namespace dz {

OpConst make_opconst(const dehaze_params& p) {
  OpConst c{};
  const int R = p.g_radius;
  double s = 0.0;
  double g[9];
  for (int a = -R; a <= R; ++a) {
    g[a + R] = std::exp(-(a * a) / (2.0 * p.sigma * p.sigma));
    s += g[a + R];
  }
  for (int a = 0; a < 2 * R + 1; ++a) c.w[a] = static_cast<float>(g[a] / s);
  c.wc2 = static_cast<float>((g[R] / s) * (g[R] / s));
  c.eps = static_cast<float>(p.eps);
  c.theta = static_cast<float>(p.theta);
  c.tau = static_cast<float>(p.tau);
  c.R = R;
  c.nonlocal_term = p.nonlocal_term;
  c.edge_preserving = p.edge_preserving;
  return c;
}

namespace {

constexpr int kTX = 64;
constexpr int kTY = 16;
constexpr int kThreads = 256;
constexpr int kPix = kTX * kTY / kThreads;  // output pixels per thread per channel

__device__ __forceinline__ float face_d(float gn, float gt, float eps, int edge) {
  return edge ? __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(gn * gn + gt * gt) + eps) : 1.0f;
}

template <int R, int MODE>
__global__ __launch_bounds__(kThreads) void k_sweep(const float* __restrict__ uin, float* __restrict__ uout,
                                                     const float* __restrict__ phi,
                                                     const float* __restrict__ lam, int H, int W, int P,
                                                     OpConst oc, double* __restrict__ partials) {
  constexpr int HALO = R > 1 ? R : 1;
  constexpr int SX = kTX + 2 * HALO;
  constexpr int SY = kTY + 2 * HALO;
  __shared__ float us[SY][SX];
  __shared__ float gh[kTY + 2 * R][kTX];
  __shared__ float qx[kTY][kTX + 1];
  __shared__ float dxs[kTY][kTX + 1];
  __shared__ float qy[kTY + 1][kTX];
  __shared__ float dys[kTY + 1][kTX];
  __shared__ double red[2][kThreads / 64];

  const int x0 = blockIdx.x * kTX;
  const int y0 = blockIdx.y * kTY;
  const int tid = threadIdx.x;
  const int tx = tid & (kTX - 1);
  const int ty = tid / kTX;
  const int gx = x0 + tx;
  const size_t plane = static_cast<size_t>(H) * P;

  float lv[kPix];
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    const int gy = y0 + ty + (kThreads / kTX) * k;
    lv[k] = (oc.nonlocal_term && gx < W && gy < H) ? lam[static_cast<size_t>(gy) * P + gx] : 0.0f;
  }
  float w[2 * R + 1];
#pragma unroll
  for (int a = 0; a < 2 * R + 1; ++a) w[a] = oc.w[a];

  double rr = 0.0, pp = 0.0;
  for (int c = 0; c < 3; ++c) {
    const float* ui = uin + c * plane;
    for (int i = tid; i < SY * SX; i += kThreads) {
      const int ly = i / SX, lx = i - (i / SX) * SX;
      const int yy = y0 - HALO + ly, xx = x0 - HALO + lx;
      us[ly][lx] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? ui[static_cast<size_t>(yy) * P + xx] : 0.0f;
    }
    __syncthreads();
    if (oc.nonlocal_term) {
      for (int i = tid; i < (kTY + 2 * R) * kTX; i += kThreads) {
        const int j = i / kTX, lx = i - (i / kTX) * kTX;
        const float* row = &us[HALO - R + j][HALO + lx - R];
        float s = 0.0f;
#pragma unroll
        for (int a = 0; a < 2 * R + 1; ++a) s += w[a] * row[a];
        gh[j][lx] = s;
      }
    }
    for (int i = tid; i < kTY * (kTX + 1); i += kThreads) {
      const int ly = i / (kTX + 1), f = i - (i / (kTX + 1)) * (kTX + 1);
      const int cy = HALO + ly, cx = HALO + f - 1;  // lower-index cell of the face
      const float gn = us[cy][cx + 1] - us[cy][cx];
      const float gt = 0.5f * (us[cy + 1][cx] - us[cy - 1][cx]);
      const float D = face_d(gn, gt, oc.eps, oc.edge_preserving);
      qx[ly][f] = D * gn;
      dxs[ly][f] = D;
    }
    for (int i = tid; i < (kTY + 1) * kTX; i += kThreads) {
      const int f = i / kTX, lx = i - (i / kTX) * kTX;
      const int cy = HALO + f - 1, cx = HALO + lx;
      const float gn = us[cy + 1][cx] - us[cy][cx];
      const float gt = 0.5f * (us[cy][cx + 1] - us[cy][cx - 1]);
      const float D = face_d(gn, gt, oc.eps, oc.edge_preserving);
      qy[f][lx] = D * gn;
      dys[f][lx] = D;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
      const int ly = ty + (kThreads / kTX) * k;
      const int gy = y0 + ly;
      const float div = (qx[ly][tx + 1] - qx[ly][tx]) + (qy[ly + 1][tx] - qy[ly][tx]);
      float G = 0.0f;
      if (oc.nonlocal_term) {
#pragma unroll
        for (int b = 0; b < 2 * R + 1; ++b) G += w[b] * gh[ly + b][tx];
      }
      const float u = us[HALO + ly][HALO + tx];
      if (gx < W && gy < H) {
        const size_t e = c * plane + static_cast<size_t>(gy) * P + gx;
        const float ph = phi[e];
        const float r = ph - (lv[k] * G - div);
        float out;
        if (MODE == kExplicit) {
          out = u + oc.tau * r;
        } else if (MODE == kJacobi) {
          const float d = (dxs[ly][tx] + dxs[ly][tx + 1]) + (dys[ly][tx] + dys[ly + 1][tx]) + lv[k] * oc.wc2;
          out = u + oc.theta * r * __builtin_amdgcn_rcpf(d);
        } else {
          out = r;
        }
        if (uout) uout[e] = out;
        rr += static_cast<double>(r) * r;
        pp += static_cast<double>(ph) * ph;
      }
    }
    __syncthreads();
  }
  if (partials) {
    for (int off = 32; off > 0; off >>= 1) {
      rr += __shfl_down(rr, off, 64);
      pp += __shfl_down(pp, off, 64);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = rr;
      red[1][tid >> 6] = pp;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int i = 0; i < kThreads / 64; ++i) {
        a += red[0][i];
        b += red[1][i];
      }
      const size_t blk = static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x;
      partials[2 * blk] = a;
      partials[2 * blk + 1] = b;
    }
  }
}

__global__ __launch_bounds__(256) void k_reduce_pairs(const double* __restrict__ in, int n, double* out) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    a += in[2 * i];
    b += in[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

template <int R>
int launch_sweep_r(int mode, const float* uin, float* uout, const float* phi, const float* lam, int H,
                   int W, int P, const OpConst& c, double* partials, hipStream_t s) {
  dim3 grid((W + kTX - 1) / kTX, (H + kTY - 1) / kTY);
  switch (mode) {
    case kExplicit:
      hipLaunchKernelGGL((k_sweep<R, kExplicit>), grid, dim3(kThreads), 0, s, uin, uout, phi, lam, H, W, P, c,
                         partials);
      break;
    case kJacobi:
      hipLaunchKernelGGL((k_sweep<R, kJacobi>), grid, dim3(kThreads), 0, s, uin, uout, phi, lam, H, W, P, c,
                         partials);
      break;
    default:
      hipLaunchKernelGGL((k_sweep<R, kResidual>), grid, dim3(kThreads), 0, s, uin, uout, phi, lam, H, W, P, c,
                         partials);
      break;
  }
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace

int sweep_num_blocks(int H, int W) { return ((W + kTX - 1) / kTX) * ((H + kTY - 1) / kTY); }

int launch_sweep(int mode, const float* uin, float* uout, const float* phi, const float* lam, int H, int W,
                 int P, const OpConst& c, double* partials, hipStream_t s) {
  switch (c.R) {
    case 0: return launch_sweep_r<0>(mode, uin, uout, phi, lam, H, W, P, c, partials, s);
    case 1: return launch_sweep_r<1>(mode, uin, uout, phi, lam, H, W, P, c, partials, s);
    case 2: return launch_sweep_r<2>(mode, uin, uout, phi, lam, H, W, P, c, partials, s);
    case 3: return launch_sweep_r<3>(mode, uin, uout, phi, lam, H, W, P, c, partials, s);
    case 4: return launch_sweep_r<4>(mode, uin, uout, phi, lam, H, W, P, c, partials, s);
    default: set_error("g_radius %d outside 0..4", c.R); return DEHAZE_EINVAL;
  }
}

int launch_reduce_pairs(const double* partials, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, s, partials, n, out);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace dz
