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
#include <utility>

#include "internal.hpp"
#include "wave.hpp"

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

// rho = ||r|| / ||Phi|| from the two sums (sum r^2, sum Phi^2); the norm of r
// alone when Phi vanishes.  Correctly rounded float64 square roots and
// division, as on the host.
__global__ void k_rho_from_sums(const double* __restrict__ sums, double* __restrict__ rho) {
  if (threadIdx.x == 0) {
    const double a = sums[0], b = sums[1];
    rho[0] = b > 0.0 ? sqrt(a) / sqrt(b) : sqrt(a);
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

// ------------------------------------------------------------ strip kernel
// Register-resident sweeps for the 5x5 Gaussian (R = 2).  Each wavefront owns
// one colour channel of a 64-column group and walks down a strip of S output
// rows.  Lane l holds column x0 - 2K + l; horizontal neighbours arrive through
// wavefront-wide DPP shifts, vertical ones through per-row register windows,
// so the kernel touches no LDS and needs no barrier.  K sweeps are pipelined
// in the same walk: sweep s consumes the rows sweep s-1 produced two rows
// earlier, so one launch reads u, Phi and lambda once and writes u once for K
// sweeps.  Each sweep leaves 2 more lanes on either side without valid
// neighbours, so a wave produces 64 - 4K output columns; the first rows of a
// strip warm the windows up.  Floating-point contraction is off in this
// kernel and every fused multiply-add is explicit, so an output value is
// computed by the same operation sequence whatever K and S are: the results
// do not depend on the launch shape the tuner picks.

// Register state of one sweep level, per column c of the lane: windows over
// the last four rows it received (rows j-2 .. j+1 when it is about to
// produce row j) of u, of its left and right neighbours and of the
// horizontal Gaussian pass; the flux and coefficient of the face above row
// j; and its Phi / lambda prefetch rings.
template <int C, int PF>
struct StripLevel {
  float U[C][4], SL[C][4], SR[C][4], GH[C][4];
  float qT[C], DT[C];
  float ph[C][PF], la[C][PF];
};

// fs, feps, fone: the face coefficient is formed as 1 / (fs |g| + feps), or
// fone without edge preservation.  The explicit update takes fs = fone = 1,
// feps = eps, i.e. D itself.  The Jacobi update takes D / theta (fs = theta,
// feps = theta eps, fone = 1 / theta) and wc2 / theta, which folds the
// damping into the diagonal: theta r / d = (Phi - lambda G + theta div') / d'
// with div' and d' formed from D / theta.
struct StripConst {
  float w0, w1, w2, wc2, theta, tau;
  float fs, feps, fone;
};

// Face coefficient 1 / (|(gn, gt)| + eps) of Appendix A-2 (scaled as above),
// or its value without edge preservation.
template <bool EDGE>
__device__ __forceinline__ float strip_face(float gn, float gt, const StripConst& k) {
  return EDGE ? __builtin_amdgcn_rcpf(__builtin_fmaf(k.fs, __builtin_amdgcn_sqrtf(__builtin_fmaf(gn, gn, gt * gt)), k.feps))
              : k.fone;
}

// Values at column offset d (-2..2) of every column of the lane: columns
// c + d inside the lane are registers, the others come from the neighbouring
// lane (one shift, or two when a lane holds a single column).
template <int C>
struct Shifted {
  float l1[C], r1[C], l2[C], r2[C];
  __device__ __forceinline__ explicit Shifted(const float (&v)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      l1[c] = from_left(v[c]);
      r1[c] = from_right(v[c]);
    }
    if (C == 1) {
      l2[0] = from_left(l1[0]);
      r2[0] = from_right(r1[0]);
    }
  }
  __device__ __forceinline__ float at(const float (&v)[C], int c, int d) const {
    const int sc = c + d;
    if (sc >= 0 && sc < C) return v[sc];
    if (sc < 0) return sc >= -C ? l1[sc + C] : l2[sc + 2 * C];
    return sc < 2 * C ? r1[sc - C] : r2[sc - 2 * C];
  }
};

// One row step of level L: takes the level's input row v (row j + 2, one
// value per column of the lane), shifts the windows and, when ACTIVE,
// returns the updated values of row j.  FIRST marks the level's first active
// row, whose top face is formed from the windows instead of the previous row.
template <int C, int MODE, bool EDGE, bool ACTIVE, bool FIRST, int PF>
__device__ __forceinline__ void strip_level(StripLevel<C, PF>& L, const float (&v)[C], float (&out)[C], int q,
                                            const StripConst& k) {
#pragma clang fp contract(off)
  const Shifted<C> sh(v);
  float ghn[C], sl1[C], sr1[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    sl1[c] = sh.at(v, c, -1);
    sr1[c] = sh.at(v, c, 1);
    ghn[c] = __builtin_fmaf(k.w2, sh.at(v, c, -2) + sh.at(v, c, 2), __builtin_fmaf(k.w1, sl1[c] + sr1[c], k.w0 * v[c]));
    out[c] = 0.0f;
  }
  if (ACTIVE) {
    float DR[C], qR[C], DB[C], qB[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float up = L.U[c][1], u0 = L.U[c][2], dn = L.U[c][3];
      if (FIRST) {
        const float gny_t = u0 - up;
        const float gty_t = 0.5f * (L.SR[c][1] - L.SL[c][1]);
        L.DT[c] = strip_face<EDGE>(gny_t, gty_t, k);
        L.qT[c] = L.DT[c] * gny_t;
      }
      // face right of (x, j): normal u(x+1) - u(x), tangential at this cell
      const float gnx = L.SR[c][2] - u0;
      const float gtx = 0.5f * (dn - up);
      DR[c] = strip_face<EDGE>(gnx, gtx, k);
      qR[c] = DR[c] * gnx;
      // face below (x, j): normal u(j+1) - u(j), tangential at this cell
      const float gny = dn - u0;
      const float gty = 0.5f * (L.SR[c][2] - L.SL[c][2]);
      DB[c] = strip_face<EDGE>(gny, gty, k);
      qB[c] = DB[c] * gny;
    }
    // the face left of column 0 is the right face of the left lane's last column
    const float DLx = from_left(DR[C - 1]), qLx = from_left(qR[C - 1]);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float u0 = L.U[c][2];
      const float DL = c > 0 ? DR[c - 1] : DLx, qL = c > 0 ? qR[c - 1] : qLx;
      const float G =
          __builtin_fmaf(k.w2, L.GH[c][0] + ghn[c], __builtin_fmaf(k.w1, L.GH[c][1] + L.GH[c][3], k.w0 * L.GH[c][2]));
      const float div = (qR[c] - qL) + (qB[c] - L.qT[c]);
      const float phc = L.ph[c][q], lac = L.la[c][q];
      if (MODE == kExplicit) {
        const float r_ = phc - __builtin_fmaf(lac, G, -div);
        out[c] = __builtin_fmaf(k.tau, r_, u0);
      } else {
        // theta r, with div and d formed from D / theta
        const float r_ = __builtin_fmaf(k.theta, div, __builtin_fmaf(-lac, G, phc));
        const float d = __builtin_fmaf(lac, k.wc2, (DL + DR[c]) + (L.DT[c] + DB[c]));
        out[c] = __builtin_fmaf(r_, __builtin_amdgcn_rcpf(d), u0);
      }
      L.qT[c] = qB[c];
      L.DT[c] = DB[c];
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      L.U[c][i] = L.U[c][i + 1];
      L.SL[c][i] = L.SL[c][i + 1];
      L.SR[c][i] = L.SR[c][i + 1];
      L.GH[c][i] = L.GH[c][i + 1];
    }
    L.U[c][3] = v[c];
    L.SL[c][3] = sl1[c];
    L.SR[c][3] = sr1[c];
    L.GH[c][3] = ghn[c];
  }
}

// Sweep level s lags level s - 1 by two rows and must produce rows
// [y0 - 2(K-1-s), y1 - 1 + 2(K-1-s)].  The walk starts at input row
// y0 - 2K; level s is first active at step 4 + 4s, so in head block b
// (steps 4b .. 4b+3, b = 0..K) levels 0 .. b-1 are active, and after the
// head every level is.  The walk ends with the last level at row y1 - 1.
// Rows of the earlier levels beyond their range are computed and unused.
// A lane holds C adjacent columns; a wavefront covers 64 C columns, of which
// 2K on either side are halo.
// Wavefronts per workgroup.  They share nothing; four (one per SIMD of a
// compute unit) measured faster than one per workgroup (127k against 120k
// Mpix-iters/s at 1024x1024).
constexpr int kStripWaves = 4;

template <int K, int C, int MODE, bool EDGE>
__global__ __launch_bounds__(64 * kStripWaves) void k_sweep_strip(const float* __restrict__ uin, float* __restrict__ uout,
                                                      const float* __restrict__ phi, const float* __restrict__ lam,
                                                      int H, int W, int P, int S, int ncols, int nwaves, OpConst oc) {
#pragma clang fp contract(off)
  constexpr int OW = 64 * C - 4 * K;
  constexpr int PF = 4;  // rows in flight; also the unroll of the walk
  const int lane = threadIdx.x & 63;
  // the wavefront index is uniform: keep everything derived from it scalar
  const int gw = blockIdx.x * kStripWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (gw >= nwaves) return;  // uniform per wavefront
  const int ch = gw % 3;
  const int rest = gw / 3;
  const int col = rest % ncols, strip = rest / ncols;
  const int x0 = col * OW - 2 * K + C * lane;  // column of the lane's first value
  const int y0 = strip * S;
  const int y1 = min(y0 + S, H);
  const int rs = y0 - 2 * K;  // first input row of the walk
  const unsigned plane_bytes = static_cast<unsigned>(H) * P * 4u;
  const size_t plane = static_cast<size_t>(H) * P;
  const __amdgpu_buffer_rsrc_t ru = plane_rsrc(uin + ch * plane, plane_bytes);
  const __amdgpu_buffer_rsrc_t rp = plane_rsrc(phi + ch * plane, plane_bytes);
  const __amdgpu_buffer_rsrc_t rl = plane_rsrc(lam, plane_bytes);
  const __amdgpu_buffer_rsrc_t ro = plane_rsrc(uout + ch * plane, plane_bytes);
  int voff[C];
  bool out_col[C];
  unsigned long long live[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int x = x0 + c;
    const bool xin = x >= 0 && x < W;
    voff[c] = min(max(x, 0), W - 1) * 4;
    live[c] = __builtin_amdgcn_ballot_w64(xin);
    out_col[c] = xin && x >= col * OW && x < (col + 1) * OW;
  }
  StripConst k;
  // without the nonlocal term every Gaussian weight is zero, so lambda G(u)
  // and its diagonal vanish
  const bool nl = oc.nonlocal_term != 0;
  k.w0 = nl ? oc.w[2] : 0.0f;
  k.w1 = nl ? oc.w[1] : 0.0f;
  k.w2 = nl ? oc.w[0] : 0.0f;
  k.theta = oc.theta;
  if (MODE == kJacobi) {
    k.fs = oc.theta;
    k.feps = oc.theta * oc.eps;
    k.fone = 1.0f / oc.theta;
    k.wc2 = nl ? oc.wc2 / oc.theta : 0.0f;
  } else {
    k.fs = 1.0f;
    k.feps = oc.eps;
    k.fone = 1.0f;
    k.wc2 = nl ? oc.wc2 : 0.0f;
  }
  k.tau = oc.tau;

  // Loads are unconditional from clamped rows and columns.  u of a row or
  // column outside the image is zeroed when it is consumed; Phi and lambda
  // need no mask, since every value computed from them for a ghost cell is
  // masked before it is used.
  auto soff = [&](int r) { return min(max(r, 0), H - 1) * P * 4; };
  auto load = [&](__amdgpu_buffer_rsrc_t rs_, int c, int row) -> float {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_, voff[c], soff(row), 0));
  };

  StripLevel<C, PF> lv[K];
  float qv[C][PF];
#pragma unroll
  for (int s = 0; s < K; ++s) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
      for (int i = 0; i < 4; ++i) lv[s].U[c][i] = lv[s].SL[c][i] = lv[s].SR[c][i] = lv[s].GH[c][i] = 0.0f;
      lv[s].qT[c] = lv[s].DT[c] = 0.0f;
    }
  }
  // step r serves level s with Phi / lambda of row r - 2(s + 1); a load
  // issued at step r fills the ring slot that step r + PF - 1 reads
#pragma unroll
  for (int q = 0; q < PF - 1; ++q) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      qv[c][q] = load(ru, c, rs + q);
#pragma unroll
      for (int s = 0; s < K; ++s) {
        lv[s].ph[c][q] = load(rp, c, rs + q - 2 * (s + 1));
        lv[s].la[c][q] = load(rl, c, rs + q - 2 * (s + 1));
      }
    }
  }

  // One row step: levels below NACT are active, level NACT only fills its
  // windows, the levels above it wait.  Outputs of levels below K - 1 feed
  // the next level and are zeroed outside the image; the last level stores
  // rows [y0, y1) of the lane's output columns.
  auto step = [&](auto nact_c, auto first_c, int r, int q) __attribute__((always_inline)) {
    constexpr int NACT = decltype(nact_c)::value;
    constexpr int FIRSTLV = decltype(first_c)::value;  // level whose first row this is, or -1
    const bool row_in = r >= 0 && r < H;
    float v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      v[c] = keep_lanes(qv[c][q], row_in ? live[c] : 0ull);
      qv[c][(q + PF - 1) % PF] = load(ru, c, r + PF - 1);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int j = r - 2 * (s + 1);
      float out[C];
      if (s < NACT) {
        if (s == FIRSTLV) strip_level<C, MODE, EDGE, true, true>(lv[s], v, out, q, k);
        else strip_level<C, MODE, EDGE, true, false>(lv[s], v, out, q, k);
      } else {
        if (s == NACT) strip_level<C, MODE, EDGE, false, false>(lv[s], v, out, q, k);
#pragma unroll
        for (int c = 0; c < C; ++c) out[c] = 0.0f;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        lv[s].ph[c][(q + PF - 1) % PF] = load(rp, c, r + PF - 1 - 2 * (s + 1));
        lv[s].la[c][(q + PF - 1) % PF] = load(rl, c, r + PF - 1 - 2 * (s + 1));
      }
      if (s < NACT) {
        if (s < K - 1) {
          const bool jin = j >= 0 && j < H;
#pragma unroll
          for (int c = 0; c < C; ++c) out[c] = keep_lanes(out[c], jin ? live[c] : 0ull);
        } else if (j >= y0 && j < y1) {
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (out_col[c])
              __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, out[c]), ro, voff[c], j * P * 4, 0);
        }
      }
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = out[c];
    }
  };
  // head: block b (0..K) has levels 0 .. b-1 active, level b-1 from its first
  // row on
  int r = rs;
  [&]<int... B>(std::integer_sequence<int, B...>) {
    (([&] {
       constexpr int b = B;
       step(std::integral_constant<int, b>{}, std::integral_constant<int, b - 1>{}, r, 0);
#pragma unroll
       for (int q = 1; q < PF; ++q) step(std::integral_constant<int, b>{}, std::integral_constant<int, -1>{}, r + q, q);
       r += PF;
     }()), ...);
  }(std::make_integer_sequence<int, K + 1>{});
  // body: every level active
  const int rend = y1 - 1 + 2 * K;  // last step: the last level at row y1 - 1
  for (; r <= rend; r += PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) step(std::integral_constant<int, K>{}, std::integral_constant<int, -1>{}, r + q, q);
  }
}

template <int K, int C, bool EDGE>
void launch_strip_ke(int mode, dim3 grid, const float* uin, float* uout, const float* phi, const float* lam, int H,
                     int W, int P, int S, int ncols, int nwaves, const OpConst& c, hipStream_t s) {
  if (mode == kExplicit)
    hipLaunchKernelGGL((k_sweep_strip<K, C, kExplicit, EDGE>), grid, dim3(64 * kStripWaves), 0, s, uin, uout, phi, lam, H, W, P,
                       S, ncols, nwaves, c);
  else
    hipLaunchKernelGGL((k_sweep_strip<K, C, kJacobi, EDGE>), grid, dim3(64 * kStripWaves), 0, s, uin, uout, phi, lam, H, W, P,
                       S, ncols, nwaves, c);
}

template <int K, int C>
int launch_strip_k(int mode, const float* uin, float* uout, const float* phi, const float* lam, int H, int W, int P,
                   int S, const OpConst& c, hipStream_t s) {
  constexpr int OW = 64 * C - 4 * K;
  const int ncols = (W + OW - 1) / OW;
  const int nstrips = (H + S - 1) / S;
  const int nwaves = 3 * ncols * nstrips;
  dim3 grid((nwaves + kStripWaves - 1) / kStripWaves);
  if (c.edge_preserving)
    launch_strip_ke<K, C, true>(mode, grid, uin, uout, phi, lam, H, W, P, S, ncols, nwaves, c, s);
  else
    launch_strip_ke<K, C, false>(mode, grid, uin, uout, phi, lam, H, W, P, S, ncols, nwaves, c, s);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace

int launch_sweep_strip(int mode, int K, int S, int C, const float* uin, float* uout, const float* phi,
                       const float* lam, int H, int W, int P, const OpConst& c, hipStream_t s) {
  if (c.R != 2 || S < 1 || (mode != kExplicit && mode != kJacobi) || (C != 1 && C != 2)) {
    set_error("strip sweep needs R = 2, S >= 1, 1 or 2 columns per lane and an update mode");
    return DEHAZE_EINVAL;
  }
  if (!strip_fits(H, P)) {
    set_error("plane of %d x %d elements exceeds the strip kernel's 32-bit byte offsets", H, P);
    return DEHAZE_EINVAL;
  }
  switch (K * 2 + (C - 1)) {
    case 2: return launch_strip_k<1, 1>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 3: return launch_strip_k<1, 2>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 4: return launch_strip_k<2, 1>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 5: return launch_strip_k<2, 2>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 6: return launch_strip_k<3, 1>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 7: return launch_strip_k<3, 2>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 8: return launch_strip_k<4, 1>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 9: return launch_strip_k<4, 2>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    default: set_error("sweeps per launch %d outside 1..4", K); return DEHAZE_EINVAL;
  }
}

bool strip_fits(int H, int P) { return static_cast<long long>(H) * P * 4 < (1LL << 31); }

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

int launch_rho_from_sums(const double* sums, double* rho, hipStream_t s) {
  hipLaunchKernelGGL(k_rho_from_sums, dim3(1), dim3(64), 0, s, sums, rho);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace dz
