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

// lane i <- lane i - 1 (column x - 1); lane 0 receives 0 (bound_ctrl)
__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
// lane i <- lane i + 1 (column x + 1); lane 63 receives 0 (bound_ctrl)
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

template <int K, int MODE>
__global__ __launch_bounds__(256) void k_sweep_strip(const float* __restrict__ uin, float* __restrict__ uout,
                                                      const float* __restrict__ phi, const float* __restrict__ lam,
                                                      int H, int W, int P, int S, int ncols, int nwaves, OpConst oc) {
  // Contraction off and every fused multiply-add spelled out: the operation
  // sequence of an output value is then fixed, whatever K and S are.
#pragma clang fp contract(off)
  constexpr int OW = 64 - 4 * K;
  const int lane = threadIdx.x & 63;
  // the wavefront index is uniform: keep everything derived from it scalar
  const int gw = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (gw >= nwaves) return;  // uniform per wavefront
  const int c = gw % 3;
  const int rest = gw / 3;
  const int col = rest % ncols, strip = rest / ncols;
  const int x = col * OW - 2 * K + lane;
  const bool xin = x >= 0 && x < W;
  const int y0 = strip * S;
  const int r0 = y0 - 2 * K - 2;
  const int r1 = min(y0 + S, H) + 2 * K - 1;
  const bool out_lane = lane >= 2 * K && lane < 2 * K + OW && xin;
  const size_t plane = static_cast<size_t>(H) * P;
  const float* ui = uin + c * plane;
  const float* ph = phi + c * plane;
  float* uo = uout + c * plane;
  const float w0 = oc.w[2], w1 = oc.w[1], w2 = oc.w[0];
  const float eps = oc.eps;
  const float wc2 = oc.wc2;
  const bool nonlocal = oc.nonlocal_term != 0;
  const bool edge = oc.edge_preserving != 0;

  float U[K][4], SL[K][3], SR[K][3], GH[K][5], qT[K], DT[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
#pragma unroll
    for (int i = 0; i < 4; ++i) U[s][i] = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) SL[s][i] = SR[s][i] = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) GH[s][i] = 0.0f;
    qT[s] = DT[s] = 0.0f;
  }
  // Loads are unconditional from clamped addresses and then selected, so no
  // branch surrounds them and the compiler can keep PF rows in flight.
  const int xc = min(max(x, 0), W - 1);
  auto row_ok = [&](int r) -> bool { return r >= 0 && r < H; };
  auto addr = [&](int r) -> size_t { return static_cast<size_t>(min(max(r, 0), H - 1)) * P + xc; };
  // invalid lanes are zeroed with a bit mask (a select would be turned back
  // into a branch around the load)
  const int xmask = xin ? -1 : 0;
  auto masked = [&](float v, bool ok) -> float {
    return __builtin_bit_cast(float, __builtin_bit_cast(int, v) & (ok ? xmask : 0));
  };
  auto load_u = [&](int r) -> float { return masked(ui[addr(r)], row_ok(r)); };
  auto load_ph = [&](int j) -> float { return masked(ph[addr(j)], row_ok(j)); };
  auto load_lam = [&](int j) -> float { return masked(lam[addr(j)], nonlocal && row_ok(j)); };
  constexpr int PF = 4;  // rows in flight
  // Phi and lambda are loaded once per row, for the first sweep level (row
  // r - 2); level s uses the row of 2s steps earlier, kept in a delay line.
  constexpr int NH = 2 * (K - 1) + 1;
  float qv[PF], qph[PF], qla[PF];
  float hph[NH], hla[NH];
#pragma unroll
  for (int d = 0; d < NH; ++d) hph[d] = hla[d] = 0.0f;
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    qv[q] = load_u(r0 + q);
    qph[q] = load_ph(r0 + q - 2);
    qla[q] = load_lam(r0 + q - 2);
  }
  // the walk is padded to a multiple of PF; the extra rows are never stored
  const int nsteps = (r1 - r0 + 1 + PF - 1) / PF * PF;
  for (int rb = r0; rb < r0 + nsteps; rb += PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
    const int r = rb + q;
    float v = qv[q];
#pragma unroll
    for (int d = NH - 1; d > 0; --d) {
      hph[d] = hph[d - 1];
      hla[d] = hla[d - 1];
    }
    hph[0] = qph[q];
    hla[0] = qla[q];
    qv[q] = load_u(r + PF);
    qph[q] = load_ph(r + PF - 2);
    qla[q] = load_lam(r + PF - 2);
    float phc[K], lac[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      phc[s] = hph[2 * s];
      lac[s] = hla[2 * s];
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
      // level s + 1 receives row j + 2 of level s and produces row j
      const int j = r - 2 * (s + 1);
      const float sl1 = from_left(v), sr1 = from_right(v);
      const float sl2 = from_left(sl1), sr2 = from_right(sr1);
      const float ghn = __builtin_fmaf(w2, sl2 + sr2, __builtin_fmaf(w1, sl1 + sr1, w0 * v));
      U[s][0] = U[s][1]; U[s][1] = U[s][2]; U[s][2] = U[s][3]; U[s][3] = v;
      SL[s][0] = SL[s][1]; SL[s][1] = SL[s][2]; SL[s][2] = sl1;
      SR[s][0] = SR[s][1]; SR[s][1] = SR[s][2]; SR[s][2] = sr1;
      GH[s][0] = GH[s][1]; GH[s][1] = GH[s][2]; GH[s][2] = GH[s][3]; GH[s][3] = GH[s][4]; GH[s][4] = ghn;
      const float u0 = U[s][1];
      const float G = __builtin_fmaf(w2, GH[s][0] + GH[s][4], __builtin_fmaf(w1, GH[s][1] + GH[s][3], w0 * GH[s][2]));
      // face right of (x, j): normal u(x+1) - u(x), tangential at this cell
      const float gnx = SR[s][0] - u0;
      const float gtx = 0.5f * (U[s][2] - U[s][0]);
      const float DR =
          edge ? __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(__builtin_fmaf(gnx, gnx, gtx * gtx)) + eps) : 1.0f;
      const float qR = DR * gnx;
      const float DL = from_left(DR), qL = from_left(qR);
      // face below (x, j): normal u(j+1) - u(j), tangential at this cell
      const float gny = U[s][2] - u0;
      const float gty = 0.5f * (SR[s][0] - SL[s][0]);
      const float DB =
          edge ? __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(__builtin_fmaf(gny, gny, gty * gty)) + eps) : 1.0f;
      const float qB = DB * gny;
      const float div = (qR - qL) + (qB - qT[s]);
      const float r_ = phc[s] - __builtin_fmaf(lac[s], G, -div);
      float out;
      if (MODE == kExplicit) {
        out = __builtin_fmaf(oc.tau, r_, u0);
      } else {
        const float d = __builtin_fmaf(lac[s], wc2, (DL + DR) + (DT[s] + DB));
        out = __builtin_fmaf(oc.theta * r_, __builtin_amdgcn_rcpf(d), u0);
      }
      qT[s] = qB;
      DT[s] = DB;
      out = masked(out, j >= 0 && j < H);  // ghost cells stay zero
      if (s == K - 1 && out_lane && j >= y0 && j < y0 + S && j < H) uo[static_cast<size_t>(j) * P + x] = out;
      v = out;
    }
    }
  }
}

template <int K>
int launch_strip_k(int mode, const float* uin, float* uout, const float* phi, const float* lam, int H, int W, int P,
                   int S, const OpConst& c, hipStream_t s) {
  constexpr int OW = 64 - 4 * K;
  const int ncols = (W + OW - 1) / OW;
  const int nstrips = (H + S - 1) / S;
  const int nwaves = 3 * ncols * nstrips;
  dim3 grid((nwaves + 3) / 4);
  if (mode == kExplicit)
    hipLaunchKernelGGL((k_sweep_strip<K, kExplicit>), grid, dim3(256), 0, s, uin, uout, phi, lam, H, W, P, S, ncols,
                       nwaves, c);
  else
    hipLaunchKernelGGL((k_sweep_strip<K, kJacobi>), grid, dim3(256), 0, s, uin, uout, phi, lam, H, W, P, S, ncols,
                       nwaves, c);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace

int launch_sweep_strip(int mode, int K, int S, const float* uin, float* uout, const float* phi, const float* lam,
                       int H, int W, int P, const OpConst& c, hipStream_t s) {
  if (c.R != 2 || S < 1 || (mode != kExplicit && mode != kJacobi)) {
    set_error("strip sweep needs R = 2, S >= 1 and an update mode");
    return DEHAZE_EINVAL;
  }
  switch (K) {
    case 1: return launch_strip_k<1>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 2: return launch_strip_k<2>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 3: return launch_strip_k<3>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    case 4: return launch_strip_k<4>(mode, uin, uout, phi, lam, H, W, P, S, c, s);
    default: set_error("sweeps per launch %d outside 1..4", K); return DEHAZE_EINVAL;
  }
}

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
