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

// Buffer resource of one plane: the row offset then travels in a scalar
// register and the lane's column offset is fixed, so no per-load address
// arithmetic is left in the vector ALU.  Word 3 is the gfx9-family default
// (32-bit dwords, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, static_cast<int>(bytes), 0x00020000);
}

// out where the lane's bit of `live` is set, else 0 (one v_cndmask)
__device__ __forceinline__ float keep_lanes(float out, unsigned long long live) {
  float r;
  asm volatile("v_cndmask_b32 %0, 0, %1, %2" : "=v"(r) : "v"(out), "s"(live));
  return r;
}

// Register state of one sweep level: windows over the last four rows it
// received (rows j-2 .. j+1 when it is about to produce row j), the flux and
// coefficient of the face above row j, and its Phi / lambda prefetch rings.
template <int PF>
struct StripLevel {
  float U[4], SL[4], SR[4], GH[4];
  float qT, DT;
  float ph[PF], la[PF];
};

struct StripConst {
  float w0, w1, w2, eps, wc2, theta, tau;
};

// Face coefficient 1 / (|(gn, gt)| + eps) of Appendix A-2, or 1 without edge
// preservation.
template <bool EDGE>
__device__ __forceinline__ float strip_face(float gn, float gt, float eps) {
  return EDGE ? __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(__builtin_fmaf(gn, gn, gt * gt)) + eps) : 1.0f;
}

// One row step of level L: takes the level's input row v (row j + 2), shifts
// the windows and, when ACTIVE, returns the updated value of row j.  FIRST
// marks the level's first active row, whose top face is formed from the
// windows instead of the previous row.
template <int MODE, bool EDGE, bool ACTIVE, bool FIRST, int PF>
__device__ __forceinline__ float strip_level(StripLevel<PF>& L, float v, int q, const StripConst& k) {
#pragma clang fp contract(off)
  const float sl1 = from_left(v), sr1 = from_right(v);
  const float sl2 = from_left(sl1), sr2 = from_right(sr1);
  const float ghn = __builtin_fmaf(k.w2, sl2 + sr2, __builtin_fmaf(k.w1, sl1 + sr1, k.w0 * v));
  float out = 0.0f;
  if (ACTIVE) {
    const float up = L.U[1], u0 = L.U[2], dn = L.U[3];
    if (FIRST) {
      const float gny_t = u0 - up;
      const float gty_t = 0.5f * (L.SR[1] - L.SL[1]);
      L.DT = strip_face<EDGE>(gny_t, gty_t, k.eps);
      L.qT = L.DT * gny_t;
    }
    const float G = __builtin_fmaf(k.w2, L.GH[0] + ghn, __builtin_fmaf(k.w1, L.GH[1] + L.GH[3], k.w0 * L.GH[2]));
    // face right of (x, j): normal u(x+1) - u(x), tangential at this cell
    const float gnx = L.SR[2] - u0;
    const float gtx = 0.5f * (dn - up);
    const float DR = strip_face<EDGE>(gnx, gtx, k.eps);
    const float qR = DR * gnx;
    const float DL = from_left(DR), qL = from_left(qR);
    // face below (x, j): normal u(j+1) - u(j), tangential at this cell
    const float gny = dn - u0;
    const float gty = 0.5f * (L.SR[2] - L.SL[2]);
    const float DB = strip_face<EDGE>(gny, gty, k.eps);
    const float qB = DB * gny;
    const float div = (qR - qL) + (qB - L.qT);
    const float phc = L.ph[q], lac = L.la[q];
    const float r_ = phc - __builtin_fmaf(lac, G, -div);
    if (MODE == kExplicit) {
      out = __builtin_fmaf(k.tau, r_, u0);
    } else {
      const float d = __builtin_fmaf(lac, k.wc2, (DL + DR) + (L.DT + DB));
      out = __builtin_fmaf(k.theta * r_, __builtin_amdgcn_rcpf(d), u0);
    }
    L.qT = qB;
    L.DT = DB;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    L.U[i] = L.U[i + 1];
    L.SL[i] = L.SL[i + 1];
    L.SR[i] = L.SR[i + 1];
    L.GH[i] = L.GH[i + 1];
  }
  L.U[3] = v;
  L.SL[3] = sl1;
  L.SR[3] = sr1;
  L.GH[3] = ghn;
  return out;
}

// Sweep level s lags level s - 1 by two rows and must produce rows
// [y0 - 2(K-1-s), y1 - 1 + 2(K-1-s)].  The walk starts at input row
// y0 - 2K; level s is first active at step 4 + 4s, so in head block b
// (steps 4b .. 4b+3, b = 0..K) levels 0 .. b-1 are active, and after the
// head every level is.  The walk ends with the last level at row y1 - 1.
// Rows of the earlier levels beyond their range are computed and unused.
template <int K, int MODE, bool EDGE>
__global__ __launch_bounds__(256) void k_sweep_strip(const float* __restrict__ uin, float* __restrict__ uout,
                                                      const float* __restrict__ phi, const float* __restrict__ lam,
                                                      int H, int W, int P, int S, int ncols, int nwaves, OpConst oc) {
#pragma clang fp contract(off)
  constexpr int OW = 64 - 4 * K;
  constexpr int PF = 4;  // rows in flight; also the unroll of the walk
  const int lane = threadIdx.x & 63;
  // the wavefront index is uniform: keep everything derived from it scalar
  const int gw = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (gw >= nwaves) return;  // uniform per wavefront
  const int c = gw % 3;
  const int rest = gw / 3;
  const int col = rest % ncols, strip = rest / ncols;
  const int x = col * OW - 2 * K + lane;
  const bool xin = x >= 0 && x < W;
  const unsigned long long live = __builtin_amdgcn_ballot_w64(xin);
  const int y0 = strip * S;
  const int y1 = min(y0 + S, H);
  const int rs = y0 - 2 * K;  // first input row of the walk
  const bool out_lane = lane >= 2 * K && lane < 2 * K + OW && xin;
  const unsigned plane_bytes = static_cast<unsigned>(H) * P * 4u;
  const size_t plane = static_cast<size_t>(H) * P;
  const __amdgpu_buffer_rsrc_t ru = plane_rsrc(uin + c * plane, plane_bytes);
  const __amdgpu_buffer_rsrc_t rp = plane_rsrc(phi + c * plane, plane_bytes);
  const __amdgpu_buffer_rsrc_t rl = plane_rsrc(lam, plane_bytes);
  const __amdgpu_buffer_rsrc_t ro = plane_rsrc(uout + c * plane, plane_bytes);
  const int voff = min(max(x, 0), W - 1) * 4;
  StripConst k;
  // without the nonlocal term every Gaussian weight is zero, so lambda G(u)
  // and its diagonal vanish
  const bool nl = oc.nonlocal_term != 0;
  k.w0 = nl ? oc.w[2] : 0.0f;
  k.w1 = nl ? oc.w[1] : 0.0f;
  k.w2 = nl ? oc.w[0] : 0.0f;
  k.wc2 = nl ? oc.wc2 : 0.0f;
  k.eps = oc.eps;
  k.theta = oc.theta;
  k.tau = oc.tau;

  // Loads are unconditional from clamped rows; u of a row or column outside
  // the image is zeroed with a bit mask (a select would be turned back into a
  // branch around the load).  Phi and lambda need no mask: every value
  // computed from them for a ghost cell is masked before it is used.
  auto soff = [&](int r) { return min(max(r, 0), H - 1) * P * 4; };
  // u of a row or column outside the image is zeroed when it is consumed
  auto load_u = [&](int r) -> float {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ru, voff, soff(r), 0));
  };
  auto load_f = [&](__amdgpu_buffer_rsrc_t rs_, int j) -> float {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_, voff, soff(j), 0));
  };

  StripLevel<PF> lv[K];
  float qv[PF];
#pragma unroll
  for (int s = 0; s < K; ++s) {
#pragma unroll
    for (int i = 0; i < 4; ++i) lv[s].U[i] = lv[s].SL[i] = lv[s].SR[i] = lv[s].GH[i] = 0.0f;
    lv[s].qT = lv[s].DT = 0.0f;
  }
  // step r serves level s with Phi / lambda of row r - 2(s + 1)
#pragma unroll
  for (int q = 0; q < PF - 1; ++q) {
    qv[q] = load_u(rs + q);
#pragma unroll
    for (int s = 0; s < K; ++s) {
      lv[s].ph[q] = load_f(rp, rs + q - 2 * (s + 1));
      lv[s].la[q] = load_f(rl, rs + q - 2 * (s + 1));
    }
  }

  // One row step; levels >= NACT only shift their windows.  Outputs of
  // levels below K - 1 feed the next level and are zeroed outside the image;
  // the last level stores rows [y0, y1) of its own lanes.
  auto step = [&](auto nact_c, auto first_c, int r, int q) {
    constexpr int NACT = decltype(nact_c)::value;
    constexpr int FIRSTLV = decltype(first_c)::value;  // level whose first row this is, or -1
    float v = keep_lanes(qv[q], (r >= 0 && r < H) ? live : 0ull);
    qv[(q + PF - 1) % PF] = load_u(r + PF - 1);
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int j = r - 2 * (s + 1);
      float out;
      if (s < NACT) {
        if (s == FIRSTLV) out = strip_level<MODE, EDGE, true, true>(lv[s], v, q, k);
        else out = strip_level<MODE, EDGE, true, false>(lv[s], v, q, k);
      } else {
        out = strip_level<MODE, EDGE, false, false>(lv[s], v, q, k);
      }
      lv[s].ph[(q + PF - 1) % PF] = load_f(rp, r + PF - 1 - 2 * (s + 1));
      lv[s].la[(q + PF - 1) % PF] = load_f(rl, r + PF - 1 - 2 * (s + 1));
      if (s < NACT) {
        if (s < K - 1) {
          out = keep_lanes(out, (j >= 0 && j < H) ? live : 0ull);
        } else if (j >= y0 && j < y1) {
          if (out_lane) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, out), ro, voff, j * P * 4, 0);
        }
      }
      v = out;
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

template <int K, bool EDGE>
void launch_strip_ke(int mode, dim3 grid, const float* uin, float* uout, const float* phi, const float* lam, int H,
                     int W, int P, int S, int ncols, int nwaves, const OpConst& c, hipStream_t s) {
  if (mode == kExplicit)
    hipLaunchKernelGGL((k_sweep_strip<K, kExplicit, EDGE>), grid, dim3(256), 0, s, uin, uout, phi, lam, H, W, P, S,
                       ncols, nwaves, c);
  else
    hipLaunchKernelGGL((k_sweep_strip<K, kJacobi, EDGE>), grid, dim3(256), 0, s, uin, uout, phi, lam, H, W, P, S,
                       ncols, nwaves, c);
}

template <int K>
int launch_strip_k(int mode, const float* uin, float* uout, const float* phi, const float* lam, int H, int W, int P,
                   int S, const OpConst& c, hipStream_t s) {
  constexpr int OW = 64 - 4 * K;
  const int ncols = (W + OW - 1) / OW;
  const int nstrips = (H + S - 1) / S;
  const int nwaves = 3 * ncols * nstrips;
  dim3 grid((nwaves + 3) / 4);
  if (c.edge_preserving)
    launch_strip_ke<K, true>(mode, grid, uin, uout, phi, lam, H, W, P, S, ncols, nwaves, c, s);
  else
    launch_strip_ke<K, false>(mode, grid, uin, uout, phi, lam, H, W, P, S, ncols, nwaves, c, s);
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
  if (!strip_fits(H, P)) {
    set_error("plane of %d x %d elements exceeds the strip kernel's 32-bit byte offsets", H, P);
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

}  // namespace dz
