// Front end of the method (Sections II-A and II-D): input conversion, the
// per-channel patch minimum (van Herk / Gil-Werman min filter, a row pass then
// a column pass), the raw dark channel, the dark-channel-prior airlight (a
// radix select of the top HW/divisor dark-channel values followed by an
// argmax of R+G+B), and the fused t_d / t / lambda / Phi kernel.
//
// Every value produced here is either an exact copy of an input value
// (minima, A) or a correctly rounded function of them (t_d through a float64
// quotient rounded once to float32; t, lambda, Phi evaluated in float64 and
// rounded once), so the results are reproducible bit for bit.
#include <cmath>

#include "internal.hpp"

namespace dz {

namespace {

// 8-bit code -> float32 intensity code / 255.  The float64 quotient rounded to
// float32 is the correctly rounded float32 quotient (53 >= 2 * 24 + 2).
__device__ __forceinline__ float u8_to_unit(uint32_t code) {
  return static_cast<float>(static_cast<double>(code) / 255.0);
}

__device__ __forceinline__ float load_input(const void* I, int dtype, int layout, int H, int pitch,
                                            int c, int y, int x) {
  const size_t idx = layout == DEHAZE_HWC ? (static_cast<size_t>(y) * pitch + x) * 3 + c
                                          : (static_cast<size_t>(c) * H + y) * pitch + x;
  if (dtype == DEHAZE_U8) return u8_to_unit(static_cast<const uint8_t*>(I)[idx]);
  return static_cast<const float*>(I)[idx];
}

// ------------------------------------------------------------ conversion
__global__ __launch_bounds__(256) void k_to_planar(const void* __restrict__ I, int dtype, int layout,
                                                    int H, int W, int pitch, float* __restrict__ Ip,
                                                    int P) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    Ip[(static_cast<size_t>(c) * H + y) * P + x] = load_input(I, dtype, layout, H, pitch, c, y, x);
}

// ------------------------------------------------------------ row pass
// One block per (row, 256-column segment).  The segment plus a halo of r
// columns each side is staged in LDS (+inf outside the image, so the window
// is clipped to the image), split into aligned runs of `patch` values, and
// each run gets its prefix minimum g and suffix minimum h.  The minimum over
// the window starting at local index q is min(h[q], g[q + patch - 1]): the
// window covers the tail of one run and the head of the next.
constexpr int kRowTile = 256;

__global__ __launch_bounds__(256) void k_rowmin(const void* __restrict__ I, int dtype, int layout,
                                                 int H, int W, int pitch, int patch,
                                                 float* __restrict__ Ip, float* __restrict__ mrow,
                                                 int P) {
  extern __shared__ float sh[];
  const int r = patch >> 1;
  const int L = (kRowTile + 2 * r + patch - 1) / patch * patch;
  float* g = sh;
  float* h = sh + 3 * L;
  const int x0 = blockIdx.x * kRowTile;
  const int y = blockIdx.y;
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    const int x = x0 - r + q;
    const bool in = x >= 0 && x < W;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v = in ? load_input(I, dtype, layout, H, pitch, c, y, x) : INFINITY;
      g[c * L + q] = v;
      h[c * L + q] = v;
      if (in && x >= x0 && x < x0 + kRowTile) Ip[(static_cast<size_t>(c) * H + y) * P + x] = v;
    }
  }
  __syncthreads();
  const int nb = L / patch;
  for (int k = threadIdx.x; k < 3 * nb; k += blockDim.x) {
    float* gg = g + (k / nb) * L + (k % nb) * patch;
    float* hh = h + (k / nb) * L + (k % nb) * patch;
    for (int i = 1; i < patch; ++i) gg[i] = fminf(gg[i], gg[i - 1]);
    for (int i = patch - 2; i >= 0; --i) hh[i] = fminf(hh[i], hh[i + 1]);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kRowTile; q += blockDim.x) {
    const int x = x0 + q;
    if (x >= W) break;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      mrow[(static_cast<size_t>(c) * H + y) * P + x] = fminf(h[c * L + q], g[c * L + q + patch - 1]);
  }
}

// ------------------------------------------------------------ column pass
// 64 x 64 output tile per block; the column strip with r rows of halo is
// staged in LDS and processed as in the row pass.  The minimum over the three
// channels (the raw dark channel) is accumulated in registers.
constexpr int kColX = 64;
constexpr int kColY = 64;
constexpr int kColPerThread = kColY / 4;

__global__ __launch_bounds__(256) void k_colmin(const float* __restrict__ mrow, float* __restrict__ m,
                                                 float* __restrict__ dc, int H, int W, int P, int patch,
                                                 float* __restrict__ dark, uint8_t* __restrict__ dark_u8) {
  extern __shared__ float sh[];
  const int r = patch >> 1;
  const int Ly = (kColY + 2 * r + patch - 1) / patch * patch;
  float* g = sh;
  float* h = sh + Ly * kColX;
  const int x0 = blockIdx.x * kColX;
  const int y0 = blockIdx.y * kColY;
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;
  const int x = x0 + tx;
  float dmin[kColPerThread];
#pragma unroll
  for (int k = 0; k < kColPerThread; ++k) dmin[k] = INFINITY;
  for (int c = 0; c < 3; ++c) {
    for (int q = threadIdx.x; q < Ly * kColX; q += blockDim.x) {
      const int y = y0 - r + q / kColX;
      const int xx = x0 + q % kColX;
      const float v = (y >= 0 && y < H && xx < W) ? mrow[(static_cast<size_t>(c) * H + y) * P + xx]
                                                  : INFINITY;
      g[q] = v;
      h[q] = v;
    }
    __syncthreads();
    const int nb = Ly / patch;
    for (int k = threadIdx.x; k < nb * kColX; k += blockDim.x) {
      const int base = (k / kColX) * patch * kColX + (k % kColX);
      for (int i = 1; i < patch; ++i)
        g[base + i * kColX] = fminf(g[base + i * kColX], g[base + (i - 1) * kColX]);
      for (int i = patch - 2; i >= 0; --i)
        h[base + i * kColX] = fminf(h[base + i * kColX], h[base + (i + 1) * kColX]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kColPerThread; ++k) {
      const int ly = ty + 4 * k;
      const float v = fminf(h[ly * kColX + tx], g[(ly + patch - 1) * kColX + tx]);
      const int y = y0 + ly;
      if (y < H && x < W) m[(static_cast<size_t>(c) * H + y) * P + x] = v;
      dmin[k] = fminf(dmin[k], v);
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kColPerThread; ++k) {
    const int y = y0 + ty + 4 * k;
    if (y < H && x < W) {
      dc[static_cast<size_t>(y) * P + x] = dmin[k];
      if (dark) dark[static_cast<size_t>(y) * W + x] = dmin[k];
      if (dark_u8) dark_u8[static_cast<size_t>(y) * W + x] = static_cast<uint8_t>(rintf(dmin[k] * 255.0f));
    }
  }
}

// Column pass held in registers, for a compile-time patch.  A thread owns
// one column and a segment of PATCH output rows starting at bs; the row
// c = bs + r lies in every window [y - r, y + r] of the segment, so each
// output is min(min(rows y - r .. c), min(rows c .. y + r)): one suffix and
// one prefix scan over 4r + 1 rows, no shared memory and no barrier.
template <int PATCH>
__global__ __launch_bounds__(256) void k_colmin_reg(const float* __restrict__ mrow, float* __restrict__ m,
                                                    float* __restrict__ dc, int H, int W, int P,
                                                    float* __restrict__ dark, uint8_t* __restrict__ dark_u8) {
  constexpr int r = PATCH / 2;
  constexpr int NR = 4 * r + 1;  // rows bs - r .. bs + 3r
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  const int bs = blockIdx.y * PATCH;
  float dmin[PATCH];
#pragma unroll
  for (int i = 0; i < PATCH; ++i) dmin[i] = INFINITY;
  for (int ch = 0; ch < 3; ++ch) {
    const float* src = mrow + static_cast<size_t>(ch) * H * P + x;
    float v[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int y = bs - r + i;
      v[i] = (y >= 0 && y < H) ? src[static_cast<size_t>(y) * P] : INFINITY;
    }
    // v[i] <- min(v[i .. 2r]) below the split row, min(v[2r .. i]) above it
#pragma unroll
    for (int i = 2 * r - 1; i >= 0; --i) v[i] = fminf(v[i], v[i + 1]);
#pragma unroll
    for (int i = 2 * r + 1; i < NR; ++i) v[i] = fminf(v[i], v[i - 1]);
    float* dst = m + static_cast<size_t>(ch) * H * P + x;
#pragma unroll
    for (int i = 0; i < PATCH; ++i) {
      const int y = bs + i;
      const float o = fminf(v[i], v[i + 2 * r]);
      if (y < H) dst[static_cast<size_t>(y) * P] = o;
      dmin[i] = fminf(dmin[i], o);
    }
  }
#pragma unroll
  for (int i = 0; i < PATCH; ++i) {
    const int y = bs + i;
    if (y < H) {
      dc[static_cast<size_t>(y) * P + x] = dmin[i];
      if (dark) dark[static_cast<size_t>(y) * W + x] = dmin[i];
      if (dark_u8) dark_u8[static_cast<size_t>(y) * W + x] = static_cast<uint8_t>(rintf(dmin[i] * 255.0f));
    }
  }
}

// ------------------------------------------------------------ airlight
// Order-preserving map of a float to uint32 (larger key <-> larger value);
// -0 is folded onto +0 so that equal values have equal keys.
__device__ __forceinline__ uint32_t order_key(float f) {
  uint32_t u = __float_as_uint(f);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int kSelBins = 2048;
constexpr int kSelChunk = 2048;  // logical indices per block in the candidate kernels

struct SelState {
  uint32_t prefix;    // fixed high bits of the threshold key
  uint32_t k_rem;     // how many keys equal to the final threshold are taken
  uint32_t count_gt;  // keys strictly above the threshold range so far
  uint32_t best;      // linear index of the chosen pixel
  uint32_t hist[kSelBins];
};

struct SelBest {
  double s;
  uint32_t q;
  uint32_t pad;
};

__host__ __device__ constexpr int sel_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }
__host__ __device__ constexpr uint32_t sel_fixed_mask(int pass) {
  return pass == 0 ? 0u : (pass == 1 ? 0xFFE00000u : 0xFFFFFC00u);
}
__host__ __device__ constexpr int sel_bins(int pass) { return pass == 2 ? 1024 : 2048; }

__global__ __launch_bounds__(256) void k_sel_init(SelState* st, uint32_t k) {
  if (threadIdx.x == 0) {
    st->prefix = 0;
    st->k_rem = k;
    st->count_gt = 0;
    st->best = 0xFFFFFFFFu;
  }
  for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) st->hist[i] = 0;
}

__global__ __launch_bounds__(256) void k_sel_hist(const float* __restrict__ dc, int H, int W, int P,
                                                   SelState* st, int pass) {
  __shared__ uint32_t lh[kSelBins];
  const int nb = sel_bins(pass);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const uint32_t fixed = sel_fixed_mask(pass);
  const uint32_t prefix = st->prefix;
  const int shift = sel_shift(pass);
  const size_t n = static_cast<size_t>(H) * W;
  for (size_t q = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(q / W);
    const int x = static_cast<int>(q - static_cast<size_t>(y) * W);
    const uint32_t key = order_key(dc[static_cast<size_t>(y) * P + x]);
    if ((key & fixed) == prefix) atomicAdd(&lh[(key >> shift) & (nb - 1)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (lh[i]) atomicAdd(&st->hist[i], lh[i]);
}

// Finds the bin holding the k_rem-th largest key among those matching the
// prefix, narrows the prefix to it and clears the histogram.
__global__ __launch_bounds__(256) void k_sel_pick(SelState* st, int pass) {
  __shared__ uint32_t part[256];
  __shared__ uint32_t chosen_bin, above_bin;
  const int nb = sel_bins(pass);
  const int per = nb / 256;
  // thread t owns bins [hi - per, hi) counted from the top
  const int hi = nb - threadIdx.x * per;
  uint32_t s = 0;
  for (int b = hi - 1; b >= hi - per; --b) s += st->hist[b];
  part[threadIdx.x] = s;
  __syncthreads();
  // inclusive scan (Hillis-Steele) of counts from the top
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const uint32_t k = st->k_rem;
  const uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  if (before < k && part[threadIdx.x] >= k) {
    uint32_t acc = before;
    for (int b = hi - 1; b >= hi - per; --b) {
      const uint32_t cnt = st->hist[b];
      if (acc + cnt >= k) {
        chosen_bin = static_cast<uint32_t>(b);
        above_bin = acc;
        break;
      }
      acc += cnt;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->prefix |= chosen_bin << sel_shift(pass);
    st->k_rem = k - above_bin;
    st->count_gt += above_bin;
  }
  for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) st->hist[i] = 0;
}

__device__ __forceinline__ uint32_t key_at(const float* dc, int W, int P, uint32_t q) {
  const uint32_t y = q / static_cast<uint32_t>(W);
  const uint32_t x = q - y * static_cast<uint32_t>(W);
  return order_key(dc[static_cast<size_t>(y) * P + x]);
}

__global__ __launch_bounds__(256) void k_sel_eqcount(const float* __restrict__ dc, int H, int W, int P,
                                                      const SelState* st, uint32_t* eq_count) {
  __shared__ uint32_t wsum[4];
  const uint32_t T = st->prefix;
  const uint32_t n = static_cast<uint32_t>(H) * W;
  const uint32_t q0 = blockIdx.x * kSelChunk;
  uint32_t c = 0;
  for (uint32_t q = q0 + threadIdx.x; q < min(n, q0 + kSelChunk); q += blockDim.x)
    c += key_at(dc, W, P, q) == T;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) eq_count[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__device__ __forceinline__ bool better(double s, uint32_t q, double bs, uint32_t bq) {
  return s > bs || (s == bs && q < bq);
}

// Candidates: keys above the threshold, plus the first k_rem keys equal to it
// in linear-index order.  Each block keeps its best (largest (R+G)+B in
// float64, lowest index on ties).
__global__ __launch_bounds__(256) void k_sel_cand(const float* __restrict__ dc, const float* __restrict__ Ip,
                                                   int H, int W, int P, const SelState* st,
                                                   const uint32_t* __restrict__ eq_count,
                                                   SelBest* block_best) {
  __shared__ uint32_t wcnt[4];
  __shared__ uint32_t sh_off;
  __shared__ double bs_sh[4];
  __shared__ uint32_t bq_sh[4];
  const uint32_t T = st->prefix;
  const uint32_t k_rem = st->k_rem;
  const uint32_t n = static_cast<uint32_t>(H) * W;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // rank offset: equal keys in all earlier chunks
  uint32_t o = 0;
  for (uint32_t b = threadIdx.x; b < blockIdx.x; b += blockDim.x) o += eq_count[b];
  for (int off = 32; off > 0; off >>= 1) o += __shfl_down(o, off, 64);
  if (lane == 0) wcnt[wave] = o;
  __syncthreads();
  if (threadIdx.x == 0) sh_off = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
  __syncthreads();
  uint32_t running = sh_off;
  double best_s = -INFINITY;
  uint32_t best_q = 0xFFFFFFFFu;
  const size_t plane = static_cast<size_t>(H) * P;
  const uint32_t q0 = blockIdx.x * kSelChunk;
  for (uint32_t base = q0; base < min(n, q0 + kSelChunk); base += blockDim.x) {
    const uint32_t q = base + threadIdx.x;
    const bool valid = q < n;
    const uint32_t key = valid ? key_at(dc, W, P, q) : 0u;
    const bool eq = valid && key == T;
    const uint64_t ball = __ballot(eq);
    const uint32_t rank_in_wave = __popcll(ball & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) wcnt[wave] = __popcll(ball);
    __syncthreads();
    uint32_t wave_off = 0;
    for (int w = 0; w < wave; ++w) wave_off += wcnt[w];
    const uint32_t rank = running + wave_off + rank_in_wave;
    const bool cand = valid && (key > T || (eq && rank < k_rem));
    if (cand) {
      const uint32_t y = q / static_cast<uint32_t>(W);
      const uint32_t x = q - y * static_cast<uint32_t>(W);
      const size_t e = static_cast<size_t>(y) * P + x;
      const double s = (static_cast<double>(Ip[e]) + static_cast<double>(Ip[plane + e])) +
                       static_cast<double>(Ip[2 * plane + e]);
      if (better(s, q, best_s, best_q)) {
        best_s = s;
        best_q = q;
      }
    }
    running += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double s2 = __shfl_down(best_s, off, 64);
    const uint32_t q2 = __shfl_down(best_q, off, 64);
    if (better(s2, q2, best_s, best_q)) {
      best_s = s2;
      best_q = q2;
    }
  }
  __syncthreads();
  if (lane == 0) {
    bs_sh[wave] = best_s;
    bq_sh[wave] = best_q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      if (better(bs_sh[w], bq_sh[w], best_s, best_q)) {
        best_s = bs_sh[w];
        best_q = bq_sh[w];
      }
    block_best[blockIdx.x] = SelBest{best_s, best_q, 0u};
  }
}

__global__ __launch_bounds__(256) void k_sel_final(const SelBest* __restrict__ block_best, int nblk,
                                                    const float* __restrict__ Ip, int H, int W, int P,
                                                    SelState* st, float* A_out) {
  __shared__ double bs_sh[4];
  __shared__ uint32_t bq_sh[4];
  double best_s = -INFINITY;
  uint32_t best_q = 0xFFFFFFFFu;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    if (better(block_best[b].s, block_best[b].q, best_s, best_q)) {
      best_s = block_best[b].s;
      best_q = block_best[b].q;
    }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const double s2 = __shfl_down(best_s, off, 64);
    const uint32_t q2 = __shfl_down(best_q, off, 64);
    if (better(s2, q2, best_s, best_q)) {
      best_s = s2;
      best_q = q2;
    }
  }
  if (lane == 0) {
    bs_sh[wave] = best_s;
    bq_sh[wave] = best_q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      if (better(bs_sh[w], bq_sh[w], best_s, best_q)) {
        best_s = bs_sh[w];
        best_q = bq_sh[w];
      }
    // k >= 1 candidates always exist; the guard only keeps a broken
    // selection state from indexing outside the image
    st->best = best_q;
    if (best_q >= static_cast<uint32_t>(H) * static_cast<uint32_t>(W)) {
      A_out[0] = A_out[1] = A_out[2] = NAN;
      return;
    }
    const uint32_t y = best_q / static_cast<uint32_t>(W);
    const uint32_t x = best_q - y * static_cast<uint32_t>(W);
    const size_t e = static_cast<size_t>(y) * P + x;
    const size_t plane = static_cast<size_t>(H) * P;
    A_out[0] = Ip[e];
    A_out[1] = Ip[plane + e];
    A_out[2] = Ip[2 * plane + e];
  }
}

// ------------------------------------------------------------ fused t / lambda / Phi
struct FusedParams {
  double omega, t0, lambda0, beta;
  int adaptive;
};

__global__ __launch_bounds__(256) void k_prior_fused(const float* __restrict__ m, const float* __restrict__ Ip,
                                                      int P, const float* __restrict__ t_in, int t_pitch,
                                                      const float* __restrict__ A, int H, int W,
                                                      FusedParams fp, FusedOut o, const double* __restrict__ tds,
                                                      double inv_scales) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  const double a0 = A[0], a1 = A[1], a2 = A[2];
  const size_t e = static_cast<size_t>(y) * P + x;
  const size_t plane = static_cast<size_t>(H) * P;
  const size_t oe = static_cast<size_t>(y) * o.op + x;
  // the airlight of the scattering model is positive in every channel; a
  // caller-supplied A that is not (A lives on the device and is never read
  // back) turns every output into NaN, which the solve reports as non-finite
  if (!(a0 > 0.0 && a1 > 0.0 && a2 > 0.0 && a0 < INFINITY && a1 < INFINITY && a2 < INFINITY)) {
    const float nan = __builtin_nanf("");
    if (o.t_d) o.t_d[static_cast<size_t>(y) * o.tp + x] = nan;
    if (o.t && (m || tds || o.t != t_in)) o.t[static_cast<size_t>(y) * o.tp + x] = nan;
    if (o.lam) o.lam[oe] = nan;
    if (o.phi) {
      const size_t oplane = static_cast<size_t>(H) * o.op;
      o.phi[oe] = o.phi[oplane + oe] = o.phi[2 * oplane + oe] = nan;
    }
    return;
  }
  float t32;
  if (tds) {
    // multiscale: the mean over the scales of the per-scale t_d, rounded once
    const float td = static_cast<float>(tds[e] * inv_scales);
    if (o.t_d) o.t_d[static_cast<size_t>(y) * o.tp + x] = td;
    double t = 1.0 - fp.omega * static_cast<double>(td);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    t32 = static_cast<float>(t);
    if (o.t) o.t[static_cast<size_t>(y) * o.tp + x] = t32;
  } else if (m) {
    // float64 quotients of float32 operands rounded once to float32 are the
    // correctly rounded float32 quotients; min commutes with that rounding.
    const float q0 = static_cast<float>(static_cast<double>(m[e]) / a0);
    const float q1 = static_cast<float>(static_cast<double>(m[plane + e]) / a1);
    const float q2 = static_cast<float>(static_cast<double>(m[2 * plane + e]) / a2);
    const float td = fminf(fminf(q0, q1), q2);
    if (o.t_d) o.t_d[static_cast<size_t>(y) * o.tp + x] = td;
    double t = 1.0 - fp.omega * static_cast<double>(td);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    t32 = static_cast<float>(t);
    if (o.t) o.t[static_cast<size_t>(y) * o.tp + x] = t32;
  } else {
    t32 = t_in[static_cast<size_t>(y) * t_pitch + x];
    if (o.t && o.t != t_in) o.t[static_cast<size_t>(y) * o.tp + x] = t32;
  }
  const double t = static_cast<double>(t32);
  if (o.lam) {
    const double lam = fp.adaptive ? fp.lambda0 * exp(-fp.beta * (1.0 - t)) : fp.lambda0;
    o.lam[oe] = static_cast<float>(lam);
  }
  if (o.phi) {
    const double den = t > fp.t0 ? t : fp.t0;
    const size_t oplane = static_cast<size_t>(H) * o.op;
    o.phi[oe] = static_cast<float>((static_cast<double>(Ip[e]) - a0 * (1.0 - t)) / den);
    o.phi[oplane + oe] = static_cast<float>((static_cast<double>(Ip[plane + e]) - a1 * (1.0 - t)) / den);
    o.phi[2 * oplane + oe] = static_cast<float>((static_cast<double>(Ip[2 * plane + e]) - a2 * (1.0 - t)) / den);
  }
}

// ------------------------------------------------------------ refinements
// One scale's t_d = min_c fl32(m^c / A^c) (as in the fused pass) added to the
// float64 sum over the scales of the multiscale dark channel.
__global__ __launch_bounds__(256) void k_td_acc(const float* __restrict__ m, int P, const float* __restrict__ A,
                                                 int H, int W, double* __restrict__ tds, int first) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  const size_t e = static_cast<size_t>(y) * P + x;
  const size_t plane = static_cast<size_t>(H) * P;
  const float q0 = static_cast<float>(static_cast<double>(m[e]) / static_cast<double>(A[0]));
  const float q1 = static_cast<float>(static_cast<double>(m[plane + e]) / static_cast<double>(A[1]));
  const float q2 = static_cast<float>(static_cast<double>(m[2 * plane + e]) / static_cast<double>(A[2]));
  const double td = static_cast<double>(fminf(fminf(q0, q1), q2));
  tds[e] = first ? td : tds[e] + td;
}

// Guided filter (He, Sun and Tang) with the channel mean of I as guide g and
// t as input q, windows (2r+1)^2 clipped to the image, in float64.  Window
// sums are sliding sums: one thread walks a row (row passes) or a column
// (column passes, coalesced across the threads).
__device__ __forceinline__ double guide_at(const float* Ip, size_t plane, size_t e) {
  return ((static_cast<double>(Ip[e]) + static_cast<double>(Ip[plane + e])) + static_cast<double>(Ip[2 * plane + e])) /
         3.0;
}

// Row window sums of g, q, g^2 and g q into gf[0..3] (dense H x W planes).
__global__ __launch_bounds__(256) void k_gf_rows4(const float* __restrict__ Ip, int P, const float* __restrict__ q,
                                                   int qp, int H, int W, int r, double* __restrict__ gf) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= H) return;
  const size_t plane = static_cast<size_t>(H) * P, n = static_cast<size_t>(H) * W;
  auto val = [&](int x, double (&v)[4]) {
    const double g = guide_at(Ip, plane, static_cast<size_t>(y) * P + x);
    const double t = q[static_cast<size_t>(y) * qp + x];
    v[0] = g; v[1] = t; v[2] = g * g; v[3] = g * t;
  };
  double sum[4] = {0.0, 0.0, 0.0, 0.0}, v[4];
  for (int x = 0; x <= r && x < W; ++x) {
    val(x, v);
    for (int k = 0; k < 4; ++k) sum[k] += v[k];
  }
  for (int x = 0; x < W; ++x) {
    const size_t o = static_cast<size_t>(y) * W + x;
    for (int k = 0; k < 4; ++k) gf[k * n + o] = sum[k];
    if (x + r + 1 < W) {
      val(x + r + 1, v);
      for (int k = 0; k < 4; ++k) sum[k] += v[k];
    }
    if (x - r >= 0) {
      val(x - r, v);
      for (int k = 0; k < 4; ++k) sum[k] -= v[k];
    }
  }
}

__device__ __forceinline__ int win_count(int i, int r, int n) { return min(i + r, n - 1) - max(i - r, 0) + 1; }

// Column window sums of the four row sums -> window means -> a, b of the
// local linear model, into gf[4], gf[5].
__global__ __launch_bounds__(256) void k_gf_cols_ab(double* __restrict__ gf, int H, int W, int r, double eps) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  const size_t n = static_cast<size_t>(H) * W;
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int y = 0; y <= r && y < H; ++y)
    for (int k = 0; k < 4; ++k) sum[k] += gf[k * n + static_cast<size_t>(y) * W + x];
  const int cx = win_count(x, r, W);
  for (int y = 0; y < H; ++y) {
    const double cnt = static_cast<double>(cx) * win_count(y, r, H);
    const double mg = sum[0] / cnt, mq = sum[1] / cnt;
    const double var = sum[2] / cnt - mg * mg, cov = sum[3] / cnt - mg * mq;
    const double a = cov / (var + eps);
    const size_t o = static_cast<size_t>(y) * W + x;
    gf[4 * n + o] = a;
    gf[5 * n + o] = mq - a * mg;
    if (y + r + 1 < H)
      for (int k = 0; k < 4; ++k) sum[k] += gf[k * n + static_cast<size_t>(y + r + 1) * W + x];
    if (y - r >= 0)
      for (int k = 0; k < 4; ++k) sum[k] -= gf[k * n + static_cast<size_t>(y - r) * W + x];
  }
}

// Row window sums of a and b into gf[0], gf[1].
__global__ __launch_bounds__(256) void k_gf_rows2(double* __restrict__ gf, int H, int W, int r) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= H) return;
  const size_t n = static_cast<size_t>(H) * W, row = static_cast<size_t>(y) * W;
  double sa = 0.0, sb = 0.0;
  for (int x = 0; x <= r && x < W; ++x) {
    sa += gf[4 * n + row + x];
    sb += gf[5 * n + row + x];
  }
  for (int x = 0; x < W; ++x) {
    gf[row + x] = sa;
    gf[n + row + x] = sb;
    if (x + r + 1 < W) {
      sa += gf[4 * n + row + x + r + 1];
      sb += gf[5 * n + row + x + r + 1];
    }
    if (x - r >= 0) {
      sa -= gf[4 * n + row + x - r];
      sb -= gf[5 * n + row + x - r];
    }
  }
}

// Column window sums of those -> mean a, mean b -> out = mean_a g + mean_b,
// clamped to [0, 1] and rounded once.
__global__ __launch_bounds__(256) void k_gf_cols_out(const double* __restrict__ gf, const float* __restrict__ Ip,
                                                      int P, int H, int W, int r, float* __restrict__ out, int op) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  const size_t n = static_cast<size_t>(H) * W, plane = static_cast<size_t>(H) * P;
  double sa = 0.0, sb = 0.0;
  for (int y = 0; y <= r && y < H; ++y) {
    sa += gf[static_cast<size_t>(y) * W + x];
    sb += gf[n + static_cast<size_t>(y) * W + x];
  }
  const int cx = win_count(x, r, W);
  for (int y = 0; y < H; ++y) {
    const double cnt = static_cast<double>(cx) * win_count(y, r, H);
    const double g = guide_at(Ip, plane, static_cast<size_t>(y) * P + x);
    double v = (sa / cnt) * g + sb / cnt;
    v = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    out[static_cast<size_t>(y) * op + x] = static_cast<float>(v);
    if (y + r + 1 < H) {
      sa += gf[static_cast<size_t>(y + r + 1) * W + x];
      sb += gf[n + static_cast<size_t>(y + r + 1) * W + x];
    }
    if (y - r >= 0) {
      sa -= gf[static_cast<size_t>(y - r) * W + x];
      sb -= gf[n + static_cast<size_t>(y - r) * W + x];
    }
  }
}

__global__ __launch_bounds__(256) void k_copy3(const float* __restrict__ src, int sp, float* __restrict__ dst,
                                                int dp, int H, int W) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    dst[(static_cast<size_t>(c) * H + y) * dp + x] = src[(static_cast<size_t>(c) * H + y) * sp + x];
}

__global__ __launch_bounds__(256) void k_copy3_wide(const float* __restrict__ src, int sp, double* __restrict__ dst,
                                                     int dp, int H, int W) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    dst[(static_cast<size_t>(c) * H + y) * dp + x] =
        static_cast<double>(src[(static_cast<size_t>(c) * H + y) * sp + x]);
}

// Analytic part of the warm start: where the solution is smooth G(u) ~ u and
// the diffusion term is small, so the main PDE reduces to lambda u = Phi and
// B = Phi / lambda.  Without lambda G (or with lambda = 0) B = Phi.  With add,
// u0 already holds the network's correction and B is added to it.  u0 is
// planar with pitch W; Phi and lambda have pitch P.
__global__ __launch_bounds__(256) void k_warm_base(float* __restrict__ u0, const float* __restrict__ phi,
                                                    const float* __restrict__ lam, int P, int H, int W, int nonlocal,
                                                    int add) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  const size_t e = static_cast<size_t>(y) * P + x;
  const float l = lam[e];
  const bool divide = nonlocal && l > 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float ph = phi[static_cast<size_t>(c) * H * P + e];
    const float b = divide ? ph / l : ph;
    float* o = u0 + (static_cast<size_t>(c) * H + y) * W + x;
    *o = add ? *o + b : b;
  }
}

int sel_chunks(int H, int W) {
  const size_t n = static_cast<size_t>(H) * W;
  return static_cast<int>((n + kSelChunk - 1) / kSelChunk);
}

}  // namespace

size_t carve_prior(void* ws, int H, int W, const dehaze_params& p, PriorBufs* b) {
  const int P = padded_pitch(W);
  const size_t plane = static_cast<size_t>(H) * P, dense = static_cast<size_t>(H) * W;
  Carver cv(ws, ~size_t(0));
  b->P = P;
  b->Ip = cv.take<float>(3 * plane);
  b->mrow = cv.take<float>(3 * plane);
  b->m = cv.take<float>(3 * plane);
  b->dc = cv.take<float>(plane);
  b->sel = cv.take<char>(prior_scratch_bytes(H, W));
  b->tds = p.dark_scales > 1 ? cv.take<double>(plane) : nullptr;
  b->traw = p.guided_radius > 0 ? cv.take<float>(dense) : nullptr;
  b->tref = p.guided_radius > 0 ? cv.take<float>(dense) : nullptr;
  b->gf = p.guided_radius > 0 ? cv.take<double>(6 * dense) : nullptr;
  return cv.used();
}

size_t prior_scratch_bytes(int H, int W) {
  const int nch = sel_chunks(H, W);
  return align_up(sizeof(SelState), 256) + align_up(sizeof(uint32_t) * nch, 256) +
         align_up(sizeof(SelBest) * nch, 256);
}

int launch_to_planar(const void* I, int dtype, int layout, int H, int W, int pitch, float* Ip, int P,
                     hipStream_t s) {
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(k_to_planar, grid, dim3(256), 0, s, I, dtype, layout, H, W, pitch, Ip, P);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int launch_patch_min(const void* I, int dtype, int layout, int H, int W, int pitch, int patch,
                     const PriorBufs& b, float* dark, uint8_t* dark_u8, hipStream_t s) {
  const int r = patch >> 1;
  {
    const int L = (kRowTile + 2 * r + patch - 1) / patch * patch;
    dim3 grid((W + kRowTile - 1) / kRowTile, H);
    hipLaunchKernelGGL(k_rowmin, grid, dim3(256), 6 * L * sizeof(float), s, I, dtype, layout, H, W,
                       pitch, patch, b.Ip, b.mrow, b.P);
    DZ_CHECK_LAUNCH();
  }
  if (patch == 15) {
    dim3 grid((W + 255) / 256, (H + 14) / 15);
    hipLaunchKernelGGL(k_colmin_reg<15>, grid, dim3(256), 0, s, b.mrow, b.m, b.dc, H, W, b.P, dark, dark_u8);
    DZ_CHECK_LAUNCH();
  } else {
    const int Ly = (kColY + 2 * r + patch - 1) / patch * patch;
    dim3 grid((W + kColX - 1) / kColX, (H + kColY - 1) / kColY);
    hipLaunchKernelGGL(k_colmin, grid, dim3(256), 2 * Ly * kColX * sizeof(float), s, b.mrow, b.m,
                       b.dc, H, W, b.P, patch, dark, dark_u8);
    DZ_CHECK_LAUNCH();
  }
  return DEHAZE_OK;
}

int launch_airlight(const PriorBufs& b, int H, int W, int atm_divisor, float* A_out, hipStream_t s) {
  const size_t n = static_cast<size_t>(H) * W;
  const uint32_t k = static_cast<uint32_t>(std::max<size_t>(1, n / static_cast<size_t>(atm_divisor)));
  const int nch = sel_chunks(H, W);
  Carver cv(b.sel, ~size_t(0));
  SelState* st = cv.take<SelState>(1);
  uint32_t* eq = cv.take<uint32_t>(nch);
  SelBest* best = cv.take<SelBest>(nch);
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, st, k);
  DZ_CHECK_LAUNCH();
  const int hist_blocks = static_cast<int>(std::min<size_t>(1024, (n + 4095) / 4096));
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(k_sel_hist, dim3(hist_blocks), dim3(256), 0, s, b.dc, H, W, b.P, st, pass);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, st, pass);
    DZ_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_sel_eqcount, dim3(nch), dim3(256), 0, s, b.dc, H, W, b.P, st, eq);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sel_cand, dim3(nch), dim3(256), 0, s, b.dc, b.Ip, H, W, b.P, st, eq, best);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sel_final, dim3(1), dim3(256), 0, s, best, nch, b.Ip, H, W, b.P, st, A_out);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int launch_prior_fused(const float* m, const float* Ip, int P, const float* t_in, int t_pitch,
                       const float* A, int H, int W, const dehaze_params& p, const FusedOut& o,
                       hipStream_t s) {
  FusedParams fp{p.omega, p.t0, p.lambda0, p.beta_lambda, p.adaptive};
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(k_prior_fused, grid, dim3(256), 0, s, m, Ip, P, t_in, t_pitch, A, H, W, fp, o, nullptr, 0.0);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int launch_prior_estimated(const void* I, int dtype, int layout, int H, int W, int pitch, const dehaze_params& p,
                           const PriorBufs& b, const float* A, const FusedOut& o, hipStream_t s) {
  FusedParams fp{p.omega, p.t0, p.lambda0, p.beta_lambda, p.adaptive};
  const dim3 grid((W + 255) / 256, H);
  int rc;
  const int scales = p.dark_scales;
  if (scales > 1) {
    // the base scale's minima are in b.m; the other scales overwrite them
    hipLaunchKernelGGL(k_td_acc, grid, dim3(256), 0, s, b.m, b.P, A, H, W, b.tds, 1);
    DZ_CHECK_LAUNCH();
    for (int k = 1; k < scales; ++k) {
      const int side = ((p.patch - 1) >> k) | 1;
      if ((rc = launch_patch_min(I, dtype, layout, H, W, pitch, side, b, nullptr, nullptr, s))) return rc;
      hipLaunchKernelGGL(k_td_acc, grid, dim3(256), 0, s, b.m, b.P, A, H, W, b.tds, 0);
      DZ_CHECK_LAUNCH();
    }
  }
  const float* m = scales > 1 ? nullptr : b.m;
  const double* tds = scales > 1 ? b.tds : nullptr;
  const double inv = 1.0 / scales;
  if (p.guided_radius <= 0) {
    hipLaunchKernelGGL(k_prior_fused, grid, dim3(256), 0, s, m, b.Ip, b.P, nullptr, 0, A, H, W, fp, o, tds, inv);
    DZ_CHECK_LAUNCH();
    return DEHAZE_OK;
  }
  // t before refinement, then the guided filter, then lambda and Phi from it
  FusedOut o1{o.t_d, b.traw, nullptr, nullptr, o.op, W};
  hipLaunchKernelGGL(k_prior_fused, grid, dim3(256), 0, s, m, b.Ip, b.P, nullptr, 0, A, H, W, fp, o1, tds, inv);
  DZ_CHECK_LAUNCH();
  const int r = p.guided_radius;
  hipLaunchKernelGGL(k_gf_rows4, dim3((H + 255) / 256), dim3(256), 0, s, b.Ip, b.P, b.traw, W, H, W, r, b.gf);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gf_cols_ab, dim3((W + 255) / 256), dim3(256), 0, s, b.gf, H, W, r, p.guided_eps);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gf_rows2, dim3((H + 255) / 256), dim3(256), 0, s, b.gf, H, W, r);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gf_cols_out, dim3((W + 255) / 256), dim3(256), 0, s, b.gf, b.Ip, b.P, H, W, r, b.tref, W);
  DZ_CHECK_LAUNCH();
  FusedOut o2{nullptr, o.t, o.lam, o.phi, o.op, o.tp};
  hipLaunchKernelGGL(k_prior_fused, grid, dim3(256), 0, s, nullptr, b.Ip, b.P, b.tref, W, A, H, W, fp, o2, nullptr,
                     0.0);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int launch_warm_base(float* u0, const float* phi, const float* lam, int P, int H, int W, bool nonlocal, bool add,
                     hipStream_t s) {
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(k_warm_base, grid, dim3(256), 0, s, u0, phi, lam, P, H, W, nonlocal ? 1 : 0, add ? 1 : 0);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int launch_copy3(const float* src, int sp, float* dst, int dp, int H, int W, hipStream_t s) {
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(k_copy3, grid, dim3(256), 0, s, src, sp, dst, dp, H, W);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int launch_copy3_wide(const float* src, int sp, double* dst, int dp, int H, int W, hipStream_t s) {
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(k_copy3_wide, grid, dim3(256), 0, s, src, sp, dst, dp, H, W);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace dz
