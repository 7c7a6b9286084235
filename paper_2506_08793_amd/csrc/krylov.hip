// Kernels of the lagged-diffusivity solve (see krylov.hpp for the scheme).
//
// All kernels walk the tiles of every image in the batch (one 64 x 16 tile
// per workgroup).  Per-image sums (norms, BiCGSTAB inner products) are formed
// deterministically: each tile writes its partial sums, and a reduction
// kernel with one workgroup per image adds them in a fixed order and updates
// the image's scalars for the next launch.  (A last-tile-done counter would
// need a device-scope release fence in every workgroup, which on a part with
// one L2 per XCD writes the L2 back each time.)
#include <cmath>

#include "krylov.hpp"
#include "wave.hpp"

namespace dz {

KConst make_kconst(const dehaze_params& p) {
  KConst c{};
  const int R = p.g_radius;
  double g[9], s = 0.0;
  for (int a = -R; a <= R; ++a) {
    g[a + R] = std::exp(-(a * a) / (2.0 * p.sigma * p.sigma));
    s += g[a + R];
  }
  for (int a = 0; a < 2 * R + 1; ++a) {
    c.w64[a] = g[a] / s;
    c.w[a] = static_cast<float>(c.w64[a]);
  }
  c.wc2_64 = c.w64[R] * c.w64[R];
  c.wc2 = static_cast<float>(c.wc2_64);
  c.eps = static_cast<float>(p.eps);
  c.eps64 = p.eps;
  c.rel_tol = p.rel_tol;
  c.eta = p.inner_rtol;
  c.R = R;
  c.nonlocal_term = p.nonlocal_term;
  c.edge_preserving = p.edge_preserving;
  c.stall_window = p.stall_window;
  c.max_inner = p.max_inner;
  c.max_outer = p.max_outer;
  c.ng_m = p.ngmres_depth;
  return c;
}

int krylov_tiles(int H, int W) { return ((W + kKTX - 1) / kKTX) * ((H + kKTY - 1) / kKTY); }
int krylov_units(int H, int W, int us) { return 3 * ((W + kUOW - 1) / kUOW) * ((H + us - 1) / us); }
int krylov_blocks(int H, int W) { return krylov_units(H, W, kSBlk); }
bool krylov_strips_fit(int H, int W) {
  return static_cast<long long>(H + 1) * padded_pitch(W + 1) * 4 < (1LL << 31);
}

// Taller strips cost less per row (fewer halo rows and partial sums) but give
// fewer wavefronts.  In a small launch each image takes the tallest of 128,
// 64, 32 and 16 rows that still gives it at least 768 wavefronts (three
// quarters of the 1024 SIMDs), else 16.  A launch that would carry more than
// 32768 wavefronts at 32 rows runs 32 rows everywhere: there the wavefronts
// queue in many rounds, and long ones lengthen the last round.  Timed against
// 32 rows everywhere (batches solved to rho 1e-5): 1920x1080 x 1, 4, 8 (128 rows)
// 8.0%, 4.8%, 4.8% faster, x 16 5.9% slower; 512x512 x 8 and 256x256 x 16
// (16 rows) 3.2% and 8.1% faster.
void krylov_strip_rows(int n, const int* H, const int* W, int* us) {
  long long at32 = 0;
  for (int i = 0; i < n; ++i) at32 += krylov_units(H[i], W[i], 32);
  for (int i = 0; i < n; ++i) {
    us[i] = 16;
    if (at32 > 32768) {
      us[i] = 32;
      continue;
    }
    for (int r = 128; r > 16; r /= 2)
      if (krylov_units(H[i], W[i], r) >= 768) {
        us[i] = r;
        break;
      }
  }
}

namespace {

struct KCarve {
  KImg img;
  size_t bytes;
};

KCarve carve(void* base, int H, int W, int tile0, int unit0, int blk0, int us, int ng_m) {
  KCarve k{};
  const int P = padded_pitch(W + 1);
  const size_t plane = static_cast<size_t>(H) * P;
  const size_t plane_y = static_cast<size_t>(H + 1) * P;
  Carver cv(base, ~size_t(0));
  KImg& m = k.img;
  m.H = H;
  m.W = W;
  m.P = P;
  m.tiles_x = (W + kKTX - 1) / kKTX;
  m.ntiles = krylov_tiles(H, W);
  m.tile0 = tile0;
  m.ucols = (W + kUOW - 1) / kUOW;
  m.us = us;
  m.nunits = krylov_units(H, W, us);
  m.unit0 = unit0;
  m.nblk = krylov_blocks(H, W);
  m.blk0 = blk0;
  m.phi = cv.take<float>(3 * plane);
  m.lam = cv.take<float>(plane);
  m.u = cv.take<double>(3 * plane);
  m.un = cv.take<double>(3 * plane);
  m.Dx = cv.take<float>(3 * plane);
  m.Dy = cv.take<float>(3 * plane_y);
  m.invd = cv.take<float>(3 * plane);
  m.rhat = cv.take<float>(3 * plane);
  m.r = cv.take<float>(3 * plane);
  m.p[0] = cv.take<float>(3 * plane);
  m.p[1] = cv.take<float>(3 * plane);
  m.v[0] = cv.take<float>(3 * plane);
  m.v[1] = cv.take<float>(3 * plane);
  m.s = cv.take<float>(3 * plane);
  m.t = cv.take<float>(3 * plane);
  m.x = cv.take<float>(3 * plane);
  m.Uh = ng_m > 0 ? cv.take<double>(3 * plane * ng_m) : nullptr;
  m.Rh = ng_m > 0 ? cv.take<float>(3 * plane * ng_m) : nullptr;
  k.bytes = cv.used();
  return k;
}

// One of a ping-pong pair, chosen without indexing the descriptor's array at
// run time (a run-time index sends the whole descriptor to scratch memory).
template <typename T>
__device__ __forceinline__ T* pick(T* const (&pair)[2], int which) {
  return which ? pair[1] : pair[0];
}

constexpr int NT = 256;
constexpr int kPixPerThread = kKTX * kKTY / NT;  // 4

struct TilePos {
  int im, local, x0, y0;
};

__device__ __forceinline__ TilePos tile_pos(const KImg& I, int im, int g) {
  TilePos t;
  t.im = im;
  t.local = g - I.tile0;
  t.x0 = (t.local % I.tiles_x) * kKTX;
  t.y0 = (t.local / I.tiles_x) * kKTY;
  return t;
}

// Block sum of N doubles; the result is valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  __shared__ double red[N][NT / 64];
  for (int k = 0; k < N; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
    for (int k = 0; k < N; ++k) red[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[k][w];
      v[k] = s;
    }
}

// Writes this tile's N partial sums (block sum; thread 0 stores them).
template <int N, int STRIDE = kKPart>
__device__ __forceinline__ void write_partials(double (&v)[N], double* part, int gtile) {
  block_sum<N>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < N; ++k) part[static_cast<size_t>(gtile) * STRIDE + k] = v[k];
}

// Image totals of the tile partials, summed over tiles in index order with a
// fixed assignment to threads and a fixed tree; valid in thread 0.  Run by
// the per-image reduction kernels (one workgroup per image) after the kernel
// that wrote the partials, so plain loads see them.
template <int N, bool UNITS = false, int STRIDE = kKPart>
__device__ __forceinline__ void image_sums(const KImg& I, const double* part, double (&tot)[N]) {
  for (int k = 0; k < N; ++k) tot[k] = 0.0;
  const int n = UNITS ? I.nblk : I.ntiles, first = UNITS ? I.blk0 : I.tile0;
  for (int q = threadIdx.x; q < n; q += NT)
    for (int k = 0; k < N; ++k) tot[k] += part[static_cast<size_t>(first + q) * STRIDE + k];
  block_sum<N>(tot);
}

// ------------------------------------------------------------ init / output
__global__ __launch_bounds__(NT) void k_scal_reset(KScal* scal, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  KScal z{};
  z.converged = 0;
  z.inner_done = 1;  // no inner solve running: the next residual pass starts one
  scal[i] = z;
}

__global__ __launch_bounds__(NT) void k_tile_map(int* tile_img, int tile0, int ntiles, int im) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntiles) tile_img[tile0 + i] = im;
}

__global__ __launch_bounds__(NT) void k_set_desc(KImg* d, int i, KImg h) { d[i] = h; }

__global__ __launch_bounds__(NT) void k_init_u(KImg I, const float* __restrict__ u0, KScal* sc) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x == 0 && y == 0) sc->warm = u0 ? 1 : 0;
  if (x >= I.W) return;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  for (int c = 0; c < 3; ++c) {
    const size_t e = c * plane + static_cast<size_t>(y) * I.P + x;
    const float v = u0 ? u0[(static_cast<size_t>(c) * I.H + y) * I.W + x] : I.phi[e];
    I.u[e] = static_cast<double>(v);
  }
}

__global__ __launch_bounds__(NT) void k_out_u(KImg I, float* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= I.W) return;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  for (int c = 0; c < 3; ++c)
    out[(static_cast<size_t>(c) * I.H + y) * I.W + x] =
        static_cast<float>(I.u[c * plane + static_cast<size_t>(y) * I.P + x]);
}

__global__ __launch_bounds__(NT) void k_out_u64(KImg I, double* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= I.W) return;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  for (int c = 0; c < 3; ++c)
    out[(static_cast<size_t>(c) * I.H + y) * I.W + x] = I.u[c * plane + static_cast<size_t>(y) * I.P + x];
}

// ------------------------------------------------------------ residual pass
// LINEAR = 0: r_n = Phi - L_{D(u_n)} u_n in float64 at the iterate u; stores D
// per face (float32), the inverse Jacobi diagonal and r_n (float32) as the
// inner right-hand side, and tests rho_n against rel_tol.
// LINEAR = 1: Phi - L_{D(u_n)} u with D recomputed (float64, bit-identical to
// the first pass) from the snapshot u_n and the operator applied to the
// current u: the right-hand side of a defect-correction pass.
template <int R, int LINEAR>
__global__ __launch_bounds__(NT) void k_res(const KImg* __restrict__ imgs, KScal* scal,
                                             const int* __restrict__ tile_img, double* part, KConst kc,
                                             int final) {
  constexpr int HALO = R > 1 ? R : 1;
  constexpr int SX = kKTX + 2 * HALO, SY = kKTY + 2 * HALO;
  __shared__ double us[SY][SX];                       // field the operator is applied to
  __shared__ double ud[LINEAR ? SY : 1][LINEAR ? SX : 1];  // field D is taken from (LINEAR)
  __shared__ double gh[kKTY + 2 * R][kKTX];
  __shared__ double qx[kKTY][kKTX + 1];
  __shared__ float dx[kKTY][kKTX + 1];
  __shared__ double qy[kKTY + 1][kKTX];
  __shared__ float dy[kKTY + 1][kKTX];
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  // a residual pass serves images between inner solves (the defect-correction
  // pass of LINEAR follows a finished one too)
  if (!final && (sc->converged || sc->exhausted || !sc->inner_done)) return;
  const TilePos tp = tile_pos(I, im, g);
  const int tid = threadIdx.x, tx = tid & (kKTX - 1), ty = tid / kKTX;
  const int gx = tp.x0 + tx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  const size_t plane_y = static_cast<size_t>(I.H + 1) * I.P;
  double lv[kPixPerThread];
  for (int k = 0; k < kPixPerThread; ++k) {
    const int gy = tp.y0 + ty + 4 * k;
    lv[k] = (kc.nonlocal_term && gx < I.W && gy < I.H) ? static_cast<double>(I.lam[static_cast<size_t>(gy) * I.P + gx])
                                                      : 0.0;
  }
  double acc[3] = {0.0, 0.0, 0.0};  // ||r||^2 (float64), ||Phi||^2, ||r||^2 of the float32 copy
  // a restart replaces the iterate by Phi: every tile of the image reads Phi
  // in place of u (halo included) and writes it over its own part of u
  const bool restart = !LINEAR && !final && sc->restart;
  for (int c = 0; c < 3; ++c) {
    const double* uc = I.u + c * plane;
    const double* unc = I.un + c * plane;
    const float* pc = I.phi + c * plane;
    for (int i = tid; i < SY * SX; i += NT) {
      const int ly = i / SX, lx = i - (i / SX) * SX;
      const int yy = tp.y0 - HALO + ly, xx = tp.x0 - HALO + lx;
      const bool in = yy >= 0 && yy < I.H && xx >= 0 && xx < I.W;
      const size_t e = static_cast<size_t>(yy) * I.P + xx;
      // the output pass reads the iterate as the float32 value it is returned as
      us[ly][lx] = in ? (restart ? static_cast<double>(pc[e])
                                 : (final == 2 ? static_cast<double>(static_cast<float>(uc[e])) : uc[e]))
                      : 0.0;
      if (LINEAR) ud[ly][lx] = in ? unc[e] : 0.0;
    }
    if (restart) {
      for (int k = 0; k < kPixPerThread; ++k) {
        const int gy = tp.y0 + ty + 4 * k;
        if (gx < I.W && gy < I.H) {
          const size_t e = static_cast<size_t>(gy) * I.P + gx;
          I.u[c * plane + e] = static_cast<double>(pc[e]);
        }
      }
    }
    __syncthreads();
    auto UD = [&](int y, int x) -> double { return LINEAR ? ud[y][x] : us[y][x]; };
    if (kc.nonlocal_term) {
      for (int i = tid; i < (kKTY + 2 * R) * kKTX; i += NT) {
        const int j = i / kKTX, lx = i - (i / kKTX) * kKTX;
        double s = 0.0;
        for (int a = 0; a < 2 * R + 1; ++a) s += kc.w64[a] * us[HALO - R + j][HALO + lx - R + a];
        gh[j][lx] = s;
      }
    }
    for (int i = tid; i < kKTY * (kKTX + 1); i += NT) {
      const int ly = i / (kKTX + 1), f = i - (i / (kKTX + 1)) * (kKTX + 1);
      const int cy = HALO + ly, cx = HALO + f - 1;
      const double gnd = UD(cy, cx + 1) - UD(cy, cx);
      const double gtd = 0.5 * (UD(cy + 1, cx) - UD(cy - 1, cx));
      const double D = kc.edge_preserving ? 1.0 / (sqrt(gnd * gnd + gtd * gtd) + kc.eps64) : 1.0;
      qx[ly][f] = D * (us[cy][cx + 1] - us[cy][cx]);
      dx[ly][f] = static_cast<float>(D);
      const int y = tp.y0 + ly, gf = tp.x0 + f;
      if (!LINEAR && y < I.H && ((f < kKTX && gf <= I.W) || (f == kKTX && gf == I.W)))
        I.Dx[c * plane + static_cast<size_t>(y) * I.P + gf] = static_cast<float>(D);
    }
    for (int i = tid; i < (kKTY + 1) * kKTX; i += NT) {
      const int f = i / kKTX, lx = i - (i / kKTX) * kKTX;
      const int cy = HALO + f - 1, cx = HALO + lx;
      const double gnd = UD(cy + 1, cx) - UD(cy, cx);
      const double gtd = 0.5 * (UD(cy, cx + 1) - UD(cy, cx - 1));
      const double D = kc.edge_preserving ? 1.0 / (sqrt(gnd * gnd + gtd * gtd) + kc.eps64) : 1.0;
      qy[f][lx] = D * (us[cy + 1][cx] - us[cy][cx]);
      dy[f][lx] = static_cast<float>(D);
      const int x = tp.x0 + lx, gf = tp.y0 + f;
      if (!LINEAR && x < I.W && ((f < kKTY && gf <= I.H) || (f == kKTY && gf == I.H)))
        I.Dy[c * plane_y + static_cast<size_t>(gf) * I.P + x] = static_cast<float>(D);
    }
    __syncthreads();
    for (int k = 0; k < kPixPerThread; ++k) {
      const int ly = ty + 4 * k, gy = tp.y0 + ly;
      if (gx < I.W && gy < I.H) {
        const double div = (qx[ly][tx + 1] - qx[ly][tx]) + (qy[ly + 1][tx] - qy[ly][tx]);
        double G = 0.0;
        if (kc.nonlocal_term)
          for (int b = 0; b < 2 * R + 1; ++b) G += kc.w64[b] * gh[ly + b][tx];
        const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
        const double ph = I.phi[e];
        const double r = ph - (lv[k] * G - div);
        const float b32 = static_cast<float>(r);
        I.rhat[e] = b32;
        if (!LINEAR) {
          const float d = (dx[ly][tx] + dx[ly][tx + 1]) + (dy[ly][tx] + dy[ly + 1][tx]) +
                          static_cast<float>(lv[k]) * kc.wc2;
          I.invd[e] = 1.0f / d;
        }
        acc[0] += r * r;
        acc[1] += ph * ph;
        acc[2] += static_cast<double>(b32) * b32;
      }
    }
    __syncthreads();
  }
  write_partials<3>(acc, part, g);
}

template <int LINEAR>
__global__ __launch_bounds__(NT) void k_red_res(const KImg* __restrict__ imgs, KScal* scal, const double* part,
                                                 KConst kc, int final) {
  const int im = blockIdx.x;
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (!final && (sc->converged || sc->exhausted || !sc->inner_done)) return;
  double tot[3];
  image_sums<3>(I, part, tot);
  if (threadIdx.x != 0) return;
  if (!LINEAR && final == 2) {
    sc->rel_out = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : sqrt(tot[0]);
    return;
  }
  if (!LINEAR) {
    if (sc->inner_this > 0) {  // account for the update applied since the last pass
      sc->outer += 1;
      sc->inner_total += sc->inner_this;
      sc->inner_this = 0;
    }
    sc->res_evals += 1;
    // a pass beyond max_outer steps only records the residual (the final
    // pass of the loop)
    const bool over = !final && ++sc->passes > kc.max_outer;
    if (over) {
      sc->res_evals -= 1;
      sc->exhausted = 1;
    }
    const double rel = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : sqrt(tot[0]);
    if (sc->res_evals == 1) sc->rel0 = rel;
    sc->rel = rel;
    if (!isfinite(rel)) {
      sc->nonfinite = 1;
      sc->converged = 1;
    } else if (kc.rel_tol > 0.0 && rel <= kc.rel_tol) {
      sc->converged = 1;
    }
    if (!final && !sc->converged && !over) {
      if (sc->res_evals == 1 || sc->restart) {  // a new start: open a window
        sc->restart = 0;
        sc->best = sc->mark = rel;
        sc->since = 0;
        sc->ng_nh = 0;
        sc->ng_slot = 0;
        sc->ng_best = rel;
      } else if (kc.stall_window > 0) {
        sc->best = fmin(sc->best, rel);
        if (++sc->since >= kc.stall_window) {
          if (!(sc->best < 0.5 * sc->mark)) {
            if (sc->warm && !sc->restarted) {
              sc->restart = 1;
              sc->restarted = 1;
            } else if (kc.rel_tol > 0.0) {
              sc->stalled = 1;
              sc->converged = 1;  // done iterating; reported as not converged
            }
          }
          sc->mark = sc->best;
          sc->since = 0;
        }
      }
    }
  } else {
    sc->res_evals += 1;
  }
  if (!final) {
    sc->bnorm2 = tot[2];
    sc->rho = tot[2];
    sc->alpha = 1.0;
    sc->omega = 1.0;
    sc->beta = 0.0;
    sc->half_done = 0;
    sc->pass_inner = 0;
    sc->it = 1;
    // no inner solve on a step that decided a restart (the next residual pass
    // replaces the iterate), nor once the iteration stops
    const bool go = tot[2] > 0.0 && isfinite(tot[2]) && !sc->restart && !sc->converged && !sc->exhausted;
    sc->inner_done = go ? 0 : 1;
    if (!LINEAR && kc.ng_m > 0) {
      // nonlinear GMRES: the mix comes first and starts the inner solve; a
      // trial rho above twice the lowest since the last drop drops the history
      sc->ng_pending = go ? 1 : 0;
      sc->inner_done = 1;
      if (go && sc->res_evals > 1) {
        if (sc->rel > 2.0 * sc->ng_best) {
          sc->ng_nh = 0;
          sc->ng_drops += 1;
          sc->ng_best = sc->rel;
        }
        sc->ng_best = fmin(sc->ng_best, sc->rel);
      }
    }
  }
}

__global__ __launch_bounds__(NT) void k_snapshot(const KImg* __restrict__ imgs, const KScal* __restrict__ scal,
                                                  const int* __restrict__ tile_img) {
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  if (scal[im].converged) return;
  const TilePos tp = tile_pos(I, im, g);
  const int tid = threadIdx.x, tx = tid & (kKTX - 1), ty = tid / kKTX;
  const int gx = tp.x0 + tx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < kPixPerThread; ++k) {
      const int gy = tp.y0 + ty + 4 * k;
      if (gx < I.W && gy < I.H) {
        const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
        I.un[e] = I.u[e];
      }
    }
}

// ------------------------------------------------------------ operator tile
// Applies L_D (frozen D) to the field f staged in LDS (tile + halo) at the
// tile's interior pixel (tx, ly); f is zero outside the image.
template <int R, int HALO>
__device__ __forceinline__ float apply_L(const float (&fs)[kKTY + 2 * HALO][kKTX + 2 * HALO],
                                         const float (&gh)[kKTY + 2 * R][kKTX], const KImg& I, const KConst& kc,
                                         int c, int gx, int gy, int tx, int ly, float lam) {
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  const size_t plane_y = static_cast<size_t>(I.H + 1) * I.P;
  const float* Dx = I.Dx + c * plane + static_cast<size_t>(gy) * I.P + gx;
  const float* Dy = I.Dy + c * plane_y + static_cast<size_t>(gy) * I.P + gx;
  const int cy = HALO + ly, cx = HALO + tx;
  const float f0 = fs[cy][cx];
  const float div = Dx[1] * (fs[cy][cx + 1] - f0) - Dx[0] * (f0 - fs[cy][cx - 1]) +
                    Dy[I.P] * (fs[cy + 1][cx] - f0) - Dy[0] * (f0 - fs[cy - 1][cx]);
  float G = 0.0f;
  if (kc.nonlocal_term)
    for (int b = 0; b < 2 * R + 1; ++b) G += kc.w[b] * gh[ly + b][tx];
  return lam * G - div;
}

template <int R, int HALO>
__device__ __forceinline__ void horiz_gauss(const float (&fs)[kKTY + 2 * HALO][kKTX + 2 * HALO],
                                            float (&gh)[kKTY + 2 * R][kKTX], const KConst& kc) {
  if (!kc.nonlocal_term) return;
  for (int i = threadIdx.x; i < (kKTY + 2 * R) * kKTX; i += NT) {
    const int j = i / kKTX, lx = i - (i / kKTX) * kKTX;
    float s = 0.0f;
    for (int a = 0; a < 2 * R + 1; ++a) s += kc.w[a] * fs[HALO - R + j][HALO + lx - R + a];
    gh[j][lx] = s;
  }
}

// ------------------------------------------------------------ BiCGSTAB
// (a) p = r + beta (p - omega v); v = L M^-1 p; sigma = (rhat, v); alpha = rho / sigma.
template <int R>
__global__ __launch_bounds__(NT) void k_bicg_a(const KImg* __restrict__ imgs, KScal* scal,
                                                const int* __restrict__ tile_img, double* part, KConst kc) {
  constexpr int HALO = R > 1 ? R : 1;
  constexpr int SX = kKTX + 2 * HALO, SY = kKTY + 2 * HALO;
  __shared__ float fs[SY][SX];
  __shared__ float gh[kKTY + 2 * R][kKTX];
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || sc->inner_done) return;
  const int first = sc->it == 1, par = sc->it & 1;
  const TilePos tp = tile_pos(I, im, g);
  const float beta = first ? 0.0f : static_cast<float>(sc->beta);
  const float omega = static_cast<float>(sc->omega);
  const float* rs = first ? I.rhat : I.r;
  const float* po = pick(I.p, 1 - par);
  const float* vo = pick(I.v, 1 - par);
  float* pn_out = pick(I.p, par);
  float* vn_out = pick(I.v, par);
  const int tid = threadIdx.x, tx = tid & (kKTX - 1), ty = tid / kKTX;
  const int gx = tp.x0 + tx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  float lv[kPixPerThread];
  for (int k = 0; k < kPixPerThread; ++k) {
    const int gy = tp.y0 + ty + 4 * k;
    lv[k] = (kc.nonlocal_term && gx < I.W && gy < I.H) ? I.lam[static_cast<size_t>(gy) * I.P + gx] : 0.0f;
  }
  double acc[1] = {0.0};
  for (int c = 0; c < 3; ++c) {
    for (int i = tid; i < SY * SX; i += NT) {
      const int ly = i / SX, lx = i - (i / SX) * SX;
      const int yy = tp.y0 - HALO + ly, xx = tp.x0 - HALO + lx;
      float f = 0.0f;
      if (yy >= 0 && yy < I.H && xx >= 0 && xx < I.W) {
        const size_t e = c * plane + static_cast<size_t>(yy) * I.P + xx;
        const float pn = first ? rs[e] : rs[e] + beta * (po[e] - omega * vo[e]);
        f = I.invd[e] * pn;
        if (ly >= HALO && ly < HALO + kKTY && lx >= HALO && lx < HALO + kKTX) pn_out[e] = pn;
      }
      fs[ly][lx] = f;
    }
    __syncthreads();
    horiz_gauss<R, HALO>(fs, gh, kc);
    __syncthreads();
    for (int k = 0; k < kPixPerThread; ++k) {
      const int ly = ty + 4 * k, gy = tp.y0 + ly;
      if (gx < I.W && gy < I.H) {
        const float v = apply_L<R, HALO>(fs, gh, I, kc, c, gx, gy, tx, ly, lv[k]);
        const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
        vn_out[e] = v;
        acc[0] += static_cast<double>(I.rhat[e]) * v;
      }
    }
    __syncthreads();
  }
  write_partials<1>(acc, part, g);
}

template <bool UNITS>
__global__ __launch_bounds__(NT) void k_red_a(const KImg* __restrict__ imgs, KScal* scal, const double* part) {
  const int im = blockIdx.x;
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || sc->inner_done) return;
  double tot[1];
  image_sums<1, UNITS>(I, part, tot);
  if (threadIdx.x != 0) return;
  const double sigma = tot[0];
  if (sigma == 0.0 || !isfinite(sigma)) sc->inner_done = 1;
  else sc->alpha = sc->rho / sigma;
}

// (b) s = r - alpha v; t = L M^-1 s; omega = (t, s) / (t, t); ||s|| test.
template <int R>
__global__ __launch_bounds__(NT) void k_bicg_b(const KImg* __restrict__ imgs, KScal* scal,
                                                const int* __restrict__ tile_img, double* part, KConst kc) {
  constexpr int HALO = R > 1 ? R : 1;
  constexpr int SX = kKTX + 2 * HALO, SY = kKTY + 2 * HALO;
  __shared__ float fs[SY][SX];
  __shared__ float gh[kKTY + 2 * R][kKTX];
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || sc->inner_done) return;
  const int first = sc->it == 1, par = sc->it & 1;
  const TilePos tp = tile_pos(I, im, g);
  const float alpha = static_cast<float>(sc->alpha);
  const float* rs = first ? I.rhat : I.r;
  const float* vn = pick(I.v, par);
  const int tid = threadIdx.x, tx = tid & (kKTX - 1), ty = tid / kKTX;
  const int gx = tp.x0 + tx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  float lv[kPixPerThread];
  for (int k = 0; k < kPixPerThread; ++k) {
    const int gy = tp.y0 + ty + 4 * k;
    lv[k] = (kc.nonlocal_term && gx < I.W && gy < I.H) ? I.lam[static_cast<size_t>(gy) * I.P + gx] : 0.0f;
  }
  double acc[3] = {0.0, 0.0, 0.0};  // (t, s), (t, t), (s, s)
  for (int c = 0; c < 3; ++c) {
    for (int i = tid; i < SY * SX; i += NT) {
      const int ly = i / SX, lx = i - (i / SX) * SX;
      const int yy = tp.y0 - HALO + ly, xx = tp.x0 - HALO + lx;
      float f = 0.0f;
      if (yy >= 0 && yy < I.H && xx >= 0 && xx < I.W) {
        const size_t e = c * plane + static_cast<size_t>(yy) * I.P + xx;
        const float sv = rs[e] - alpha * vn[e];
        f = I.invd[e] * sv;
        if (ly >= HALO && ly < HALO + kKTY && lx >= HALO && lx < HALO + kKTX) I.s[e] = sv;
      }
      fs[ly][lx] = f;
    }
    __syncthreads();
    horiz_gauss<R, HALO>(fs, gh, kc);
    __syncthreads();
    for (int k = 0; k < kPixPerThread; ++k) {
      const int ly = ty + 4 * k, gy = tp.y0 + ly;
      if (gx < I.W && gy < I.H) {
        const float t = apply_L<R, HALO>(fs, gh, I, kc, c, gx, gy, tx, ly, lv[k]);
        const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
        I.t[e] = t;
        const float s_e = rs[e] - alpha * vn[e];
        acc[0] += static_cast<double>(t) * s_e;
        acc[1] += static_cast<double>(t) * t;
        acc[2] += static_cast<double>(s_e) * s_e;
      }
    }
    __syncthreads();
  }
  write_partials<3>(acc, part, g);
}

template <bool UNITS>
__global__ __launch_bounds__(NT) void k_red_b(const KImg* __restrict__ imgs, KScal* scal, const double* part,
                                               KConst kc) {
  const int im = blockIdx.x;
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || sc->inner_done) return;
  double tot[3];
  image_sums<3, UNITS>(I, part, tot);
  if (threadIdx.x != 0) return;
  if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2])) {
    sc->inner_done = 1;
  } else {
    if (tot[2] <= kc.eta * kc.eta * sc->bnorm2) sc->half_done = 1;
    sc->omega = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
  }
}

// ------------------------------------------------------------ BiCGSTAB, strips
// Depth of the strip kernels' load rings (rows in flight per wavefront + 1).
constexpr int kRing = 4;

// The operator kernels (a) and (b) for the radius-2 Gaussian as register-
// resident strip walks: one wavefront per (image, channel, group of kUOW
// columns, strip of I.us rows); lane = column with a 2-column halo on each
// side, horizontal neighbours by DPP shifts, vertical ones in 4-row windows.
// Step r of the walk forms f = M^-1 q at input row r (q = p in (a), s in (b))
// and applies the operator at row j = r - 2.  Loads go through buffer
// resources with scalar row offsets, RING - 1 rows ahead into RING-slot
// rings (RING divides kSBlk).
// MODE 0 is (a): p = r + beta (p - omega v); v = L M^-1 p; partial (rhat, v).
// MODE 1 is (b): s = r - alpha v; t = L M^-1 s; partials (t, s), (t, t), (s, s).
template <int MODE, bool FIRST, int RING>
__global__ __launch_bounds__(256) void k_bicg_strip(const KImg* __restrict__ imgs, KScal* scal,
                                                     const int* __restrict__ unit_img, double* upart, KConst kc,
                                                     int nunits) {
#pragma clang fp contract(off)
  constexpr int NACC = MODE == 0 ? 1 : 3;  // dot products: (rhat, v); (t, s), (t, t), (s, s)
  constexpr int AHEAD = RING - 1;
  constexpr int HEAD = 4;                  // steps that fill the 4-row windows
  static_assert(kSBlk % RING == 0 && RING >= HEAD, "RING must divide kSBlk and cover the head");
  constexpr int TPB = kSBlk / RING;        // loop trips per block of kSBlk output rows
  const int gw = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (gw >= nunits) return;
  // uniform per wavefront: keeps the descriptor and everything from it scalar
  const int im = __builtin_amdgcn_readfirstlane(unit_img[gw]);
  const KImg I = imgs[im];
  const KScal* sc = scal + im;
  // uniform per wavefront; the first iteration of an inner solve has its own
  // instantiation (launch-shape trials run regardless, on whatever the
  // buffers hold, and their outputs are overwritten before use)
  if (!kc.trial && (sc->converged || sc->inner_done || (sc->it == 1) != FIRST)) return;
  const int par = kc.trial ? 1 : (sc->it & 1);
  const int u = gw - I.unit0;
  // column group fastest: the four wavefronts of a workgroup (one XCD, one
  // L2) take adjacent column groups and share the cache lines between them
  const int col = u % I.ucols, rest = u / I.ucols;
  const int c = rest % 3, strip = rest / 3;
  const int lane = threadIdx.x & 63;
  const int x = col * kUOW - 2 + lane;
  const bool xin = x >= 0 && x < I.W;
  const unsigned long long live = __builtin_amdgcn_ballot_w64(xin);
  const bool out_lane = lane >= 2 && lane < 2 + kUOW && xin;
  const int y0 = strip * I.us, y1 = min(y0 + I.us, I.H);
  const int H = I.H, P = I.P;
  const unsigned pb = static_cast<unsigned>(H) * P * 4u, pby = static_cast<unsigned>(H + 1) * P * 4u;
  const size_t plane = static_cast<size_t>(H) * P, plane_y = static_cast<size_t>(H + 1) * P;
  const float* rsrc = FIRST ? I.rhat : I.r;
  const __amdgpu_buffer_rsrc_t b_rs = plane_rsrc(rsrc + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_id = plane_rsrc(I.invd + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_dx = plane_rsrc(I.Dx + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_dy = plane_rsrc(I.Dy + c * plane_y, pby);
  const __amdgpu_buffer_rsrc_t b_la = plane_rsrc(I.lam, pb);
  // (a): old p and v, rhat for the dot product; (b): v of this iteration
  const __amdgpu_buffer_rsrc_t b_po = plane_rsrc(MODE == 0 ? pick(I.p, 1 - par) + c * plane : pick(I.v, par) + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_vo = plane_rsrc(pick(I.v, 1 - par) + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_rh = plane_rsrc(I.rhat + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_qo = plane_rsrc(MODE == 0 ? pick(I.p, par) + c * plane : I.s + c * plane, pb);
  const __amdgpu_buffer_rsrc_t b_lo = plane_rsrc(MODE == 0 ? pick(I.v, par) + c * plane : I.t + c * plane, pb);
  const int vx = min(max(x, 0), I.W - 1) * 4;   // cell columns
  const int vf = min(max(x, 0), I.W) * 4;       // x-face columns (W + 1 faces)
  const float beta = FIRST || kc.trial ? 0.0f : static_cast<float>(sc->beta);
  const float omega = kc.trial ? 0.0f : static_cast<float>(sc->omega);
  const float alpha = kc.trial ? 0.0f : static_cast<float>(sc->alpha);
  const bool nl = kc.nonlocal_term != 0;
  const float w0 = nl ? kc.w[2] : 0.0f, w1 = nl ? kc.w[1] : 0.0f, w2 = nl ? kc.w[0] : 0.0f;

  auto soff = [&](int row) { return min(max(row, 0), H - 1) * P * 4; };
  auto ld = [&](__amdgpu_buffer_rsrc_t b, int vo, int so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b, vo, so, 0));
  };
  // ring slots: inputs of row r (rs, the old p or v, old v, invd) and the
  // operator's data of row r - 2 (Dx, Dy above and below, lambda, rhat)
  float q_rs[RING], q_po[RING], q_vo[RING], q_id[RING];
  float q_dx[RING], q_dya[RING], q_dyb[RING], q_la[RING], q_rh[RING];
  auto issue = [&](int slot, int r) {
    const int so = soff(r);
    q_rs[slot] = ld(b_rs, vx, so);
    if (MODE == 1 || !FIRST) q_po[slot] = ld(b_po, vx, so);
    if (MODE == 0 && !FIRST) q_vo[slot] = ld(b_vo, vx, so);
    q_id[slot] = ld(b_id, vx, so);
    const int j = r - 2, sj = soff(j);
    q_dx[slot] = ld(b_dx, vf, sj);
    q_dya[slot] = ld(b_dy, vx, min(max(j, 0), H) * P * 4);
    q_dyb[slot] = ld(b_dy, vx, min(max(j + 1, 0), H) * P * 4);
    q_la[slot] = ld(b_la, vx, sj);
    if (MODE == 0) q_rh[slot] = ld(b_rh, vx, sj);
  };
  float F[4] = {0.0f, 0.0f, 0.0f, 0.0f}, GH[4] = {0.0f, 0.0f, 0.0f, 0.0f}, Q[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  double acc[3] = {0.0, 0.0, 0.0};
  const int rs0 = y0 - 2;
#pragma unroll
  for (int q = 0; q < AHEAD; ++q) issue(q, rs0 + q);

  // step r: slot q holds row r's inputs and row r - 2's operator data
  auto step = [&](int r, int q, bool out) __attribute__((always_inline)) {
    const float rv = q_rs[q], idv = q_id[q];
    float qv;
    if (MODE == 0) qv = FIRST ? rv : rv + beta * (q_po[q] - omega * q_vo[q]);
    else qv = rv - alpha * q_po[q];
    const bool rin = r >= 0 && r < H;
    const float f = keep_lanes(idv * qv, rin ? live : 0ull);
    const float dx = q_dx[q], dya = q_dya[q], dyb = q_dyb[q], la = q_la[q], rh = q_rh[q];
    issue((q + AHEAD) % RING, r + AHEAD);
    if (rin && r >= y0 && r < y1 && out_lane)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, qv), b_qo, vx, r * P * 4, 0);
    const float fl1 = from_left(f), fr1 = from_right(f);
    const float fl2 = from_left(fl1), fr2 = from_right(fr1);
    const float ghn = __builtin_fmaf(w2, fl2 + fr2, __builtin_fmaf(w1, fl1 + fr1, w0 * f));
    if (out) {
      const int j = r - 2;
      const float up = F[1], f0 = F[2], dn = F[3];
      const float G = __builtin_fmaf(w2, GH[0] + ghn, __builtin_fmaf(w1, GH[1] + GH[3], w0 * GH[2]));
      const float dxr = from_right(dx);
      const float div = (dxr * (from_right(f0) - f0) - dx * (f0 - from_left(f0))) + (dyb * (dn - f0) - dya * (f0 - up));
      const float lv = __builtin_fmaf(la, G, -div);
      if (j < y1 && out_lane) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, lv), b_lo, vx, j * P * 4, 0);
        if (MODE == 0) {
          acc[0] += static_cast<double>(rh) * lv;
        } else {
          const float se = Q[2];
          acc[0] += static_cast<double>(lv) * se;
          acc[1] += static_cast<double>(lv) * lv;
          acc[2] += static_cast<double>(se) * se;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      F[i] = F[i + 1];
      GH[i] = GH[i + 1];
      Q[i] = Q[i + 1];
    }
    F[3] = f;
    GH[3] = ghn;
    Q[3] = qv;
  };
  // the sums of each block of kSBlk output rows go to that block's own slot
  // (column group fastest, then channel, then block), whatever the strip
  // height, so the per-image totals are summed in one fixed order
  auto flush = [&](int blk) {
    const size_t slot = static_cast<size_t>(I.blk0 + (blk * 3 + c) * I.ucols + col) * kKPart;
    for (int k = 0; k < NACC; ++k) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) upart[slot + k] = v;
      acc[k] = 0.0;
    }
  };
  // head: rows y0 - 2 .. y0 + 1 fill the windows; then rows j = y0 .. y1 - 1,
  // RING per loop trip, a block complete after every TPB trips (y0 is a
  // multiple of kSBlk); row r always sits in slot (r - rs0) % RING
  int r = rs0;
#pragma unroll
  for (int q = 0; q < HEAD; ++q) step(r + q, q, false);
  r += HEAD;
  int trips = 0;
  for (; r - 2 < y1; r += RING) {
#pragma unroll
    for (int i = 0; i < RING; ++i) step(r + i, (HEAD + i) % RING, true);
    if (++trips % TPB == 0) flush(y0 / kSBlk + trips / TPB - 1);
  }
  if (trips % TPB) flush(y0 / kSBlk + trips / TPB);
}

// (c) x += alpha M^-1 p + omega M^-1 s; r = s - omega t; rho = (rhat, r); beta.
__global__ __launch_bounds__(NT) void k_bicg_c(const KImg* __restrict__ imgs, KScal* scal,
                                                const int* __restrict__ tile_img, double* part, KConst kc) {
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || sc->inner_done) return;
  const int first = sc->it == 1, par = sc->it & 1;
  const TilePos tp = tile_pos(I, im, g);
  const float alpha = static_cast<float>(sc->alpha);
  const float omega = static_cast<float>(sc->omega);
  const int half = sc->half_done;
  const float* pn = pick(I.p, par);
  // thread: 4 adjacent pixels of one row (16-byte accesses; rows start on
  // 256-byte boundaries and the pitch holds every aligned group that starts
  // inside the image)
  const int ly = threadIdx.x >> 4, lx = (threadIdx.x & 15) * 4;
  const int gy = tp.y0 + ly, gx = tp.x0 + lx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  double acc[2] = {0.0, 0.0};  // (rhat, r), (r, r)
  if (gy < I.H && gx < I.W) {
    const int nv = min(4, I.W - gx);  // pixels inside the image
    auto ld4 = [](const float* q) { return *reinterpret_cast<const float4*>(q); };
    for (int c = 0; c < 3; ++c) {
      const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
      const float4 id4 = ld4(I.invd + e), p4 = ld4(pn + e);
      const float4 x4 = first ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : ld4(I.x + e);
      const float id[4] = {id4.x, id4.y, id4.z, id4.w}, pv[4] = {p4.x, p4.y, p4.z, p4.w};
      const float xo[4] = {x4.x, x4.y, x4.z, x4.w};
      float xn[4], rn[4];
      if (half) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xn[k] = xo[k] + alpha * (id[k] * pv[k]);
      } else {
        const float4 s4 = ld4(I.s + e), t4 = ld4(I.t + e), h4 = ld4(I.rhat + e);
        const float sv[4] = {s4.x, s4.y, s4.z, s4.w}, tv[4] = {t4.x, t4.y, t4.z, t4.w};
        const float hv[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          xn[k] = xo[k] + alpha * (id[k] * pv[k]) + omega * (id[k] * sv[k]);
          rn[k] = sv[k] - omega * tv[k];
          if (k < nv) {
            acc[0] += static_cast<double>(hv[k]) * rn[k];
            acc[1] += static_cast<double>(rn[k]) * rn[k];
          }
        }
      }
      if (nv == 4) {
        *reinterpret_cast<float4*>(I.x + e) = make_float4(xn[0], xn[1], xn[2], xn[3]);
        if (!half) *reinterpret_cast<float4*>(I.r + e) = make_float4(rn[0], rn[1], rn[2], rn[3]);
      } else {
        for (int k = 0; k < nv; ++k) {
          I.x[e + k] = xn[k];
          if (!half) I.r[e + k] = rn[k];
        }
      }
    }
  }
  write_partials<2>(acc, part, g);
}

__global__ __launch_bounds__(NT) void k_red_c(const KImg* __restrict__ imgs, KScal* scal, const double* part,
                                               KConst kc) {
  const int im = blockIdx.x;
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || sc->inner_done) return;
  const int half = sc->half_done;
  double tot[2];
  image_sums<2>(I, part, tot);
  if (threadIdx.x != 0) return;
  sc->inner_this += 1;
  sc->pass_inner += 1;
  if (sc->it >= kc.max_inner) sc->inner_done = 1;
  sc->it += 1;
  if (half) {
    sc->inner_done = 1;
  } else {
    const double rho_new = tot[0];
    if (!isfinite(tot[1]) || tot[1] <= kc.eta * kc.eta * sc->bnorm2 || sc->omega == 0.0 || rho_new == 0.0) {
      sc->inner_done = 1;
    } else {
      sc->beta = (rho_new / sc->rho) * (sc->alpha / sc->omega);
      sc->rho = rho_new;
    }
  }
}

// u += delta where this outer step ran at least one inner iteration.
__global__ __launch_bounds__(NT) void k_update(const KImg* __restrict__ imgs, const KScal* __restrict__ scal,
                                                const int* __restrict__ tile_img) {
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  const KScal* sc = scal + im;
  // once per inner solve: after it ended, before the next residual pass
  if (sc->converged || !sc->inner_done || sc->pass_inner < 1) return;
  const TilePos tp = tile_pos(I, im, g);
  const int tid = threadIdx.x, tx = tid & (kKTX - 1), ty = tid / kKTX;
  const int gx = tp.x0 + tx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < kPixPerThread; ++k) {
      const int gy = tp.y0 + ty + 4 * k;
      if (gx < I.W && gy < I.H) {
        const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
        I.u[e] += static_cast<double>(I.x[e]);
      }
    }
}

// ------------------------------------------------------------ nonlinear GMRES
// Gram sums of the residual differences d_j = r - R_j (r the trial residual,
// float32, in rhat): (d_j, d_l) for j <= l < nh and (d_j, r), summed in
// float64 per tile.  Four pixels of one row per thread, 16-byte accesses.
template <int M>
__global__ __launch_bounds__(NT) void k_ngm_dots(const KImg* __restrict__ imgs, const KScal* __restrict__ scal,
                                                  const int* __restrict__ tile_img, double* npart) {
  constexpr int NG = M * (M + 1) / 2 + M;
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  const KScal* sc = scal + im;
  const int nh = sc->ng_nh;
  if (sc->converged || !sc->ng_pending || nh == 0) return;
  const TilePos tp = tile_pos(I, im, g);
  const int ly = threadIdx.x >> 4, lx = (threadIdx.x & 15) * 4;
  const int gy = tp.y0 + ly, gx = tp.x0 + lx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  double acc[NG];
  for (int k = 0; k < NG; ++k) acc[k] = 0.0;
  if (gy < I.H && gx < I.W) {
    const int nv = min(4, I.W - gx);
    for (int c = 0; c < 3; ++c) {
      const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
      const float4 r4 = *reinterpret_cast<const float4*>(I.rhat + e);
      const float rv[4] = {r4.x, r4.y, r4.z, r4.w};
      float d[M][4];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        if (j < nh) {
          const float4 h4 = *reinterpret_cast<const float4*>(I.Rh + static_cast<size_t>(j) * 3 * plane + e);
          d[j][0] = rv[0] - h4.x;
          d[j][1] = rv[1] - h4.y;
          d[j][2] = rv[2] - h4.z;
          d[j][3] = rv[3] - h4.w;
        } else {
          d[j][0] = d[j][1] = d[j][2] = d[j][3] = 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q >= nv) break;
        int k = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
          for (int l = j; l < M; ++l) acc[k++] += static_cast<double>(d[j][q]) * d[l][q];
          acc[M * (M + 1) / 2 + j] += static_cast<double>(d[j][q]) * rv[q];
        }
      }
    }
  }
  write_partials<NG, kNPart>(acc, npart, g);
}

// Per image: the mixing coefficients b solve (A + s I) b = -h, A the Gram
// matrix of the nh residual differences, h their products with r, s = 1e-10
// trace(A) / nh; Gaussian elimination with partial pivoting in float64.  A
// system that cannot be solved, or a non-finite b, gives b = 0 (a plain step).
template <int M>
__global__ __launch_bounds__(NT) void k_red_ngm(const KImg* __restrict__ imgs, KScal* scal, const double* npart) {
  constexpr int NG = M * (M + 1) / 2 + M;
  const int im = blockIdx.x;
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  const int nh = sc->ng_nh;
  if (sc->converged || !sc->ng_pending || nh == 0) return;
  double tot[NG];
  image_sums<NG, false, kNPart>(I, npart, tot);
  if (threadIdx.x != 0) return;
  double A[M][M + 1];
  int k = 0;
  for (int j = 0; j < M; ++j) {
    for (int l = j; l < M; ++l) {
      A[j][l] = A[l][j] = tot[k];
      ++k;
    }
    A[j][M] = -tot[M * (M + 1) / 2 + j];
  }
  double tr = 0.0;
  for (int j = 0; j < nh; ++j) tr += A[j][j];
  for (int j = 0; j < nh; ++j) A[j][j] += 1e-10 * tr / nh;
  bool ok = tr > 0.0 && isfinite(tr);
  for (int col = 0; col < nh && ok; ++col) {
    int piv = col;
    for (int r = col + 1; r < nh; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (!(fabs(A[piv][col]) > 0.0)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int q = col; q <= M; ++q) {
        const double t = A[col][q];
        A[col][q] = A[piv][q];
        A[piv][q] = t;
      }
    for (int r = col + 1; r < nh; ++r) {
      const double f = A[r][col] / A[col][col];
      for (int q = col; q < nh; ++q) A[r][q] -= f * A[col][q];
      A[r][M] -= f * A[col][M];
    }
  }
  double b[M];
  for (int j = nh - 1; j >= 0 && ok; --j) {
    double s = A[j][M];
    for (int q = j + 1; q < nh; ++q) s -= A[j][q] * b[q];
    b[j] = s / A[j][j];
    ok = isfinite(b[j]);
  }
  for (int j = 0; j < M; ++j) sc->ngb[j] = (ok && j < nh) ? b[j] : 0.0;
}

// u_mix = ut + sum_j b_j (ut - U_j), r_mix = r + sum_j b_j (r - R_j); (ut, r)
// goes into history slot ng_slot first.  Partial sum of r_mix^2 (the inner
// solve's reference norm).
template <int M>
__global__ __launch_bounds__(NT) void k_ngm_mix(const KImg* __restrict__ imgs, const KScal* __restrict__ scal,
                                                 const int* __restrict__ tile_img, double* part) {
  const int g = blockIdx.x;
  const int im = tile_img[g];
  const KImg I = imgs[im];
  const KScal* sc = scal + im;
  if (sc->converged || !sc->ng_pending) return;
  const int nh = sc->ng_nh, slot = sc->ng_slot;
  double bj[M];
  for (int j = 0; j < M; ++j) bj[j] = j < nh ? sc->ngb[j] : 0.0;
  const TilePos tp = tile_pos(I, im, g);
  const int tid = threadIdx.x, tx = tid & (kKTX - 1), ty = tid / kKTX;
  const int gx = tp.x0 + tx;
  const size_t plane = static_cast<size_t>(I.H) * I.P;
  double acc[1] = {0.0};
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < kPixPerThread; ++k) {
      const int gy = tp.y0 + ty + 4 * k;
      if (gx < I.W && gy < I.H) {
        const size_t e = c * plane + static_cast<size_t>(gy) * I.P + gx;
        const double ut = I.u[e];
        const float rt = I.rhat[e];
        double um = ut, rm = rt;
#pragma unroll
        for (int j = 0; j < M; ++j)
          if (j < nh) {
            const size_t h = static_cast<size_t>(j) * 3 * plane + e;
            um += bj[j] * (ut - I.Uh[h]);
            rm += bj[j] * static_cast<double>(rt - I.Rh[h]);
          }
        const size_t hs = static_cast<size_t>(slot) * 3 * plane + e;
        I.Uh[hs] = ut;
        I.Rh[hs] = rt;
        I.u[e] = um;
        const float r32 = static_cast<float>(rm);
        I.rhat[e] = r32;
        acc[0] += static_cast<double>(r32) * r32;
      }
    }
  write_partials<1>(acc, part, g);
}

// Starts the inner solve on the mixed right-hand side and advances the
// history ring.
__global__ __launch_bounds__(NT) void k_red_mix(const KImg* __restrict__ imgs, KScal* scal, const double* part,
                                                 KConst kc) {
  const int im = blockIdx.x;
  const KImg I = imgs[im];
  KScal* sc = scal + im;
  if (sc->converged || !sc->ng_pending) return;
  double tot[1];
  image_sums<1>(I, part, tot);
  if (threadIdx.x != 0) return;
  sc->ng_pending = 0;
  sc->ng_slot = (sc->ng_slot + 1) % kc.ng_m;
  sc->ng_nh = min(sc->ng_nh + 1, kc.ng_m);
  sc->bnorm2 = tot[0];
  sc->rho = tot[0];
  sc->alpha = 1.0;
  sc->omega = 1.0;
  sc->beta = 0.0;
  sc->half_done = 0;
  sc->pass_inner = 0;
  sc->it = 1;
  sc->inner_done = (tot[0] > 0.0 && isfinite(tot[0])) ? 0 : 1;
}

#define DZ_KRYLOV_DISPATCH(R_, LAUNCH) \
  switch (R_) {                        \
    case 0: LAUNCH(0); break;          \
    case 1: LAUNCH(1); break;          \
    case 2: LAUNCH(2); break;          \
    case 3: LAUNCH(3); break;          \
    case 4: LAUNCH(4); break;          \
    default: set_error("g_radius outside 0..4"); return DEHAZE_EINVAL; \
  }

}  // namespace

size_t krylov_image_bytes(int H, int W, int ng_m) { return carve(nullptr, H, W, 0, 0, 0, 32, ng_m).bytes; }

KImg krylov_carve(void* base, int H, int W, int tile0, int unit0, int blk0, int us, int ng_m) {
  return carve(base, H, W, tile0, unit0, blk0, us, ng_m).img;
}

int krylov_upload_strips(const KrylovBatch& b, const KImg* h_imgs, hipStream_t s) {
  for (int i = 0; i < b.nimg; ++i) {
    const KImg& m = h_imgs[i];
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, s, const_cast<KImg*>(b.d_imgs), i, m);
    DZ_CHECK_LAUNCH();
    if (b.d_unit_img && b.nunits > 0) {
      hipLaunchKernelGGL(k_tile_map, dim3((m.nunits + NT - 1) / NT), dim3(NT), 0, s,
                         const_cast<int*>(b.d_unit_img), m.unit0, m.nunits, i);
      DZ_CHECK_LAUNCH();
    }
  }
  return DEHAZE_OK;
}

int krylov_init(const KrylovBatch& b, const KImg* h_imgs, const float* const* u0, hipStream_t s) {
  hipLaunchKernelGGL(k_scal_reset, dim3((b.nimg + NT - 1) / NT), dim3(NT), 0, s, b.d_scal, b.nimg);
  DZ_CHECK_LAUNCH();
  int rc = krylov_upload_strips(b, h_imgs, s);
  if (rc) return rc;
  for (int i = 0; i < b.nimg; ++i) {
    const KImg& m = h_imgs[i];
    hipLaunchKernelGGL(k_tile_map, dim3((m.ntiles + NT - 1) / NT), dim3(NT), 0, s,
                       const_cast<int*>(b.d_tile_img), m.tile0, m.ntiles, i);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_init_u, dim3((m.W + NT - 1) / NT, m.H), dim3(NT), 0, s, m, u0 ? u0[i] : nullptr,
                       b.d_scal + i);
    DZ_CHECK_LAUNCH();
  }
  return DEHAZE_OK;
}

int krylov_residual(const KrylovBatch& b, const KConst& c, int final, hipStream_t s) {
#define L_RES(R) hipLaunchKernelGGL((k_res<R, 0>), dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, \
                                    b.d_part, c, final)
  DZ_KRYLOV_DISPATCH(c.R, L_RES)
#undef L_RES
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_red_res<0>), dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_part, c, final);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int krylov_linear_residual(const KrylovBatch& b, const KConst& c, hipStream_t s) {
#define L_RES(R) hipLaunchKernelGGL((k_res<R, 1>), dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, \
                                    b.d_part, c, 0)
  DZ_KRYLOV_DISPATCH(c.R, L_RES)
#undef L_RES
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_red_res<1>), dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_part, c, 0);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int krylov_snapshot(const KrylovBatch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_snapshot, dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int krylov_time_strips(const KrylovBatch& b, const KConst& c, int reps, hipStream_t s, float* us) {
  KConst t = c;
  t.trial = 1;
  const dim3 ug((b.nunits + 3) / 4);
  hipEvent_t e0, e1;
  DZ_HIP(hipEventCreate(&e0));
  DZ_HIP(hipEventCreate(&e1));
  int rc = DEHAZE_OK;
  // one untimed launch first: caches, clocks
  for (int i = 0; i <= reps && rc == DEHAZE_OK; ++i) {
    if (i == 1 && hipEventRecord(e0, s) != hipSuccess) rc = DEHAZE_EHIP;
    hipLaunchKernelGGL((k_bicg_strip<0, false, kRing>), ug, dim3(256), 0, s, b.d_imgs, b.d_scal, b.d_unit_img, b.d_upart, t,
                       b.nunits);
    if (hipGetLastError() != hipSuccess) rc = DEHAZE_EHIP;
  }
  float ms = 0.0f;
  if (rc == DEHAZE_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = DEHAZE_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    set_error("timing the BiCGSTAB strip kernel failed");
    return rc;
  }
  *us = 1000.0f * ms / static_cast<float>(reps);
  return DEHAZE_OK;
}

int krylov_inner(const KrylovBatch& b, const KConst& c, hipStream_t s) {
  // one BiCGSTAB iteration for every image inside an inner solve; each image
  // carries its own iteration count, so the first-iteration kernels run
  // beside the others
  if (c.R == 2 && b.nunits > 0) {
    const dim3 ug((b.nunits + 3) / 4);
    hipLaunchKernelGGL((k_bicg_strip<0, true, kRing>), ug, dim3(256), 0, s, b.d_imgs, b.d_scal, b.d_unit_img, b.d_upart, c,
                       b.nunits);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL((k_bicg_strip<0, false, kRing>), ug, dim3(256), 0, s, b.d_imgs, b.d_scal, b.d_unit_img, b.d_upart, c,
                       b.nunits);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_red_a<true>, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_upart);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL((k_bicg_strip<1, true, kRing>), ug, dim3(256), 0, s, b.d_imgs, b.d_scal, b.d_unit_img, b.d_upart, c,
                       b.nunits);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL((k_bicg_strip<1, false, kRing>), ug, dim3(256), 0, s, b.d_imgs, b.d_scal, b.d_unit_img, b.d_upart, c,
                       b.nunits);
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_red_b<true>, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_upart, c);
    DZ_CHECK_LAUNCH();
  } else {
#define L_A(R) hipLaunchKernelGGL((k_bicg_a<R>), dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, \
                                  b.d_part, c)
#define L_B(R) hipLaunchKernelGGL((k_bicg_b<R>), dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, \
                                  b.d_part, c)
    DZ_KRYLOV_DISPATCH(c.R, L_A)
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_red_a<false>, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_part);
    DZ_CHECK_LAUNCH();
    DZ_KRYLOV_DISPATCH(c.R, L_B)
    DZ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_red_b<false>, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_part, c);
    DZ_CHECK_LAUNCH();
#undef L_A
#undef L_B
  }
  hipLaunchKernelGGL(k_bicg_c, dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, b.d_part, c);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_c, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_part, c);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

template <int M>
int launch_ngmres(const KrylovBatch& b, const KConst& c, hipStream_t s) {
  hipLaunchKernelGGL(k_ngm_dots<M>, dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, b.d_npart);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_ngm<M>, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_npart);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ngm_mix<M>, dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img, b.d_part);
  DZ_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_mix, dim3(b.nimg), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_part, c);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int krylov_ngmres(const KrylovBatch& b, const KConst& c, hipStream_t s) {
  if (c.ng_m <= 0) return DEHAZE_OK;
  if (!b.d_npart) {
    set_error("nonlinear GMRES buffers missing");
    return DEHAZE_EINVAL;
  }
  switch (c.ng_m) {
    case 1: return launch_ngmres<1>(b, c, s);
    case 2: return launch_ngmres<2>(b, c, s);
    case 3: return launch_ngmres<3>(b, c, s);
    case 4: return launch_ngmres<4>(b, c, s);
    case 5: return launch_ngmres<5>(b, c, s);
    case 6: return launch_ngmres<6>(b, c, s);
    case 7: return launch_ngmres<7>(b, c, s);
    case 8: return launch_ngmres<8>(b, c, s);
    default: set_error("ngmres_depth %d outside 0..%d", c.ng_m, kNgMax); return DEHAZE_EINVAL;
  }
}

int krylov_update(const KrylovBatch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(b.ntiles), dim3(NT), 0, s, b.d_imgs, b.d_scal, b.d_tile_img);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int krylov_output(const KImg& img, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_out_u, dim3((img.W + NT - 1) / NT, img.H), dim3(NT), 0, s, img, out);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

int krylov_output64(const KImg& img, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_out_u64, dim3((img.W + NT - 1) / NT, img.H), dim3(NT), 0, s, img, out);
  DZ_CHECK_LAUNCH();
  return DEHAZE_OK;
}

}  // namespace dz
