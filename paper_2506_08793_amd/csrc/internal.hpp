// Internal declarations shared by the HIP translation units of the library.
// Not part of the C ABI (that is include/dehaze.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/dehaze.h"

namespace dz {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define DZ_HIP(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::dz::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                      __FILE__, __LINE__);                                      \
      return DEHAZE_EHIP;                                                       \
    }                                                                           \
  } while (0)

#define DZ_CHECK_LAUNCH() DZ_HIP(hipGetLastError())

// ---------------------------------------------------------------- geometry
// Internal planes are stored with the row pitch rounded up to 64 floats
// (256 bytes), so every row of a tile starts on a 256-byte boundary.
constexpr int kPitchAlign = 64;
// Largest dark-channel patch the column pass can stage in 64 KiB of LDS.
constexpr int kMaxPatch = 31;
inline int padded_pitch(int W) { return (W + kPitchAlign - 1) / kPitchAlign * kPitchAlign; }

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace.  Every block is 256-byte aligned.
struct Carver {
  char* base;
  size_t cap;
  size_t off = 0;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t n) {
    size_t o = align_up(off, 256);
    off = o + n * sizeof(T);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
  bool ok() const { return off <= cap; }
  size_t used() const { return align_up(off, 256); }
};

// ---------------------------------------------------------------- context
struct GraphCache;  // captured outer-step graphs (solver.hip)
struct CnnState;    // warm-start network weights and optimiser state (cnn.hip)
struct SweepTune;   // autotuned sweep launch shapes per image size (solver.hip)
struct KrylovTune;  // autotuned BiCGSTAB strip heights per batch composition (solver.hip)
struct Ctx {
  int device = 0;
  int num_cus = 256;
  int lds_bytes = 65536;
  GraphCache* graphs = nullptr;
  CnnState* cnn = nullptr;
  SweepTune* tune = nullptr;
  KrylovTune* ktune = nullptr;
};

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `s` and returns DEHAZE_OK or DEHAZE_EHIP.

// Input conversion to planar float32 with pitch P (Section II-A's I).
int launch_to_planar(const void* I, int dtype, int layout, int H, int W, int pitch,
                     float* Ip, int P, hipStream_t s);

// Outputs of the fused t / lambda / Phi pass (all nullable).
struct FusedOut {
  float* t_d; float* t; float* lam; float* phi;
  int op;          // pitch of lam and phi (elements)
  int tp;          // pitch of t_d and t (elements)
};

struct PriorBufs {
  float* Ip;      // 3 planes, pitch P: float32 intensities
  float* mrow;    // 3 planes, pitch P: row-pass minima
  float* m;       // 3 planes, pitch P: patch minima
  float* dc;      // 1 plane, pitch P: min over channels
  void* sel;      // airlight selection scratch
  int P;
  // refinements (carved only when the parameters ask for them)
  double* tds;    // 1 plane, pitch P: sum of t_d over the dark-channel scales
  float* traw;    // 1 plane, pitch W: t before the guided filter
  float* tref;    // 1 plane, pitch W: t after it
  double* gf;     // 6 planes H x W: guided-filter window sums
};
size_t prior_scratch_bytes(int H, int W);
// Carves the front-end buffers for an H x W image out of `ws` (nullptr: size
// only); returns the bytes used.
size_t carve_prior(void* ws, int H, int W, const dehaze_params& p, PriorBufs* b);
// t_d, t, lambda and Phi from the patch minima in b (after launch_patch_min
// and the airlight), with the multiscale dark channel and the guided-filter
// refinement of t when the parameters ask for them.
int launch_prior_estimated(const void* I, int dtype, int layout, int H, int W, int pitch, const dehaze_params& p,
                           const PriorBufs& b, const float* A, const FusedOut& o, hipStream_t s);
// Per-channel patch minimum (van Herk / Gil-Werman, rows then columns) and the
// raw dark channel.  dark/dark_u8 are dense (pitch W) and nullable.
int launch_patch_min(const void* I, int dtype, int layout, int H, int W, int pitch, int patch,
                     const PriorBufs& b, float* dark, uint8_t* dark_u8, hipStream_t s);
// Dark-channel-prior airlight; writes A_out[3] (device).
int launch_airlight(const PriorBufs& b, int H, int W, int atm_divisor, float* A_out, hipStream_t s);
// t_d, t, lambda, Phi from the patch minima (or, with m == nullptr, from a
// given t) and A.  All outputs nullable; strided outputs use pitch `op`.
int launch_prior_fused(const float* m, const float* Ip, int P, const float* t_in, int t_pitch,
                       const float* A, int H, int W, const dehaze_params& p,
                       const FusedOut& o, hipStream_t s);

// Warm start u0 (planar, pitch W) = B (+ u0 when add), B = Phi / lambda, or Phi
// without the nonlocal term; Phi and lambda have pitch P.
int launch_warm_base(float* u0, const float* phi, const float* lam, int P, int H, int W, bool nonlocal, bool add,
                     hipStream_t s);

// Strided 3-plane copy (pitches in elements), and the same widened to float64.
int launch_copy3(const float* src, int sp, float* dst, int dp, int H, int W, hipStream_t s);
int launch_copy3_wide(const float* src, int sp, double* dst, int dp, int H, int W, hipStream_t s);

// Sweep constants derived from the parameters.
struct OpConst {
  float w[9];      // 1-D Gaussian taps w_{-R..R}
  float wc2;       // centre tap of the 2-D kernel, w_0^2
  float eps;
  float theta;
  float tau;
  int R;
  int nonlocal_term;
  int edge_preserving;
};
OpConst make_opconst(const dehaze_params& p);

// One sweep over the planar field uin -> uout (pitch P), scheme explicit or
// Jacobi, or (mode RESIDUAL) r = Phi - L_{D(u)} u written to uout.
// If `partials` is non-null every block writes (sum r^2, sum phi^2) there.
enum SweepMode { kExplicit = 0, kJacobi = 1, kResidual = 2 };
int sweep_num_blocks(int H, int W);
int launch_sweep(int mode, const float* uin, float* uout, const float* phi, const float* lam,
                 int H, int W, int P, const OpConst& c, double* partials, hipStream_t s);
// K (1..4) pipelined sweeps in one launch, register-resident strips of S
// output rows with C (1 or 2) columns per lane (R = 2, explicit or Jacobi);
// uin and uout must differ.
constexpr int kMaxSweepsPerLaunch = 4;
// Whether a plane of H rows of pitch P is addressable by the strip kernel
// (byte offsets below 2^31); larger planes use the tile kernel.
bool strip_fits(int H, int P);
// Launch shape of the strip kernel: K sweeps per launch, S output rows per
// wavefront, C adjacent columns per lane (a wavefront spans 64 C columns).
struct StripShape {
  int K = 0, S = 0, C = 0;
};
int launch_sweep_strip(int mode, int K, int S, int C, const float* uin, float* uout, const float* phi,
                       const float* lam, int H, int W, int P, const OpConst& c, hipStream_t s);
// Deterministic sum of `n` (a, b) double pairs into out[0..1].
int launch_reduce_pairs(const double* partials, int n, double* out, hipStream_t s);
// rho[0] = sqrt(sums[0]) / sqrt(sums[1]) (sqrt(sums[0]) when sums[1] is 0), on the device.
int launch_rho_from_sums(const double* sums, double* rho, hipStream_t s);

}  // namespace dz
