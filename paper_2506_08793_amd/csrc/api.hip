// C ABI entry points: argument checks, workspace carving and the order of
// kernel launches.  All arithmetic happens in the kernels of the other
// translation units.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cnn.hpp"
#include "internal.hpp"
#include "solver.hpp"

namespace dz {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

int check_params(const dehaze_params* p) {
  if (!p) { set_error("params is NULL"); return DEHAZE_EINVAL; }
  if (p->patch < 1 || p->patch % 2 == 0 || p->patch > kMaxPatch) {
    set_error("patch %d must be odd and in 1..%d", p->patch, kMaxPatch);
    return DEHAZE_EINVAL;
  }
  if (p->g_radius < 0 || p->g_radius > 4) { set_error("g_radius %d outside 0..4", p->g_radius); return DEHAZE_EINVAL; }
  if (!(p->t0 > 0.0) || !(p->eps > 0.0) || !(p->sigma > 0.0)) {
    set_error("t0, eps and sigma must be positive"); return DEHAZE_EINVAL;
  }
  if (!(p->omega > 0.0 && p->omega <= 1.0)) { set_error("omega must lie in (0, 1]"); return DEHAZE_EINVAL; }
  if (!(p->lambda0 >= 0.0) || !std::isfinite(p->beta_lambda)) {
    set_error("lambda0 must be >= 0 and beta finite"); return DEHAZE_EINVAL;
  }
  if (p->atm_divisor < 1) { set_error("atm_divisor must be >= 1"); return DEHAZE_EINVAL; }
  if (p->scheme < DEHAZE_PAPER_EXPLICIT || p->scheme > DEHAZE_PICARD_KRYLOV) {
    set_error("unknown scheme %d", p->scheme); return DEHAZE_EINVAL;
  }
  if (p->max_outer < 0 || p->max_inner < 1 || p->check_every < 1) {
    set_error("max_outer >= 0, max_inner >= 1 and check_every >= 1 required"); return DEHAZE_EINVAL;
  }
  if (!(p->theta > 0.0) || !std::isfinite(p->tau)) { set_error("theta must be positive"); return DEHAZE_EINVAL; }
  if (p->sweeps_per_launch < 0) { set_error("sweeps_per_launch must be >= 0"); return DEHAZE_EINVAL; }
  if (p->inner_refine < 0) { set_error("inner_refine must be >= 0"); return DEHAZE_EINVAL; }
  if (p->strip_rows < 0) { set_error("strip_rows must be >= 0"); return DEHAZE_EINVAL; }
  if (p->lane_columns < 0 || p->lane_columns > 2) { set_error("lane_columns must be 0, 1 or 2"); return DEHAZE_EINVAL; }
  if (p->stall_window < 0) { set_error("stall_window must be >= 0"); return DEHAZE_EINVAL; }
  if (p->warm_start < 0 || p->warm_start > 2) { set_error("warm_start must be 0, 1 or 2"); return DEHAZE_EINVAL; }
  if (p->guided_radius < 0 || p->guided_radius > 1024) {
    set_error("guided_radius must lie in 0..1024");
    return DEHAZE_EINVAL;
  }
  if (p->guided_radius > 0 && !(p->guided_eps > 0.0 && std::isfinite(p->guided_eps))) {
    set_error("guided_eps must be positive and finite");
    return DEHAZE_EINVAL;
  }
  if (p->dark_scales < 1 || p->dark_scales > 4) { set_error("dark_scales must lie in 1..4"); return DEHAZE_EINVAL; }
  if (p->krylov_rows < 0 || p->krylov_rows > 512 || p->krylov_rows % 16 != 0) {
    set_error("krylov_rows must be 0 or a multiple of 16 up to 512");
    return DEHAZE_EINVAL;
  }
  if (p->ngmres_depth < 0 || p->ngmres_depth > 8) { set_error("ngmres_depth must lie in 0..8"); return DEHAZE_EINVAL; }
  if (p->ngmres_depth > 0 && p->inner_refine > 0) {
    set_error("ngmres_depth needs inner_refine = 0");
    return DEHAZE_EINVAL;
  }
  if (p->u_state != DEHAZE_U_F32 && p->u_state != DEHAZE_U_F64) {
    set_error("u_state must be DEHAZE_U_F32 or DEHAZE_U_F64");
    return DEHAZE_EINVAL;
  }
  for (int r : p->reserved)
    if (r != 0) { set_error("reserved fields of dehaze_params must be zero"); return DEHAZE_EINVAL; }
  if (!(p->inner_rtol > 0.0)) { set_error("inner_rtol must be positive"); return DEHAZE_EINVAL; }
  return DEHAZE_OK;
}

int check_image(const void* I, int dtype, int layout, int H, int W, int pitch) {
  if (!I) { set_error("image pointer is NULL"); return DEHAZE_EINVAL; }
  if (H < 1 || W < 1) { set_error("image must be at least 1 x 1 (got %d x %d)", H, W); return DEHAZE_EINVAL; }
  if (static_cast<long long>(H) * W > (1LL << 30)) { set_error("image too large"); return DEHAZE_EINVAL; }
  if (pitch < W) { set_error("pitch %d < width %d", pitch, W); return DEHAZE_EINVAL; }
  if (dtype != DEHAZE_U8 && dtype != DEHAZE_F32) { set_error("unknown dtype %d", dtype); return DEHAZE_EINVAL; }
  if (layout != DEHAZE_HWC && layout != DEHAZE_CHW) { set_error("unknown layout %d", layout); return DEHAZE_EINVAL; }
  return DEHAZE_OK;
}

// ------------------------------------------------------------ allocation-free scratch
// Device memory of dehaze_residual_noalloc: the summed pair (sum r^2, sum Phi^2)
// in the first 256 bytes, then one pair per residual block.  Each GPU holds its
// own copy for the life of the process.  In host code `scratch` is a host-side
// stand-in, not a device address: the address of the current device's copy is
// looked up once per device (in dehaze_ctx_create) and only that is used.
constexpr size_t kNoallocHead = 256;
constexpr size_t kNoallocBytes = kNoallocHead + 2 * sizeof(double) * DEHAZE_NOALLOC_MAX_BLOCKS;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Looks up this device's copy of `scratch`; the device must be current.
static int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d outside 0..%d", device, kMaxDevices - 1);
    return DEHAZE_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return DEHAZE_OK;
  void* ptr = nullptr;
  DZ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) {
    set_error("no device address for the allocation-free scratch on device %d", device);
    return DEHAZE_EHIP;
  }
  g_scratch_ptr[device] = ptr;
  return DEHAZE_OK;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

// ------------------------------------------------------------ workspace plans
struct PriorPlan {
  PriorBufs b{};
  size_t bytes = 0;
};

static PriorPlan plan_prior(void* ws, int H, int W, const dehaze_params& p) {
  PriorPlan pl;
  pl.bytes = carve_prior(ws, H, W, p, &pl.b);
  return pl;
}

}  // namespace dz

using namespace dz;

struct dehaze_ctx {
  Ctx c;
};

extern "C" {

int dehaze_params_default(dehaze_params* p) {
  if (!p) { set_error("params is NULL"); return DEHAZE_EINVAL; }
  std::memset(p, 0, sizeof(*p));
  p->patch = 15;
  p->g_radius = 2;
  p->omega = 0.95;
  p->t0 = 0.1;
  p->eps = 1e-3;
  p->sigma = 1.5;
  p->lambda0 = 0.5;
  p->beta_lambda = 3.0;
  p->tau = 0.2;
  p->theta = 0.8;
  p->rel_tol = 1e-5;
  p->inner_rtol = 0.2;
  p->scheme = DEHAZE_PICARD_KRYLOV;
  p->max_outer = 5000;
  p->max_inner = 128;
  p->check_every = 16;
  p->atm_divisor = 1000;
  p->warm_start = 0;
  p->nonlocal_term = 1;
  p->adaptive = 1;
  p->edge_preserving = 1;
  p->sweeps_per_launch = 0;
  p->strip_rows = 0;
  p->lane_columns = 0;
  p->stall_window = 256;
  p->guided_radius = 0;
  p->dark_scales = 1;
  p->guided_eps = 1e-3;
  return DEHAZE_OK;
}

size_t dehaze_params_size(void) { return sizeof(dehaze_params); }
size_t dehaze_stats_size(void) { return sizeof(dehaze_stats); }

const char* dehaze_last_error(void) { return dz::g_err; }

const char* dehaze_strerror(int code) {
  switch (code) {
    case DEHAZE_OK: return "ok";
    case DEHAZE_EINVAL: return "invalid argument";
    case DEHAZE_ENOMEM: return "workspace too small";
    case DEHAZE_EHIP: return "HIP runtime error";
    case DEHAZE_ENOTCONV: return "tolerance not reached";
    case DEHAZE_ENONFINITE: return "non-finite value";
    default: return "unknown error";
  }
}

int dehaze_ctx_create(dehaze_ctx** out, int device) {
  clear_error();
  if (!out) { set_error("ctx pointer is NULL"); return DEHAZE_EINVAL; }
  *out = nullptr;
  DZ_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  DZ_HIP(hipGetDeviceProperties(&prop, device));
  int rc = scratch_setup(device);
  if (rc) return rc;
  dehaze_ctx* ctx = new (std::nothrow) dehaze_ctx();
  if (!ctx) { set_error("out of host memory"); return DEHAZE_EINVAL; }
  ctx->c.device = device;
  ctx->c.num_cus = prop.multiProcessorCount;
  ctx->c.lds_bytes = static_cast<int>(prop.sharedMemPerBlock);
  *out = ctx;
  return DEHAZE_OK;
}

void dehaze_ctx_destroy(dehaze_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  solver_release(ctx->c);
  cnn_release(ctx->c.cnn);
  ctx->c.cnn = nullptr;
  delete ctx;
}

size_t dehaze_prior_workspace_size(int H, int W, const dehaze_params* p) {
  if (H < 1 || W < 1) return 0;
  dehaze_params d;
  if (!p) {
    dehaze_params_default(&d);
    p = &d;
  }
  return plan_prior(nullptr, H, W, *p).bytes;
}

int dehaze_prior(dehaze_ctx* ctx, const void* I, int dtype, int layout, int H, int W, int pitch,
                 const dehaze_params* p, const float* A_in, float* dark, uint8_t* dark_u8, float* t_d,
                 float* t, float* lam, float* phi, float* A_out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!ctx) { set_error("ctx is NULL"); return DEHAZE_EINVAL; }
  int rc = check_image(I, dtype, layout, H, W, pitch);
  if (rc) return rc;
  if ((rc = check_params(p))) return rc;
  if (!A_out) { set_error("A_out is NULL"); return DEHAZE_EINVAL; }
  if (dark_u8 && dtype != DEHAZE_U8) { set_error("dark_u8 needs 8-bit input"); return DEHAZE_EINVAL; }
  PriorPlan pl = plan_prior(ws, H, W, *p);
  if (!ws || ws_bytes < pl.bytes) {
    set_error("prior workspace needs %zu bytes, got %zu", pl.bytes, ws_bytes);
    return DEHAZE_ENOMEM;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  DZ_HIP(hipSetDevice(ctx->c.device));
  if ((rc = launch_patch_min(I, dtype, layout, H, W, pitch, p->patch, pl.b, dark, dark_u8, s))) return rc;
  const float* A = A_out;
  if (A_in) {
    if (A_in != A_out) DZ_HIP(hipMemcpyAsync(A_out, A_in, 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else {
    if ((rc = launch_airlight(pl.b, H, W, p->atm_divisor, A_out, s))) return rc;
  }
  FusedOut o{t_d, t, lam, phi, W, W};
  return launch_prior_estimated(I, dtype, layout, H, W, pitch, *p, pl.b, A, o, s);
}

size_t dehaze_solve_workspace_size(int H, int W, const dehaze_params* p) {
  if (H < 1 || W < 1 || !p) return 0;
  return solver_workspace_bytes(H, W, *p);
}

int dehaze_solve(dehaze_ctx* ctx, const void* I, int dtype, int layout, int H, int W, int pitch, const float* t,
                 const float* A, const dehaze_params* p, const float* u0, float* u, void* ws, size_t ws_bytes,
                 dehaze_stats* stats, void* stream) {
  clear_error();
  if (!ctx) { set_error("ctx is NULL"); return DEHAZE_EINVAL; }
  int rc = check_image(I, dtype, layout, H, W, pitch);
  if (rc) return rc;
  if ((rc = check_params(p))) return rc;
  if (!t || !A || !u) { set_error("t, A and u are required"); return DEHAZE_EINVAL; }
  const size_t need = solver_workspace_bytes(H, W, *p);
  if (!ws || ws_bytes < need) {
    set_error("solve workspace needs %zu bytes, got %zu", need, ws_bytes);
    return DEHAZE_ENOMEM;
  }
  DZ_HIP(hipSetDevice(ctx->c.device));
  SolveArgs a{I, dtype, layout, H, W, pitch, t, A, u0, u, ws, ws_bytes};
  return solve_one(ctx->c, a, *p, stats, static_cast<hipStream_t>(stream));
}

static int check_batch(int n, const dehaze_image* imgs) {
  if (n < 1 || !imgs) { set_error("batch needs n >= 1 images"); return DEHAZE_EINVAL; }
  for (int i = 0; i < n; ++i) {
    const dehaze_image& m = imgs[i];
    if (!m.I || !m.u) { set_error("image %d: I and u are required", i); return DEHAZE_EINVAL; }
    if (m.H < 1 || m.W < 1 || m.pitch < m.W) { set_error("image %d: bad size %d x %d pitch %d", i, m.H, m.W, m.pitch); return DEHAZE_EINVAL; }
    if (static_cast<long long>(m.H) * m.W > (1LL << 30)) { set_error("image %d too large", i); return DEHAZE_EINVAL; }
  }
  return DEHAZE_OK;
}

size_t dehaze_batch_workspace_size(int n, const dehaze_image* imgs, const dehaze_params* p) {
  if (!p || check_batch(n, imgs)) return 0;
  return batch_workspace_bytes(n, imgs, *p);
}

int dehaze_batch(dehaze_ctx* ctx, int n, const dehaze_image* imgs, int dtype, int layout, const dehaze_params* p,
                 void* ws, size_t ws_bytes, dehaze_stats* stats, void* stream) {
  clear_error();
  if (!ctx) { set_error("ctx is NULL"); return DEHAZE_EINVAL; }
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_batch(n, imgs))) return rc;
  if (dtype != DEHAZE_U8 && dtype != DEHAZE_F32) { set_error("unknown dtype %d", dtype); return DEHAZE_EINVAL; }
  if (layout != DEHAZE_HWC && layout != DEHAZE_CHW) { set_error("unknown layout %d", layout); return DEHAZE_EINVAL; }
  if (p->scheme != DEHAZE_PICARD_KRYLOV) { set_error("the batch solve runs DEHAZE_PICARD_KRYLOV only"); return DEHAZE_EINVAL; }
  const size_t need = batch_workspace_bytes(n, imgs, *p);
  if (!ws || ws_bytes < need) {
    set_error("batch workspace needs %zu bytes, got %zu", need, ws_bytes);
    return DEHAZE_ENOMEM;
  }
  DZ_HIP(hipSetDevice(ctx->c.device));
  return solve_batch(ctx->c, n, imgs, dtype, layout, *p, ws, stats, static_cast<hipStream_t>(stream));
}

int dehaze_batch_strip_rows(const dehaze_ctx* ctx, int n, const dehaze_image* imgs, const dehaze_params* p,
                            int* rows, int* tuned) {
  clear_error();
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_batch(n, imgs))) return rc;
  if (!rows || !tuned) { set_error("rows and tuned are required"); return DEHAZE_EINVAL; }
  return batch_strip_rows(ctx ? &ctx->c : nullptr, n, imgs, *p, rows, tuned);
}

size_t dehaze_cnn_param_count(void) { return cnn_param_count(); }

int dehaze_cnn_set_weights(dehaze_ctx* ctx, const float* w, size_t count) {
  clear_error();
  if (!ctx || !w) { set_error("ctx and weights are required"); return DEHAZE_EINVAL; }
  DZ_HIP(hipSetDevice(ctx->c.device));
  return cnn_set_weights(ctx->c, w, count, nullptr);
}

int dehaze_cnn_get_weights(dehaze_ctx* ctx, float* w, size_t count) {
  clear_error();
  if (!ctx || !w) { set_error("ctx and output are required"); return DEHAZE_EINVAL; }
  DZ_HIP(hipSetDevice(ctx->c.device));
  return cnn_get_weights(ctx->c, w, count, nullptr);
}

size_t dehaze_cnn_workspace_size(int n, int H, int W, int training) {
  if (n < 1 || H < 1 || W < 1) return 0;
  return training ? cnn_train_bytes(n, H, W) : cnn_forward_bytes(n, H, W);
}

static int check_cnn_call(dehaze_ctx* ctx, int n, int H, int W, const void* I, const void* t, const void* A,
                          size_t ws_bytes, size_t need, const void* ws) {
  if (!ctx) { set_error("ctx is NULL"); return DEHAZE_EINVAL; }
  if (n < 1 || H < 1 || W < 1 || static_cast<long long>(n) * H * W > (1LL << 31)) {
    set_error("bad network batch %d x %d x %d", n, H, W);
    return DEHAZE_EINVAL;
  }
  if (!I || !t || !A) { set_error("I, t and A are required"); return DEHAZE_EINVAL; }
  if (!cnn_ready(ctx->c)) { set_error("no network weights loaded"); return DEHAZE_EINVAL; }
  if (!ws || ws_bytes < need) { set_error("network workspace needs %zu bytes, got %zu", need, ws_bytes); return DEHAZE_ENOMEM; }
  return DEHAZE_OK;
}

int dehaze_cnn_forward(dehaze_ctx* ctx, int n, int H, int W, const float* I, const float* t, const float* A, float* u,
                       void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int rc = check_cnn_call(ctx, n, H, W, I, t, A, ws_bytes, cnn_forward_bytes(n, H, W), ws);
  if (rc) return rc;
  if (!u) { set_error("u is required"); return DEHAZE_EINVAL; }
  DZ_HIP(hipSetDevice(ctx->c.device));
  const size_t plane = static_cast<size_t>(H) * W;
  return cnn_forward(ctx->c, n, H, W, I, W, plane, 3 * plane, t, W, plane, A, u, W, 3 * plane, ws,
                     static_cast<hipStream_t>(stream));
}

int dehaze_cnn_grad(dehaze_ctx* ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                    const float* target, float* grad, double* loss, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int rc = check_cnn_call(ctx, n, H, W, I, t, A, ws_bytes, cnn_train_bytes(n, H, W), ws);
  if (rc) return rc;
  if (!target) { set_error("target is required"); return DEHAZE_EINVAL; }
  DZ_HIP(hipSetDevice(ctx->c.device));
  return cnn_grad(ctx->c, n, H, W, I, t, A, target, grad, loss, ws, static_cast<hipStream_t>(stream));
}

int dehaze_cnn_train_step(dehaze_ctx* ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                          const float* target, float lr, double* loss, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int rc = check_cnn_call(ctx, n, H, W, I, t, A, ws_bytes, cnn_train_bytes(n, H, W), ws);
  if (rc) return rc;
  if (!target || !(lr > 0.0f)) { set_error("target and lr > 0 are required"); return DEHAZE_EINVAL; }
  DZ_HIP(hipSetDevice(ctx->c.device));
  return cnn_train_step(ctx->c, n, H, W, I, t, A, target, lr, loss, ws, static_cast<hipStream_t>(stream));
}

int dehaze_sweep_shape(const dehaze_ctx* ctx, int H, int W, int scheme, int* sweeps_per_launch, int* strip_rows,
                       int* lane_columns) {
  clear_error();
  if (!ctx || !sweeps_per_launch || !strip_rows || !lane_columns) {
    set_error("ctx and outputs are required");
    return DEHAZE_EINVAL;
  }
  return sweep_shape(ctx->c, H, W, scheme, sweeps_per_launch, strip_rows, lane_columns);
}

size_t dehaze_residual_workspace_size(int H, int W, const dehaze_params* p) {
  (void)p;
  if (H < 1 || W < 1) return 0;
  Carver cv(nullptr, ~size_t(0));
  cv.take<double>(2 * static_cast<size_t>(sweep_num_blocks(H, W)));
  cv.take<double>(2);
  return cv.used();
}

int dehaze_residual(dehaze_ctx* ctx, const float* u, const float* phi, const float* lam, int H, int W,
                    const dehaze_params* p, float* r, double* rho, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!ctx) { set_error("ctx is NULL"); return DEHAZE_EINVAL; }
  if (!u || !phi || !lam || !rho) { set_error("u, phi, lam and rho are required"); return DEHAZE_EINVAL; }
  if (H < 1 || W < 1) { set_error("image must be at least 1 x 1"); return DEHAZE_EINVAL; }
  int rc = check_params(p);
  if (rc) return rc;
  const size_t need = dehaze_residual_workspace_size(H, W, p);
  if (!ws || ws_bytes < need) {
    set_error("residual workspace needs %zu bytes, got %zu", need, ws_bytes);
    return DEHAZE_ENOMEM;
  }
  DZ_HIP(hipSetDevice(ctx->c.device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(ws, ws_bytes);
  const int nb = sweep_num_blocks(H, W);
  double* part = cv.take<double>(2 * static_cast<size_t>(nb));
  double* sums = cv.take<double>(2);
  const OpConst oc = make_opconst(*p);
  if ((rc = launch_sweep(kResidual, u, r, phi, lam, H, W, W, oc, part, s))) return rc;
  if ((rc = launch_reduce_pairs(part, nb, sums, s))) return rc;
  double h[2];
  DZ_HIP(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
  DZ_HIP(hipStreamSynchronize(s));
  *rho = h[1] > 0.0 ? std::sqrt(h[0]) / std::sqrt(h[1]) : std::sqrt(h[0]);
  if (!std::isfinite(*rho)) { set_error("residual is not finite"); return DEHAZE_ENONFINITE; }
  return DEHAZE_OK;
}

int dehaze_residual_noalloc(dehaze_ctx* ctx, const float* u, const float* phi, const float* lam, int H, int W,
                            const dehaze_params* p, float* r, double* rho, void* stream) {
  clear_error();
  if (!ctx) { set_error("ctx is NULL"); return DEHAZE_EINVAL; }
  if (!u || !phi || !lam || !rho) { set_error("u, phi, lam and rho are required"); return DEHAZE_EINVAL; }
  if (H < 1 || W < 1) { set_error("image must be at least 1 x 1"); return DEHAZE_EINVAL; }
  int rc = check_params(p);
  if (rc) return rc;
  const long long nb = (static_cast<long long>(W) + 63) / 64 * ((static_cast<long long>(H) + 15) / 16);
  if (nb > DEHAZE_NOALLOC_MAX_BLOCKS) {
    set_error("%d x %d needs %lld residual blocks; the allocation-free scratch holds %d (ceil(W/64) * ceil(H/16))",
              H, W, nb, DEHAZE_NOALLOC_MAX_BLOCKS);
    return DEHAZE_EINVAL;
  }
  char* base = static_cast<char*>(scratch_ptr(ctx->c.device));
  if (!base) { set_error("allocation-free scratch not set up on device %d", ctx->c.device); return DEHAZE_EINVAL; }
  DZ_HIP(hipSetDevice(ctx->c.device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* sums = reinterpret_cast<double*>(base);
  double* part = reinterpret_cast<double*>(base + kNoallocHead);
  // every block writes its pair and the reduction overwrites `sums`, so the
  // array needs no clearing between calls
  const OpConst oc = make_opconst(*p);
  if ((rc = launch_sweep(kResidual, u, r, phi, lam, H, W, W, oc, part, s))) return rc;
  if ((rc = launch_reduce_pairs(part, static_cast<int>(nb), sums, s))) return rc;
  return launch_rho_from_sums(sums, rho, s);
}

}  // extern "C"
