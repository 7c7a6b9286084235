/*
 * dehaze.h - C ABI of the MI355X (gfx950) PDE dehazing library.
 *
 * The library computes, for a hazy RGB image I, the front end of Section II-D
 * (dark channel, transmission t, adaptive weight lambda(t)) with the
 * atmospheric light A, the reconstruction Phi(I, t, A) of Section II-A, and
 * solves the main PDE
 *
 *     -div(D(grad u) grad u) + lambda(t) G(u) = Phi(I, t, A),
 *     D(grad u) = (|grad u| + eps)^-1,  u = 0 outside the image,
 *
 * discretised as in Appendix A-2 (face coefficients from the forward normal
 * difference and the central tangential difference at the lower-index cell;
 * G a (2R+1)^2 Gaussian with taps normalised to sum 1, zero outside the
 * image), by one of three fixed-point iterations (Appendix A-1 and the
 * lagged-diffusivity reading of it).
 *
 * Conventions for every entry point:
 *   - Image pointers are DEVICE pointers owned by the caller.  The library
 *     never frees them and keeps no reference after the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Outputs are valid once that stream has been synchronised, except where
 *     an entry point says it synchronises itself.
 *   - Planar ("CHW") float images hold 3 planes of H rows; row r of plane c
 *     starts at element (c * H + r) * pitch.  Interleaved ("HWC") images hold
 *     3 values per pixel; row r starts at element 3 * r * pitch.  pitch >= W
 *     counts pixels.  Outputs written by the library (u, t, t_d, lambda, ...)
 *     use pitch W (dense) unless stated otherwise.
 *   - Scratch memory ("workspace") is passed in by the caller: `ws` must be
 *     a device buffer of at least the size the matching *_workspace_size call
 *     reports, aligned to 256 bytes.  Its contents need not be initialised.
 *   - Return value: DEHAZE_OK (0) or a negative DEHAZE_E* code; no exception
 *     crosses the ABI.  dehaze_last_error() gives a message for the calling
 *     thread's last failure.
 *   - Calls on different contexts may run concurrently from different host
 *     threads; one context must not be used by two threads at once.
 */
#ifndef DEHAZE_H
#define DEHAZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define DEHAZE_OK          0
#define DEHAZE_EINVAL     -1  /* bad size, parameter or NULL required pointer */
#define DEHAZE_ENOMEM     -2  /* workspace too small */
#define DEHAZE_EHIP       -3  /* a HIP runtime call failed (see dehaze_last_error) */
#define DEHAZE_ENOTCONV   -4  /* rel_tol not reached within max_outer; u holds the last iterate */
#define DEHAZE_ENONFINITE -5  /* NaN or Inf met in the input or the residual */

/* ------------------------------------------------------------ enumerations */
#define DEHAZE_U8  0          /* 8-bit codes; intensity = code / 255, correctly rounded */
#define DEHAZE_F32 1          /* float32 intensities (not clipped) */

#define DEHAZE_HWC 0          /* interleaved RGB */
#define DEHAZE_CHW 1          /* planar RGB */

#define DEHAZE_U_F32 0         /* u is returned as float32 (u points to 3 planes of float) */
#define DEHAZE_U_F64 1         /* u is returned as float64 (u points to 3 planes of double) */

#define DEHAZE_PAPER_EXPLICIT 0  /* u += tau r(u), Appendix A-1 as printed */
#define DEHAZE_JACOBI         1  /* u += theta r(u) / diag(L_D(u)), D recomputed every sweep */
#define DEHAZE_PICARD_KRYLOV  2  /* lagged diffusivity: u_{n+1} = L_{D(u_n)}^-1 Phi, each
                                    linear solve by Jacobi-preconditioned BiCGSTAB */

/* ------------------------------------------------------------ parameters */
typedef struct dehaze_params {
  int32_t patch;            /* dark-channel patch side, odd (Section II-D: 15) */
  int32_t g_radius;         /* Gaussian radius R, kernel (2R+1)^2 (Appendix A-2: 2), 0..4 */
  double  omega;            /* t = 1 - omega t_d (Section II-D: 0.95) */
  double  t0;               /* Phi threshold (Section II-A: "small"; 0.1) */
  double  eps;              /* D stabiliser (Section II-B: 1e-3) */
  double  sigma;            /* Gaussian width (Section II-C: 2.0; default 1.5) */
  double  lambda0;          /* lambda = lambda0 exp(-beta (1 - t)) (Section II-D: 0.5) */
  double  beta_lambda;      /* (Section II-D: 3.0) */
  double  tau;              /* explicit relaxation (Appendix A-1: 0.2) */
  double  theta;            /* Jacobi damping (0.8) */
  double  rel_tol;          /* stop when ||r||/||Phi|| <= rel_tol; <= 0: run exactly max_outer */
  double  inner_rtol;       /* Krylov solve tolerance relative to its start residual */
  int32_t scheme;           /* DEHAZE_PAPER_EXPLICIT, DEHAZE_JACOBI, DEHAZE_PICARD_KRYLOV */
  int32_t max_outer;        /* sweeps (explicit, Jacobi) or lagged-diffusivity steps */
  int32_t max_inner;        /* BiCGSTAB iterations per lagged-diffusivity step */
  int32_t check_every;      /* with inner_refine > 0: outer steps per captured graph, after which the host
                               reads the stopping flags (>= 1); the default loop ignores it */
  int32_t atm_divisor;      /* A from the top max(1, HW / atm_divisor) dark-channel pixels */
  int32_t warm_start;       /* starting iterate of the lagged-diffusivity solve (u0 must then be NULL):
                               0 = Phi (or u0); 2 = B = Phi / lambda, the solution of lambda u = Phi,
                               to which the main PDE reduces where u is smooth (B = Phi without the
                               nonlocal term or with lambda = 0); 1 = B plus the network's learned
                               correction (needs loaded weights) */
  int32_t nonlocal_term;    /* 0: drop lambda G (ablation) */
  int32_t adaptive;         /* 0: lambda = lambda0 everywhere (ablation) */
  int32_t edge_preserving;  /* 0: D = 1 (ablation; the solve becomes linear) */
  int32_t sweeps_per_launch;/* explicit/Jacobi sweeps fused per kernel launch (1..4, temporal blocking;
                               R = 2 only); 0 = time the launch shapes on the first solve of each image
                               size (synchronises once) and keep the fastest in the context */
  int32_t inner_refine;     /* extra defect-correction passes per lagged-diffusivity step: with D frozen
                               at u_n, re-form Phi - L_{D(u_n)} u in float64 and solve again (0 = one solve) */
  int32_t strip_rows;       /* output rows per wavefront of the register-resident sweep kernel; 0 = the
                               tuned value (every value gives bit-identical results) */
  int32_t lane_columns;     /* adjacent columns per lane of that kernel (1 or 2); 0 = tuned */
  int32_t stall_window;     /* lagged-diffusivity solves: if over this many outer steps the lowest rho did
                               not fall below half its value at the window's start, an image that
                               started from a given iterate (u0 or a warm start) restarts once from Phi;
                               otherwise, when rel_tol > 0, its solve stops there (DEHAZE_ENOTCONV,
                               stats.stalled = 1).  0 = never; default 256 */
  int32_t guided_radius;    /* > 0: refine the estimated t with a guided filter (guide: channel mean of I,
                               window (2r+1)^2 clipped to the image, He-Sun-Tang).  Table II ablates a
                               guided filter without defining it; 0 (default) = the printed method */
  int32_t dark_scales;      /* t_d averaged over patch sides ((patch - 1) >> k) | 1, k < dark_scales: a
                               reading of the multiscale dark channel Table II ablates; 1 (default) = off */
  double  guided_eps;       /* guided-filter regulariser (default 1e-3) */
  int32_t u_state;          /* precision of the returned u: DEHAZE_U_F32 (default) rounds the solution to
                               float32; DEHAZE_U_F64 returns it in float64, and then the `u` argument of
                               dehaze_solve and the `u` of every dehaze_image must point to 3 * H * W
                               doubles (cast to float*).  The lagged-diffusivity solve iterates in float64,
                               so only DEHAZE_U_F64 hands back an iterate whose residual meets rel_tol
                               (rel_residual_out == rel_residual); the sweep schemes iterate in float32
                               and return that iterate widened */
  int32_t krylov_rows;      /* rows per wavefront of the BiCGSTAB strip kernels (lagged-diffusivity
                               solves, R = 2): a multiple of 16 up to 512; 0 = time the candidates on the
                               first solve of each batch composition (synchronises) and keep the fastest
                               in the context.  Every value gives bit-identical results */
  int32_t ngmres_depth;     /* lagged-diffusivity solves: 0 = the plain iteration; 1..8 = accelerate it by
                               nonlinear GMRES over that many earlier iterates (each outer step mixes the
                               current iterate with them to minimise the linearised residual, then takes
                               the lagged-diffusivity correction from the mix; same fixed point).  Needs
                               inner_refine = 0; the workspace grows by 36 bytes per pixel and depth */
  int32_t reserved[1];      /* must be zero */
} dehaze_params;

typedef struct dehaze_stats {
  int32_t outer;            /* outer steps taken (sweeps or lagged-diffusivity steps) */
  int32_t converged;        /* 1 if rel_tol was reached */
  int64_t inner;            /* BiCGSTAB iterations in total */
  int64_t applications;     /* operator applications (sweeps or matrix-vector products) */
  double  rel_residual;     /* ||Phi - L_{D(u)} u|| / ||Phi|| (float64 sum) at the final iterate; the
                               lagged-diffusivity solves iterate in float64, and rel_tol is tested
                               against this value */
  double  rel_residual0;    /* the same at the starting iterate */
  float   A[3];             /* atmospheric light used */
  int32_t status;           /* DEHAZE_OK, DEHAZE_ENOTCONV or DEHAZE_ENONFINITE for this image */
  int32_t restarts;         /* 1 if the solve stalled from its given start and restarted from Phi */
  int32_t stalled;          /* 1 if the solve stopped early because rho stopped falling */
  double  rel_residual_out; /* the same residual at the returned u.  With DEHAZE_U_F32, rounding u to
                               float32 perturbs each flux by up to ulp(u) / eps, so where u is large
                               and flat this sits at a floor well above rel_residual (e.g. 7.6e-4 for
                               a 1080p image with u near 32 whose iterate met 1e-5); with DEHAZE_U_F64
                               it equals rel_residual.  The sweep schemes iterate in float32 and report
                               rel_residual here too */
} dehaze_stats;

typedef struct dehaze_ctx dehaze_ctx;

/* Fills *p with the defaults listed above (scheme = DEHAZE_PICARD_KRYLOV,
   max_outer = 5000, max_inner = 128, rel_tol = 1e-5, inner_rtol = 0.2,
   check_every = 16, inner_refine = 0, stall_window = 256).  Returns DEHAZE_EINVAL for NULL. */
int dehaze_params_default(dehaze_params* p);

/* sizeof(dehaze_params) and sizeof(dehaze_stats), so bindings can check their mirrors. */
size_t dehaze_params_size(void);
size_t dehaze_stats_size(void);

/* Creates a context on HIP device `device` (it becomes current for the
   calling thread).  The context owns kernel-launch tables, captured graphs
   and the network weights.  DEHAZE_EHIP if the device cannot be used. */
int dehaze_ctx_create(dehaze_ctx** ctx, int device);
void dehaze_ctx_destroy(dehaze_ctx* ctx);

/* Message for the calling thread's last failure ("" if none). */
const char* dehaze_last_error(void);
const char* dehaze_strerror(int code);

/* ------------------------------------------------------------ front end
 * Section II-D (dark channel, t = clamp(1 - omega t_d, 0, 1), lambda(t)) and
 * Section II-A (Phi), with A from the dark-channel-prior rule (the paper
 * takes A as given): the top max(1, HW / atm_divisor) pixels of the raw dark
 * channel (ties to the lower linear index), then the one with the largest
 * R+G+B summed in float64 as (R+G)+B (ties to the lower index).
 *
 *   I        image (dtype, layout, pitch as above), H, W >= 1
 *   A_in     3 floats on the device, or NULL to estimate A
 *   dark     raw dark channel min_c min_patch I^c (H x W float, nullable)
 *   dark_u8  the same as 8-bit codes (H x W, nullable; only for DEHAZE_U8)
 *   t_d      min_c min_patch I^c / A^c, float32 division (H x W, nullable)
 *   t, lam   transmission and lambda(t) (H x W, nullable)
 *   phi      Phi^c = (I^c - A^c (1 - t)) / max(t, t0) (planar, pitch W, nullable)
 *   A_out    3 floats on the device receiving A (required)
 * Errors: EINVAL (H or W < 1, pitch < W, even or non-positive patch,
 * t0, eps or sigma <= 0, omega outside (0, 1], unknown dtype or layout, NULL
 * I or A_out), ENOMEM (ws_bytes too small), EHIP.  A_in lives on the device
 * and is not read back: an A_in (or, in dehaze_solve and dehaze_batch, an A)
 * with a channel that is not positive and finite makes t_d, t, lam and phi
 * NaN, which dehaze_solve and dehaze_batch report as DEHAZE_ENONFINITE. */
size_t dehaze_prior_workspace_size(int H, int W, const dehaze_params* p);
int dehaze_prior(dehaze_ctx* ctx, const void* I, int dtype, int layout, int H, int W, int pitch,
                 const dehaze_params* p, const float* A_in,
                 float* dark, uint8_t* dark_u8, float* t_d, float* t, float* lam, float* phi,
                 float* A_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ one image solve
 * Builds lambda(t) and Phi(I, t, A) from the given t (H x W, pitch W) and A
 * (3 device floats), then iterates p->scheme from u0 (planar, pitch W;
 * NULL = Phi, or the warm start p->warm_start selects) into u (planar, pitch W).
 *   DEHAZE_PAPER_EXPLICIT, DEHAZE_JACOBI: p->max_outer sweeps, each one pass
 *     of the face-coefficient recompute and the update (Appendix A-1).
 *   DEHAZE_PICARD_KRYLOV: lagged-diffusivity steps; the residual of the
 *     current iterate is formed in float64 from the float64 iterate, each
 *     correction L_{D(u_n)} delta = r_n is solved by BiCGSTAB in float32
 *     (to inner_rtol, at most max_inner iterations).
 * With rel_tol > 0 the solve stops once rho <= rel_tol (tested on the device
 * after every step) and returns DEHAZE_ENOTCONV if max_outer passes first.
 * `stats` (host, nullable) is filled.  The sweep schemes synchronise
 * `stream` when stats is non-NULL or rel_tol > 0; DEHAZE_PICARD_KRYLOV always
 * does (the host reads the per-image state between graph replays).
 * u is not clipped: the solution of the PDE exceeds the [0, 1] range. */
size_t dehaze_solve_workspace_size(int H, int W, const dehaze_params* p);
int dehaze_solve(dehaze_ctx* ctx, const void* I, int dtype, int layout, int H, int W, int pitch,
                 const float* t, const float* A, const dehaze_params* p, const float* u0,
                 float* u, void* ws, size_t ws_bytes, dehaze_stats* stats, void* stream);

/* ------------------------------------------------------------ batch solve
 * Many images of uneven size solved together by the lagged-diffusivity
 * scheme (DEHAZE_PICARD_KRYLOV only): every kernel launch covers the tiles of
 * all images still iterating, the per-image reductions and stopping tests run
 * on the device, and groups of 64 ticks are captured once in a HIP graph and
 * replayed until every image reaches rel_tol (or max_outer, or stalls).  In a
 * tick each image does the next thing it needs (the residual pass that
 * starts a step, one BiCGSTAB iteration, or the update that ends the step),
 * at its own pace.  With inner_refine > 0, groups of check_every outer steps
 * of max_inner iterations per pass are captured instead.
 * Per image, t and A are taken as given or, when NULL, estimated by the
 * front end of dehaze_prior (Section II-D); lambda(t) and Phi follow
 * (Sections II-A, II-D).  The call synchronises `stream`.  stats (host, n
 * entries, nullable) receives each image's counts, residuals, A and status.  Returns DEHAZE_OK, or the worst
 * per-image status (DEHAZE_ENONFINITE before DEHAZE_ENOTCONV), or an error.
 * The context keeps the captured graph for reuse by a later call with the
 * same workspace, batch layout and parameters. */
typedef struct dehaze_image {
  const void* I;        /* image (the call's dtype and layout) */
  int32_t H, W, pitch;  /* size and pitch in pixels, pitch >= W */
  int32_t reserved;     /* must be zero */
  float* u;             /* output: planar, pitch W */
  const float* t;       /* H x W transmission, or NULL to estimate it */
  const float* A;       /* 3 device floats, or NULL to estimate them */
  const float* u0;      /* starting iterate (planar, pitch W), or NULL for Phi */
  float* t_out;         /* nullable: receives the estimated t (H x W) */
  float* A_out;         /* nullable: receives the estimated A (3 floats) */
} dehaze_image;

size_t dehaze_batch_workspace_size(int n, const dehaze_image* imgs, const dehaze_params* p);
/* Rows per wavefront of the BiCGSTAB strip kernels that a lagged-diffusivity
 * solve of this batch (or, with n = 1, dehaze_solve of that image) uses for
 * each image: rows[i] (host, n entries) is the height the context timed as
 * fastest for this composition of image sizes (*tuned = 1), else
 * p->krylov_rows or the size rule the timing starts from (*tuned = 0).
 * rows[i] = 0 for every image when the tile kernels run instead: g_radius !=
 * 2, or some image's planes exceed the strips' 32-bit byte offsets ((H + 1) *
 * roundup(W + 1, 64) * 4 >= 2^31).  Only the sizes of imgs are read; ctx may
 * be NULL (the rule alone).  Host only, no device work.  Errors: EINVAL. */
int dehaze_batch_strip_rows(const dehaze_ctx* ctx, int n, const dehaze_image* imgs, const dehaze_params* p,
                            int* rows, int* tuned);
int dehaze_batch(dehaze_ctx* ctx, int n, const dehaze_image* imgs, int dtype, int layout,
                 const dehaze_params* p, void* ws, size_t ws_bytes, dehaze_stats* stats, void* stream);

/* ------------------------------------------------------------ warm-start network
 * The paper ends its introduction by pointing at hybrids of the PDE with
 * learned models; this network corrects the analytic start B = Phi / lambda
 * (see warm_start): the lagged-diffusivity solve starts from B + network
 * (warm_start = 1) and then runs to its own residual test exactly as from a
 * cold start.  The network is trained on u* - B for converged solutions u*.
 * Architecture: six 3x3 convolutions 7 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3,
 * ReLU after the first five, zero padding, input [I^R, I^G, I^B, t, A^R,
 * A^G, A^B] per pixel, output (u - B) / 8 (dehaze_cnn_forward returns the
 * output multiplied by 8, i.e. the correction itself).  bfloat16 weights
 * and activations, float32 accumulation on the matrix cores.
 *
 * Parameters are float32 on the host, layer by layer: W[co][ci][3][3] then
 * b[co] (dehaze_cnn_param_count() values in all).  The context keeps a
 * float32 master copy, the Adam moments and the bfloat16 packings.
 * Training images are dense and share one size: I is n x 3 x H x W planar
 * float, t n x H x W, A n x 3, target (converged solutions) n x 3 x H x W,
 * all on the device.  The loss is the mean squared error of u against target.
 * Errors: EINVAL (no weights loaded, wrong count, bad sizes), ENOMEM, EHIP. */
size_t dehaze_cnn_param_count(void);
int dehaze_cnn_set_weights(dehaze_ctx* ctx, const float* w, size_t count);   /* host; resets Adam */
int dehaze_cnn_get_weights(dehaze_ctx* ctx, float* w, size_t count);         /* host */
size_t dehaze_cnn_workspace_size(int n, int H, int W, int training);
/* u (n x 3 x H x W planar) = the network's output times 8: its correction to B. */
int dehaze_cnn_forward(dehaze_ctx* ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                       float* u, void* ws, size_t ws_bytes, void* stream);
/* Gradient of the loss wrt the parameters (device, param_count floats, layout
   as above) and the loss itself (host, synchronises). */
int dehaze_cnn_grad(dehaze_ctx* ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                    const float* target, float* grad, double* loss, void* ws, size_t ws_bytes, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr;
   loss (host, nullable) receives the loss before the step. */
int dehaze_cnn_train_step(dehaze_ctx* ctx, int n, int H, int W, const float* I, const float* t, const float* A,
                          const float* target, float lr, double* loss, void* ws, size_t ws_bytes, void* stream);

/* Launch shape the context's tuner chose for explicit/Jacobi sweeps of an
   H x W image: *sweeps_per_launch (0 if none has been chosen yet, or if the
   tile kernel is used because g_radius != 2 or a plane exceeds 2 GiB),
   *strip_rows and *lane_columns.  Host pointers; EINVAL if any is NULL. */
int dehaze_sweep_shape(const dehaze_ctx* ctx, int H, int W, int scheme, int* sweeps_per_launch, int* strip_rows,
                       int* lane_columns);

/* ------------------------------------------------------------ residual
 * rho = ||Phi - L_{D(u)} u||_2 / ||Phi||_2 over all channels, for planar
 * u, phi (pitch W) and lam (H x W): the quantity the main PDE sets to zero.
 * r (planar, pitch W, nullable) receives Phi - L_{D(u)} u.  Synchronises
 * `stream` and writes *rho (host). */
size_t dehaze_residual_workspace_size(int H, int W, const dehaze_params* p);
int dehaze_residual(dehaze_ctx* ctx, const float* u, const float* phi, const float* lam,
                    int H, int W, const dehaze_params* p, float* r, double* rho,
                    void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ allocation-free residual
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * what dehaze_residual computes, with the same kernels, but takes no
 * workspace, allocates nothing and does not synchronise: its per-block
 * partial sums live in a library-owned device array of 256 bytes + 16 bytes
 * per block (1 MiB + 256 bytes), one per GPU, held until the process ends,
 * and rho is written to device memory.
 *   u, phi, lam, H, W, p, r   as in dehaze_residual (r nullable)
 *   rho    ONE DEVICE double receiving ||Phi - L_{D(u)} u|| / ||Phi||; it is
 *          NaN or Inf when the residual is not finite (no host-side check)
 * Limit: ceil(W / 64) * ceil(H / 16) <= DEHAZE_NOALLOC_MAX_BLOCKS (e.g. 8192
 * x 8192); larger images return DEHAZE_EINVAL.  Every call on one GPU shares
 * that GPU's array and leaves its own sums there: calls that overlap on one
 * GPU (different streams, threads or contexts) race, so the caller must
 * order them.  Errors: EINVAL (NULL pointer, size, parameters), EHIP. */
#define DEHAZE_NOALLOC_MAX_BLOCKS 65536
int dehaze_residual_noalloc(dehaze_ctx* ctx, const float* u, const float* phi, const float* lam,
                            int H, int W, const dehaze_params* p, float* r, double* rho, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DEHAZE_H */
