// Lagged-diffusivity (Picard) solve of the main PDE over a list of images.
//
// Every solve is watched: when over stall_window outer steps its lowest rho
// has not fallen below half its value at the window's start, an image
// started from a given iterate (the caller's u0 or a warm start)
// restarts once from Phi; any other image of a tolerance-terminated solve
// stops there, reported as stalled.  The fixed-point iteration of this
// discretisation can level off short of the tolerance (the tangential
// differences make the operator nonsymmetric), and from some starting points
// more than from Phi, the start the plain method uses.
//
// Outer step n (for every image that has not converged):
//   1. r_n = Phi - L_{D(u_n)} u_n, formed in float64 from the float64 iterate
//      u_n; D(u_n) is stored per face (float32) for the inner solve, together
//      with the inverse Jacobi diagonal; rho_n = ||r_n|| / ||Phi||.
//   2. L_{D(u_n)} delta = r_n is solved by right-preconditioned BiCGSTAB
//      (Jacobi preconditioner) in float32 until ||r_k|| <= inner_rtol ||r_n||
//      or max_inner iterations.
//   3. u_{n+1} = u_n + delta  (= L_{D(u_n)}^-1 Phi up to the inner tolerance).
// With nonlinear GMRES acceleration (KConst::ng_m > 0, depth m), step 1 is
// preceded by a least-squares mix: the current (trial) iterate ut with its
// exact residual r(ut) is combined with the last m trial iterates U_j and
// residuals R_j, u_mix = ut + sum_j b_j (ut - U_j) with b minimising
// ||r(ut) + sum_j b_j (r(ut) - R_j)||; that combination of residuals is the
// right-hand side of step 2, D stays frozen at ut, and step 3 applies the
// correction to u_mix.  (ut, r(ut)) then joins the history.  A step whose
// trial rho exceeds twice the lowest so far drops the history.
// Every launch covers the tiles of all images; per-image scalars and flags
// live on the device, so one outer step is a fixed launch sequence that can be
// captured in a HIP graph and replayed.
#pragma once

#include "internal.hpp"

namespace dz {

constexpr int kKTX = 64;   // tile width of the Krylov kernels
constexpr int kKTY = 16;   // tile height
constexpr int kKPart = 4;  // doubles of partial sums per tile

// Strip wavefronts of the BiCGSTAB operator kernels (Gaussian radius 2): one
// wavefront per (channel, group of kUOW columns, strip of KImg::us rows).
constexpr int kUOW = 60;
// Their dot products are summed per block of kSBlk rows (strip heights are
// multiples of it), so the sums, and every rounding that follows from them,
// do not depend on the strip height.
constexpr int kSBlk = 16;
// Nonlinear GMRES: at most kNgMax earlier iterates; per tile, the Gram
// entries (r - R_j).(r - R_l) for j <= l and (r - R_j).r.
constexpr int kNgMax = 8;
constexpr int kNPart = kNgMax * (kNgMax + 1) / 2 + kNgMax;

struct KImg {
  int H, W, P;             // P: pitch of every plane, >= W + 1
  int tiles_x, ntiles, tile0;
  int ucols, nunits, unit0; // strip wavefronts: column groups, count, first global index
  int us;                   // rows per strip wavefront (a multiple of kSBlk)
  int nblk, blk0;           // partial-sum blocks (channel, column group, kSBlk rows): count, first index
  const float* phi;        // 3 planes
  const float* lam;        // 1 plane
  double* u;               // 3 planes, the iterate
  double* un;              // 3 planes, u_n: D stays frozen at it during defect-correction passes
  float* Dx;               // 3 planes of H rows: face f of row j sits left of column f (f = 0..W)
  float* Dy;               // 3 planes of H + 1 rows: face f of column i sits above row f (f = 0..H)
  float* invd;             // 3 planes: 1 / diag(L_D)
  float* rhat;             // 3 planes: r_n, also the BiCGSTAB shadow residual
  float* r;                // 3 planes
  float* p[2];             // search direction, ping-pong between iterations
  float* v[2];             // L M^-1 p, ping-pong between iterations
  float* s;
  float* t;
  float* x;                // 3 planes: the correction delta
  double* Uh;              // nonlinear GMRES: m earlier trial iterates, 3 planes each (nullptr if m = 0)
  float* Rh;               // their residuals, 3 planes each
};

struct KScal {
  double rho, alpha, omega, beta;
  double bnorm2;           // ||r_n||^2 in float32 terms
  double rel;              // rho_n = ||r_n|| / ||Phi|| (float64)
  double rel0;             // rho at the starting iterate
  int converged;           // rho <= rel_tol reached (or stopped on a non-finite value)
  int nonfinite;
  int inner_done, half_done;
  int inner_this;          // BiCGSTAB iterations of the current outer step
  int pass_inner;          // BiCGSTAB iterations of the current solve pass
  int outer;               // updates applied
  long long inner_total;
  long long res_evals;
  // stall watch (solves started from a given iterate): lowest rho so far, its
  // value at the start of the current window, steps into the window
  double best, mark;
  int since;
  int warm;                // started from a given iterate
  int restart;             // restart from Phi at the next residual pass
  int restarted;           // restarted once already
  int stalled;             // stopped: rho stopped falling (tolerance-terminated solves)
  double rel_out;          // rho of the iterate rounded to float32 (the returned u)
  int it;                  // BiCGSTAB iteration of the current inner solve (1-based)
  int passes;              // residual passes that may start a step (defect-correction passes excluded)
  int exhausted;           // max_outer steps taken: done iterating
  // nonlinear GMRES: mixing coefficients, lowest trial rho since the history
  // was last dropped, entries in the history, slot of the next entry, and
  // whether this step's mix is due
  double ngb[kNgMax];
  double ng_best;
  int ng_nh, ng_slot, ng_pending;
  int ng_drops;            // times the history was dropped
};

struct KConst {
  float w[9];
  float wc2;
  float eps;
  double eps64;
  double w64[9];
  double wc2_64;
  double rel_tol;
  double eta;
  int R;
  int nonlocal_term;
  int edge_preserving;
  int stall_window;        // 0: never restart
  int max_inner;
  int max_outer;
  int trial;               // launch-shape trials: the strip kernels skip the per-image state tests
  int ng_m;                // nonlinear GMRES depth (0: plain lagged diffusivity)
};
KConst make_kconst(const dehaze_params& p);

// Bytes of one image's planes (internal pitch; ng_m earlier iterates for
// nonlinear GMRES) and its tile count.
size_t krylov_image_bytes(int H, int W, int ng_m);
int krylov_tiles(int H, int W);
int krylov_units(int H, int W, int us);
int krylov_blocks(int H, int W);
// Whether the strip kernels can address an image (32-bit byte offsets within
// every plane, the y-face plane of H + 1 rows included).
bool krylov_strips_fit(int H, int W);
// Rows per strip wavefront of each image of a launch of n images (us[i]) by
// the size rule, the tuner's starting point and fallback.
void krylov_strip_rows(int n, const int* H, const int* W, int* us);
// Fills a descriptor whose planes live at `base` (krylov_image_bytes bytes,
// 256-byte aligned); phi/lam are carved here too and returned through the
// descriptor (the front end writes them).
KImg krylov_carve(void* base, int H, int W, int tile0, int unit0, int blk0, int us, int ng_m);

struct KrylovBatch {
  const KImg* d_imgs;      // device copy of the descriptors
  KScal* d_scal;           // device scalars, one per image
  const int* d_tile_img;   // image index of every tile
  double* d_part;          // kKPart doubles per tile
  int nimg;
  int ntiles;
  const int* d_unit_img;   // image index of every strip wavefront
  double* d_upart;         // kKPart doubles per strip wavefront
  int nunits;
  double* d_npart;         // nonlinear GMRES: kNPart doubles per tile (nullptr if unused)
};

// Uploads the descriptors and the strip-wavefront -> image map (b.nunits
// wavefronts in all; none when b.nunits is 0).
int krylov_upload_strips(const KrylovBatch& b, const KImg* h_imgs, hipStream_t s);
// Starting iterate: u = u0 (float, dense pitch W) or Phi; resets the scalars
// and uploads the descriptors and maps.
int krylov_init(const KrylovBatch& b, const KImg* h_imgs, const float* const* u0, hipStream_t s);
// Residual pass (final != 0: evaluate every image, converged or not).
int krylov_residual(const KrylovBatch& b, const KConst& c, int final, hipStream_t s);
// Linear residual Phi - L_{D(u_n)} u with D frozen at the snapshot u_n, as the
// right-hand side of a defect-correction pass.
int krylov_linear_residual(const KrylovBatch& b, const KConst& c, hipStream_t s);
// u_n := u for every image still iterating.
int krylov_snapshot(const KrylovBatch& b, hipStream_t s);
// Times one launch of the strip operator kernel (a) over every image with the
// descriptors currently on the device (trial mode: no state tests, results
// discarded); *us receives the average in microseconds over `reps` launches.
int krylov_time_strips(const KrylovBatch& b, const KConst& c, int reps, hipStream_t s, float* us);
// One BiCGSTAB iteration of every image inside an inner solve (each image
// keeps its own iteration count; an inner solve ends at its tolerance or after
// max_inner iterations).
int krylov_inner(const KrylovBatch& b, const KConst& c, hipStream_t s);
// Nonlinear GMRES mix for every image whose residual pass just ended a step
// (Gram sums, least squares, mix and history update); it then starts the
// image's inner solve.  Nothing to do when c.ng_m = 0.
int krylov_ngmres(const KrylovBatch& b, const KConst& c, hipStream_t s);
// u += delta.
int krylov_update(const KrylovBatch& b, hipStream_t s);
// u (float64) -> out (float, dense pitch W), or unchanged into a double array.
int krylov_output(const KImg& img, float* out, hipStream_t s);
int krylov_output64(const KImg& img, double* out, hipStream_t s);

}  // namespace dz
