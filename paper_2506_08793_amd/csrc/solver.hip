// One-image solve: builds lambda(t) and Phi(I, t, A) (Sections II-A, II-D),
// picks the starting iterate and runs the chosen fixed-point iteration
// (Appendix A-1) with its stopping rule.
#include <cmath>

#include "internal.hpp"
#include "krylov.hpp"
#include "solver.hpp"

namespace dz {

namespace {

struct SweepPlan {
  int P = 0;
  float* Ip = nullptr;   // 3 planes
  float* phi = nullptr;  // 3 planes
  float* lam = nullptr;  // 1 plane
  float* ua = nullptr;   // 3 planes
  float* ub = nullptr;   // 3 planes
  double* part = nullptr;
  double* sums = nullptr;
  size_t bytes = 0;
};

SweepPlan plan_sweeps(void* ws, int H, int W) {
  SweepPlan pl;
  pl.P = padded_pitch(W);
  const size_t plane = static_cast<size_t>(H) * pl.P;
  Carver cv(ws, ~size_t(0));
  pl.Ip = cv.take<float>(3 * plane);
  pl.phi = cv.take<float>(3 * plane);
  pl.lam = cv.take<float>(plane);
  pl.ua = cv.take<float>(3 * plane);
  pl.ub = cv.take<float>(3 * plane);
  pl.part = cv.take<double>(2 * static_cast<size_t>(sweep_num_blocks(H, W)));
  pl.sums = cv.take<double>(2);
  pl.bytes = cv.used();
  return pl;
}

// rho = ||Phi - L_{D(u)} u|| / ||Phi|| of the planar field u; synchronises s.
int residual_of(const float* u, const SweepPlan& pl, int H, int W, const OpConst& oc, double* rho,
                hipStream_t s) {
  int rc = launch_sweep(kResidual, u, nullptr, pl.phi, pl.lam, H, W, pl.P, oc, pl.part, s);
  if (rc) return rc;
  if ((rc = launch_reduce_pairs(pl.part, sweep_num_blocks(H, W), pl.sums, s))) return rc;
  double h[2];
  DZ_HIP(hipMemcpyAsync(h, pl.sums, sizeof(h), hipMemcpyDeviceToHost, s));
  DZ_HIP(hipStreamSynchronize(s));
  *rho = h[1] > 0.0 ? std::sqrt(h[0]) / std::sqrt(h[1]) : std::sqrt(h[0]);
  return DEHAZE_OK;
}

int run_sweeps(const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  const int H = a.H, W = a.W;
  SweepPlan pl = plan_sweeps(a.ws, H, W);
  int rc;
  if ((rc = launch_to_planar(a.I, a.dtype, a.layout, H, W, a.pitch, pl.Ip, pl.P, s))) return rc;
  FusedOut fo{nullptr, nullptr, pl.lam, pl.phi, pl.P};
  if ((rc = launch_prior_fused(nullptr, pl.Ip, pl.P, a.t, W, a.A, H, W, p, fo, s))) return rc;
  if (a.u0) rc = launch_copy3(a.u0, W, pl.ua, pl.P, H, W, s);
  else rc = launch_copy3(pl.phi, pl.P, pl.ua, pl.P, H, W, s);
  if (rc) return rc;

  const OpConst oc = make_opconst(p);
  const int mode = p.scheme == DEHAZE_PAPER_EXPLICIT ? kExplicit : kJacobi;
  float* cur = pl.ua;
  float* nxt = pl.ub;
  int done = 0;
  bool conv = false;
  double rho0 = NAN, rho = NAN;
  int status = DEHAZE_OK;
  if (p.rel_tol > 0.0) {
    for (;;) {
      if ((rc = residual_of(cur, pl, H, W, oc, &rho, s))) return rc;
      if (done == 0) rho0 = rho;
      if (!std::isfinite(rho)) { status = DEHAZE_ENONFINITE; break; }
      if (rho <= p.rel_tol) { conv = true; break; }
      if (done >= p.max_outer) { status = DEHAZE_ENOTCONV; break; }
      const int k = std::min(p.check_every, p.max_outer - done);
      for (int i = 0; i < k; ++i) {
        if ((rc = launch_sweep(mode, cur, nxt, pl.phi, pl.lam, H, W, pl.P, oc, nullptr, s))) return rc;
        std::swap(cur, nxt);
      }
      done += k;
    }
  } else {
    if (st && (rc = residual_of(cur, pl, H, W, oc, &rho0, s))) return rc;
    for (int i = 0; i < p.max_outer; ++i) {
      if ((rc = launch_sweep(mode, cur, nxt, pl.phi, pl.lam, H, W, pl.P, oc, nullptr, s))) return rc;
      std::swap(cur, nxt);
    }
    done = p.max_outer;
    if (st) {
      if ((rc = residual_of(cur, pl, H, W, oc, &rho, s))) return rc;
      if (!std::isfinite(rho)) status = DEHAZE_ENONFINITE;
    }
  }
  if ((rc = launch_copy3(cur, pl.P, a.u, W, H, W, s))) return rc;
  if (st) {
    st->outer = done;
    st->converged = conv ? 1 : 0;
    st->inner = 0;
    st->applications = done;
    st->rel_residual = rho;
    st->rel_residual0 = rho0;
    DZ_HIP(hipMemcpyAsync(st->A, a.A, 3 * sizeof(float), hipMemcpyDeviceToHost, s));
    DZ_HIP(hipStreamSynchronize(s));
    st->status = status;
  }
  if (status == DEHAZE_ENONFINITE) set_error("residual is not finite");
  else if (status == DEHAZE_ENOTCONV) set_error("rel_tol %g not reached in %d sweeps (rho %g)", p.rel_tol, done, rho);
  return status;
}

struct KrylovPlan {
  KImg img{};
  float* Ip = nullptr;
  KImg* d_imgs = nullptr;
  KScal* d_scal = nullptr;
  int* d_tile_img = nullptr;
  double* d_part = nullptr;
  size_t bytes = 0;
};

KrylovPlan plan_krylov(void* ws, int H, int W) {
  KrylovPlan pl;
  Carver cv(ws, ~size_t(0));
  char* arena = cv.take<char>(krylov_image_bytes(H, W));
  pl.img = krylov_carve(arena, H, W, 0);
  const int nt = krylov_tiles(H, W);
  pl.Ip = cv.take<float>(3 * static_cast<size_t>(H) * pl.img.P);
  pl.d_imgs = cv.take<KImg>(1);
  pl.d_scal = cv.take<KScal>(1);
  pl.d_tile_img = cv.take<int>(nt);
  pl.d_part = cv.take<double>(static_cast<size_t>(kKPart) * nt);
  pl.bytes = cv.used();
  return pl;
}

int read_scalars(const KrylovBatch& b, KScal* h, hipStream_t s) {
  DZ_HIP(hipMemcpyAsync(h, b.d_scal, sizeof(KScal) * b.nimg, hipMemcpyDeviceToHost, s));
  DZ_HIP(hipStreamSynchronize(s));
  return DEHAZE_OK;
}

void fill_stats(const KScal& k, dehaze_stats* st) {
  st->outer = k.outer;
  st->converged = (k.converged && !k.nonfinite) ? 1 : 0;
  st->inner = k.inner_total;
  st->applications = 2 * k.inner_total + k.res_evals;
  st->rel_residual = k.rel;
  st->rel_residual0 = k.rel0;
  st->status = k.nonfinite ? DEHAZE_ENONFINITE : DEHAZE_OK;
}

int run_krylov(const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  const int H = a.H, W = a.W;
  KrylovPlan pl = plan_krylov(a.ws, H, W);
  const int P = pl.img.P;
  int rc;
  if ((rc = launch_to_planar(a.I, a.dtype, a.layout, H, W, a.pitch, pl.Ip, P, s))) return rc;
  FusedOut fo{nullptr, nullptr, const_cast<float*>(pl.img.lam), const_cast<float*>(pl.img.phi), P};
  if ((rc = launch_prior_fused(nullptr, pl.Ip, P, a.t, W, a.A, H, W, p, fo, s))) return rc;
  KrylovBatch b{pl.d_imgs, pl.d_scal, pl.d_tile_img, pl.d_part, 1, pl.img.ntiles};
  const float* u0 = a.u0;
  if ((rc = krylov_init(b, &pl.img, &u0, s))) return rc;
  const KConst kc = make_kconst(p);
  KScal hs{};
  for (int n = 0; n < p.max_outer; ++n) {
    if ((rc = krylov_residual(b, kc, 0, s))) return rc;
    if (p.inner_refine > 0 && (rc = krylov_snapshot(b, s))) return rc;
    for (int pass = 0; pass <= p.inner_refine; ++pass) {
      if (pass > 0 && (rc = krylov_linear_residual(b, kc, s))) return rc;
      for (int it = 1; it <= p.max_inner; ++it)
        if ((rc = krylov_inner(b, kc, it, s))) return rc;
      if ((rc = krylov_update(b, s))) return rc;
    }
    if (p.rel_tol > 0.0 && (n + 1) % p.check_every == 0) {
      if ((rc = read_scalars(b, &hs, s))) return rc;
      if (hs.converged) break;
    }
  }
  if ((rc = krylov_residual(b, kc, 1, s))) return rc;
  if ((rc = krylov_output(pl.img, a.u, s))) return rc;
  if (!st && p.rel_tol <= 0.0) return DEHAZE_OK;
  if ((rc = read_scalars(b, &hs, s))) return rc;
  int status = hs.nonfinite ? DEHAZE_ENONFINITE
                            : ((p.rel_tol > 0.0 && !hs.converged) ? DEHAZE_ENOTCONV : DEHAZE_OK);
  if (st) {
    fill_stats(hs, st);
    st->status = status;
    DZ_HIP(hipMemcpyAsync(st->A, a.A, 3 * sizeof(float), hipMemcpyDeviceToHost, s));
    DZ_HIP(hipStreamSynchronize(s));
  }
  if (status == DEHAZE_ENONFINITE) set_error("residual is not finite");
  else if (status == DEHAZE_ENOTCONV)
    set_error("rel_tol %g not reached in %d outer steps (rho %g)", p.rel_tol, hs.outer, hs.rel);
  return status;
}

}  // namespace

size_t solver_workspace_bytes(int H, int W, const dehaze_params& p) {
  if (p.scheme == DEHAZE_PICARD_KRYLOV) return plan_krylov(nullptr, H, W).bytes;
  return plan_sweeps(nullptr, H, W).bytes;
}

int solve_one(Ctx& ctx, const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  (void)ctx;
  if (p.warm_start) { set_error("warm start needs loaded network weights"); return DEHAZE_EINVAL; }
  if (p.scheme == DEHAZE_PICARD_KRYLOV) return run_krylov(a, p, st, s);
  return run_sweeps(a, p, st, s);
}

void solver_release(Ctx& ctx) { (void)ctx; }

}  // namespace dz
