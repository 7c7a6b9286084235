// One-image solve: builds lambda(t) and Phi(I, t, A) (Sections II-A, II-D),
// picks the starting iterate and runs the chosen fixed-point iteration
// (Appendix A-1) with its stopping rule.
#include <cmath>

#include "internal.hpp"
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

}  // namespace

size_t solver_workspace_bytes(int H, int W, const dehaze_params& p) {
  (void)p;
  return plan_sweeps(nullptr, H, W).bytes;
}

int solve_one(Ctx& ctx, const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  (void)ctx;
  if (p.warm_start) { set_error("warm start needs loaded network weights"); return DEHAZE_EINVAL; }
  if (p.scheme == DEHAZE_PICARD_KRYLOV) { set_error("scheme not available"); return DEHAZE_EINVAL; }
  return run_sweeps(a, p, st, s);
}

void solver_release(Ctx& ctx) { (void)ctx; }

}  // namespace dz
