// One-image solve: builds lambda(t) and Phi(I, t, A) (Sections II-A, II-D),
// picks the starting iterate and runs the chosen fixed-point iteration
// (Appendix A-1) with its stopping rule.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "cnn.hpp"
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

}  // namespace

// Launch shape of the strip sweep kernel chosen per (H, W, mode): sweeps per
// launch K, strip height S and columns per lane C.  Every shape computes the
// same values, so the choice only affects speed.
struct SweepTune {
  std::map<std::tuple<int, int, int>, std::array<int, 3>> best;
};

namespace {

constexpr int kStripHeights[] = {8, 12, 16, 20, 24, 28, 32, 40, 48, 64, 96, 128};

// Times every shape on sweeps from u to scratch (the caller's starting
// iterate and the other half of its ping-pong pair), so the trial launches
// touch the same buffers as the solve.  A forced K, S or C (> 0) is taken as
// given; the others come from the tuned shape when there is one, else from
// defaults.
int pick_strip_shape(Ctx& ctx, int mode, int H, int W, int P, const float* u, const float* phi, const float* lam,
                     float* scratch, const OpConst& oc, const dehaze_params& p, hipStream_t s, StripShape* out) {
  *out = StripShape{};
  if (oc.R != 2 || !strip_fits(H, P)) return DEHAZE_OK;  // the tile kernel handles these
  if (!ctx.tune) ctx.tune = new SweepTune();
  const auto key = std::make_tuple(H, W, mode);
  auto it = ctx.tune->best.find(key);
  const bool tuned = it != ctx.tune->best.end();
  if (p.sweeps_per_launch > 0 || p.strip_rows > 0 || p.lane_columns > 0) {
    out->K = p.sweeps_per_launch > 0 ? std::min(p.sweeps_per_launch, kMaxSweepsPerLaunch) : (tuned ? it->second[0] : 2);
    out->S = p.strip_rows > 0 ? p.strip_rows : (tuned ? it->second[1] : 32);
    out->C = p.lane_columns > 0 ? p.lane_columns : (tuned ? it->second[2] : 1);
    return DEHAZE_OK;
  }
  if (tuned) {
    *out = StripShape{it->second[0], it->second[1], it->second[2]};
    return DEHAZE_OK;
  }
  hipEvent_t e0, e1;
  DZ_HIP(hipEventCreate(&e0));
  DZ_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  StripShape bst{1, 32, 1};
  int rc = DEHAZE_OK;
  for (int c = 1; c <= 2 && rc == DEHAZE_OK; ++c) {
    for (int k = 1; k <= kMaxSweepsPerLaunch && rc == DEHAZE_OK; ++k) {
      int prev_strips = -1;
      for (int sh : kStripHeights) {
        // heights that give the same strip count as the previous one add nothing
        const int strips = (H + sh - 1) / sh;
        if (strips == prev_strips) continue;
        prev_strips = strips;
        if ((rc = launch_sweep_strip(mode, k, sh, c, u, scratch, phi, lam, H, W, P, oc, s))) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = DEHAZE_EHIP; break; }
        for (int i = 0; i < 3 && rc == DEHAZE_OK; ++i)
          rc = launch_sweep_strip(mode, k, sh, c, u, scratch, phi, lam, H, W, P, oc, s);
        if (rc) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = DEHAZE_EHIP; break; }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = DEHAZE_EHIP; break; }
        const float per_sweep = ms / (3.0f * k);
        if (per_sweep < best) {
          best = per_sweep;
          bst = StripShape{k, sh, c};
        }
      }
    }
  }
  // refine the strip height around the winner: the balance of wavefronts
  // over the compute units changes quickly with the strip count
  const StripShape coarse = bst;
  for (int sh = std::max(4, coarse.S - 3); sh <= coarse.S + 3 && rc == DEHAZE_OK; ++sh) {
    if (sh == coarse.S) continue;
    if ((rc = launch_sweep_strip(mode, coarse.K, sh, coarse.C, u, scratch, phi, lam, H, W, P, oc, s))) break;
    if (hipEventRecord(e0, s) != hipSuccess) { rc = DEHAZE_EHIP; break; }
    for (int i = 0; i < 3 && rc == DEHAZE_OK; ++i)
      rc = launch_sweep_strip(mode, coarse.K, sh, coarse.C, u, scratch, phi, lam, H, W, P, oc, s);
    if (rc) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = DEHAZE_EHIP; break; }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = DEHAZE_EHIP; break; }
    const float per_sweep = ms / (3.0f * coarse.K);
    if (per_sweep < best) {
      best = per_sweep;
      bst = StripShape{coarse.K, sh, coarse.C};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == DEHAZE_EHIP) set_error("timing the sweep launch shapes failed");
  if (rc) return rc;
  ctx.tune->best[key] = {bst.K, bst.S, bst.C};
  *out = bst;
  return DEHAZE_OK;
}

int run_sweeps(Ctx& ctx, const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  const int H = a.H, W = a.W;
  SweepPlan pl = plan_sweeps(a.ws, H, W);
  int rc;
  if ((rc = launch_to_planar(a.I, a.dtype, a.layout, H, W, a.pitch, pl.Ip, pl.P, s))) return rc;
  FusedOut fo{nullptr, nullptr, pl.lam, pl.phi, pl.P, pl.P};
  if ((rc = launch_prior_fused(nullptr, pl.Ip, pl.P, a.t, W, a.A, H, W, p, fo, s))) return rc;
  if (a.u0) rc = launch_copy3(a.u0, W, pl.ua, pl.P, H, W, s);
  else rc = launch_copy3(pl.phi, pl.P, pl.ua, pl.P, H, W, s);
  if (rc) return rc;

  const OpConst oc = make_opconst(p);
  const int mode = p.scheme == DEHAZE_PAPER_EXPLICIT ? kExplicit : kJacobi;
  StripShape sh;
  if ((rc = pick_strip_shape(ctx, mode, H, W, pl.P, pl.ua, pl.phi, pl.lam, pl.ub, oc, p, s, &sh))) return rc;
  const int K = sh.K;
  float* cur = pl.ua;
  float* nxt = pl.ub;
  // n sweeps from cur, ending with the result in cur
  auto sweeps = [&](int n) -> int {
    while (n > 0) {
      const int k = K > 0 ? std::min(K, n) : 1;
      const int e = K > 0 ? launch_sweep_strip(mode, k, sh.S, sh.C, cur, nxt, pl.phi, pl.lam, H, W, pl.P, oc, s)
                          : launch_sweep(mode, cur, nxt, pl.phi, pl.lam, H, W, pl.P, oc, nullptr, s);
      if (e) return e;
      std::swap(cur, nxt);
      n -= k;
    }
    return DEHAZE_OK;
  };
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
      if ((rc = sweeps(k))) return rc;
      done += k;
    }
  } else {
    if (st && (rc = residual_of(cur, pl, H, W, oc, &rho0, s))) return rc;
    if ((rc = sweeps(p.max_outer))) return rc;
    done = p.max_outer;
    if (st) {
      if ((rc = residual_of(cur, pl, H, W, oc, &rho, s))) return rc;
      if (!std::isfinite(rho)) status = DEHAZE_ENONFINITE;
    }
  }
  if (p.u_state == DEHAZE_U_F64) rc = launch_copy3_wide(cur, pl.P, reinterpret_cast<double*>(a.u), W, H, W, s);
  else rc = launch_copy3(cur, pl.P, a.u, W, H, W, s);
  if (rc) return rc;
  if (st) {
    st->outer = done;
    st->converged = conv ? 1 : 0;
    st->inner = 0;
    st->applications = done;
    st->rel_residual = rho;
    st->rel_residual0 = rho0;
    st->rel_residual_out = rho;
    st->restarts = 0;
    st->stalled = 0;
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
  int* d_unit_img = nullptr;
  double* d_upart = nullptr;
  double* d_npart = nullptr;
  float* u0w = nullptr;   // warm start B (+ the network's correction), planar pitch W
  char* cnn_ws = nullptr;
  size_t bytes = 0;
};

KrylovPlan plan_krylov(void* ws, int H, int W, const dehaze_params& p) {
  const bool warm = p.warm_start != 0;
  const int ng = p.ngmres_depth;
  KrylovPlan pl;
  Carver cv(ws, ~size_t(0));
  char* arena = cv.take<char>(krylov_image_bytes(H, W, ng));
  int us = 32;
  krylov_strip_rows(1, &H, &W, &us);
  pl.img = krylov_carve(arena, H, W, 0, 0, 0, us, ng);
  const int nt = krylov_tiles(H, W);
  // room for the most strip wavefronts (kSBlk rows each), one partial-sum
  // slot per block
  const int nu = pl.img.nblk;
  pl.Ip = cv.take<float>(3 * static_cast<size_t>(H) * pl.img.P);
  pl.d_imgs = cv.take<KImg>(1);
  pl.d_scal = cv.take<KScal>(1);
  pl.d_tile_img = cv.take<int>(nt);
  pl.d_part = cv.take<double>(static_cast<size_t>(kKPart) * nt);
  pl.d_unit_img = cv.take<int>(nu);
  pl.d_upart = cv.take<double>(static_cast<size_t>(kKPart) * nu);
  if (ng > 0) pl.d_npart = cv.take<double>(static_cast<size_t>(kNPart) * nt);
  if (warm) {
    pl.u0w = cv.take<float>(3 * static_cast<size_t>(H) * W);
    pl.cnn_ws = cv.take<char>(cnn_forward_bytes(1, H, W));
  }
  pl.bytes = cv.used();
  return pl;
}

int read_scalars(const KrylovBatch& b, KScal* h, hipStream_t s) {
  DZ_HIP(hipMemcpyAsync(h, b.d_scal, sizeof(KScal) * b.nimg, hipMemcpyDeviceToHost, s));
  DZ_HIP(hipStreamSynchronize(s));
  return DEHAZE_OK;
}

void fill_stats(const KScal& k, const dehaze_params& p, dehaze_stats* st) {
  st->outer = k.outer;
  st->converged = (k.converged && !k.nonfinite && !k.stalled) ? 1 : 0;
  st->inner = k.inner_total;
  st->applications = 2 * k.inner_total + k.res_evals;
  st->rel_residual = k.rel;
  st->rel_residual0 = k.rel0;
  // a float64 output is the iterate itself
  st->rel_residual_out = p.u_state == DEHAZE_U_F64 ? k.rel : k.rel_out;
  st->status = k.nonfinite ? DEHAZE_ENONFINITE : DEHAZE_OK;
  st->restarts = k.restarted;
  st->stalled = k.stalled;
}

// With defect-correction passes (inner_refine > 0): one lagged-diffusivity
// step for every image still iterating, each pass max_inner iterations long.
int outer_step(const KrylovBatch& b, const KConst& kc, const dehaze_params& p, hipStream_t s) {
  int rc;
  if ((rc = krylov_residual(b, kc, 0, s))) return rc;
  if (p.inner_refine > 0 && (rc = krylov_snapshot(b, s))) return rc;
  for (int pass = 0; pass <= p.inner_refine; ++pass) {
    if (pass > 0 && (rc = krylov_linear_residual(b, kc, s))) return rc;
    for (int it = 1; it <= p.max_inner; ++it)
      if ((rc = krylov_inner(b, kc, s))) return rc;
    if ((rc = krylov_update(b, s))) return rc;
  }
  return DEHAZE_OK;
}

// Without them (the default): one tick.  Images between inner solves get
// their residual pass (and start the next inner solve), images inside one get
// a BiCGSTAB iteration, and images whose inner solve just ended apply the
// correction.  Every image advances at its own pace, so a replayed group of
// ticks holds no iterations that only wait for the slowest inner solve.
int tick_step(const KrylovBatch& b, const KConst& kc, hipStream_t s) {
  int rc;
  if ((rc = krylov_residual(b, kc, 0, s))) return rc;
  if ((rc = krylov_ngmres(b, kc, s))) return rc;
  if ((rc = krylov_inner(b, kc, s))) return rc;
  return krylov_update(b, s);
}

// Ticks per captured graph.
constexpr int kTicks = 64;

}  // namespace

// A captured group of `steps` outer steps, replayed until the images converge.
// The key holds everything the captured kernel arguments depend on.
struct GraphCache {
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  KrylovBatch b{};
  KConst kc{};
  int steps = 0, max_inner = 0, refine = 0;
};

namespace {

bool same_key(const GraphCache& g, const KrylovBatch& b, const KConst& kc, int steps, const dehaze_params& p) {
  return g.exec && g.b.d_imgs == b.d_imgs && g.b.d_scal == b.d_scal && g.b.d_tile_img == b.d_tile_img &&
         g.b.d_part == b.d_part && g.b.nimg == b.nimg && g.b.ntiles == b.ntiles &&
         g.b.d_unit_img == b.d_unit_img && g.b.d_upart == b.d_upart && g.b.nunits == b.nunits && g.b.d_npart == b.d_npart && g.steps == steps &&
         g.max_inner == p.max_inner && g.refine == p.inner_refine && std::memcmp(&g.kc, &kc, sizeof(kc)) == 0;
}

int graph_for(Ctx& ctx, const KrylovBatch& b, const KConst& kc, int steps, const dehaze_params& p,
              hipGraphExec_t* out) {
  if (!ctx.graphs) ctx.graphs = new GraphCache();
  GraphCache& g = *ctx.graphs;
  if (same_key(g, b, kc, steps, p)) {
    *out = g.exec;
    return DEHAZE_OK;
  }
  if (g.exec) {
    DZ_HIP(hipGraphExecDestroy(g.exec));
    g.exec = nullptr;
  }
  if (!g.cap) DZ_HIP(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
  DZ_HIP(hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal));
  int rc = DEHAZE_OK;
  for (int i = 0; i < steps && rc == DEHAZE_OK; ++i)
    rc = p.inner_refine > 0 ? outer_step(b, kc, p, g.cap) : tick_step(b, kc, g.cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(g.cap, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) {
    set_error("graph capture failed: %s", hipGetErrorString(e));
    return DEHAZE_EHIP;
  }
  const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    g.exec = nullptr;
    set_error("graph instantiation failed: %s", hipGetErrorString(ei));
    return DEHAZE_EHIP;
  }
  g.b = b;
  g.kc = kc;
  g.steps = steps;
  g.max_inner = p.max_inner;
  g.refine = p.inner_refine;
  *out = g.exec;
  return DEHAZE_OK;
}

// Runs outer steps (groups of check_every, replayed from a HIP graph) until
// every image has converged or max_outer steps were taken, then evaluates the
// final residual.  h (nimg entries) receives the scalars when they are read.
int krylov_loop(Ctx& ctx, const KrylovBatch& b, const dehaze_params& p, KScal* h, bool need_scalars,
                hipStream_t s) {
  const KConst kc = make_kconst(p);
  int rc;
  if (p.inner_refine > 0) {
    const int per = std::max(1, std::min(p.check_every, p.max_outer));
    hipGraphExec_t exec = nullptr;
    if (p.max_outer >= per && (rc = graph_for(ctx, b, kc, per, p, &exec))) return rc;
    int done = 0;
    while (done < p.max_outer) {
      const int k = std::min(per, p.max_outer - done);
      if (k == per && exec) {
        DZ_HIP(hipGraphLaunch(exec, s));
      } else {
        for (int i = 0; i < k; ++i)
          if ((rc = outer_step(b, kc, p, s))) return rc;
      }
      done += k;
      if (p.rel_tol > 0.0) {
        if ((rc = read_scalars(b, h, s))) return rc;
        bool all = true;
        for (int i = 0; i < b.nimg; ++i) all = all && h[i].converged;
        if (all) break;
      }
    }
  } else {
    // groups of ticks until every image has converged, stopped or taken
    // max_outer steps; a step takes at most max_inner ticks
    hipGraphExec_t exec = nullptr;
    if ((rc = graph_for(ctx, b, kc, kTicks, p, &exec))) return rc;
    const long long cap = (static_cast<long long>(p.max_outer) + 1) * std::max(1, p.max_inner) + 2;
    for (long long ticks = 0; ticks < cap; ticks += kTicks) {
      DZ_HIP(hipGraphLaunch(exec, s));
      if ((rc = read_scalars(b, h, s))) return rc;
      bool all = true;
      for (int i = 0; i < b.nimg; ++i) all = all && (h[i].converged || h[i].exhausted);
      if (all) break;
    }
  }
  if ((rc = krylov_residual(b, kc, 1, s))) return rc;
  // the float64 iterate is returned rounded to float32 (unless the caller
  // takes it in float64); its residual there is reported beside the
  // iterate's own
  if (p.u_state != DEHAZE_U_F64 && (rc = krylov_residual(b, kc, 2, s))) return rc;
  if (need_scalars || p.rel_tol > 0.0) return read_scalars(b, h, s);
  return DEHAZE_OK;
}

}  // namespace

// Strip heights of the BiCGSTAB operator kernels per batch composition: the
// key lists every image size with its count, the value the height of each
// size.  Every height gives the same results (the dot products are summed per
// block of kSBlk rows), so the choice only affects speed.
struct KrylovTune {
  std::map<std::vector<std::array<int, 3>>, std::map<std::pair<int, int>, int>> best;
};

namespace {

constexpr int kKrylovRows[] = {16, 32, 64, 128, 256};

std::vector<std::array<int, 3>> composition(const std::vector<KImg>& imgs) {
  std::map<std::pair<int, int>, int> cnt;
  for (const KImg& m : imgs) cnt[{m.H, m.W}] += 1;
  std::vector<std::array<int, 3>> key;
  for (const auto& [hw, c] : cnt) key.push_back({hw.first, hw.second, c});
  return key;
}

// Sets the strip height of every image from its size; returns the wavefronts
// of one launch.
int lay_out(std::vector<KImg>& imgs, const std::map<std::pair<int, int>, int>& rows) {
  int unit0 = 0;
  for (KImg& m : imgs) {
    m.us = rows.at({m.H, m.W});
    m.nunits = krylov_units(m.H, m.W, m.us);
    m.unit0 = unit0;
    unit0 += m.nunits;
  }
  return unit0;
}

bool strips_usable(const std::vector<KImg>& imgs, const dehaze_params& p) {
  if (p.g_radius != 2) return false;
  for (const KImg& m : imgs)
    if (!krylov_strips_fit(m.H, m.W)) return false;
  return true;
}

// Strip heights by the size rule (or forced by krylov_rows), per image size.
std::map<std::pair<int, int>, int> rule_rows(const std::vector<KImg>& imgs, const dehaze_params& p) {
  const int n = static_cast<int>(imgs.size());
  std::vector<int> hs(n), ws(n), us(n);
  for (int i = 0; i < n; ++i) {
    hs[i] = imgs[i].H;
    ws[i] = imgs[i].W;
  }
  krylov_strip_rows(n, hs.data(), ws.data(), us.data());
  std::map<std::pair<int, int>, int> rows;
  for (int i = 0; i < n; ++i) rows[{hs[i], ws[i]}] = p.krylov_rows > 0 ? p.krylov_rows : us[i];
  return rows;
}

// Chooses the strip height of every image of the launch and uploads the
// descriptors and the wavefront map; b.nunits receives the launch's
// wavefront count (0: the tile kernels run, when an image is too large for
// the strip kernels' 32-bit offsets or R != 2).  Without krylov_rows, the
// first solve of a batch composition times kernel (a) over the whole launch
// for each candidate height of each image size in turn (sizes with the most
// pixels first, the others held at their current choice), starting from the
// size rule, and the context keeps the fastest.
int choose_strips(Ctx& ctx, std::vector<KImg>& imgs, KrylovBatch& b, const dehaze_params& p, hipStream_t s) {
  if (!strips_usable(imgs, p)) {
    b.nunits = 0;
    return DEHAZE_OK;
  }
  std::map<std::pair<int, int>, int> rows = rule_rows(imgs, p);
  auto upload = [&]() -> int {
    b.nunits = lay_out(imgs, rows);
    return krylov_upload_strips(b, imgs.data(), s);
  };
  if (p.krylov_rows > 0) return upload();
  if (!ctx.ktune) ctx.ktune = new KrylovTune();
  const auto key = composition(imgs);
  auto it = ctx.ktune->best.find(key);
  if (it != ctx.ktune->best.end()) {
    rows = it->second;
    return upload();
  }
  const KConst kc = make_kconst(p);
  int rc;
  float best = 0.0f;
  if ((rc = upload()) || (rc = krylov_time_strips(b, kc, 3, s, &best))) return rc;
  std::vector<std::pair<long long, std::pair<int, int>>> order;
  for (const auto& k : key) order.push_back({-static_cast<long long>(k[0]) * k[1] * k[2], {k[0], k[1]}});
  std::sort(order.begin(), order.end());
  for (const auto& [neg, hw] : order) {
    const int keep = rows[hw];
    int chosen = keep;
    std::vector<int> seen{(hw.first + keep - 1) / keep};
    for (int cand : kKrylovRows) {
      const int strips = (hw.first + cand - 1) / cand;
      if (std::find(seen.begin(), seen.end(), strips) != seen.end()) continue;
      seen.push_back(strips);
      rows[hw] = cand;
      float t = 0.0f;
      if ((rc = upload()) || (rc = krylov_time_strips(b, kc, 3, s, &t))) return rc;
      if (t < best) {
        best = t;
        chosen = cand;
      }
    }
    rows[hw] = chosen;
  }
  ctx.ktune->best[key] = rows;
  return upload();
}

int image_status(const KScal& k, const dehaze_params& p) {
  if (k.nonfinite) return DEHAZE_ENONFINITE;
  if (p.rel_tol > 0.0 && (!k.converged || k.stalled)) return DEHAZE_ENOTCONV;
  return DEHAZE_OK;
}

int run_krylov(Ctx& ctx, const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  const int H = a.H, W = a.W;
  KrylovPlan pl = plan_krylov(a.ws, H, W, p);
  const int P = pl.img.P;
  int rc;
  if ((rc = launch_to_planar(a.I, a.dtype, a.layout, H, W, a.pitch, pl.Ip, P, s))) return rc;
  FusedOut fo{nullptr, nullptr, const_cast<float*>(pl.img.lam), const_cast<float*>(pl.img.phi), P, P};
  if ((rc = launch_prior_fused(nullptr, pl.Ip, P, a.t, W, a.A, H, W, p, fo, s))) return rc;
  KrylovBatch b{pl.d_imgs, pl.d_scal, pl.d_tile_img, pl.d_part, 1, pl.img.ntiles,
                pl.d_unit_img, pl.d_upart, pl.img.nunits, pl.d_npart};
  const float* u0 = a.u0;
  if (p.warm_start) {
    const size_t plane = static_cast<size_t>(H) * P;
    if (p.warm_start == 1 &&
        (rc = cnn_forward(ctx, 1, H, W, pl.Ip, P, plane, 3 * plane, a.t, W, static_cast<size_t>(H) * W, a.A, pl.u0w,
                          W, 3 * static_cast<size_t>(H) * W, pl.cnn_ws, s)))
      return rc;
    if ((rc = launch_warm_base(pl.u0w, pl.img.phi, pl.img.lam, P, H, W, p.nonlocal_term != 0, p.warm_start == 1, s)))
      return rc;
    u0 = pl.u0w;
  }
  if ((rc = krylov_init(b, &pl.img, &u0, s))) return rc;
  std::vector<KImg> one{pl.img};
  if ((rc = choose_strips(ctx, one, b, p, s))) return rc;
  pl.img = one[0];
  KScal hs{};
  if ((rc = krylov_loop(ctx, b, p, &hs, st != nullptr, s))) return rc;
  rc = p.u_state == DEHAZE_U_F64 ? krylov_output64(pl.img, reinterpret_cast<double*>(a.u), s)
                                 : krylov_output(pl.img, a.u, s);
  if (rc) return rc;
  if (!st && p.rel_tol <= 0.0) return DEHAZE_OK;
  const int status = image_status(hs, p);
  if (st) {
    fill_stats(hs, p, st);
    st->status = status;
    DZ_HIP(hipMemcpyAsync(st->A, a.A, 3 * sizeof(float), hipMemcpyDeviceToHost, s));
    DZ_HIP(hipStreamSynchronize(s));
  }
  if (status == DEHAZE_ENONFINITE) set_error("residual is not finite");
  else if (status == DEHAZE_ENOTCONV)
    set_error("rel_tol %g not reached in %d outer steps (rho %g%s)", p.rel_tol, hs.outer, hs.rel,
              hs.stalled ? ", stopped: rho stopped falling" : "");
  return status;
}

// ------------------------------------------------------------ batch
struct BatchPlan {
  char* prior_ws = nullptr;
  std::vector<KImg> imgs;
  std::vector<float*> t_int;
  std::vector<float*> A_int;
  KImg* d_imgs = nullptr;
  KScal* d_scal = nullptr;
  int* d_tile_img = nullptr;
  double* d_part = nullptr;
  int* d_unit_img = nullptr;
  double* d_upart = nullptr;
  double* d_npart = nullptr;
  std::vector<float*> u0w;  // warm starts B (+ the network's correction)
  char* cnn_ws = nullptr;
  int ntiles = 0;
  int nunits = 0;
  size_t bytes = 0;
};

BatchPlan plan_batch(void* ws, int n, const dehaze_image* im, const dehaze_params& p) {
  const bool warm = p.warm_start != 0;
  BatchPlan pl;
  Carver cv(ws, ~size_t(0));
  size_t prior_max = 0, cnn_max = 0;
  for (int i = 0; i < n; ++i) {
    PriorBufs tmp{};
    prior_max = std::max(prior_max, carve_prior(nullptr, im[i].H, im[i].W, p, &tmp));
    cnn_max = std::max(cnn_max, cnn_forward_bytes(1, im[i].H, im[i].W));
  }
  pl.prior_ws = cv.take<char>(prior_max);
  if (warm) pl.cnn_ws = cv.take<char>(cnn_max);
  std::vector<int> hs(n), wsz(n), us(n);
  for (int i = 0; i < n; ++i) {
    hs[i] = im[i].H;
    wsz[i] = im[i].W;
  }
  krylov_strip_rows(n, hs.data(), wsz.data(), us.data());
  int tile0 = 0, unit0 = 0, blk0 = 0;
  for (int i = 0; i < n; ++i) {
    char* arena = cv.take<char>(krylov_image_bytes(im[i].H, im[i].W, p.ngmres_depth));
    pl.imgs.push_back(krylov_carve(arena, im[i].H, im[i].W, tile0, unit0, blk0, us[i], p.ngmres_depth));
    tile0 += pl.imgs.back().ntiles;
    unit0 += pl.imgs.back().nunits;
    blk0 += pl.imgs.back().nblk;
    const bool need_t = !im[i].t && !im[i].t_out;
    const bool need_A = !im[i].A && !im[i].A_out;
    pl.t_int.push_back(need_t ? cv.take<float>(static_cast<size_t>(im[i].H) * im[i].W) : nullptr);
    pl.A_int.push_back(need_A ? cv.take<float>(4) : nullptr);
    pl.u0w.push_back(warm ? cv.take<float>(3 * static_cast<size_t>(im[i].H) * im[i].W) : nullptr);
  }
  pl.ntiles = tile0;
  pl.nunits = unit0;
  pl.d_imgs = cv.take<KImg>(n);
  pl.d_scal = cv.take<KScal>(n);
  pl.d_tile_img = cv.take<int>(tile0);
  pl.d_part = cv.take<double>(static_cast<size_t>(kKPart) * tile0);
  // room for the most strip wavefronts (kSBlk rows each), one partial-sum
  // slot per block
  pl.d_unit_img = cv.take<int>(blk0);
  pl.d_upart = cv.take<double>(static_cast<size_t>(kKPart) * blk0);
  if (p.ngmres_depth > 0) pl.d_npart = cv.take<double>(static_cast<size_t>(kNPart) * tile0);
  pl.bytes = cv.used();
  return pl;
}

// Front end of one batch image: t and A as given, or estimated (Section II-D);
// lambda and Phi go straight into the image's solver planes.
int batch_front_end(Ctx& ctx, const BatchPlan& pl, int i, const dehaze_image& m, int dtype, int layout,
                    const dehaze_params& p, const float** A_used, hipStream_t s) {
  PriorBufs pb{};
  carve_prior(pl.prior_ws, m.H, m.W, p, &pb);
  const KImg& K = pl.imgs[i];
  int rc;
  const float* A = m.A;
  float* t_dst = nullptr;
  if (!m.t || !m.A) {
    if ((rc = launch_patch_min(m.I, dtype, layout, m.H, m.W, m.pitch, p.patch, pb, nullptr, nullptr, s)))
      return rc;
    if (!m.A) {
      float* A_dst = m.A_out ? m.A_out : pl.A_int[i];
      if ((rc = launch_airlight(pb, m.H, m.W, p.atm_divisor, A_dst, s))) return rc;
      A = A_dst;
    }
    if (!m.t) t_dst = m.t_out ? m.t_out : pl.t_int[i];
  } else if ((rc = launch_to_planar(m.I, dtype, layout, m.H, m.W, m.pitch, pb.Ip, pb.P, s))) {
    return rc;
  }
  if (m.A && m.A_out && m.A_out != m.A)
    DZ_HIP(hipMemcpyAsync(m.A_out, m.A, 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
  FusedOut fo{nullptr, t_dst, const_cast<float*>(K.lam), const_cast<float*>(K.phi), K.P, m.W};
  if (m.t) rc = launch_prior_fused(nullptr, pb.Ip, pb.P, m.t, m.W, A, m.H, m.W, p, fo, s);
  else rc = launch_prior_estimated(m.I, dtype, layout, m.H, m.W, m.pitch, p, pb, A, fo, s);
  if (rc) return rc;
  if (p.warm_start) {
    const size_t plane = static_cast<size_t>(m.H) * pb.P;
    const float* t_used = m.t ? m.t : t_dst;
    if (p.warm_start == 1 &&
        (rc = cnn_forward(ctx, 1, m.H, m.W, pb.Ip, pb.P, plane, 3 * plane, t_used, m.W,
                          static_cast<size_t>(m.H) * m.W, A, pl.u0w[i], m.W, 3 * static_cast<size_t>(m.H) * m.W,
                          pl.cnn_ws, s)))
      return rc;
    if ((rc = launch_warm_base(pl.u0w[i], K.phi, K.lam, K.P, m.H, m.W, p.nonlocal_term != 0, p.warm_start == 1, s)))
      return rc;
  }
  *A_used = A;
  return DEHAZE_OK;
}

}  // namespace

size_t solver_workspace_bytes(int H, int W, const dehaze_params& p) {
  if (p.scheme == DEHAZE_PICARD_KRYLOV) return plan_krylov(nullptr, H, W, p).bytes;
  return plan_sweeps(nullptr, H, W).bytes;
}

static int check_warm(const Ctx& ctx, const dehaze_params& p, bool has_u0) {
  if (!p.warm_start) return DEHAZE_OK;
  if (p.warm_start == 1 && !cnn_ready(ctx)) {
    set_error("warm start from the network needs loaded weights");
    return DEHAZE_EINVAL;
  }
  if (has_u0) { set_error("warm start and an explicit u0 exclude each other"); return DEHAZE_EINVAL; }
  if (p.scheme != DEHAZE_PICARD_KRYLOV) { set_error("warm start applies to DEHAZE_PICARD_KRYLOV"); return DEHAZE_EINVAL; }
  return DEHAZE_OK;
}

int solve_one(Ctx& ctx, const SolveArgs& a, const dehaze_params& p, dehaze_stats* st, hipStream_t s) {
  int rc = check_warm(ctx, p, a.u0 != nullptr);
  if (rc) return rc;
  if (p.scheme == DEHAZE_PICARD_KRYLOV) return run_krylov(ctx, a, p, st, s);
  return run_sweeps(ctx, a, p, st, s);
}

int sweep_shape(const Ctx& ctx, int H, int W, int scheme, int* K, int* S, int* C) {
  *K = *S = *C = 0;
  if (!ctx.tune) return DEHAZE_OK;
  const int mode = scheme == DEHAZE_PAPER_EXPLICIT ? kExplicit : kJacobi;
  auto it = ctx.tune->best.find(std::make_tuple(H, W, mode));
  if (it != ctx.tune->best.end()) {
    *K = it->second[0];
    *S = it->second[1];
    *C = it->second[2];
  }
  return DEHAZE_OK;
}

int batch_strip_rows(const Ctx* ctx, int n, const dehaze_image* im, const dehaze_params& p, int* rows, int* tuned) {
  std::vector<KImg> imgs(n);
  for (int i = 0; i < n; ++i) {
    imgs[i] = KImg{};
    imgs[i].H = im[i].H;
    imgs[i].W = im[i].W;
  }
  *tuned = 0;
  if (!strips_usable(imgs, p)) {
    for (int i = 0; i < n; ++i) rows[i] = 0;
    return DEHAZE_OK;
  }
  std::map<std::pair<int, int>, int> r = rule_rows(imgs, p);
  if (p.krylov_rows <= 0 && ctx && ctx->ktune) {
    auto it = ctx->ktune->best.find(composition(imgs));
    if (it != ctx->ktune->best.end()) {
      r = it->second;
      *tuned = 1;
    }
  }
  for (int i = 0; i < n; ++i) rows[i] = r.at({im[i].H, im[i].W});
  return DEHAZE_OK;
}

size_t batch_workspace_bytes(int n, const dehaze_image* imgs, const dehaze_params& p) {
  return plan_batch(nullptr, n, imgs, p).bytes;
}

int solve_batch(Ctx& ctx, int n, const dehaze_image* im, int dtype, int layout, const dehaze_params& p, void* ws,
                dehaze_stats* st, hipStream_t s) {
  bool any_u0 = false;
  for (int i = 0; i < n; ++i) any_u0 = any_u0 || im[i].u0;
  int rc0 = check_warm(ctx, p, any_u0);
  if (rc0) return rc0;
  BatchPlan pl = plan_batch(ws, n, im, p);
  std::vector<const float*> A_used(n, nullptr), u0(n, nullptr);
  int rc;
  for (int i = 0; i < n; ++i) {
    if ((rc = batch_front_end(ctx, pl, i, im[i], dtype, layout, p, &A_used[i], s))) return rc;
    u0[i] = p.warm_start ? pl.u0w[i] : im[i].u0;
  }
  KrylovBatch b{pl.d_imgs, pl.d_scal, pl.d_tile_img, pl.d_part, n, pl.ntiles, pl.d_unit_img, pl.d_upart, pl.nunits,
                pl.d_npart};
  if ((rc = krylov_init(b, pl.imgs.data(), u0.data(), s))) return rc;
  if ((rc = choose_strips(ctx, pl.imgs, b, p, s))) return rc;
  std::vector<KScal> hs(n);
  if ((rc = krylov_loop(ctx, b, p, hs.data(), st != nullptr, s))) return rc;
  for (int i = 0; i < n; ++i) {
    rc = p.u_state == DEHAZE_U_F64 ? krylov_output64(pl.imgs[i], reinterpret_cast<double*>(im[i].u), s)
                                   : krylov_output(pl.imgs[i], im[i].u, s);
    if (rc) return rc;
  }
  if (!st && p.rel_tol <= 0.0) return DEHAZE_OK;
  int worst = DEHAZE_OK;
  std::vector<float> Ah(3 * static_cast<size_t>(n));
  for (int i = 0; i < n; ++i)
    DZ_HIP(hipMemcpyAsync(&Ah[3 * i], A_used[i], 3 * sizeof(float), hipMemcpyDeviceToHost, s));
  DZ_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) {
    const int status = image_status(hs[i], p);
    if (status == DEHAZE_ENONFINITE || (status == DEHAZE_ENOTCONV && worst == DEHAZE_OK)) worst = status;
    if (st) {
      fill_stats(hs[i], p, &st[i]);
      st[i].status = status;
      for (int c = 0; c < 3; ++c) st[i].A[c] = Ah[3 * i + c];
    }
  }
  if (worst == DEHAZE_ENONFINITE) set_error("a residual is not finite");
  else if (worst == DEHAZE_ENOTCONV) set_error("rel_tol %g not reached for every image", p.rel_tol);
  return worst;
}

void solver_release(Ctx& ctx) {
  delete ctx.tune;
  ctx.tune = nullptr;
  delete ctx.ktune;
  ctx.ktune = nullptr;
  if (!ctx.graphs) return;
  if (ctx.graphs->exec) (void)hipGraphExecDestroy(ctx.graphs->exec);
  if (ctx.graphs->cap) (void)hipStreamDestroy(ctx.graphs->cap);
  delete ctx.graphs;
  ctx.graphs = nullptr;
}

}  // namespace dz
