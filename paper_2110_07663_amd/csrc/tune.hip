// Run-time preconditioner selection (Sec. 5): exhaustive search over a small
// parameter space at the first solve, on the problem and hardware at hand.
//
// The space follows the paper's table for pMG (Cheby-ASM and Cheby-RAS with the
// short schedule, Cheby-Jacobi with the long one) and adds the knobs this
// implementation exposes: Chebyshev order, smoother precision (FP64, FP32, FP32
// with FP16 matrix-core FDM) and, at p = 7, the Ax kernel shape.  Each candidate
// is set up in the caller's workspace, solved from x = 0 and timed with HIP
// events on the caller's stream; the fastest converged candidate wins.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "sem_internal.h"

namespace sem {
struct TuneSched {
  int n;
  int p[8];
};

static void schedules_for(int p, TuneSched &schwarz, TuneSched &jac) {
  auto set = [](TuneSched &t, std::initializer_list<int> v) {
    t.n = 0;
    for (int x : v) t.p[t.n++] = x;
  };
  if (p == 7) {
    set(schwarz, {7, 3, 1});
    set(jac, {7, 5, 3, 1});
  } else if (p == 9) {
    set(schwarz, {9, 5, 1});
    set(jac, {9, 7, 5, 1});
  } else {
    // generic: halve toward 1 for Schwarz, step by 2 for Jacobi
    schwarz.n = 0;
    for (int q = p; q > 1; q = std::max(1, q / 2)) schwarz.p[schwarz.n++] = q;
    schwarz.p[schwarz.n++] = 1;
    jac.n = 0;
    for (int q = p; q > 1 && jac.n < 7; q -= 2) jac.p[jac.n++] = q;
    jac.p[jac.n++] = 1;
    if (p == 1) {
      schwarz.n = jac.n = 1;
      schwarz.p[0] = jac.p[0] = 1;
    }
  }
}
}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_tune_space(int32_t p, const sem_opts *base, sem_tune_request *req) {
  if (!base || !req || p < 1 || p > kMaxP) return SEM_EINVAL;
  TuneSched sch, jac;
  schedules_for(p, sch, jac);
  req->ncand = 0;
  req->repeats = 3;
  req->rtol = 1e-8;
  req->maxit = 200;
  const int smoothers[3] = {SEM_SMOOTH_ASM, SEM_SMOOTH_RAS, SEM_SMOOTH_JACOBI};
  // (smoother, FDM contraction inputs, geometric factors of the smoothed
  // levels); at p = 7 the FP16 factors are tried with the one-wavefront Ax
  // shapes (ax_variant 1, 2) only, which keeps the space within SEM_TUNE_MAX
  const int precs[4][3] = {{SEM_F64, SEM_F64, SEM_F32},
                           {SEM_F32, SEM_F32, SEM_F32},
                           {SEM_F32, SEM_F16, SEM_F32},
                           {SEM_F32, SEM_F32, SEM_F16}};
  const int nax = p == 7 ? 3 : 1;
  for (int sm = 0; sm < 3; ++sm) {
    const TuneSched &t = smoothers[sm] == SEM_SMOOTH_JACOBI ? jac : sch;
    if (smoothers[sm] != SEM_SMOOTH_JACOBI && t.n > 1 && t.p[t.n - 2] < 2) continue;
    for (int order = 1; order <= 3; ++order)
      for (int pr = 0; pr < 4; ++pr) {
        if (smoothers[sm] == SEM_SMOOTH_JACOBI && precs[pr][1] == SEM_F16) continue;
        const bool g16 = precs[pr][2] == SEM_F16;
        for (int ax = g16 && nax > 1 ? 1 : 0; ax < nax; ++ax) {
          if (req->ncand >= SEM_TUNE_MAX) return SEM_OK;
          sem_opts o = *base;
          o.precond = SEM_PRECOND_PMG;
          o.nlevels = t.n;
          for (int l = 0; l < 8; ++l) o.p_levels[l] = l < t.n ? t.p[l] : 0;
          o.smoother = smoothers[sm];
          o.cheb_order = order;
          o.smoother_prec = precs[pr][0];
          o.fdm_prec = precs[pr][1];
          o.geom_prec = precs[pr][2];
          o.ax_variant = nax > 1 ? ax : -1;
          for (int l = 0; l < 8; ++l) o.lambda_override[l] = 0.0;
          req->cand[req->ncand++] = o;
        }
      }
  }
  return SEM_OK;
}

sem_status sem_tune_plan(const sem_mesh *mesh, int32_t p, const int8_t bc[6],
                         const sem_tune_request *req, size_t *bytes) {
  if (!req || !bytes || req->ncand < 1 || req->ncand > SEM_TUNE_MAX) return SEM_EINVAL;
  size_t best = 0;
  for (int k = 0; k < req->ncand; ++k) {
    size_t b = 0;
    sem_status st = sem_plan(mesh, p, bc, &req->cand[k], &b);
    if (st == SEM_OK) best = std::max(best, b);
  }
  *bytes = best;
  return best ? SEM_OK : SEM_EINVAL;
}

sem_status sem_tune(const sem_mesh *mesh, int32_t p, const int8_t bc[6],
                    const sem_tune_request *req, const double *b, double *x, void *ws,
                    size_t bytes, void *stream, sem_tune_result *out) {
  if (!req || !out || !b || !x || req->ncand < 1 || req->ncand > SEM_TUNE_MAX) return SEM_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::memset(out, 0, sizeof(*out));
  out->best = -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SEM_EHIP;
  const int reps = std::max(1, req->repeats);
  for (int k = 0; k < req->ncand; ++k) {
    sem_ctx *ctx = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    sem_status st = sem_setup(mesh, p, bc, &req->cand[k], ws, bytes, stream, &ctx);
    out->setup_ms[k] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    out->status[k] = st;
    out->ms[k] = -1.0;
    if (st != SEM_OK) continue;
    sem_level_desc d;
    sem_level_info(ctx, 0, &d);
    std::vector<double> times;
    sem_solve_info info;
    for (int r = 0; r <= reps && st == SEM_OK; ++r) {
      try {
        launch_fill(d.nlocal, 0.0, x, s);
      } catch (const Error &err) {
        st = err.status;
        break;
      }
      (void)hipEventRecord(e0, s);
      st = sem_solve(ctx, b, x, req->rtol, req->maxit, &info, stream);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) times.push_back(ms);  // the first solve warms up
      out->iters[k] = info.iters;
    }
    out->status[k] = st;
    if (st == SEM_OK && !times.empty()) {
      std::sort(times.begin(), times.end());
      out->ms[k] = times[times.size() / 2];
    }
    sem_destroy(ctx);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // fastest converged; near-ties (1%) go to the lower order, then fewer levels
  for (int k = 0; k < req->ncand; ++k) {
    if (out->status[k] != SEM_OK || out->ms[k] < 0) continue;
    int bi = out->best;
    if (bi < 0) {
      out->best = k;
      continue;
    }
    double mk = out->ms[k], mb = out->ms[bi];
    bool tie = std::fabs(mk - mb) <= 0.01 * std::min(mk, mb);
    const sem_opts &ok = req->cand[k], &ob = req->cand[bi];
    if ((!tie && mk < mb) ||
        (tie && (ok.cheb_order < ob.cheb_order ||
                 (ok.cheb_order == ob.cheb_order && ok.nlevels < ob.nlevels))))
      out->best = k;
  }
  return out->best >= 0 ? SEM_OK : SEM_ENOCONV;
}

}  // extern "C"
