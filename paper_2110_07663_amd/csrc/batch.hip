// Batched solves: many independent problems and right-hand sides advanced
// together, one recorded HIP graph per outer iteration of the whole batch.
//
// Each (problem, right side) pair is a lane running flexible CG (the same
// recurrence as sem_solve) with every scalar on the device: the inner product
// kernels close with a last-block reduction that also forms alpha, beta and the
// convergence flag, and every lane kernel is a no-op once its lane is done.
// One outer iteration of all active lanes is recorded as a single graph: one
// branch per problem (lanes of a problem share its V-cycle work vectors and run
// in sequence inside the branch), branches spread over a few streams so that
// small problems run concurrently.  The graph is replayed a few times between
// host checks of the lane flags, and recorded again when lanes finish.  The
// coarse solve inside a recorded V-cycle runs a fixed number of iterations
// (the count the eager first V-cycle needed, plus a margin, capped by
// coarse_maxit); flexible CG absorbs the variation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sem_internal.h"

namespace sem {

struct LaneScalars {
  double rz, pq, alpha, beta, rr, rr0, tol2, pad;
  int done, iters, maxit, breakdown;
};

// Lane reductions in two launches: the blocks write partials, then one
// workgroup per lane sums them in block order and applies the scalar step (a
// ticket counter taken by every block would serialise on one address).
template <int ND>
__device__ inline void lane_tree(double (&acc)[ND], double (*sh)[256]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < ND; ++j) sh[j][tid] = acc[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int j = 0; j < ND; ++j) sh[j][tid] += sh[j][tid + h];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = sh[j][0];
}
template <int ND>
__device__ inline void lane_partials(double (&acc)[ND], double *partials) {
  __shared__ double sh[ND][256];
  lane_tree<ND>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) partials[blockIdx.x * 8 + j] = acc[j];
  }
}
// sum of the nb block partials, in block order, in every thread
template <int ND>
__device__ inline void lane_sum(double (&acc)[ND], const double *partials, int nb) {
  __shared__ double sh[ND][256];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[j] += partials[b * 8 + j];
  lane_tree<ND>(acc, sh);
}

__global__ void k_lane_init(LaneScalars *L, double rz, double rr0, double tol2, int maxit) {
  L->rz = rz;
  L->rr0 = rr0;
  L->rr = rr0;
  L->tol2 = tol2;
  L->maxit = maxit;
  L->iters = 0;
  L->breakdown = 0;
  L->alpha = L->beta = L->pq = 0.0;
  L->done = (rr0 == 0.0 || maxit <= 0) ? 1 : 0;
}

// The lane kernels run over blockIdx.y = lanes lane0, lane0 + 1, ... of one
// problem: vectors n apart, reduction partials kRedBlocks * 8 apart, scalars
// consecutive.  A finished lane's blocks return at once.
#define SEM_LANE_OFFSETS(...)                        \
  do {                                               \
    const int64_t y = blockIdx.y;                    \
    partials += y * kRedBlocks * 8;                  \
    L += y;                                          \
    __VA_ARGS__                                      \
  } while (0)

// pq = (p, q)_w; alpha = rz / pq
__global__ __launch_bounds__(256) void k_lane_pq(int64_t n, const double *__restrict__ w,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ q, double *partials,
                                                 LaneScalars *L) {
  SEM_LANE_OFFSETS(p += y * n; q += y * n;);
  if (L->done) return;
  double acc[1] = {0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    acc[0] += w[t] * p[t] * q[t];
  lane_partials<1>(acc, partials);
}
__global__ __launch_bounds__(256) void k_lane_pq_fin(int nb, double *partials, LaneScalars *L) {
  SEM_LANE_OFFSETS();
  if (L->done) return;
  double acc[1];
  lane_sum<1>(acc, partials, nb);
  if (threadIdx.x == 0) {
    L->pq = acc[0];
    if (acc[0] > 0.0) {
      L->alpha = L->rz / acc[0];
    } else {
      L->alpha = 0.0;
      L->breakdown = 1;
      L->done = 1;
    }
  }
}

// x += alpha p; r -= alpha q; (r, r) and the stopping test
__global__ __launch_bounds__(256) void k_lane_update(int64_t n, const double *__restrict__ w,
                                                     double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ p,
                                                     const double *__restrict__ q,
                                                     double *partials, LaneScalars *L) {
  SEM_LANE_OFFSETS(x += y * n; r += y * n; p += y * n; q += y * n;);
  if (L->done) return;
  const double alpha = L->alpha;
  double acc[1] = {0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    x[t] += alpha * p[t];
    double rv = r[t] - alpha * q[t];
    r[t] = rv;
    acc[0] += w[t] * rv * rv;
  }
  lane_partials<1>(acc, partials);
}
__global__ __launch_bounds__(256) void k_lane_update_fin(int nb, double *partials,
                                                         LaneScalars *L) {
  SEM_LANE_OFFSETS();
  if (L->done) return;
  double acc[1];
  lane_sum<1>(acc, partials, nb);
  if (threadIdx.x == 0) {
    L->rr = acc[0];
    L->iters += 1;
    if (acc[0] <= L->tol2 * L->rr0 || L->iters >= L->maxit || !(acc[0] == acc[0])) L->done = 1;
  }
}

// beta = (r.z - r.z_old) / rz (flexible CG, Polak-Ribiere)
__global__ __launch_bounds__(256) void k_lane_beta(int64_t n, const double *__restrict__ w,
                                                   const double *__restrict__ r,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ zo, double *partials,
                                                   LaneScalars *L) {
  SEM_LANE_OFFSETS(r += y * n; z += y * n; zo += y * n;);
  if (L->done) return;
  double acc[2] = {0.0, 0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double wr = w[t] * r[t];
    acc[0] += wr * z[t];
    acc[1] += wr * zo[t];
  }
  lane_partials<2>(acc, partials);
}
__global__ __launch_bounds__(256) void k_lane_beta_fin(int nb, double *partials, LaneScalars *L) {
  SEM_LANE_OFFSETS();
  if (L->done) return;
  double acc[2];
  lane_sum<2>(acc, partials, nb);
  if (threadIdx.x == 0) {
    L->beta = (acc[0] - acc[1]) / L->rz;
    L->rz = acc[0];
  }
}

// p = z + beta p; z_old = z
__global__ void k_lane_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                         double *__restrict__ zo, const LaneScalars *L) {
  {
    const int64_t y = blockIdx.y;
    z += y * n;
    p += y * n;
    zo += y * n;
    L += y;
  }
  if (L->done) return;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double zv = z[t];
  p[t] = zv + L->beta * p[t];
  zo[t] = zv;
}

static inline unsigned rgrid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > kRedBlocks) g = kRedBlocks;
  return (unsigned)(g < 1 ? 1 : g);
}
static inline unsigned egrid(int64_t n) { return (unsigned)((n + 255) / 256); }

// eager helpers from solver.hip (nv right sides nloc apart)
void batch_opA(const Ctx &c, const Level &L, const double *u, double *Au, hipStream_t s,
               int nv = 1);
void batch_precondition(Ctx &c, const double *r, double *z, hipStream_t s, int nv = 1);
double batch_wnorm2(Ctx &c, const double *a, const double *b, hipStream_t s);

struct Lane {
  Ctx *c;
  int ci;  // index of its problem (context) in the batch
  int k;   // right side index inside its problem
  const double *b;
  double *x;
  double *r, *z, *zo, *p, *q;
  LaneScalars *sc;
  bool active;
};

// one flexible-CG iteration of nv consecutive lanes starting at ln (nv > 1:
// the lanes share each operator application and V-cycle; their x vectors, which
// the caller owns, are updated one lane per launch)
static void lane_iteration(Lane *ln, int nv, hipStream_t s) {
  Ctx &c = *ln->c;
  const Level &F = c.lev[0];
  const int64_t n = F.nloc;
  const int k = ln->k;
  double *part = c.lpartials + (int64_t)k * kRedBlocks * 8;
  const int nb = (int)rgrid(n);
  const dim3 rg(rgrid(n), (unsigned)nv), eg(egrid(n), (unsigned)nv), fg(1, (unsigned)nv);
  batch_opA(c, F, ln->p, ln->q, s, nv);
  hipLaunchKernelGGL(k_lane_pq, rg, dim3(256), 0, s, n, F.w64, ln->p, ln->q, part, ln->sc);
  SEM_LAUNCH("k_lane_pq");
  hipLaunchKernelGGL(k_lane_pq_fin, fg, dim3(256), 0, s, nb, part, ln->sc);
  SEM_LAUNCH("k_lane_pq_fin");
  for (int j = 0; j < nv; ++j) {
    Lane &lj = ln[j];
    double *pj = part + (int64_t)j * kRedBlocks * 8;
    hipLaunchKernelGGL(k_lane_update, dim3(rgrid(n)), dim3(256), 0, s, n, F.w64, lj.x, lj.r, lj.p,
                       lj.q, pj, lj.sc);
    SEM_LAUNCH("k_lane_update");
    hipLaunchKernelGGL(k_lane_update_fin, dim3(1), dim3(256), 0, s, nb, pj, lj.sc);
    SEM_LAUNCH("k_lane_update_fin");
  }
  batch_precondition(c, ln->r, ln->z, s, nv);
  hipLaunchKernelGGL(k_lane_beta, rg, dim3(256), 0, s, n, F.w64, ln->r, ln->z, ln->zo, part,
                     ln->sc);
  SEM_LAUNCH("k_lane_beta");
  hipLaunchKernelGGL(k_lane_beta_fin, fg, dim3(256), 0, s, nb, part, ln->sc);
  SEM_LAUNCH("k_lane_beta_fin");
  hipLaunchKernelGGL(k_lane_p, eg, dim3(256), 0, s, n, ln->z, ln->p, ln->zo, ln->sc);
  SEM_LAUNCH("k_lane_p");
}

struct BatchStreams {
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> ev;
  hipEvent_t fork = nullptr;
  ~BatchStreams() {
    for (auto s : st) (void)hipStreamDestroy(s);
    for (auto e : ev) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
};

// The lane scalars of every context on the host: copies to each context's
// pinned buffer, enqueued together, then one wait (not one per context).
static void poll_lanes(const std::vector<Ctx *> &cs, int nrhs, std::vector<LaneScalars> &out,
                       hipStream_t s) {
  const size_t bytes = (size_t)nrhs * sizeof(LaneScalars);
  if (bytes <= 4096) {  // the size of every context's pinned buffer
    for (auto *c : cs)
      SEM_HIP(hipMemcpyAsync(c->hres, c->lanes, bytes, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < cs.size(); ++i)
      std::memcpy(&out[i * nrhs], cs[i]->hres, bytes);
    return;
  }
  for (size_t i = 0; i < cs.size(); ++i) {
    SEM_HIP(hipMemcpyAsync(&out[i * nrhs], cs[i]->lanes, bytes, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace sem

using namespace sem;

extern "C" sem_status sem_batch_solve(int32_t nctx, sem_ctx *const *ctxs, int32_t nrhs,
                                      const double *const *b, double *const *x, double rtol,
                                      int32_t maxit, int32_t iters_per_launch,
                                      sem_solve_info *infos, void *stream) {
  sem_status status = SEM_OK;
  std::vector<Ctx *> cs;
  try {
    if (nctx < 1 || nrhs < 1 || !ctxs || !b || !x || !(rtol > 0) || maxit < 0)
      fail(SEM_EINVAL, "bad batch arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int ipl = std::max(1, iters_per_launch);
    for (int i = 0; i < nctx; ++i) {
      Ctx *c = reinterpret_cast<Ctx *>(ctxs[i]);
      if (!c) fail(SEM_EINVAL, "null context in batch");
      if (c->nlanes < nrhs) fail(SEM_EINVAL, "context was set up with fewer batch lanes than nrhs");
      if (c->opts.krylov != SEM_KRYLOV_FCG && c->opts.krylov != SEM_KRYLOV_PCG)
        fail(SEM_EUNSUPPORTED, "batched solves use flexible CG");
      cs.push_back(c);
    }
    // lanes and their eager start: r = b - A x, z = M r, p = z_old = z
    std::vector<Lane> lanes;
    for (int i = 0; i < nctx; ++i) {
      Ctx &c = *cs[i];
      const Level &F = c.lev[0];
      for (int k = 0; k < nrhs; ++k) {
        Lane ln;
        ln.c = &c;
        ln.ci = i;
        ln.k = k;
        ln.b = b[i * nrhs + k];
        ln.x = x[i * nrhs + k];
        if (!ln.b || !ln.x) fail(SEM_EINVAL, "null vector in batch");
        // [5][nlanes][nloc]: the r (z, z_old, p, q) of consecutive lanes are adjacent
        const size_t blk = (size_t)c.nlanes * F.nloc;
        ln.r = c.lanev + (size_t)k * F.nloc;
        ln.z = ln.r + blk;
        ln.zo = ln.z + blk;
        ln.p = ln.zo + blk;
        ln.q = ln.p + blk;
        ln.sc = reinterpret_cast<LaneScalars *>(c.lanes) + k;
        batch_opA(c, F, ln.x, ln.q, s);
        launch_sub<double>(F.nloc, ln.b, ln.q, ln.r, s);
        double rr0 = batch_wnorm2(c, ln.r, ln.r, s);
        batch_precondition(c, ln.r, ln.z, s);
        launch_copy<double>(F.nloc, ln.z, ln.p, s);
        launch_copy<double>(F.nloc, ln.z, ln.zo, s);
        double rz = batch_wnorm2(c, ln.r, ln.z, s);
        hipLaunchKernelGGL(k_lane_init, dim3(1), dim3(1), 0, s, ln.sc, rz, rr0, rtol * rtol, maxit);
        SEM_LAUNCH("k_lane_init");
        ln.active = rr0 > 0.0 && maxit > 0;
        lanes.push_back(ln);
      }
      c.capture_coarse_iters = std::min(c.opts.coarse_maxit, c.last_coarse_iters + 4);
    }
    // lanes of one problem share each operator application and V-cycle when the
    // context holds work vectors for all of them (SEM_BATCH_JOINT=0: one at a time)
    std::vector<char> joint(nctx, 0);
    {
      const char *j = getenv("SEM_BATCH_JOINT");
      const bool allow = !(j && j[0] == '0');
      for (int i = 0; i < nctx; ++i) joint[i] = allow && nrhs > 1 && cs[i]->nvmax >= nrhs;
    }
    // streams for concurrent branches
    BatchStreams bs;
    const int nbs = std::min(nctx, 8);
    for (int q = 0; q < nbs; ++q) {
      hipStream_t t;
      SEM_HIP(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
      bs.st.push_back(t);
      hipEvent_t e;
      SEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      bs.ev.push_back(e);
    }
    SEM_HIP(hipEventCreateWithFlags(&bs.fork, hipEventDisableTiming));
    hipStream_t cap;
    SEM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    bs.st.push_back(cap);

    std::vector<LaneScalars> host_all((size_t)nctx * nrhs);
    std::vector<char> recorded(nctx, 0), recorded_lane((size_t)nctx * nrhs, 0);
    // SEM_BATCH_RECORD_ONCE=1: keep replaying the first graph to the end (the
    // finished lanes' kernels return at once; their problems' V-cycles still run)
    const char *once_env = getenv("SEM_BATCH_RECORD_ONCE");
    const bool record_once = once_env && once_env[0] == '1';
    // one outer iteration of every active lane, forked from `root` onto the
    // branch streams and joined back (recorded into a graph, or launched)
    auto enqueue_iteration = [&](hipStream_t root) {
      SEM_HIP(hipEventRecord(bs.fork, root));
      for (int i = 0; i < nctx; ++i) {
        hipStream_t br = bs.st[i % nbs];
        SEM_HIP(hipStreamWaitEvent(br, bs.fork, 0));
        Lane *first = &lanes[(size_t)i * nrhs];
        bool any_active = false;
        for (int k = 0; k < nrhs; ++k) {
          any_active = any_active || first[k].active;
          recorded_lane[(size_t)i * nrhs + k] = first[k].active;
        }
        recorded[i] = any_active;
        if (!any_active) continue;
        if (joint[i]) {
          lane_iteration(first, nrhs, br);  // finished lanes' own kernels return at once
        } else {
          for (int k = 0; k < nrhs; ++k)
            if (first[k].active) lane_iteration(first + k, 1, br);
        }
      }
      for (int q = 0; q < nbs; ++q) {
        SEM_HIP(hipEventRecord(bs.ev[q], bs.st[q]));
        SEM_HIP(hipStreamWaitEvent(root, bs.ev[q], 0));
      }
    };
    // SEM_BATCH_GRAPH=0: launch every iteration's kernels directly (the same
    // kernels on the same streams, no recording)
    const char *graph_env = getenv("SEM_BATCH_GRAPH");
    const bool use_graph = !(graph_env && graph_env[0] == '0');
    int iterations = 0;
    while (!use_graph) {
      bool any = false;
      for (auto &ln : lanes) any = any || ln.active;
      if (!any || iterations >= maxit) break;
      const int k = std::min(ipl, maxit - iterations);
      for (auto *c : cs) c->capturing = true;  // no host interaction inside
      try {
        for (int q = 0; q < k; ++q) enqueue_iteration(s);
      } catch (...) {
        for (auto *c : cs) c->capturing = false;
        throw;
      }
      for (auto *c : cs) c->capturing = false;
      iterations += k;
      poll_lanes(cs, nrhs, host_all, s);
      for (auto &ln : lanes)
        if (ln.active) {
          const LaneScalars &h = host_all[(size_t)ln.ci * nrhs + ln.k];
          if (!(h.rr == h.rr)) fail(SEM_ENAN, "NaN in a batched solve");
          if (h.done) ln.active = false;
        }
    }
    while (use_graph) {
      bool any = false;
      for (auto &ln : lanes) any = any || ln.active;
      if (!any || iterations >= maxit) break;
      // record one outer iteration of every active lane
      for (auto *c : cs) c->capturing = true;
      SEM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      hipGraph_t graph = nullptr;
      try {
        enqueue_iteration(cap);
      } catch (...) {
        (void)hipStreamEndCapture(cap, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto *c : cs) c->capturing = false;
        throw;
      }
      SEM_HIP(hipStreamEndCapture(cap, &graph));
      for (auto *c : cs) c->capturing = false;
      hipGraphExec_t exec = nullptr;
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        SEM_HIP(ie);
      }
      // replay until some lane finishes
      bool changed = false;
      while (!changed && iterations < maxit) {
        if (record_once) {
          bool left = false;
          for (auto &ln : lanes) left = left || ln.active;
          if (!left) break;
        }
        const int k = std::min(ipl, maxit - iterations);
        for (int q = 0; q < k; ++q) SEM_HIP(hipGraphLaunch(exec, s));
        iterations += k;
        poll_lanes(cs, nrhs, host_all, s);
        for (auto &ln : lanes)
          if (ln.active) {
            const LaneScalars &h = host_all[(size_t)ln.ci * nrhs + ln.k];
            if (!(h.rr == h.rr)) fail(SEM_ENAN, "NaN in a batched solve");
            if (h.done) ln.active = false;
          }
        // the recorded graph changes only when a problem sharing its launches
        // finishes all its lanes, or a lane running on its own finishes (the
        // kernels of a finished lane of a shared problem return at once)
        for (int i = 0; i < nctx && !changed && !record_once; ++i) {
          const Lane *first = &lanes[(size_t)i * nrhs];
          bool any_active = false;
          for (int k = 0; k < nrhs; ++k) any_active = any_active || first[k].active;
          if (joint[i]) {
            changed = !any_active && recorded[i];
          } else {
            for (int k = 0; k < nrhs; ++k) changed = changed || (recorded_lane[(size_t)i * nrhs + k] && !first[k].active);
          }
        }
      }
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
    }
    // true residuals and per-lane results
    bool all = true;
    poll_lanes(cs, nrhs, host_all, s);
    for (size_t li = 0; li < lanes.size(); ++li) {
      Lane &ln = lanes[li];
      Ctx &c = *ln.c;
      const Level &F = c.lev[0];
      const LaneScalars &h = host_all[(size_t)ln.ci * nrhs + ln.k];
      batch_opA(c, F, ln.x, ln.q, s);
      launch_sub<double>(F.nloc, ln.b, ln.q, ln.r, s);
      double tr = batch_wnorm2(c, ln.r, ln.r, s);
      sem_solve_info *inf = infos ? &infos[li] : nullptr;
      double rel = h.rr0 > 0 ? std::sqrt(h.rr / h.rr0) : 0.0;
      double trel = h.rr0 > 0 ? std::sqrt(tr / h.rr0) : 0.0;
      bool conv = trel <= rtol;
      all = all && conv;
      if (inf) {
        std::memset(inf, 0, sizeof(*inf));
        inf->iters = h.iters;
        inf->converged = conv ? 1 : 0;
        inf->rel_res = rel;
        inf->true_rel_res = trel;
        inf->r0_norm = std::sqrt(h.rr0);
        inf->coarse_iters = c.capture_coarse_iters;
        for (int l = 0; l < c.nlev; ++l) inf->lambda_tilde[l] = c.lev[l].lam_tilde;
      }
    }
    SEM_HIP(hipStreamSynchronize(s));
    if (!all) {
      set_last_error("a batched lane did not reach rtol within maxit");
      status = SEM_ENOCONV;
    }
  } catch (const Error &e) {
    for (auto *c : cs) c->capturing = false;
    set_last_error(e.msg);
    status = e.status;
  } catch (...) {
    for (auto *c : cs) c->capturing = false;
    set_last_error("unexpected exception in a batched solve");
    status = SEM_EHIP;
  }
  return status;
}
