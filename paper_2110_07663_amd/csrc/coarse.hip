// Coarse-grid solve of the V-cycle (Algorithm 1, "solve" on the coarsest level):
// Jacobi-preconditioned CG on the assembled p = 1 operator.
//
// At p = 1 every node is an element vertex, so the E-vector form (8 copies per
// interior node and a gather-scatter per product) wastes most of its traffic.
// The coarsest level is therefore assembled once into its 27-point stencil
// (row = global node, column = the node offset by (dx, dy, dz) in {-1,0,1}^3),
// with identity rows for Dirichlet nodes, and CG runs on global vectors (36K
// unknowns for a 32^3 mesh, all L2/MALL resident).
//
// The iteration is the Chronopoulos-Gear form of PCG (the same iterates as the
// textbook recurrence in exact arithmetic): one pointwise kernel (update of
// p, s = A p, x, r, z = D^{-1} r and the products (r,z), (r,r)) and one stencil
// kernel (w = A z and (w,z), then alpha and beta) per iteration, both closing
// with a fixed-order last-block reduction.  All scalars stay on the device; a
// finished or broken-down iteration turns every later kernel into a no-op, so a
// chunk of iterations is recorded once as a HIP graph and replayed.
#include "sem_internal.h"

namespace sem {

struct CoarseGrid {
  int nex, ney, nez;
  int64_t nx, ny, nz;
  int bc[6];
};

static CoarseGrid cgrid(const Ctx &c) {
  CoarseGrid g;
  g.nex = c.nex; g.ney = c.ney; g.nez = c.nez;
  g.nx = c.nex + 1; g.ny = c.ney + 1; g.nz = c.nez + 1;
  for (int f = 0; f < 6; ++f) g.bc[f] = c.bc[f];
  return g;
}

__device__ inline bool cg_dirichlet(const CoarseGrid &g, int64_t x, int64_t y, int64_t z) {
  return (g.bc[0] && x == 0) || (g.bc[1] && x == g.nx - 1) || (g.bc[2] && y == 0) ||
         (g.bc[3] && y == g.ny - 1) || (g.bc[4] && z == 0) || (g.bc[5] && z == g.nz - 1);
}

// element matrix of a p = 1 element: A[q][q'] = sum_{q''} sum_{b,c} (D_b)_{q''q} G_bc(q'') (D_c)_{q''q'}
__global__ void k_coarse_elem(int64_t E, const double *__restrict__ G, const double *__restrict__ D,
                              double *__restrict__ Ae) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  const double *Ge = G + e * 6 * 8;
  const int pr[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  double *A = Ae + e * 64;
  for (int q = 0; q < 64; ++q) A[q] = 0.0;
  for (int qq = 0; qq < 8; ++qq) {
    int i2 = qq & 1, j2 = (qq >> 1) & 1, k2 = qq >> 2;
    // grad of basis function q at point qq along r, s, t: Db[qq][q]
    double gr[3][8];
    for (int q = 0; q < 8; ++q) {
      int i = q & 1, j = (q >> 1) & 1, k = q >> 2;
      gr[0][q] = (j == j2 && k == k2) ? D[i2 * 2 + i] : 0.0;
      gr[1][q] = (i == i2 && k == k2) ? D[j2 * 2 + j] : 0.0;
      gr[2][q] = (i == i2 && j == j2) ? D[k2 * 2 + k] : 0.0;
    }
    double Gm[3][3];
    for (int c = 0; c < 6; ++c) {
      double v = Ge[c * 8 + qq];
      Gm[pr[c][0]][pr[c][1]] = v;
      Gm[pr[c][1]][pr[c][0]] = v;
    }
    for (int q = 0; q < 8; ++q)
      for (int q2 = 0; q2 < 8; ++q2) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b)
          for (int cc = 0; cc < 3; ++cc) s += gr[b][q] * Gm[b][cc] * gr[cc][q2];
        A[q * 8 + q2] += s;
      }
  }
}

// stencil row of every global node, gathered from its (up to 8) elements in a
// fixed order; Dirichlet rows become identity, Dirichlet columns are dropped
__global__ void k_coarse_assemble(CoarseGrid g, const double *__restrict__ Ae,
                                  double *__restrict__ St, double *__restrict__ dinv) {
  int64_t n = g.nx * g.ny * g.nz;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  int64_t x = t % g.nx, y = (t / g.nx) % g.ny, z = t / (g.nx * g.ny);
  double row[27];
  for (int m = 0; m < 27; ++m) row[m] = 0.0;
  bool dir = cg_dirichlet(g, x, y, z);
  if (!dir) {
    for (int ez = (int)z - 1; ez <= (int)z; ++ez)
      for (int ey = (int)y - 1; ey <= (int)y; ++ey)
        for (int ex = (int)x - 1; ex <= (int)x; ++ex) {
          if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nex || ey >= g.ney || ez >= g.nez) continue;
          int64_t e = ((int64_t)ez * g.ney + ey) * g.nex + ex;
          int q = (int)((z - ez) * 4 + (y - ey) * 2 + (x - ex));
          for (int q2 = 0; q2 < 8; ++q2) {
            int64_t cx = ex + (q2 & 1), cy = ey + ((q2 >> 1) & 1), cz = ez + (q2 >> 2);
            if (cg_dirichlet(g, cx, cy, cz)) continue;
            int m = (int)((cz - z + 1) * 9 + (cy - y + 1) * 3 + (cx - x + 1));
            row[m] += Ae[e * 64 + q * 8 + q2];
          }
        }
  } else {
    row[13] = 1.0;
  }
  for (int m = 0; m < 27; ++m) St[m * n + t] = row[m];
  dinv[t] = dir ? 0.0 : 1.0 / row[13];
}

// b_g[node] = b_L at the node's owner copy (the element with the smallest index)
__global__ void k_coarse_to_global(CoarseGrid g, const double *__restrict__ bl,
                                   double *__restrict__ bg) {
  int64_t n = g.nx * g.ny * g.nz;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  int64_t x = t % g.nx, y = (t / g.nx) % g.ny, z = t / (g.nx * g.ny);
  int64_t ex = x < g.nex ? x : g.nex - 1, ey = y < g.ney ? y : g.ney - 1,
          ez = z < g.nez ? z : g.nez - 1;
  int q = (int)((z - ez) * 4 + (y - ey) * 2 + (x - ex));
  bg[t] = bl[((ez * g.ney + ey) * g.nex + ex) * 8 + q];
}

__device__ inline double stencil_apply(const CoarseGrid &g, const double *__restrict__ St,
                                       const double *__restrict__ u, int64_t t, int64_t n) {
  int64_t x = t % g.nx, y = (t / g.nx) % g.ny, z = t / (g.nx * g.ny);
  double acc = 0.0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        int m = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        int64_t cx = x + dx, cy = y + dy, cz = z + dz;
        bool in = cx >= 0 && cy >= 0 && cz >= 0 && cx < g.nx && cy < g.ny && cz < g.nz;
        if (in) acc += St[m * n + t] * u[(cz * g.ny + cy) * g.nx + cx];
      }
  return acc;
}

struct CgPtrs {
  const double *St, *dinv, *b;
  double *x, *r, *u, *w, *p, *s;
  double *partials;
  unsigned *counter;
  CoarseScalars *sc;
};

template <int ND>
__device__ inline bool cg_last_block(double (&acc)[ND], double *partials, unsigned *counter) {
  __shared__ double sh[ND][256];
  __shared__ bool is_last;
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
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) partials[blockIdx.x * 4 + j] = sh[j][0];
    __threadfence();
    is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  for (int b = tid; b < (int)gridDim.x; b += 256)
#pragma unroll
    for (int j = 0; j < ND; ++j)
      acc[j] += __hip_atomic_load(&partials[b * 4 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
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
  if (tid == 0) *counter = 0u;
  return true;
}

// start from x = 0: r = b, z = D^{-1} r, p = s = 0; (r,z), (r,r)
__global__ __launch_bounds__(256) void k_cg_start(int64_t n, CgPtrs P, double tol2, int maxit) {
  double acc[2] = {0.0, 0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double rv = P.b[t], zv = P.dinv[t] * rv;
    P.x[t] = 0.0;
    P.r[t] = rv;
    P.u[t] = zv;
    P.p[t] = 0.0;
    P.s[t] = 0.0;
    acc[0] += rv * zv;
    acc[1] += rv * rv;
  }
  if (cg_last_block<2>(acc, P.partials, P.counter) && threadIdx.x == 0) {
    CoarseScalars *c = P.sc;
    c->gamma = acc[0];
    c->rr = acc[1];
    c->rr0 = acc[1];
    c->tol2 = tol2;
    c->maxit = maxit;
    c->iters = 0;
    c->alpha = 0.0;
    c->beta = 0.0;
    c->done = (acc[1] == 0.0 || maxit <= 0 || !(acc[0] > 0.0)) ? 1 : 0;
  }
}

// w = A z, delta = (w, z); then alpha, beta for the next update
__global__ __launch_bounds__(256) void k_cg_spmv(int64_t n, CoarseGrid g, CgPtrs P, int first) {
  if (P.sc->done) return;
  double acc[1] = {0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double wv = stencil_apply(g, P.St, P.u, t, n);
    P.w[t] = wv;
    acc[0] += wv * P.u[t];
  }
  if (cg_last_block<1>(acc, P.partials, P.counter) && threadIdx.x == 0) {
    CoarseScalars *c = P.sc;
    const double delta = acc[0];
    double alpha, beta;
    if (first) {
      beta = 0.0;
      alpha = c->gamma / delta;
    } else {
      beta = c->gamma / c->gamma_old;
      alpha = c->gamma / (delta - beta * c->gamma / c->alpha);
    }
    c->delta = delta;
    c->beta = beta;
    c->alpha = alpha;
    if (!(alpha > 0.0) || !(delta > 0.0)) c->done = 1;  // exact breakdown (or NaN)
  }
}

// p = z + beta p; s = w + beta s; x += alpha p; r -= alpha s; z = D^{-1} r; (r,z), (r,r)
__global__ __launch_bounds__(256) void k_cg_update(int64_t n, CgPtrs P) {
  CoarseScalars *c = P.sc;
  if (c->done) return;
  const double alpha = c->alpha, beta = c->beta;
  double acc[2] = {0.0, 0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double pv = P.u[t] + beta * P.p[t];
    double sv = P.w[t] + beta * P.s[t];
    P.p[t] = pv;
    P.s[t] = sv;
    P.x[t] += alpha * pv;
    double rv = P.r[t] - alpha * sv;
    double zv = P.dinv[t] * rv;
    P.r[t] = rv;
    P.u[t] = zv;
    acc[0] += rv * zv;
    acc[1] += rv * rv;
  }
  if (cg_last_block<2>(acc, P.partials, P.counter) && threadIdx.x == 0) {
    c->gamma_old = c->gamma;
    c->gamma = acc[0];
    c->rr = acc[1];
    c->iters += 1;
    bool conv = c->tol2 > 0.0 && acc[1] <= c->tol2 * c->rr0;
    if (conv || c->iters >= c->maxit || !(acc[0] > 0.0) || !(acc[1] == acc[1])) c->done = 1;
  }
}

static inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }
// CG kernels: each thread handles `rows_per_thread` rows (fewer blocks close
// each reduction); the grid is fixed per solver so the summation order is too
static inline unsigned cg_grid(const CoarseSolver &S) {
  int64_t per = 256 * (int64_t)S.rows_per_thread;
  return (unsigned)((S.n + per - 1) / per);
}

static CgPtrs ptrs(const Ctx &c) {
  const CoarseSolver &S = *c.cs;
  CgPtrs P;
  P.St = S.St; P.dinv = S.dinv; P.b = S.b;
  P.x = S.x; P.r = S.r; P.u = S.u; P.w = S.w; P.p = S.p; P.s = S.s;
  P.partials = S.partials; P.counter = S.counter; P.sc = S.sc;
  return P;
}

bool coarse_assembled_ok(const Ctx &c, const Level &C) { return C.p == 1 && c.cs != nullptr; }

void coarse_setup(Ctx &c, Level &C, hipStream_t s) {
  CoarseSolver &S = *c.cs;
  CoarseGrid g = cgrid(c);
  hipLaunchKernelGGL(k_coarse_elem, dim3(nb(C.E)), dim3(256), 0, s, C.E, C.G64, C.D64, S.Ae);
  SEM_LAUNCH("k_coarse_elem");
  hipLaunchKernelGGL(k_coarse_assemble, dim3(nb(S.n)), dim3(256), 0, s, g, S.Ae, S.St, S.dinv);
  SEM_LAUNCH("k_coarse_assemble");
}

static void enqueue_iterations(const Ctx &c, int k, hipStream_t s) {
  CgPtrs P = ptrs(c);
  CoarseGrid g = cgrid(c);
  const int64_t n = c.cs->n;
  for (int it = 0; it < k; ++it) {
    hipLaunchKernelGGL(k_cg_update, dim3(cg_grid(*c.cs)), dim3(256), 0, s, n, P);
    SEM_LAUNCH("k_cg_update");
    hipLaunchKernelGGL(k_cg_spmv, dim3(cg_grid(*c.cs)), dim3(256), 0, s, n, g, P, 0);
    SEM_LAUNCH("k_cg_spmv");
  }
}

static void ensure_graph(Ctx &c) {
  CoarseSolver &S = *c.cs;
  if (S.exec) return;
  if (!S.cap) SEM_HIP(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
  SEM_HIP(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_iterations(c, S.chunk, S.cap);
  } catch (...) {
    hipGraph_t dummy;
    (void)hipStreamEndCapture(S.cap, &dummy);
    throw;
  }
  SEM_HIP(hipStreamEndCapture(S.cap, &S.graph));
  SEM_HIP(hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
}

// solve on the coarsest level: C.d_b (consistent, masked E-vector) -> c.cx
void coarse_solve_assembled(Ctx &c, Level &C, double tol, int maxit, hipStream_t s) {
  CoarseSolver &S = *c.cs;
  CoarseGrid g = cgrid(c);
  CgPtrs P = ptrs(c);
  hipLaunchKernelGGL(k_coarse_to_global, dim3(nb(S.n)), dim3(256), 0, s, g, C.d_b, S.b);
  SEM_LAUNCH("k_coarse_to_global");
  hipLaunchKernelGGL(k_cg_start, dim3(cg_grid(S)), dim3(256), 0, s, S.n, P,
                     tol > 0 ? tol * tol : 0.0, maxit);
  SEM_LAUNCH("k_cg_start");
  hipLaunchKernelGGL(k_cg_spmv, dim3(cg_grid(S)), dim3(256), 0, s, S.n, g, P, 1);
  SEM_LAUNCH("k_cg_spmv");
  if (c.capturing) {
    // inside a recorded batch iteration: a fixed count, no readback
    const int k = tol > 0.0 ? std::min(maxit, c.capture_coarse_iters) : maxit;
    enqueue_iterations(c, k, s);
    launch_gather(c, C, S.x, c.cx, s);
    return;
  }
  if (tol <= 0.0 || !S.use_graph) {
    // fixed iteration count (or graphs off): plain launches, one readback at most
    if (tol <= 0.0) {
      enqueue_iterations(c, maxit, s);
    } else {
      int done_it = 0;
      int chunk = std::max(8, c.last_coarse_iters + 2);
      while (true) {
        int k = std::min(chunk, maxit - done_it);
        enqueue_iterations(c, k, s);
        done_it += k;
        SEM_HIP(hipMemcpyAsync(c.hres, S.sc, sizeof(CoarseScalars), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
        const CoarseScalars *h = reinterpret_cast<const CoarseScalars *>(c.hres);
        if (h->done || done_it >= maxit) break;
        chunk = 8;
      }
    }
  } else {
    ensure_graph(c);
    int done_it = 0;
    int predicted = std::max(S.chunk, c.last_coarse_iters);
    while (true) {
      int launches = (std::min(predicted, maxit) - done_it + S.chunk - 1) / S.chunk;
      if (launches < 1) launches = 1;
      for (int q = 0; q < launches; ++q) SEM_HIP(hipGraphLaunch(S.exec, s));
      done_it += launches * S.chunk;
      SEM_HIP(hipMemcpyAsync(c.hres, S.sc, sizeof(CoarseScalars), hipMemcpyDeviceToHost, s));
      SEM_HIP(hipStreamSynchronize(s));
      const CoarseScalars *h = reinterpret_cast<const CoarseScalars *>(c.hres);
      if (h->done || done_it >= maxit) break;
      predicted = done_it + S.chunk;
    }
  }
  SEM_HIP(hipMemcpyAsync(c.hres, S.sc, sizeof(CoarseScalars), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  const CoarseScalars *h = reinterpret_cast<const CoarseScalars *>(c.hres);
  if (tol > 0.0) c.last_coarse_iters = h->iters;
  else c.last_coarse_iters = maxit;
  if (!(h->rr == h->rr)) fail(SEM_ENAN, "NaN in the coarse-grid solve");
  launch_gather(c, C, S.x, c.cx, s);
}

void coarse_release(CoarseSolver &S) {
  if (S.exec) (void)hipGraphExecDestroy(S.exec);
  if (S.graph) (void)hipGraphDestroy(S.graph);
  if (S.cap) (void)hipStreamDestroy(S.cap);
  S.exec = nullptr;
  S.graph = nullptr;
  S.cap = nullptr;
}

}  // namespace sem
