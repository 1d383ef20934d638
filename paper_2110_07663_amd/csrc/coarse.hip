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
// textbook recurrence in exact arithmetic): update p, s = A p, x, r and
// z = D^{-1} r, then w = A z, and one reduction of (r,z), (r,r), (w,z) gives
// the next alpha and beta.  Both halves run in ONE kernel per iteration: the
// stencil needs the new z of neighbouring rows, and each row recomputes those
// from the neighbours' previous r, s, w (kept in two alternating copies), so
// no grid-wide synchronisation separates the update from the product.  The
// kernel closes with a fixed-order last-block reduction.  All scalars stay on
// the device; a finished or broken-down iteration turns every later kernel
// into a no-op, so a chunk of iterations is recorded once as a HIP graph and
// replayed.
//
// Optionally (SEM_COARSE_PERSIST=1) the whole solve runs as one persistent
// cooperative launch (k_cg_persistent): each thread keeps its stencil row and
// its entries of the CG vectors in registers and the phases are separated by
// grid barriers that carry the partial sums.  On an 8-XCD device a grid
// barrier costs more than a kernel boundary, so this is not the default.
#include <algorithm>

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

// b_g[node] = b_L at the node's owner copy (the element with the smallest index);
// also clears the grid-barrier state of the persistent solve that follows
__global__ void k_coarse_to_global(CoarseGrid g, const double *__restrict__ bl,
                                   double *__restrict__ bg, unsigned *bar, int *aborted) {
  int64_t n = g.nx * g.ny * g.nz;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t == 0 && blockIdx.y == 0) {
    *bar = 0u;
    *aborted = 0;
  }
  if (t >= n) return;
  bl += blockIdx.y * (int64_t)g.nex * g.ney * g.nez * 8;  // right side blockIdx.y
  bg += blockIdx.y * n;
  int64_t x = t % g.nx, y = (t / g.nx) % g.ny, z = t / (g.nx * g.ny);
  int64_t ex = x < g.nex ? x : g.nex - 1, ey = y < g.ney ? y : g.ney - 1,
          ez = z < g.nez ? z : g.nez - 1;
  int q = (int)((z - ez) * 4 + (y - ey) * 2 + (x - ex));
  bg[t] = bl[((ez * g.ney + ey) * g.nex + ex) * 8 + q];
}

// b_g[node] = the sum of the node's copies in b_L as the restriction leaves
// it (before its gather-scatter), in FP64, the elements in increasing index
// order; 0 on Dirichlet nodes.  Also clears the grid-barrier state.
template <typename T>
__global__ void k_coarse_sum_to_global(CoarseGrid g, const T *__restrict__ bl,
                                       double *__restrict__ bg, unsigned *bar, int *aborted) {
  const int64_t n = g.nx * g.ny * g.nz;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t == 0 && blockIdx.y == 0) {
    *bar = 0u;
    *aborted = 0;
  }
  if (t >= n) return;
  bl += blockIdx.y * (int64_t)g.nex * g.ney * g.nez * 8;  // right side blockIdx.y
  bg += blockIdx.y * n;
  const int64_t x = t % g.nx, y = (t / g.nx) % g.ny, z = t / (g.nx * g.ny);
  double acc = 0.0;
  if (!cg_dirichlet(g, x, y, z)) {
    for (int64_t ez = z - 1; ez <= z; ++ez) {
      if (ez < 0 || ez >= g.nez) continue;
      for (int64_t ey = y - 1; ey <= y; ++ey) {
        if (ey < 0 || ey >= g.ney) continue;
        for (int64_t ex = x - 1; ex <= x; ++ex) {
          if (ex < 0 || ex >= g.nex) continue;
          const int q = (int)((z - ez) * 4 + (y - ey) * 2 + (x - ex));
          acc += (double)bl[((ez * g.ney + ey) * g.nex + ex) * 8 + q];
        }
      }
    }
  }
  bg[t] = acc;
}

static void launch_to_global(const CoarseSolver &S, const CoarseGrid &g, const double *bl,
                             CoarseRhs u, int nv, hipStream_t s) {
  const dim3 grid((unsigned)((S.n + 255) / 256), (unsigned)nv);
  if (!u.p) {
    hipLaunchKernelGGL(k_coarse_to_global, grid, dim3(256), 0, s, g, bl, S.b, S.counter + 32,
                       &S.sc->aborted);
  } else if (u.f32) {
    hipLaunchKernelGGL(k_coarse_sum_to_global<float>, grid, dim3(256), 0, s, g,
                       (const float *)u.p, S.b, S.counter + 32, &S.sc->aborted);
  } else {
    hipLaunchKernelGGL(k_coarse_sum_to_global<double>, grid, dim3(256), 0, s, g,
                       (const double *)u.p, S.b, S.counter + 32, &S.sc->aborted);
  }
  SEM_LAUNCH("k_coarse_to_global");
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
  double *r2, *w2, *s2;  // second copies of r, w, s (alternating iterations)
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

// first product: w = A z, delta = (w, z), alpha = gamma / delta, beta = 0
__global__ __launch_bounds__(256) void k_cg_first(int64_t n, CoarseGrid g, CgPtrs P) {
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
    const double alpha = c->gamma / delta;
    c->delta = delta;
    c->beta = 0.0;
    c->alpha = alpha;
    if (!(alpha > 0.0) || !(delta > 0.0)) c->done = 1;  // exact breakdown (or NaN)
  }
}

// new z of a row from its previous r, s, w: s' = w + beta s, r' = r - alpha s',
// z' = D^{-1} r' (the same expression for the row itself and for its neighbours)
__device__ inline double cg_next_z(double dinv, double r, double w, double s, double alpha,
                                   double beta, double &s_new, double &r_new) {
  s_new = w + beta * s;
  r_new = r - alpha * s_new;
  return dinv * r_new;
}

// Sum over a wavefront by an xor butterfly: every lane ends with the same bits
// (each step adds the same two values, in either order).
template <int ND>
__device__ inline void wave_sum(double (&acc)[ND]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[j] += __shfl_xor(acc[j], o, 64);
}

// cg_last_block for blocks of NW wavefronts: wave sums, then the NW wave sums
// in order; the last block sums the block partials the same way.
template <int ND, int NW>
__device__ inline bool cg_last_block_waves(double (&acc)[ND], double *partials,
                                           unsigned *counter) {
  __shared__ double sh[ND][NW];
  __shared__ bool is_last;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  wave_sum<ND>(acc);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) sh[j][wv] = acc[j];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += sh[j][w];
      partials[blockIdx.x * 4 + j] = t;
    }
    __threadfence();
    is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  for (int b = tid; b < (int)gridDim.x; b += 64 * NW)
#pragma unroll
    for (int j = 0; j < ND; ++j)
      acc[j] += __hip_atomic_load(&partials[b * 4 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  wave_sum<ND>(acc);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) sh[j][wv] = acc[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += sh[j][w];
    acc[j] = t;
  }
  if (tid == 0) *counter = 0u;
  return true;
}

// One iteration: p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s,
// z = D^{-1} r, w = A z, then (r,z), (r,r), (w,z) -> gamma, rr, delta and the
// next alpha, beta.  Reads r, s, w from copy `par`, writes them to copy 1-par.
// Four lanes share a row (lane q takes stencil entries q, q+4, ...), 64 rows
// per 256-thread block (four times as many blocks as 256-row, 1024-thread
// ones: at 17^3 unknowns 77 compute units share the stencil reads instead of
// 20); every load is issued before the scalars are known, so the kernel waits
// on memory about once.
constexpr int kCgRows = 256;     // rows per block of the start kernels
constexpr int kCgIterWaves = 4;  // wavefronts per block of the iteration
constexpr int kCgIterRows = 16 * kCgIterWaves;
__global__ __launch_bounds__(64 * kCgIterWaves) void k_cg_iter(int64_t n, CoarseGrid g, CgPtrs P,
                                                                int par) {
  CoarseScalars *c = P.sc;
  const double *__restrict__ R = par ? P.r2 : P.r;
  const double *__restrict__ Wv = par ? P.w2 : P.w;
  const double *__restrict__ Sv = par ? P.s2 : P.s;
  const int q = threadIdx.x & 3;
  const int64_t t = blockIdx.x * (int64_t)kCgIterRows + (threadIdx.x >> 2);
  const bool row = t < n;
  const int64_t tt = row ? t : 0;
  const int nx = (int)g.nx, ny = (int)g.ny, nz = (int)g.nz;
  // (n < 2^31 for any coarse grid this solver takes: 32-bit index arithmetic)
  const unsigned ut = (unsigned)tt, uxy = ut / (unsigned)nx;
  const int x = (int)(ut - uxy * (unsigned)nx), y = (int)(uxy % (unsigned)ny),
            z = (int)(uxy / (unsigned)ny);
  // this lane's stencil entries m = q + 4k and the neighbours' previous r, s, w
  // (unconditional loads at clamped indices, so that they all issue at once;
  // entries outside the grid get coefficient 0)
  double a[7], dj[7], rj[7], wj[7], sj[7];
  bool in[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int m = q + 4 * k;
    const int dx = m % 3 - 1, dy = (m / 3) % 3 - 1, dz = m / 9 - 1;
    in[k] = row && m < 27 && x + dx >= 0 && x + dx < nx && y + dy >= 0 && y + dy < ny &&
            z + dz >= 0 && z + dz < nz;
    const int64_t j = in[k] ? tt + dx + (int64_t)dy * nx + (int64_t)dz * nx * ny : tt;
    a[k] = P.St[(m < 27 ? m : 26) * n + tt];
    dj[k] = P.dinv[j];
    rj[k] = R[j];
    wj[k] = Wv[j];
    sj[k] = Sv[j];
  }
  const double di = P.dinv[tt], r0 = R[tt], w0 = Wv[tt], s0 = Sv[tt], p0 = P.p[tt];
  const double x0 = P.x[tt];
  if (c->done) return;
  const double alpha = c->alpha, beta = c->beta;
  const double pv = di * r0 + beta * p0;
  double sv, rv;
  const double zv = cg_next_z(di, r0, w0, s0, alpha, beta, sv, rv);
  double wq = 0.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    double s1, r1;
    const double zj = cg_next_z(dj[k], rj[k], wj[k], sj[k], alpha, beta, s1, r1);
    if (in[k]) wq += a[k] * zj;
  }
  wq += __shfl_xor(wq, 1, 64);
  wq += __shfl_xor(wq, 2, 64);
  double acc[3] = {0.0, 0.0, 0.0};
  if (row && q == 0) {
    double *__restrict__ Rn = par ? P.r : P.r2;
    double *__restrict__ Wn = par ? P.w : P.w2;
    double *__restrict__ Sn = par ? P.s : P.s2;
    P.p[t] = pv;
    P.x[t] = x0 + alpha * pv;
    Rn[t] = rv;
    Sn[t] = sv;
    Wn[t] = wq;
    acc[0] = rv * zv;
    acc[1] = rv * rv;
    acc[2] = wq * zv;
  }
  if (cg_last_block_waves<3, kCgIterWaves>(acc, P.partials, P.counter) && threadIdx.x == 0) {
    c->gamma_old = c->gamma;
    c->gamma = acc[0];
    c->rr = acc[1];
    c->iters += 1;
    const bool conv = c->tol2 > 0.0 && acc[1] <= c->tol2 * c->rr0;
    if (conv || c->iters >= c->maxit || !(acc[0] > 0.0) || !(acc[1] == acc[1])) {
      c->done = 1;
    } else {
      const double delta = acc[2];
      const double b2 = c->gamma / c->gamma_old;
      const double a2 = c->gamma / (delta - b2 * c->gamma / alpha);
      c->delta = delta;
      c->beta = b2;
      c->alpha = a2;
      if (!(a2 > 0.0) || !(delta > 0.0)) c->done = 1;  // exact breakdown (or NaN)
    }
  }
}

// ---- persistent form ------------------------------------------------------

struct GridSync {
  unsigned *count;    // arrivals, monotone within one launch (cleared before it)
  int *aborted;       // raised by a block whose wait exceeded spin_limit
  double *partials;   // [2][gridDim.x][4], alternating between barriers
  unsigned epoch;     // barriers passed so far (same in every block)
  int spin_limit;
};

// Grid barrier that also reduces: every block publishes its block sum of acc,
// waits until all blocks have arrived, then sums the gridDim.x partials in the
// order of cg_last_block, so every block ends with the same totals.  Returns
// false (in every thread of the block) if the wait was abandoned.
template <int ND>
__device__ bool grid_reduce(double (&acc)[ND], GridSync &gs) {
  __shared__ double sh[ND][256];
  __shared__ int ok;
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
  double *part = gs.partials + (size_t)(gs.epoch & 1u) * gridDim.x * 4;
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) part[blockIdx.x * 4 + j] = sh[j][0];
  }
  __threadfence();  // every wave: its stores (z and the partials) reach agent scope
  __syncthreads();
  gs.epoch += 1u;
  if (tid == 0) {
    int good = 1;
    __hip_atomic_fetch_add(gs.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = gs.epoch * gridDim.x;
    int spins = 0;
    while (__hip_atomic_load(gs.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 63) == 0 &&
          (spins > gs.spin_limit ||
           __hip_atomic_load(gs.aborted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        __hip_atomic_store(gs.aborted, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
    }
    ok = good;
  }
  __syncthreads();
  if (!ok) return false;
  __threadfence();  // acquire: later loads see the other blocks' stores
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  for (int b = tid; b < (int)gridDim.x; b += 256)
#pragma unroll
    for (int j = 0; j < ND; ++j)
      acc[j] += __hip_atomic_load(&part[b * 4 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  __syncthreads();  // sh is reused by the next call
  return true;
}

// The whole Chronopoulos-Gear PCG of k_cg_start / k_cg_first / k_cg_iter in
// one launch of ceil(n/256) blocks, thread = row.  The scalar recurrences and
// the stopping and breakdown tests are those of the two-kernel form, evaluated
// redundantly (and identically) in every block, so all blocks leave the loop
// at the same iteration.
__global__ __launch_bounds__(256) void k_cg_persistent(CoarseGrid g, CgPtrs P, double tol2,
                                                       int maxit, GridSync gs) {
  const int64_t n = g.nx * g.ny * g.nz;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = t < n;
  double a[27];
  unsigned valid = 0u;
  if (act) {
    const int64_t x = t % g.nx, y = (t / g.nx) % g.ny, z = t / (g.nx * g.ny);
#pragma unroll
    for (int m = 0; m < 27; ++m) {
      const int dx = m % 3 - 1, dy = (m / 3) % 3 - 1, dz = m / 9 - 1;
      const bool in = x + dx >= 0 && y + dy >= 0 && z + dz >= 0 && x + dx < g.nx &&
                      y + dy < g.ny && z + dz < g.nz;
      a[m] = P.St[m * n + t];
      if (in) valid |= 1u << m;
    }
  } else {
#pragma unroll
    for (int m = 0; m < 27; ++m) a[m] = 0.0;
  }
  const int64_t sy = g.nx, sz = g.nx * g.ny;
  const double *__restrict__ U = P.u;
  auto spmv = [&]() {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 27; ++m) {
      const int64_t off = (int64_t)(m / 9 - 1) * sz + (int64_t)((m / 3) % 3 - 1) * sy + (m % 3 - 1);
      if (valid & (1u << m)) acc += a[m] * U[t + off];
    }
    return acc;
  };
  const double di = act ? P.dinv[t] : 0.0;
  double rv = act ? P.b[t] : 0.0;
  double uv = di * rv, xv = 0.0, pv = 0.0, sv = 0.0, wv = 0.0;
  if (act) P.u[t] = uv;
  double acc2[2] = {rv * uv, rv * rv};
  if (!grid_reduce<2>(acc2, gs)) return;
  double gamma = acc2[0], rr = acc2[1];
  const double rr0 = rr;
  double gamma_old = 0.0, alpha = 0.0, beta = 0.0, delta = 0.0;
  int iters = 0;
  bool done = rr == 0.0 || maxit <= 0 || !(gamma > 0.0);
  if (!done) {
    wv = spmv();
    double acc1[1] = {wv * uv};
    if (!grid_reduce<1>(acc1, gs)) return;
    delta = acc1[0];
    beta = 0.0;
    alpha = gamma / delta;
    if (!(alpha > 0.0) || !(delta > 0.0)) done = true;
  }
  while (!done) {
    pv = uv + beta * pv;
    sv = wv + beta * sv;
    xv += alpha * pv;
    rv = rv - alpha * sv;
    uv = di * rv;
    if (act) P.u[t] = uv;
    acc2[0] = rv * uv;
    acc2[1] = rv * rv;
    if (!grid_reduce<2>(acc2, gs)) return;
    gamma_old = gamma;
    gamma = acc2[0];
    rr = acc2[1];
    iters += 1;
    const bool conv = tol2 > 0.0 && rr <= tol2 * rr0;
    if (conv || iters >= maxit || !(gamma > 0.0) || !(rr == rr)) break;
    wv = spmv();
    double acc1[1] = {wv * uv};
    if (!grid_reduce<1>(acc1, gs)) return;
    delta = acc1[0];
    beta = gamma / gamma_old;
    alpha = gamma / (delta - beta * gamma / alpha);
    if (!(alpha > 0.0) || !(delta > 0.0)) done = true;
  }
  if (act) {
    P.x[t] = xv;
    P.r[t] = rv;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CoarseScalars *c = P.sc;
    c->gamma = gamma;
    c->gamma_old = gamma_old;
    c->delta = delta;
    c->alpha = alpha;
    c->beta = beta;
    c->rr = rr;
    c->rr0 = rr0;
    c->tol2 = tol2;
    c->iters = iters;
    c->maxit = maxit;
    c->done = 1;
  }
}

static inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

size_t coarse_cg_partials(int64_t n) {
  const int64_t iter = 4 * ((n + kCgIterRows - 1) / kCgIterRows);  // k_cg_iter's blocks
  const int64_t persistent = 8 * ((n + 255) / 256);               // two epochs of 256-row blocks
  const int64_t start = 4 * ((n + kCgRows - 1) / kCgRows);
  return (size_t)std::max(iter, std::max(persistent, start));
}

// CG start kernels: one 256-thread block per 256 rows (the iteration: one per
// 64 rows, k_cg_iter); the grids are fixed per solver, so is the summation
// order
static inline unsigned cg_grid(const CoarseSolver &S) {
  return (unsigned)((S.n + kCgRows - 1) / kCgRows);
}

static CgPtrs ptrs(const Ctx &c) {
  const CoarseSolver &S = *c.cs;
  CgPtrs P;
  P.St = S.St; P.dinv = S.dinv; P.b = S.b;
  P.x = S.x; P.r = S.r; P.u = S.u; P.w = S.w; P.p = S.p; P.s = S.s;
  P.r2 = S.r2; P.w2 = S.w2; P.s2 = S.s2;
  P.partials = S.partials; P.counter = S.counter; P.sc = S.sc;
  return P;
}

bool coarse_assembled_ok(const Ctx &c, const Level &C) { return C.p == 1 && c.cs != nullptr; }

void coarse_setup(Ctx &c, Level &C, hipStream_t s) {
  CoarseSolver &S = *c.cs;
  CoarseGrid g = cgrid(c);
  // the persistent solve needs all ceil(n/256) blocks resident at once
  {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    SEM_HIP(hipGetDevice(&dev));
    SEM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    SEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg_persistent, 256, 0));
    const char *env = getenv("SEM_COARSE_PERSIST");
    const int64_t blocks = (S.n + 255) / 256;
    const int64_t barriers = 4 + 2 * (int64_t)c.opts.coarse_maxit;
    S.persistent = coop != 0 && blocks <= (int64_t)per_cu * cus && blocks * barriers < (1ll << 31) &&
                   env && env[0] == '1';
  }
  hipLaunchKernelGGL(k_coarse_elem, dim3(nb(C.E)), dim3(256), 0, s, C.E, C.G64, C.D64, S.Ae);
  SEM_LAUNCH("k_coarse_elem");
  hipLaunchKernelGGL(k_coarse_assemble, dim3(nb(S.n)), dim3(256), 0, s, g, S.Ae, S.St, S.dinv);
  SEM_LAUNCH("k_coarse_assemble");
  if (S.direct) coarse_direct_setup(S, g.nx, g.ny, g.nz, s);
}

// k iterations after `done` earlier ones (which fixes the copy of r, s, w read first)
static void enqueue_iterations(const Ctx &c, int k, int done, hipStream_t s) {
  CgPtrs P = ptrs(c);
  CoarseGrid g = cgrid(c);
  const int64_t n = c.cs->n;
  for (int it = 0; it < k; ++it) {
    hipLaunchKernelGGL(k_cg_iter, dim3((unsigned)((n + kCgIterRows - 1) / kCgIterRows)),
                       dim3(64 * kCgIterWaves), 0, s, n, g, P, (done + it) & 1);
    SEM_LAUNCH("k_cg_iter");
  }
}

static void ensure_graph(Ctx &c) {
  CoarseSolver &S = *c.cs;
  if (S.exec) return;
  if (!S.cap) SEM_HIP(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
  SEM_HIP(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_iterations(c, S.chunk, 0, S.cap);  // chunk is even: every replay starts on copy 0
  } catch (...) {
    hipGraph_t dummy;
    (void)hipStreamEndCapture(S.cap, &dummy);
    throw;
  }
  SEM_HIP(hipStreamEndCapture(S.cap, &S.graph));
  SEM_HIP(hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
}

// one right side: bl (consistent, masked E-vector of the coarsest level) -> xl
static void coarse_solve_one(Ctx &c, Level &C, double tol, int maxit, hipStream_t s,
                             const double *bl, double *xl, CoarseRhs u) {
  CoarseSolver &S = *c.cs;
  CoarseGrid g = cgrid(c);
  CgPtrs P = ptrs(c);
  launch_to_global(S, g, bl, u, 1, s);
  if (!c.capturing && S.persistent) {
    GridSync gs;
    gs.count = S.counter + 32;
    gs.aborted = &S.sc->aborted;
    gs.partials = S.partials;
    gs.epoch = 0u;
    gs.spin_limit = 1 << 20;
    double tol2 = tol > 0 ? tol * tol : 0.0;
    void *args[] = {&g, &P, &tol2, &maxit, &gs};
    SEM_HIP(hipLaunchCooperativeKernel((const void *)k_cg_persistent, dim3(nb(S.n)), dim3(256), args,
                                       0, s));
    SEM_HIP(hipMemcpyAsync(c.hres, S.sc, sizeof(CoarseScalars), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    const CoarseScalars *h = reinterpret_cast<const CoarseScalars *>(c.hres);
    if (h->aborted) fail(SEM_EHIP, "coarse-grid solve: a grid barrier timed out");
    c.last_coarse_iters = tol > 0.0 ? h->iters : maxit;
    if (!(h->rr == h->rr)) fail(SEM_ENAN, "NaN in the coarse-grid solve");
    launch_gather(c, C, S.x, xl, s);
    return;
  }
  hipLaunchKernelGGL(k_cg_start, dim3(cg_grid(S)), dim3(256), 0, s, S.n, P,
                     tol > 0 ? tol * tol : 0.0, maxit);
  SEM_LAUNCH("k_cg_start");
  hipLaunchKernelGGL(k_cg_first, dim3(cg_grid(S)), dim3(256), 0, s, S.n, g, P);
  SEM_LAUNCH("k_cg_first");
  if (c.capturing) {
    // inside a recorded batch iteration: a fixed count, no readback
    const int k = tol > 0.0 ? std::min(maxit, c.capture_coarse_iters) : maxit;
    enqueue_iterations(c, k, 0, s);
    launch_gather(c, C, S.x, xl, s);
    return;
  }
  if (tol <= 0.0 || !S.use_graph) {
    // fixed iteration count (or graphs off): plain launches, one readback at most
    if (tol <= 0.0) {
      enqueue_iterations(c, maxit, 0, s);
    } else {
      int done_it = 0;
      int chunk = std::max(8, c.last_coarse_iters + 2);
      while (true) {
        int k = std::min(chunk, maxit - done_it);
        enqueue_iterations(c, k, done_it, s);
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
  launch_gather(c, C, S.x, xl, s);
}

// solve on the coarsest level for nv right sides: C.d_b (consistent, masked
// E-vectors, nloc apart) -> c.cx.  The exact solve takes all right sides in one
// pair of sweeps; the iterative one solves them in turn.
void coarse_solve_assembled(Ctx &c, Level &C, double tol, int maxit, hipStream_t s, int nv,
                            CoarseRhs u) {
  CoarseSolver &S = *c.cs;
  if (nv > c.nvmax) fail(SEM_EINVAL, "coarse solve: more right sides than were set up");
  if (S.direct) {  // exact: no iteration, no host interaction (also inside a recorded graph)
    CoarseGrid g = cgrid(c);
    launch_to_global(S, g, C.d_b, u, nv, s);
    coarse_direct_apply(S, g.nx, g.ny, g.nz, S.b, S.x, s, nv);
    if (!c.capturing) c.last_coarse_iters = 0;
    launch_gather(c, C, S.x, c.cx, s, nv, S.n);
    return;
  }
  for (int v = 0; v < nv; ++v) {
    CoarseRhs uv = u;
    if (u.p) uv.p = (const char *)u.p + (size_t)v * C.nloc * (u.f32 ? sizeof(float) : sizeof(double));
    coarse_solve_one(c, C, tol, maxit, s, C.d_b + v * C.nloc, c.cx + v * C.nloc, uv);
  }
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
