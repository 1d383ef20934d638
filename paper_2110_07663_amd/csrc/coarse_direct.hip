// Exact coarse-grid solve of the V-cycle (Algorithm 1, "solve" on the
// coarsest level) for the assembled p = 1 operator.
//
// With nodes numbered plane by plane along z, the 27-point operator is block
// tridiagonal: D_k couples the nodes of plane k among themselves, A_{k,k-1} and
// A_{k,k+1} couple it to the planes below and above.  Block elimination runs
// from both ends towards the middle plane c = K/2 (a "twisted" factorisation),
// so the solve has two independent chains of half the length:
//   below c:  T_0 = D_0,  H_k = A_{k,k-1} G_{k-1},  T_k = D_k - H_k A_{k-1,k};
//   above c:  T_{K-1} = D_{K-1},  H_k = A_{k,k+1} G_{k+1},  T_k = D_k - H_k A_{k+1,k};
//   at c:     T_c = D_c - Hd_c A_{c-1,c} - Hu_c A_{c+1,c}   (both updates);
//   G_k = T_k^{-1}, and J_k = H_{k+1}^T (below c) or H_{k-1}^T (above c).
// Solve: y_0 = b_0, y_{K-1} = b_{K-1}, y_k = b_k - H_k y_{k-+1} walking inwards,
// y_c = b_c - Hd_c y_{c-1} - Hu_c y_{c+1}, x_c = G_c y_c, then outwards
// x_k = G_k y_k - J_k x_{k+-1}.  One launch advances both chains.
// Each T_k is symmetric positive definite (a Schur complement of an SPD
// matrix), so it is inverted in place by blocked Gauss-Jordan elimination
// without pivoting (32x32 blocks: invert the pivot block, scale its block row,
// update the rest, scale its block column).  Dirichlet rows of the stencil are
// identity rows, so they need no special case.  A pivot below 1e-12 of its
// row's diagonal (a numerically singular level, e.g. all-Neumann) is reported
// and the caller keeps the CG.
//
// Storage: G, H, J as K dense [Mp][Mp] FP64 blocks, Mp = nx*ny rounded up to
// 32 (identity / zero padding); Hu_c sits in J's slot c.  A solve reads each
// block once: 3 K Mp^2 * 8 bytes, in about K dependent matrix-vector launches
// with no host interaction, so it can be recorded into a graph.  Under an FP32
// smoother the sweeps read FP32 copies of the factored blocks instead (half the
// bytes; vectors and sums stay FP64): the solve is then exact to about 1e-6,
// below what the FP32 V-cycle around it resolves.
#include <algorithm>

#include "sem_internal.h"

namespace sem {

constexpr int kGB = 32;  // Gauss-Jordan block

static inline int64_t padded(int64_t m) { return (m + kGB - 1) / kGB * kGB; }

size_t coarse_direct_bytes(int64_t nx, int64_t ny, int64_t nz, bool f32) {
  const int64_t Mp = padded(nx * ny);
  return (size_t)(3 * nz * Mp * Mp + nx * ny * nz) * sizeof(double) +
         (f32 ? (size_t)(3 * nz * Mp * Mp) * sizeof(float) : 0);
}

// ---- setup kernels ----------------------------------------------------------

// stencil entry of row t for the node offset (dx, dy, dz)
__device__ inline double st_at(const double *St, int64_t n, int64_t t, int dx, int dy, int dz) {
  return St[(int64_t)((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)) * n + t];
}

// H[i][l] = sum_a A_{k,k+dz}[i][a] G_{k+dz}[a][l], A_{k,k+dz}[i][a] = stencil of
// row (k, i) towards node (k + dz, a), dz = -1 or +1
__global__ void k_bt_H(int nx, int ny, int64_t n, int k, int Mp, const double *__restrict__ St,
                       const double *__restrict__ Gp, double *__restrict__ H, int dz) {
  const int m = nx * ny;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)Mp * Mp) return;
  const int i = (int)(e / Mp), l = (int)(e - (int64_t)i * Mp);
  double h = 0.0;
  if (i < m && l < m) {
    const int xi = i % nx, yi = i / nx;
    const int64_t row = (int64_t)k * m + i;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int xa = xi + dx, ya = yi + dy;
        if (xa < 0 || xa >= nx || ya < 0 || ya >= ny) continue;
        h += st_at(St, n, row, dx, dy, dz) * Gp[(int64_t)(ya * nx + xa) * Mp + l];
      }
  }
  H[e] = h;
}

// T[i][j] = D_k[i][j] - sum_l H1[i][l] A_{k,k+dz1}[j][l] - sum_l H2[i][l] A_{k,k+dz2}[j][l]
// (A_{k+dz,k} = A_{k,k+dz}^T; absent updates are null; padding: identity).  The
// diagonal is also kept in `diag` for the pivot test of the inversion.
__device__ inline double bt_update(int nx, int ny, int64_t n, int64_t rowj, int xj, int yj, int Mp,
                                   const double *__restrict__ St, const double *__restrict__ Hi,
                                   int dz) {
  double v = 0.0;
  for (int ey = -1; ey <= 1; ++ey)
    for (int ex = -1; ex <= 1; ++ex) {
      const int xl = xj + ex, yl = yj + ey;
      if (xl < 0 || xl >= nx || yl < 0 || yl >= ny) continue;
      v += Hi[yl * nx + xl] * st_at(St, n, rowj, ex, ey, dz);
    }
  return v;
}

__global__ void k_bt_T(int nx, int ny, int64_t n, int k, int Mp, const double *__restrict__ St,
                       const double *__restrict__ H1, int dz1, const double *__restrict__ H2,
                       int dz2, double *__restrict__ T, double *__restrict__ diag) {
  const int m = nx * ny;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)Mp * Mp) return;
  const int i = (int)(e / Mp), j = (int)(e - (int64_t)i * Mp);
  if (i >= m || j >= m) {
    T[e] = i == j ? 1.0 : 0.0;
    if (i == j) diag[i] = 1.0;
    return;
  }
  const int xi = i % nx, yi = i / nx, xj = j % nx, yj = j / nx;
  const int dx = xj - xi, dy = yj - yi;
  double v = 0.0;
  if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) v = st_at(St, n, (int64_t)k * m + i, dx, dy, 0);
  const int64_t rowj = (int64_t)k * m + j;
  if (H1) v -= bt_update(nx, ny, n, rowj, xj, yj, Mp, St, H1 + (int64_t)i * Mp, dz1);
  if (H2) v -= bt_update(nx, ny, n, rowj, xj, yj, Mp, St, H2 + (int64_t)i * Mp, dz2);
  T[e] = v;
  if (i == j) diag[i] = v;
}

// in-place inverse of the pivot block (Kb, Kb) in LDS.  For an SPD matrix
// every pivot lies in (0, original diagonal]; a pivot below 1e-12 of its row's
// original diagonal marks a (numerically) singular level.
__global__ __launch_bounds__(256) void k_gj_diag(double *A, int Mp, int Kb,
                                                 const double *__restrict__ diag, int *flag) {
  __shared__ double P[kGB][kGB + 1];
  const int tid = threadIdx.x;
  double *blk = A + (int64_t)Kb * kGB * Mp + (int64_t)Kb * kGB;
  for (int e = tid; e < kGB * kGB; e += 256) P[e / kGB][e % kGB] = blk[(int64_t)(e / kGB) * Mp + e % kGB];
  __syncthreads();
  for (int p = 0; p < kGB; ++p) {
    const double piv = P[p][p];
    const double d = 1.0 / piv;
    __syncthreads();
    if (tid < kGB && tid != p) P[p][tid] *= d;
    __syncthreads();
    for (int e = tid; e < kGB * kGB; e += 256) {
      const int i = e / kGB, j = e % kGB;
      if (i != p && j != p) P[i][j] -= P[i][p] * P[p][j];
    }
    __syncthreads();
    if (tid < kGB && tid != p) P[tid][p] = -P[tid][p] * d;
    if (tid == 0) {
      P[p][p] = d;
      if (!(piv > 1e-12 * diag[Kb * kGB + p])) atomicOr(flag, 1);
    }
    __syncthreads();
  }
  for (int e = tid; e < kGB * kGB; e += 256) blk[(int64_t)(e / kGB) * Mp + e % kGB] = P[e / kGB][e % kGB];
}

// block row: A[Kb][J] <- P A[Kb][J] for J != Kb (P = inverted pivot block)
__global__ __launch_bounds__(256) void k_gj_row(double *A, int Mp, int Kb) {
  __shared__ double P[kGB][kGB + 1], B[kGB][kGB + 1];
  const int tid = threadIdx.x;
  const int J = (int)blockIdx.x < Kb ? (int)blockIdx.x : (int)blockIdx.x + 1;
  const double *pb = A + (int64_t)Kb * kGB * Mp + (int64_t)Kb * kGB;
  double *tb = A + (int64_t)Kb * kGB * Mp + (int64_t)J * kGB;
  for (int e = tid; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    P[i][j] = pb[(int64_t)i * Mp + j];
    B[i][j] = tb[(int64_t)i * Mp + j];
  }
  __syncthreads();
  for (int e = tid; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGB; ++q) s += P[i][q] * B[q][j];
    tb[(int64_t)i * Mp + j] = s;
  }
}

// rest: A[I][J] -= A[I][Kb] A[Kb][J] for I, J != Kb (block row already scaled)
__global__ __launch_bounds__(256) void k_gj_trail(double *A, int Mp, int Kb, int nbk) {
  __shared__ double L[kGB][kGB + 1], R[kGB][kGB + 1];
  const int tid = threadIdx.x;
  const int ti = (int)blockIdx.x / (nbk - 1), tj = (int)blockIdx.x % (nbk - 1);
  const int I = ti < Kb ? ti : ti + 1, J = tj < Kb ? tj : tj + 1;
  const double *lb = A + (int64_t)I * kGB * Mp + (int64_t)Kb * kGB;
  const double *rb = A + (int64_t)Kb * kGB * Mp + (int64_t)J * kGB;
  double *ob = A + (int64_t)I * kGB * Mp + (int64_t)J * kGB;
  for (int e = tid; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    L[i][j] = lb[(int64_t)i * Mp + j];
    R[i][j] = rb[(int64_t)i * Mp + j];
  }
  __syncthreads();
  for (int e = tid; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGB; ++q) s += L[i][q] * R[q][j];
    ob[(int64_t)i * Mp + j] -= s;
  }
}

// block column: A[I][Kb] <- -A[I][Kb] P for I != Kb
__global__ __launch_bounds__(256) void k_gj_col(double *A, int Mp, int Kb) {
  __shared__ double P[kGB][kGB + 1], B[kGB][kGB + 1];
  const int tid = threadIdx.x;
  const int I = (int)blockIdx.x < Kb ? (int)blockIdx.x : (int)blockIdx.x + 1;
  const double *pb = A + (int64_t)Kb * kGB * Mp + (int64_t)Kb * kGB;
  double *tb = A + (int64_t)I * kGB * Mp + (int64_t)Kb * kGB;
  for (int e = tid; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    P[i][j] = pb[(int64_t)i * Mp + j];
    B[i][j] = tb[(int64_t)i * Mp + j];
  }
  __syncthreads();
  for (int e = tid; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGB; ++q) s += B[i][q] * P[q][j];
    tb[(int64_t)i * Mp + j] = -s;
  }
}

// J[i][a] = H[a][i]
__global__ void k_bt_transpose(int Mp, const double *__restrict__ H, double *__restrict__ J) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 256 threads: 8 rows per pass
  for (int r = ty; r < 32; r += 8) t[r][tx] = H[(int64_t)(by + r) * Mp + bx + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8) J[(int64_t)(bx + r) * Mp + by + tx] = t[tx][r];
}

// ---- solve kernel -------------------------------------------------------------

// One product of a sweep: out = c + s1 * (M1 v1) - (M2 v2) (absent terms null);
// MT is the type of the stored blocks
template <typename MT>
struct BtOp {
  const MT *M1;
  const double *v1;
  const MT *M2;
  const double *v2, *c;
  double *out;
  double s1;
};

__global__ void k_bt_narrow(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Up to two independent products (the two chains of the sweep) for NV right
// sides (vectors vs apart in v1, v2, c and out); one wavefront per row, the
// matrix rows are read once for all right sides.  Each right side is summed in
// the same order for any NV (four strided partial sums per lane, then the wave
// reduction).
template <int NV, typename MT>
__global__ __launch_bounds__(256) void k_bt_mv(int m, int Mp, BtOp<MT> o0, BtOp<MT> o1,
                                               int64_t vs) {
  constexpr int W = 16 / (int)sizeof(MT);  // entries per 16-byte load
  struct alignas(16) Chunk {
    MT e[W];
  };
  const int rb = (m + 3) / 4;
  const int which = (int)blockIdx.x >= rb;
  const BtOp<MT> &o = which ? o1 : o0;
  const int row = ((int)blockIdx.x - which * rb) * 4 + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;  // whole wave
  double a1[NV], a2[NV];
  // The matrix row (16-byte aligned: Mp is a multiple of 32) streams as 16-byte
  // loads of W entries, four per lane per step (256 W entries a wave), into four
  // partial sums per right side; x (L2 resident, any alignment) is read per
  // entry.  (Issuing a whole row's loads before the first use, with the last
  // chunk guarded entry by entry, measured slower.)
  auto rowdot = [&](const MT *__restrict__ r, const double *__restrict__ x, double *acc) {
    double t[NV][4];
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v][0] = t[v][1] = t[v][2] = t[v][3] = 0.0;
    const Chunk *__restrict__ rc = reinterpret_cast<const Chunk *>(r);
    int j0 = 0;
    for (; j0 + 256 * W <= m; j0 += 256 * W) {
      Chunk q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = rc[j0 / W + 64 * u + lane];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + 64 * W * u + W * lane;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double *xv = x + v * vs;
#pragma unroll
          for (int w = 0; w < W; ++w) t[v][u] += (double)q[u].e[w] * xv[j + w];
        }
      }
    }
    for (int j = j0 + lane; j < m; j += 64) {
      const double r0 = (double)r[j];
#pragma unroll
      for (int v = 0; v < NV; ++v) t[v][0] += r0 * x[v * vs + j];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = (t[v][0] + t[v][1]) + (t[v][2] + t[v][3]);
  };
  if (o.M1) {
    rowdot(o.M1 + (int64_t)row * Mp, o.v1, a1);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) a1[v] = 0.0;
  }
  if (o.M2) {
    rowdot(o.M2 + (int64_t)row * Mp, o.v2, a2);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) a2[v] = 0.0;
  }
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      a1[v] += __shfl_xor(a1[v], sh, 64);
      a2[v] += __shfl_xor(a2[v], sh, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      o.out[v * vs + row] = (o.c ? o.c[v * vs + row] : 0.0) + o.s1 * a1[v] - a2[v];
  }
}

// ---- host side -------------------------------------------------------------------

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

static void bt_invert(double *Gk, int Mp, int nbk, const double *diag, int *flag, hipStream_t s) {
  for (int b = 0; b < nbk; ++b) {
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, s, Gk, Mp, b, diag, flag);
    SEM_LAUNCH("k_gj_diag");
    if (nbk == 1) continue;
    hipLaunchKernelGGL(k_gj_row, dim3(nbk - 1), dim3(256), 0, s, Gk, Mp, b);
    SEM_LAUNCH("k_gj_row");
    hipLaunchKernelGGL(k_gj_trail, dim3((nbk - 1) * (nbk - 1)), dim3(256), 0, s, Gk, Mp, b, nbk);
    SEM_LAUNCH("k_gj_trail");
    hipLaunchKernelGGL(k_gj_col, dim3(nbk - 1), dim3(256), 0, s, Gk, Mp, b);
    SEM_LAUNCH("k_gj_col");
  }
}

void coarse_direct_setup(CoarseSolver &S, int64_t nx, int64_t ny, int64_t nz, hipStream_t s) {
  const int m = (int)(nx * ny), K = (int)nz, c = K / 2;
  const int Mp = (int)padded(m), nbk = Mp / kGB;
  const int64_t M2 = (int64_t)Mp * Mp;
  const unsigned g2 = nblk(M2);
  SEM_HIP(hipMemsetAsync(S.dflag, 0, sizeof(int), s));
  auto G = [&](int k) { return S.dG + k * M2; };
  auto H = [&](int k) { return S.dH + k * M2; };
  auto J = [&](int k) { return S.dJ + k * M2; };
  // chain from plane 0 up to c - 1
  for (int k = 0; k < c; ++k) {
    if (k > 0) {
      hipLaunchKernelGGL(k_bt_H, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, k, Mp, S.St,
                         (const double *)G(k - 1), H(k), -1);
      SEM_LAUNCH("k_bt_H");
    }
    hipLaunchKernelGGL(k_bt_T, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, k, Mp, S.St,
                       k > 0 ? (const double *)H(k) : nullptr, -1, (const double *)nullptr, 0,
                       G(k), S.dy);
    SEM_LAUNCH("k_bt_T");
    bt_invert(G(k), Mp, nbk, S.dy, S.dflag, s);
  }
  // chain from plane K - 1 down to c + 1
  for (int k = K - 1; k > c; --k) {
    if (k < K - 1) {
      hipLaunchKernelGGL(k_bt_H, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, k, Mp, S.St,
                         (const double *)G(k + 1), H(k), 1);
      SEM_LAUNCH("k_bt_H");
    }
    hipLaunchKernelGGL(k_bt_T, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, k, Mp, S.St,
                       k < K - 1 ? (const double *)H(k) : nullptr, 1, (const double *)nullptr, 0,
                       G(k), S.dy);
    SEM_LAUNCH("k_bt_T");
    bt_invert(G(k), Mp, nbk, S.dy, S.dflag, s);
  }
  // plane c takes both updates: from below in H's slot, from above in J's slot
  if (c > 0) {
    hipLaunchKernelGGL(k_bt_H, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, c, Mp, S.St,
                       (const double *)G(c - 1), H(c), -1);
    SEM_LAUNCH("k_bt_H");
  }
  if (c < K - 1) {
    hipLaunchKernelGGL(k_bt_H, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, c, Mp, S.St,
                       (const double *)G(c + 1), J(c), 1);
    SEM_LAUNCH("k_bt_H");
  }
  hipLaunchKernelGGL(k_bt_T, dim3(g2), dim3(256), 0, s, (int)nx, (int)ny, S.n, c, Mp, S.St,
                     c > 0 ? (const double *)H(c) : nullptr, -1,
                     c < K - 1 ? (const double *)J(c) : nullptr, 1, G(c), S.dy);
  SEM_LAUNCH("k_bt_T");
  bt_invert(G(c), Mp, nbk, S.dy, S.dflag, s);
  // back-substitution blocks: J_k = H_{k+1}^T below c, H_{k-1}^T above c (Hu_c for c + 1)
  for (int k = 0; k < K; ++k) {
    if (k == c) continue;
    const double *src = k < c ? H(k + 1) : (k - 1 == c ? J(c) : H(k - 1));
    hipLaunchKernelGGL(k_bt_transpose, dim3(nbk, nbk), dim3(256), 0, s, Mp, src, J(k));
    SEM_LAUNCH("k_bt_transpose");
  }
  if (S.fG) {
    const int64_t nb = (int64_t)K * M2;
    hipLaunchKernelGGL(k_bt_narrow, dim3(nblk(nb)), dim3(256), 0, s, nb, (const double *)S.dG,
                       S.fG);
    hipLaunchKernelGGL(k_bt_narrow, dim3(nblk(nb)), dim3(256), 0, s, nb, (const double *)S.dH,
                       S.fH);
    hipLaunchKernelGGL(k_bt_narrow, dim3(nblk(nb)), dim3(256), 0, s, nb, (const double *)S.dJ,
                       S.fJ);
    SEM_LAUNCH("k_bt_narrow");
  }
  int flag = 0;
  SEM_HIP(hipMemcpyAsync(&flag, S.dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  S.direct = flag == 0;
}

template <int NV, typename MT>
static void bt_sweeps(const CoarseSolver &S, const MT *dG, const MT *dH, const MT *dJ, int m,
                      int K, int Mp, const double *b, double *x, double *y, hipStream_t s) {
  using BtOp = sem::BtOp<MT>;
  const int64_t M2 = (int64_t)Mp * Mp, vs = S.n;
  const int c = K / 2;
  const unsigned rb = (unsigned)((m + 3) / 4);
  auto G = [&](int k) { return dG + k * M2; };
  auto H = [&](int k) { return dH + k * M2; };
  auto J = [&](int k) { return dJ + k * M2; };
  // y_k of the sweep; y_0 and y_{K-1} are b itself
  auto Y = [&](int k) -> const double * {
    return (k == 0 || k == K - 1) ? b + (int64_t)k * m : (const double *)(y + (int64_t)k * m);
  };
  auto launch = [&](const BtOp &o0, const BtOp *o1) {
    const BtOp none{};
    hipLaunchKernelGGL((k_bt_mv<NV, MT>), dim3(o1 ? 2 * rb : rb), dim3(256), 0, s, m, Mp, o0,
                       o1 ? *o1 : none, vs);
    SEM_LAUNCH("k_bt_mv");
  };
  // inwards: y_k = b_k - H_k y_{k-1} (k < c), y_k = b_k - H_k y_{k+1} (k > c)
  for (int t = 1;; ++t) {
    const int kd = t, ku = K - 1 - t;
    const bool dn = kd < c, up = ku > c;
    if (!dn && !up) break;
    BtOp od{H(kd), Y(kd - 1), nullptr, nullptr, b + (int64_t)kd * m, y + (int64_t)kd * m, -1.0};
    BtOp ou{H(ku), Y(ku + 1), nullptr, nullptr, b + (int64_t)ku * m, y + (int64_t)ku * m, -1.0};
    if (dn && up) launch(od, &ou);
    else launch(dn ? od : ou, nullptr);
  }
  // plane c: y_c = b_c - Hd_c y_{c-1} - Hu_c y_{c+1}; x_c = G_c y_c
  {
    BtOp oy{c > 0 ? H(c) : nullptr, c > 0 ? Y(c - 1) : nullptr, c < K - 1 ? J(c) : nullptr,
            c < K - 1 ? Y(c + 1) : nullptr, b + (int64_t)c * m, y + (int64_t)c * m, -1.0};
    launch(oy, nullptr);
    BtOp ox{G(c), y + (int64_t)c * m, nullptr, nullptr, nullptr, x + (int64_t)c * m, 1.0};
    launch(ox, nullptr);
  }
  // outwards: x_k = G_k y_k - J_k x_{k+1} (k < c), x_k = G_k y_k - J_k x_{k-1} (k > c)
  for (int t = 1;; ++t) {
    const int kd = c - t, ku = c + t;
    const bool dn = kd >= 0, up = ku < K;
    if (!dn && !up) break;
    BtOp od{G(kd), Y(kd), J(kd), x + (int64_t)(kd + 1) * m, nullptr, x + (int64_t)kd * m, 1.0};
    BtOp ou{G(ku), Y(ku), J(ku), x + (int64_t)(ku - 1) * m, nullptr, x + (int64_t)ku * m, 1.0};
    if (dn && up) launch(od, &ou);
    else launch(dn ? od : ou, nullptr);
  }
}

template <typename MT>
static void bt_apply(const CoarseSolver &S, const MT *G, const MT *H, const MT *J, int m, int K,
                     int Mp, const double *b, double *x, hipStream_t s, int nv) {
  for (int v0 = 0; v0 < nv; v0 += 4) {  // up to four right sides per sweep
    const int64_t o = (int64_t)v0 * S.n;
    switch (std::min(4, nv - v0)) {
      case 1: bt_sweeps<1, MT>(S, G, H, J, m, K, Mp, b + o, x + o, S.dy + o, s); break;
      case 2: bt_sweeps<2, MT>(S, G, H, J, m, K, Mp, b + o, x + o, S.dy + o, s); break;
      case 3: bt_sweeps<3, MT>(S, G, H, J, m, K, Mp, b + o, x + o, S.dy + o, s); break;
      default: bt_sweeps<4, MT>(S, G, H, J, m, K, Mp, b + o, x + o, S.dy + o, s); break;
    }
  }
}

void coarse_direct_apply(const CoarseSolver &S, int64_t nx, int64_t ny, int64_t nz, const double *b,
                         double *x, hipStream_t s, int nv) {
  const int m = (int)(nx * ny), K = (int)nz;
  const int Mp = (int)padded(m);
  if (S.fG)
    bt_apply<float>(S, S.fG, S.fH, S.fJ, m, K, Mp, b, x, s, nv);
  else
    bt_apply<double>(S, S.dG, S.dH, S.dJ, m, K, Mp, b, x, s, nv);
}

}  // namespace sem
