// Geometry of the isoparametric elements (Sec. 2.1).
//
// x^e(r,s,t) = sum x_ijk h_i(r) h_j(s) h_k(t).  At every GLL point q of a level:
//   Jm[a][b] = dx_a/dr_b (1D derivative-matrix contractions of the coordinates),
//   G_q      = w_q det(Jm) Jm^{-1} Jm^{-T}   (6 unique entries: rr rs rt ss st tt),
//   B_L(q)   = w_q det(Jm)                   (diagonal GLL mass).
#include "sem_internal.h"

namespace sem {

// X[a][e][k][j][i] = sum_{c,b,a'} Jg[k][c] Jg[j][b] Jg[i][a'] xyz[e][(c*Ng+b)*Ng+a'][a]
__global__ void k_level_coords(int64_t E, int N, int Ng, const double *__restrict__ xyz,
                               const double *__restrict__ Jg, double *__restrict__ X) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int N3 = N * N * N;
  int64_t nloc = E * N3;
  if (t >= nloc) return;
  int64_t e = t / N3;
  int q = (int)(t - e * N3);
  int i = q % N, j = (q / N) % N, k = q / (N * N);
  int Ng3 = Ng * Ng * Ng;
  const double *xe = xyz + e * Ng3 * 3;
  double acc[3] = {0, 0, 0};
  for (int c = 0; c < Ng; ++c) {
    double jk = Jg[k * Ng + c];
    for (int b = 0; b < Ng; ++b) {
      double jkb = jk * Jg[j * Ng + b];
      for (int a = 0; a < Ng; ++a) {
        double f = jkb * Jg[i * Ng + a];
        const double *pt = xe + ((c * Ng + b) * Ng + a) * 3;
        acc[0] += f * pt[0];
        acc[1] += f * pt[1];
        acc[2] += f * pt[2];
      }
    }
  }
  X[t] = acc[0];
  X[nloc + t] = acc[1];
  X[2 * nloc + t] = acc[2];
}

__global__ void k_geom(int64_t E, int N, const double *__restrict__ X, const double *__restrict__ D,
                       const double *__restrict__ wq, double *__restrict__ G, float *__restrict__ G32,
                       double *__restrict__ BL, int *bad) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int N3 = N * N * N;
  int64_t nloc = E * N3;
  if (t >= nloc) return;
  int64_t e = t / N3;
  int q = (int)(t - e * N3);
  int i = q % N, j = (q / N) % N, k = q / (N * N);
  const int64_t base = e * N3;
  double Jm[3][3];
  for (int a = 0; a < 3; ++a) {
    const double *xa = X + a * nloc + base;
    double xr = 0, xs = 0, xt = 0;
    for (int l = 0; l < N; ++l) {
      xr += D[i * N + l] * xa[(k * N + j) * N + l];
      xs += D[j * N + l] * xa[(k * N + l) * N + i];
      xt += D[k * N + l] * xa[(l * N + j) * N + i];
    }
    Jm[a][0] = xr;
    Jm[a][1] = xs;
    Jm[a][2] = xt;
  }
  // cofactor form of the inverse: Jinv[b][a] = cof[a][b] / det
  double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
  double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
  double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
  double c10 = Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2];
  double c11 = Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0];
  double c12 = Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1];
  double c20 = Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1];
  double c21 = Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2];
  double c22 = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
  double det = Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
  if (!(det > 0.0)) atomicOr(bad, 1);
  // inv[b][a] = d r_b / d x_a = cof[a][b] / det
  double inv[3][3] = {{c00 / det, c10 / det, c20 / det},
                      {c01 / det, c11 / det, c21 / det},
                      {c02 / det, c12 / det, c22 / det}};
  double w = wq[i] * wq[j] * wq[k];
  double sc = w * det;
  const int pairs[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  double *Ge = G + e * 6 * N3 + q;
  for (int c = 0; c < 6; ++c) {
    int a = pairs[c][0], b = pairs[c][1];
    double m = inv[a][0] * inv[b][0] + inv[a][1] * inv[b][1] + inv[a][2] * inv[b][2];
    double g = sc * m;
    Ge[c * N3] = g;
    if (G32) G32[e * 6 * N3 + c * N3 + q] = (float)g;
  }
  if (BL) BL[t] = sc;
}

// box length per direction: mean of the 4 corner-to-corner edges along r, s, t
__global__ void k_boxlen(int64_t E, int N, const double *__restrict__ X, double *__restrict__ Lb) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  int N3 = N * N * N;
  int64_t nloc = E * N3;
  int p = N - 1;
  auto P = [&](int i, int j, int k, double *v) {
    int64_t t = e * N3 + (k * N + j) * N + i;
    v[0] = X[t];
    v[1] = X[nloc + t];
    v[2] = X[2 * nloc + t];
  };
  double sum[3] = {0, 0, 0};
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      double a[3], b[3];
      // r edges: (0,j,k)-(p,j,k), j,k in {0,p}
      P(0, u * p, v * p, a);
      P(p, u * p, v * p, b);
      sum[0] += sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                     (b[2] - a[2]) * (b[2] - a[2]));
      P(u * p, 0, v * p, a);
      P(u * p, p, v * p, b);
      sum[1] += sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                     (b[2] - a[2]) * (b[2] - a[2]));
      P(u * p, v * p, 0, a);
      P(u * p, v * p, p, b);
      sum[2] += sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                     (b[2] - a[2]) * (b[2] - a[2]));
    }
  for (int d = 0; d < 3; ++d) Lb[e * 3 + d] = sum[d] / 4.0;
}

__global__ void k_mul(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = a[t] * b[t];
}

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_level_coords(const Ctx &c, const double *xyz_in, int p_geom, const double *Jg,
                         Level &L, hipStream_t s) {
  (void)c;
  hipLaunchKernelGGL(k_level_coords, dim3(nblocks(L.nloc, 256)), dim3(256), 0, s, L.E, L.N,
                     p_geom + 1, xyz_in, Jg, L.X);
  SEM_LAUNCH("k_level_coords");
}

void launch_geom(const Ctx &c, Level &L, int *bad, hipStream_t s) {
  (void)c;
  hipLaunchKernelGGL(k_geom, dim3(nblocks(L.nloc, 256)), dim3(256), 0, s, L.E, L.N, L.X, L.D64,
                     L.wq, L.G64, L.G32, L.BL, bad);
  SEM_LAUNCH("k_geom");
}

// FP16 storage of an element's factors for the FP32 smoother's A: one
// wavefront per element takes the largest |G| of the element's six factors,
// scales them all by 2^s so that it falls in [2^13, 2^14) (FP16's largest
// finite value is 65504), and stores pairs (G0,G1), (G2,G3), (G4,G5) rounded
// to nearest; gscale[e] = 2^-s.  A power of two commutes with FP32 rounding, so
// scaling the product instead of every factor gives the same result.
__global__ __launch_bounds__(256) void k_geom16(int64_t E, int N3, const double *__restrict__ G,
                                                uint32_t *__restrict__ G16,
                                                float *__restrict__ gscale) {
  const int lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= E) return;  // whole wave
  const double *Ge = G + e * 6 * N3;
  double mx = 0.0;
  for (int q = lane; q < 6 * N3; q += 64) mx = fmax(mx, fabs(Ge[q]));
  for (int sh = 32; sh > 0; sh >>= 1) mx = fmax(mx, __shfl_xor(mx, sh, 64));
  int ex = 0;
  if (mx > 0.0) frexp(mx, &ex);  // mx < 2^ex
  const int sh = 14 - ex;
  if (lane == 0) gscale[e] = (float)ldexp(1.0, -sh);
  for (int q = lane; q < N3; q += 64)
    for (int c = 0; c < 3; ++c) {
      const _Float16 a = (_Float16)ldexp(Ge[(2 * c) * N3 + q], sh);
      const _Float16 b = (_Float16)ldexp(Ge[(2 * c + 1) * N3 + q], sh);
      G16[(e * 3 + c) * N3 + q] = (uint32_t)__builtin_bit_cast(uint16_t, a) |
                                  ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
}

void launch_geom16(Level &L, hipStream_t s) {
  if (!L.G16) return;
  hipLaunchKernelGGL(k_geom16, dim3(nblocks(L.E, 4)), dim3(256), 0, s, L.E, L.N * L.N * L.N,
                     (const double *)L.G64, L.G16, L.gscale);
  SEM_LAUNCH("k_geom16");
}

void launch_boxlen(const Ctx &c, Level &L, hipStream_t s) {
  (void)c;
  hipLaunchKernelGGL(k_boxlen, dim3(nblocks(L.E, 256)), dim3(256), 0, s, L.E, L.N, L.X, L.boxlen);
  SEM_LAUNCH("k_boxlen");
}

void launch_rhs(const Level &L, const double *f, double *b, hipStream_t s) {
  hipLaunchKernelGGL(k_mul, dim3(nblocks(L.nloc, 256)), dim3(256), 0, s, L.nloc, L.BL, f, b);
  SEM_LAUNCH("k_mul");
}

}  // namespace sem
