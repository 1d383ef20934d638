// GLL basis on the device (Sec. 2.1: degree-p Lagrange cardinal basis on the
// Gauss-Lobatto-Legendre points, GLL quadrature for the inner product).
//
//   nodes    xi_0 = -1, xi_p = 1, interior nodes = roots of P_p'
//   weights  w_j = 2 / (p (p+1) P_p(xi_j)^2)
//   D[i][j]  = h_j'(xi_i) = P_p(xi_i) / (P_p(xi_j)(xi_i - xi_j)) for i != j,
//              D[0][0] = -p(p+1)/4, D[p][p] = p(p+1)/4, otherwise 0
//   J[i][j]  = h^c_j(x_i) (coarse cardinal basis at the fine nodes)
#include "sem_internal.h"

namespace sem {

__device__ inline void legendre_pair(int p, double x, double &Pp, double &Pm1) {
  double a = 1.0, b = x;  // P_0, P_1
  if (p == 0) { Pp = 1.0; Pm1 = 0.0; return; }
  for (int k = 1; k < p; ++k) {
    double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  Pp = b;
  Pm1 = a;
}

__global__ void k_gll(int p, double *xi, double *w) {
  int t = threadIdx.x;
  if (t > p) return;
  double x;
  if (t == 0) {
    x = -1.0;
  } else if (t == p) {
    x = 1.0;
  } else {
    // Newton on f = P_p'(x); Legendre's equation gives
    // P_p'' = (2x P_p' - p(p+1) P_p) / (1 - x^2), and P_p' = p (x P_p - P_{p-1})/(x^2-1)
    x = -cos(M_PI * t / p);
    for (int it = 0; it < 100; ++it) {
      double P, Pm;
      legendre_pair(p, x, P, Pm);
      double dP = p * (x * P - Pm) / (x * x - 1.0);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double step = dP / d2P;
      x -= step;
      if (fabs(step) < 1e-16) break;
    }
  }
  double P, Pm;
  legendre_pair(p, x, P, Pm);
  xi[t] = x;
  if (w) w[t] = 2.0 / (p * (p + 1.0) * P * P);
}

__global__ void k_dmat(int p, const double *xi, double *D, float *D32) {
  int i = threadIdx.x, j = threadIdx.y;
  if (i > p || j > p) return;
  double v;
  if (i != j) {
    double Pi, Pj, t;
    legendre_pair(p, xi[i], Pi, t);
    legendre_pair(p, xi[j], Pj, t);
    v = Pi / (Pj * (xi[i] - xi[j]));
  } else if (i == 0) {
    v = -p * (p + 1.0) / 4.0;
  } else if (i == p) {
    v = p * (p + 1.0) / 4.0;
  } else {
    v = 0.0;
  }
  D[i * (p + 1) + j] = v;
  if (D32) D32[i * (p + 1) + j] = (float)v;
}

__global__ void k_interp(int pc, int pf, const double *xic, const double *xif, double *J,
                         float *J32) {
  int i = threadIdx.x, j = threadIdx.y;
  if (i > pf || j > pc) return;
  double x = xif[i], h = 1.0;
  for (int m = 0; m <= pc; ++m)
    if (m != j) h *= (x - xic[m]) / (xic[j] - xic[m]);
  J[i * (pc + 1) + j] = h;
  if (J32) J32[i * (pc + 1) + j] = (float)h;
}

void launch_gll(int p, double *xi, double *w, hipStream_t s) {
  hipLaunchKernelGGL(k_gll, dim3(1), dim3(64), 0, s, p, xi, w);
  SEM_LAUNCH("k_gll");
}

void launch_dmat(int p, const double *xi, double *D, float *D32, hipStream_t s) {
  hipLaunchKernelGGL(k_dmat, dim3(1), dim3(16, 16), 0, s, p, xi, D, D32);
  SEM_LAUNCH("k_dmat");
}

void launch_interp(int pc, int pf, const double *xic, const double *xif, double *J, float *J32,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_interp, dim3(1), dim3(16, 16), 0, s, pc, pf, xic, xif, J, J32);
  SEM_LAUNCH("k_interp");
}

}  // namespace sem
