// Eigenvalues of the small Arnoldi Hessenberg matrix (Sec. 2.2.3: lambda~ from
// a few Arnoldi steps on S A).  S A is not symmetric for Schwarz smoothers, so
// Ritz values can be complex: this is the shifted QR algorithm on a complex
// upper Hessenberg matrix (Givens rotations, Wilkinson shifts, deflation at the
// bottom).  k <= 16, host code.
#include <cmath>
#include <complex>
#include <vector>

#include "sem_internal.h"

namespace sem {

using cd = std::complex<double>;

double hessenberg_max_abs_eig(const double *H, int ldh, int k) {
  if (k <= 0) return 0.0;
  std::vector<cd> A(k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) A[i * k + j] = (i <= j + 1) ? cd(H[i * ldh + j], 0.0) : cd(0.0);
  auto at = [&](int i, int j) -> cd & { return A[i * k + j]; };
  double best = 0.0;
  int n = k;
  int iter = 0;
  std::vector<cd> gc(k), gs(k);
  while (n > 1) {
    double sub = std::abs(at(n - 1, n - 2));
    double scale = std::abs(at(n - 1, n - 1)) + std::abs(at(n - 2, n - 2));
    if (sub <= 1e-15 * (scale > 0 ? scale : 1.0) || iter > 200) {
      best = std::max(best, std::abs(at(n - 1, n - 1)));
      --n;
      iter = 0;
      continue;
    }
    ++iter;
    // Wilkinson shift: eigenvalue of the trailing 2x2 closer to the last entry
    cd a = at(n - 2, n - 2), b = at(n - 2, n - 1), c = at(n - 1, n - 2), d = at(n - 1, n - 1);
    cd tr = a + d, det = a * d - b * c;
    cd disc = std::sqrt(tr * tr - 4.0 * det);
    cd l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
    cd mu = (std::abs(l1 - d) < std::abs(l2 - d)) ? l1 : l2;
    if (iter % 11 == 10) mu += cd(0.75 * sub, 0.0);  // exceptional shift
    for (int i = 0; i < n; ++i) at(i, i) -= mu;
    // QR by Givens: rotate rows j, j+1 to zero the subdiagonal
    for (int j = 0; j < n - 1; ++j) {
      cd x = at(j, j), y = at(j + 1, j);
      double r = std::sqrt(std::norm(x) + std::norm(y));
      cd cc = r > 0 ? x / r : cd(1.0), ss = r > 0 ? y / r : cd(0.0);
      gc[j] = cc;
      gs[j] = ss;
      for (int col = j; col < n; ++col) {
        cd u = at(j, col), v = at(j + 1, col);
        at(j, col) = std::conj(cc) * u + std::conj(ss) * v;
        at(j + 1, col) = -ss * u + cc * v;
      }
    }
    // R Q: apply the adjoint rotations on the right
    for (int j = 0; j < n - 1; ++j) {
      cd cc = gc[j], ss = gs[j];
      int top = std::min(j + 2, n - 1);
      for (int row = 0; row <= top; ++row) {
        cd u = at(row, j), v = at(row, j + 1);
        at(row, j) = u * cc + v * ss;
        at(row, j + 1) = -u * std::conj(ss) + v * std::conj(cc);
      }
    }
    for (int i = 0; i < n; ++i) at(i, i) += mu;
  }
  best = std::max(best, std::abs(at(0, 0)));
  return best;
}

}  // namespace sem
