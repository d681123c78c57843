// Host FP64 tridiagonal square root for the full-mobility Krylov sample
// (Sec. II B.1 applies the same Lanczos process to M_r; Sec. III compares
// with it on the whole mobility, where the basis grows past what one
// wavefront's registers hold).
#include <cmath>
#include <vector>

#include "pse_internal.hpp"

namespace pse {

// s = T^{1/2} e_1 for the m x m symmetric tridiagonal T with diagonal d and
// off-diagonal e (e[i] couples i and i + 1), through its eigendecomposition
// T = Q diag(lambda) Q^T by implicit QL with shifts (Q accumulated; negative
// eigenvalues from rounding are taken as 0).  false if an eigenvalue does
// not converge in 60 sweeps.
bool tridiag_sqrt_e1_host(int m, const double *dd, const double *ee, double *s) {
  std::vector<double> d(dd, dd + m), e(m, 0.0), Q((size_t)m * m, 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = ee[i];
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;  // Q[row k][col j] at k m + j
  const double eps = 2.2e-16;
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    while (true) {
      int mm = l;
      for (; mm < m - 1; ++mm) {
        const double sc = std::fabs(d[mm]) + std::fabs(d[mm + 1]);
        if (std::fabs(e[mm]) <= eps * sc) break;
      }
      if (mm == l) break;
      if (++iter > 60) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + std::copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool deflated = false;
      for (int i = mm - 1; i >= l; --i) {
        const double f = sn * e[i], b = cs * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
          deflated = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * sn + 2.0 * cs * b;
        p = sn * r;
        d[i + 1] = g + p;
        g = cs * r - b;
        for (int k = 0; k < m; ++k) {
          double *row = &Q[(size_t)k * m];
          const double q1 = row[i + 1], q0 = row[i];
          row[i + 1] = sn * q0 + cs * q1;
          row[i] = cs * q0 - sn * q1;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  for (int k = 0; k < m; ++k) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += Q[(size_t)k * m + j] * std::sqrt(d[j] > 0.0 ? d[j] : 0.0) * Q[j];
    s[k] = acc;
  }
  return true;
}

}  // namespace pse
