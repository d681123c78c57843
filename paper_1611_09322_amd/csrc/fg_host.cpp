// Host-side FP64 pieces: the real-space scalar functions F, G of Appendix A,
// their small-r series and the FP32 interpolation table.
#include <cmath>
#include <vector>

#include "pse_internal.hpp"

namespace pse {

static const double kPi = 3.14159265358979323846;

// eq. (RPY_free_space) in the (I - rr, rr) basis, times 6 pi eta a
static void free_rpy(double r, double a, double *F, double *G) {
  if (r > 2.0 * a) {
    const double ci = 0.75 * a / r + 0.5 * a * a * a / (r * r * r);
    const double crr = 0.75 * a / r - 1.5 * a * a * a / (r * r * r);
    *F = ci;
    *G = ci + crr;
  } else {
    *F = 1.0 - 9.0 * r / (32.0 * a);
    *G = 1.0 - 3.0 * r / (16.0 * a);
  }
}

// Appendix A, Case 1 (r > 2a) and Case 2 (r <= 2a): F = sum f_i * basis_i.
static void fg_closed(double r, double x, double a, double *F, double *G) {
  const double sp = std::sqrt(kPi);
  const double r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
  const double x2 = x * x, x3 = x2 * x, x4 = x2 * x2;
  const double a2 = a * a;
  const double rm = r - 2.0 * a, rp = r + 2.0 * a;
  const double qp = 4.0 * a2 + 4.0 * a * r + 9.0 * r2;  // 4a^2 + 4ar + 9r^2
  const double qm = 4.0 * a2 - 4.0 * a * r + 9.0 * r2;  // 4a^2 - 4ar + 9r^2
  double f[7], g[7];
  f[1] = (18.0 * r2 * x2 + 3.0) / (64.0 * sp * a * r2 * x3);
  f[2] = (2.0 * x2 * (2.0 * a - r) * qp - 2.0 * a - 3.0 * r) / (128.0 * sp * a * r3 * x3);
  f[3] = (-2.0 * x2 * rp * qm + 2.0 * a - 3.0 * r) / (128.0 * sp * a * r3 * x3);
  f[4] = (3.0 - 36.0 * r4 * x4) / (128.0 * a * r3 * x4);
  f[5] = (4.0 * x4 * rm * rm * qp - 3.0) / (256.0 * a * r3 * x4);
  f[6] = (4.0 * x4 * rp * rp * qm - 3.0) / (256.0 * a * r3 * x4);
  g[1] = (6.0 * r2 * x2 - 3.0) / (32.0 * sp * a * r2 * x3);
  g[2] = (-2.0 * x2 * rm * rm * (2.0 * a + 3.0 * r) + 2.0 * a + 3.0 * r) / (64.0 * sp * a * r3 * x3);
  g[3] = (2.0 * x2 * rp * rp * (2.0 * a - 3.0 * r) - 2.0 * a + 3.0 * r) / (64.0 * sp * a * r3 * x3);
  g[4] = -(3.0 * (4.0 * r4 * x4 + 1.0)) / (64.0 * a * r3 * x4);
  g[5] = (3.0 - 4.0 * x4 * (2.0 * a - r) * (2.0 * a - r) * (2.0 * a - r) * (2.0 * a + 3.0 * r)) / (128.0 * a * r3 * x4);
  g[6] = (3.0 - 4.0 * x4 * (2.0 * a - 3.0 * r) * rp * rp * rp) / (128.0 * a * r3 * x4);
  if (r <= 2.0 * a) {
    f[0] = -rm * rm * qp / (32.0 * a * r3);
    g[0] = (2.0 * a - r) * (2.0 * a - r) * (2.0 * a - r) * (2.0 * a + 3.0 * r) / (16.0 * a * r3);
  } else {
    f[0] = g[0] = 0.0;
  }
  const double b[7] = {1.0,
                       std::exp(-r2 * x2),
                       std::exp(-rm * rm * x2),
                       std::exp(-rp * rp * x2),
                       std::erfc(r * x),
                       std::erfc(rm * x),
                       std::erfc(rp * x)};
  double sf = 0.0, sg = 0.0;
  for (int i = 0; i < 7; ++i) {
    sf += f[i] * b[i];
    sg += g[i] * b[i];
  }
  *F = sf;
  *G = sg;
}

double fg_self(double xi, double a) {
  const double sp = std::sqrt(kPi);
  return (1.0 - std::exp(-4.0 * a * a * xi * xi) + 4.0 * sp * a * xi * std::erfc(2.0 * a * xi)) / (4.0 * sp * xi * a);
}

static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Series of the H-weighted complement (the wave part of the pair function):
//   F_w(r) = (3a/pi) int H sinc^2(ka) K_F(kr) dk = sum_n serF[n] r^{2n}
//   G_w(r) = (6a/pi) int H sinc^2(ka) K_G(kr) dk = sum_n serG[n] r^{2n}
// from the Taylor series of the radial kernels of eqs. (int1)/(int2) and the
// moments I_n = int_0^inf H(k) sinc^2(ka) k^{2n} dk (composite Gauss-Legendre).
void fg_series_coeffs(double xi, double a, double *serF, double *serG) {
  // 16-point Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_16)
  const int q = 16;
  double t[q], w[q];
  for (int i = 0; i < q; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (q + 0.5)), pp = 0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= q; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = q * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) break;
    }
    t[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
  for (int n = 0; n < kSeriesTerms; ++n) {
    const double kmax = 2.0 * xi * (std::sqrt(2.0 * n + 2.0) + 8.0);
    const int npan = 400;
    double I = 0.0;
    for (int pnl = 0; pnl < npan; ++pnl) {
      const double lo = kmax * pnl / npan, hi = kmax * (pnl + 1) / npan;
      for (int i = 0; i < q; ++i) {
        const double k = 0.5 * (hi - lo) * t[i] + 0.5 * (hi + lo);
        const double qq = k * k / (4.0 * xi * xi);
        const double H = (1.0 + qq) * std::exp(-qq);
        const double ka = k * a;
        const double s = ka == 0.0 ? 1.0 : std::sin(ka) / ka;
        I += 0.5 * (hi - lo) * w[i] * H * s * s * std::pow(k, 2.0 * n);
      }
    }
    const int m = n + 1;  // kernel term u^{2m-2}
    const double sgn = (m % 2) ? -1.0 : 1.0;
    const double cF = sgn * (1.0 / fact(2 * m) - 1.0 / fact(2 * m + 1) - 1.0 / fact(2 * m - 1));
    const double cG = sgn * (1.0 / fact(2 * m + 1) - 1.0 / fact(2 * m));
    serF[n] = 3.0 * a / kPi * cF * I;
    serG[n] = 6.0 * a / kPi * cG * I;
  }
}

// Below this r the closed forms lose more than ~3 digits to cancellation
// (their terms grow like 1/(r^3 xi^4)); the series is used instead.
double fg_small_r_threshold(double xi, double a) { return std::cbrt(1e-3 * a * a * a / (xi * xi * xi * xi)); }

void fg_eval_host(double r, double xi, double a, const double *serF, const double *serG, double *F, double *G) {
  if (r < fg_small_r_threshold(xi, a)) {
    double Ff, Gf;
    free_rpy(r, a, &Ff, &Gf);
    const double r2 = r * r;
    double sf = 0.0, sg = 0.0;
    for (int n = kSeriesTerms - 1; n >= 0; --n) {
      sf = sf * r2 + serF[n];
      sg = sg * r2 + serG[n];
    }
    *F = Ff - sf;
    *G = Gf - sg;
  } else {
    fg_closed(r, xi, a, F, G);
  }
}

// FP32 table nodes r_k = k rc / K, k = 0 ... K + 1: (mu0 F, mu0 (G - F)),
// read two at a time for linear interpolation (the node past rc keeps the
// interpolation at r = rc inside the table).
void fg_build_table(double xi, double a, double rc, double mu0, const double *serF, const double *serG, float2 *tab) {
  for (int k = 0; k < kTableN; ++k) {
    const double r = rc * k / kTableK;
    double F, G;
    if (k == 0) {
      F = G = fg_self(xi, a);
    } else {
      fg_eval_host(r, xi, a, serF, serG, &F, &G);
    }
    tab[k] = make_float2((float)(F * mu0), (float)((G - F) * mu0));
  }
}

}  // namespace pse
