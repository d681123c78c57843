// Training targets of the learned block preconditioner (host, FP64).
//
// For particle i: M_patch is M_r (eq. Mreal, Appendix A, self term eq. self)
// restricted to i and the particles within `radius` of it (minimum image);
// the target is the symmetric square root of the ii block of M_patch^{-1},
// times (mu0 F_self)^{1/2} so that an isolated particle has target I.  The
// ii block comes from a Cholesky solve with the three unit columns of i.
// Off the sampling path: used only to build training sets.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "pse_internal.hpp"

namespace pse {

namespace {

// Symmetric 3x3 square root by cyclic Jacobi rotations.
void sqrtm3(const double S[9], double R[9]) {
  double A[9], V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int k = 0; k < 9; ++k) A[k] = S[k];
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    if (off < 1e-30 * (A[0] * A[0] + A[4] * A[4] + A[8] * A[8])) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        const double apq = A[3 * p + q];
        if (apq == 0.0) continue;
        const double th = 0.5 * (A[3 * q + q] - A[3 * p + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A G
          const double akp = A[3 * k + p], akq = A[3 * k + q];
          A[3 * k + p] = c * akp - s * akq;
          A[3 * k + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- G^T A
          const double apk = A[3 * p + k], aqk = A[3 * q + k];
          A[3 * p + k] = c * apk - s * aqk;
          A[3 * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {  // V <- V G
          const double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - s * vkq;
          V[3 * k + q] = s * vkp + c * vkq;
        }
      }
  }
  const double l[3] = {std::sqrt(std::max(A[0], 0.0)), std::sqrt(std::max(A[4], 0.0)), std::sqrt(std::max(A[8], 0.0))};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[3 * r + c] = V[3 * r] * l[0] * V[3 * c] + V[3 * r + 1] * l[1] * V[3 * c + 1] +
                                             V[3 * r + 2] * l[2] * V[3 * c + 2];
}

struct Ctx {
  const double *x;
  int n;
  double L, a, xi, rc, mu0, fself, radius;
  const double *serF, *serG;
};

inline void min_image3(const double *xi, const double *xj, double L, double d[3]) {
  for (int k = 0; k < 3; ++k) {
    double v = xi[k] - xj[k];
    v -= L * std::nearbyint(v / L);
    d[k] = v;
  }
}

bool target_one(const Ctx &c, int i, double out[9]) {
  std::vector<int> patch{i};
  for (int j = 0; j < c.n; ++j) {
    if (j == i) continue;
    double d[3];
    min_image3(c.x + 3 * i, c.x + 3 * j, c.L, d);
    if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= c.radius * c.radius) patch.push_back(j);
  }
  const int p = (int)patch.size(), N = 3 * p;
  std::vector<double> M((size_t)N * N, 0.0);
  for (int u = 0; u < p; ++u) {
    for (int k = 0; k < 3; ++k) M[(size_t)(3 * u + k) * N + 3 * u + k] = c.mu0 * c.fself;
    for (int v = u + 1; v < p; ++v) {
      double d[3];
      min_image3(c.x + 3 * patch[u], c.x + 3 * patch[v], c.L, d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 > c.rc * c.rc) continue;
      double F = c.fself, G = c.fself, h[3] = {0, 0, 0};
      if (r2 > 0) {
        const double r = std::sqrt(r2);
        fg_eval_host(r, c.xi, c.a, c.serF, c.serG, &F, &G);
        for (int k = 0; k < 3; ++k) h[k] = d[k] / r;
      }
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          const double b = c.mu0 * ((k == l ? F : 0.0) + (G - F) * h[k] * h[l]);
          M[(size_t)(3 * u + k) * N + 3 * v + l] = b;
          M[(size_t)(3 * v + l) * N + 3 * u + k] = b;
        }
    }
  }
  // Cholesky M = C C^T (lower, in place)
  for (int j = 0; j < N; ++j) {
    double s = M[(size_t)j * N + j];
    for (int k = 0; k < j; ++k) s -= M[(size_t)j * N + k] * M[(size_t)j * N + k];
    if (!(s > 0)) return false;
    const double cj = std::sqrt(s);
    M[(size_t)j * N + j] = cj;
    for (int r = j + 1; r < N; ++r) {
      double t = M[(size_t)r * N + j];
      for (int k = 0; k < j; ++k) t -= M[(size_t)r * N + k] * M[(size_t)j * N + k];
      M[(size_t)r * N + j] = t / cj;
    }
  }
  // X = M^{-1} [e_0 e_1 e_2]; only rows 0..2 are needed
  double blk[9];
  std::vector<double> y(N);
  for (int col = 0; col < 3; ++col) {
    for (int r = 0; r < N; ++r) {  // C y = e_col
      double t = r == col ? 1.0 : 0.0;
      for (int k = 0; k < r; ++k) t -= M[(size_t)r * N + k] * y[k];
      y[r] = t / M[(size_t)r * N + r];
    }
    for (int r = N - 1; r >= 0; --r) {  // C^T x = y
      double t = y[r];
      for (int k = r + 1; k < N; ++k) t -= M[(size_t)k * N + r] * y[k];
      y[r] = t / M[(size_t)r * N + r];
    }
    for (int r = 0; r < 3; ++r) blk[3 * r + col] = y[r];
  }
  for (int r = 0; r < 3; ++r)
    for (int k = r + 1; k < 3; ++k) blk[3 * r + k] = blk[3 * k + r] = 0.5 * (blk[3 * r + k] + blk[3 * k + r]);
  double R[9];
  sqrtm3(blk, R);
  const double s = std::sqrt(c.mu0 * c.fself);
  for (int k = 0; k < 9; ++k) out[k] = R[k] * s;
  return true;
}

}  // namespace

bool precond_targets(const double *x, int n, double L, double a, double xi, double rc, double mu0,
                     const double *serF, const double *serG, const int *idx, int m, double radius, double *out) {
  Ctx c{x, n, L, a, xi, rc, mu0, fg_self(xi, a), radius, serF, serG};
  const int nt = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), 32));
  std::vector<int> ok(m, 1);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int q = t; q < m; q += nt) ok[q] = target_one(c, idx[q], out + 9 * (size_t)q) ? 1 : 0;
    });
  for (auto &w : th) w.join();
  return std::all_of(ok.begin(), ok.end(), [](int v) { return v != 0; });
}

}  // namespace pse
