// Host-side FP64 error model and parameter choice (Sec. II C-D).
//
// Four error sources are controlled separately (Sec. II C): the real-space
// truncation, whose decay is eps_R = exp(-xi^2 rc^2) and whose size is set
// by the pairs just past rc (a shell integral, below), the wave-space
// truncation at k_cut = pi / h (bound of Sec. II D), the spectral-Ewald
// quadrature exp(-pi^2 P^2 / 2m^2) + erfc(m / sqrt 2), and the aliasing of
// the Gaussian window by the grid (an estimate over the grid's k-set,
// below).  The parameter choice minimises the work model of eq. (work) over
// xi with every source within its share of the tolerance.
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "pse_internal.hpp"

namespace pse {

static const double kPi = 3.14159265358979323846;

// Sec. II D, last display: bound on the relative self-mobility error of
// truncating the wave sum at kc (PSE kernel, sinc^2 bounded by (ka)^-2).
double eps_wave_bound(double kc, double xi, double a) {
  return (4.0 / kc * std::exp(-kc * kc / (4 * xi * xi)) - std::sqrt(kPi) / xi * std::erfc(kc / (2 * xi))) /
         (2 * kPi * a);
}

// Sec. II C: quadrature error of the Gaussian window truncated at m standard
// deviations over P nodes.
double eps_quad_bound(int P, double m) {
  return std::exp(-kPi * kPi * P * P / (2 * m * m)) + std::erfc(m / std::sqrt(2.0));
}

// Relative error of one spreading or interpolation with the truncated
// Gaussian window.  The window is separable, so the per-axis truncation of
// eps_quad (the mass beyond m standard deviations) is lost on each of the
// three axes; the grid aliasing is the estimate over the k-set (its k -> 0
// limit is the first term of eps_quad, counted again here as a margin).
double window_error(double eps_quad, double eps_alias) { return 3.0 * eps_quad + eps_alias; }

// Real-space tail beyond rc (eq. Mreal truncated at rc), for spheres at
// number density rho without structure beyond rc, relative to the Stokes
// mobility (F, G of Appendix A are dimensionless):
//   incoherent  sqrt(rho int_rc^inf 4 pi r^2 (2 F^2 + G^2) / 3 dr)
//               (random forces or noise: the pairs past rc add in variance)
//   coherent    rho int_rc^inf 4 pi r^2 |2 F + G| / 3 dr
//               (aligned forces, e.g. sedimentation: they add in amplitude)
// The paper's exp(-xi^2 rc^2) gives the decay; the shell of pairs just past
// rc (4 pi r^2 rho of them) sets the constant in front.  Simpson's rule on
// [rc, rc + 12 / xi].
void real_tail(double rc, double xi, double a, double rho, double *inc, double *coh) {
  const double zero[kSeriesTerms] = {};  // the series serves r < 0.3a only
  const int nq = 400;  // even: Simpson's rule
  const double hi = rc + 12.0 / xi, dr = (hi - rc) / nq;
  double s2 = 0.0, s1 = 0.0;
  for (int q = 0; q <= nq; ++q) {
    const double r = rc + q * dr;
    double F, G;
    fg_eval_host(r, xi, a, zero, zero, &F, &G);
    const double w = (q == 0 || q == nq) ? 1.0 : (q % 2 ? 4.0 : 2.0);
    s2 += w * 4.0 * kPi * r * r * (2.0 * F * F + G * G) / 3.0;
    s1 += w * 4.0 * kPi * r * r * std::fabs(2.0 * F + G) / 3.0;
  }
  *inc = std::sqrt(rho * s2 * dr / 3.0);
  *coh = rho * s1 * dr / 3.0;
}

// Smallest rc (at least 2a) whose tail estimate is at most tol (bisection;
// the tail shrinks as rc grows); +inf when even rc_max does not reach it.
double rcut_for(double tol, double xi, double a, double rho, bool coherent, double rc_max) {
  auto tail = [&](double rc) {
    double i, c;
    real_tail(rc, xi, a, rho, &i, &c);
    return coherent ? c : i;
  };
  // no cutoff below contact (2a): the pairs of hard spheres start there
  double lo = 2.0 * a, hi = rc_max;
  if (!(lo < hi) || tail(hi) > tol) return INFINITY;
  if (tail(lo) <= tol) return lo;
  for (int it = 0; it < 40 && hi - lo > 1e-9 * rc_max; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (tail(mid) > tol) lo = mid;
    else hi = mid;
  }
  return hi;
}

// rcut_for to about 1e-4 of rc, for scanning many xi: the tail integral
// accumulated once from the top of [2a, rc_max + 12 / xi] on a step of
// 0.02 / xi (trapezoid), its crossing of tol interpolated.
double rcut_scan(double tol, double xi, double a, double rho, bool coherent, double rc_max) {
  const double zero[kSeriesTerms] = {};
  const double lo = 2.0 * a;
  if (!(lo < rc_max)) return INFINITY;
  const double dr = 0.02 / xi, top = rc_max + 12.0 / xi;
  const int n = (int)std::ceil((top - lo) / dr) + 1;
  std::vector<double> g(n), C(n);
  for (int i = 0; i < n; ++i) {
    const double r = lo + i * dr;
    double F, G;
    fg_eval_host(r, xi, a, zero, zero, &F, &G);
    g[i] = 4.0 * kPi * r * r * (coherent ? std::fabs(2.0 * F + G) : 2.0 * F * F + G * G) / 3.0;
  }
  C[n - 1] = 0.0;
  for (int i = n - 2; i >= 0; --i) C[i] = C[i + 1] + 0.5 * dr * (g[i] + g[i + 1]);
  auto tail = [&](int i) { return coherent ? rho * C[i] : std::sqrt(rho * C[i]); };
  const int imax = (int)std::floor((rc_max - lo) / dr);
  if (tail(imax) > tol) return INFINITY;
  if (tail(0) <= tol) return lo;
  int i = 1;
  while (tail(i) > tol) ++i;  // tail decreases with r; tail(imax) <= tol ends the scan
  const double t0 = std::log(tail(i - 1)), t1 = std::log(std::max(tail(i), 1e-300)), lt = std::log(tol);
  return lo + (i - 1 + (t0 - lt) / (t0 - t1)) * dr;
}

// Smallest kc with eps_wave_bound(kc) <= tol (the bound decreases with kc).
double kcut_for(double tol, double xi, double a) {
  double lo = 1e-6 * xi, hi = 2.0 * xi;
  while (eps_wave_bound(hi, xi, a) > tol && hi < 1e6 * xi) hi *= 2.0;
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (eps_wave_bound(mid, xi, a) > tol) lo = mid;
    else hi = mid;
  }
  return hi;
}

// Aliasing estimate of the spectral-Ewald wave sample.  Interpolating the
// grid field with the Gaussian window (standard deviation sigma, grid
// spacing h) returns each grid mode k together with its images
// k + 2 pi n / h, weighted by ghat(k + 2 pi n / h) / ghat(k) after the
// deconvolution; with independent k-space noise the relative variance of
// that error is
//   sum_k B(k) sum_{n != 0} rho(k, n)^2 / sum_k B(k),
//   rho(k, n)^2 = prod_d exp(-sigma^2 ((k_d + 2 pi n_d / h)^2 - k_d^2)),
// over the grid k-set (k = 0 and Nyquist indices excluded), first alias
// shell n in {-1, 0, 1}^3.  The shell sum factorises over the axes,
// prod_d (1 + rho_d(-1)^2 + rho_d(+1)^2) - 1.  Summed over one octant with
// sign multiplicities; above 96 frequencies per axis the octant is sampled
// at the midpoints of blocks of s consecutive indices (s = ceil(M / 96)),
// each weighted by its index count.  Returns the relative error (the square
// root).
AliasWeights::AliasWeights(double L_, int M_, double xi, double a, int max_freq) : L(L_), M(M_) {
  const int H = M / 2;  // signed indices 0 .. H - 1 per axis (Nyquist excluded)
  const int s = std::max(1, (M + max_freq - 1) / max_freq);
  nq = (H + s - 1) / s;
  k.resize(nq);
  std::vector<double> wt(nq);
  const double dk = 2.0 * kPi / L;
  for (int q = 0; q < nq; ++q) {
    const int j0 = q * s, j1 = std::min(H, j0 + s);
    const double jm = s == 1 ? (double)j0 : 0.5 * (j0 + j1 - 1);
    k[q] = jm * dk;
    // +-j for j > 0, j = 0 once
    wt[q] = 2.0 * (j1 - j0) - (j0 == 0 ? 1.0 : 0.0);
  }
  // B(k) times the index multiplicities, over the octant (the sigma-free part)
  const double inv4x2 = 1.0 / (4.0 * xi * xi);
  w.assign((size_t)nq * nq * nq, 0.0);
  sum = 0.0;
  for (int qx = 0; qx < nq; ++qx)
    for (int qy = 0; qy < nq; ++qy)
      for (int qz = 0; qz < nq; ++qz) {
        const double k2 = k[qx] * k[qx] + k[qy] * k[qy] + k[qz] * k[qz];
        if (k2 <= 0.0) continue;
        const double kk = std::sqrt(k2), ka = kk * a;
        const double sinc = std::sin(ka) / ka;
        const double B = sinc * sinc * (1.0 + k2 * inv4x2) * std::exp(-k2 * inv4x2) / k2;
        const double v = wt[qx] * wt[qy] * wt[qz] * B;
        w[((size_t)qx * nq + qy) * nq + qz] = v;
        sum += v;
      }
}

double AliasWeights::estimate(double sigma) const {
  const double h = L / M, s2 = sigma * sigma, g = 2.0 * kPi / h;
  std::vector<double> f1(nq);
  for (int q = 0; q < nq; ++q) {
    const double rm = std::exp(-s2 * ((k[q] - g) * (k[q] - g) - k[q] * k[q]));
    const double rp = std::exp(-s2 * ((k[q] + g) * (k[q] + g) - k[q] * k[q]));
    f1[q] = 1.0 + rm + rp;
  }
  double N = 0.0;
  for (int qx = 0; qx < nq; ++qx)
    for (int qy = 0; qy < nq; ++qy) {
      const double fxy = f1[qx] * f1[qy];
      const double *row = &w[((size_t)qx * nq + qy) * nq];
      for (int qz = 0; qz < nq; ++qz) N += row[qz] * (fxy * f1[qz] - 1.0);
    }
  return sum > 0.0 ? std::sqrt(std::max(N, 0.0) / sum) : 0.0;
}

double alias_estimate(double L, int M, double xi, double a, double sigma, int max_freq) {
  return AliasWeights(L, M, xi, a, max_freq).estimate(sigma);
}

// FFT lengths with a plan: 2^k and 3 x 2^k from 16 to 512.
bool fft_size_supported(int M) {
  switch (M) {
    case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 384: case 512:
      return true;
    default: return false;
  }
}

pse_status derive_params(const pse_params &p, Derived *d) {
  if (p.n < 1 || !(p.box > 0) || !(p.a > 0) || !(p.eta > 0) || !(p.kT >= 0) || !(p.xi > 0) || !(p.rcut > 0))
    return PSE_ERR_INVALID_ARG;
  if (p.precision < PSE_FP64 || p.precision > PSE_MIXED) return PSE_ERR_INVALID_ARG;
  if (!(p.tol >= 0)) return PSE_ERR_INVALID_ARG;
  if (p.flags & ~kKnownFlags) return PSE_ERR_INVALID_ARG;
  // the full-mobility Krylov sample keeps a longer basis than the near-field one
  const int maxit = (p.flags & PSE_FLAG_FULL_LANCZOS) ? kFullMaxIter : kMaxIter;
  if (p.lanczos_max_iter < 1 || p.lanczos_max_iter > maxit || !(p.lanczos_tol > 0)) return PSE_ERR_PARAMS;
  if (!(p.rcut < 0.5 * p.box)) return PSE_ERR_PARAMS;
  if (p.support < 2 || p.support % 2 || p.support > 16 || p.grid < p.support) return PSE_ERR_PARAMS;
  if (!fft_size_supported(p.grid)) return PSE_ERR_PARAMS;
  d->L = p.box;
  d->h = p.box / p.grid;
  d->gm = p.gauss_m > 0 ? p.gauss_m : std::sqrt(kPi * p.support);
  d->sigma = p.support * d->h / (2.0 * d->gm);
  d->eta_se = 4.0 * p.xi * p.xi * d->sigma * d->sigma;
  if (!(d->eta_se < 1.0)) return PSE_ERR_PARAMS;
  d->eps_real = std::exp(-p.xi * p.xi * p.rcut * p.rcut);
  real_tail(p.rcut, p.xi, p.a, p.n / (p.box * p.box * p.box), &d->eps_real_tail, &d->eps_real_coherent);
  d->eps_wave = eps_wave_bound(kPi / d->h, p.xi, p.a);
  d->eps_quad = eps_quad_bound(p.support, d->gm);
  d->eps_alias = alias_estimate(p.box, p.grid, p.xi, p.a, d->sigma);  // 96 frequencies per axis at most
  // (a relative slack of 1e-9 admits the chooser's rc = sqrt(-ln tol) / xi
  // after rounding)
  const double lim = p.tol * (1.0 + 1e-9);
  if (p.tol > 0 && (d->eps_real_tail > lim || d->eps_wave > lim || window_error(d->eps_quad, d->eps_alias) > lim))
    return PSE_ERR_PARAMS;
  d->mu0 = 1.0 / (6.0 * kPi * p.eta * p.a);
  d->self_r = fg_self(p.xi, p.a) * d->mu0;
  int nc = (int)std::floor(p.box / p.rcut);
  if (nc < 1) nc = 1;
  if (nc > 128) nc = 128;
  d->nc = nc;
  d->cs = p.box / nc;
  return PSE_OK;
}

// Work model of one Brownian step (eq. work, with the constants of this
// implementation): n_iter + 1 near-field products (with forces) plus the
// neighbour build, about two products' worth of pair work; spreading and
// interpolation over N P^3 nodes; the FFT set over M^3 log2 M^3.
static double model_seconds(const pse_tuning &t, double n, double pairs, int M, int P, bool forces) {
  const double M3 = (double)M * M * M;
  const double nprod = t.n_iter + (forces ? 1.0 : 0.0) + 2.0;
  const double nquad = forces ? 2.0 : 1.0;
  return t.c_pair * pairs * nprod + t.c_node * n * (double)P * P * P * nquad + t.c_fft * M3 * std::log2(M3) +
         t.c_particle * n;
}

pse_status choose_params(const pse_params &base, const pse_tuning &tin, pse_params *out, pse_tuning_info *info) {
  pse_tuning t = tin;
  if (!(t.tol > 0 && t.tol < 1)) return PSE_ERR_INVALID_ARG;
  if (base.n < 1 || !(base.box > 0) || !(base.a > 0)) return PSE_ERR_INVALID_ARG;
  if (t.n_iter <= 0) t.n_iter = 5.0;
  if (t.c_pair <= 0) t.c_pair = 1.8e-12;
  if (t.c_node <= 0) t.c_node = 7.4e-13;
  if (t.c_fft <= 0) t.c_fft = 1.5e-12;
  if (t.c_particle <= 0) t.c_particle = 3.8e-10;
  if (t.max_grid <= 0) t.max_grid = 512;
  const double L = base.box, a = base.a, n = base.n;
  const double dens = n / (L * L * L);
  // error budget.  A sample (and M F with random forces): the real-space,
  // wave-space and Krylov errors are independent and add in variance, each
  // gets tol / sqrt 3.  Aligned forces (deterministic): the real-space and
  // wave-space errors are both systematic and add linearly, each gets
  // tol / 2.
  const double ts = t.deterministic ? 0.5 * t.tol : t.tol / std::sqrt(3.0);
  static const int kGrids[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
  std::vector<double> xis;
  if (t.xi > 0) xis.push_back(t.xi);
  else
    for (double xa = 0.15; xa <= 1.5 + 1e-9; xa += 0.01) xis.push_back(xa / a);
  // every (xi, M, P) that passes the cheap tests, in order of model cost:
  // the first whose quadrature and aliasing bounds hold is the optimum
  struct Cand {
    double cost, xi, rc, pairs;
    int M, P;
  };
  std::vector<Cand> cands;
  for (double xi : xis) {
    const double rc = rcut_scan(ts, xi, a, dens, t.deterministic != 0, 0.499 * L);
    if (!(rc < 0.5 * L)) continue;
    // ordered pairs at the mean density (hard-sphere structure, d_f = 3)
    const double pairs = n * dens * 4.0 / 3.0 * kPi * rc * rc * rc;
    const double kc = kcut_for(ts, xi, a);
    for (int M : kGrids) {
      if (M > t.max_grid || !fft_size_supported(M)) continue;
      const double h = L / M;
      if (kPi / h < kc || eps_wave_bound(kPi / h, xi, a) > ts) continue;
      for (int P = 2; P <= 16 && P <= M; P += 2) {
        if (!(1.0001 * P * h * xi < 1.4 * std::sqrt(kPi * P))) break;  // eta_SE < 1 needs m > P h xi
        cands.push_back({model_seconds(t, n, pairs, M, P, t.with_forces != 0), xi, rc, pairs, M, P});
      }
    }
  }
  std::sort(cands.begin(), cands.end(), [](const Cand &u, const Cand &v) { return u.cost < v.cost; });
  // B(k) weights of the aliasing estimate per (xi, M): coarse (32
  // frequencies per axis, for the width search) and full (96, to confirm)
  std::map<std::pair<double, int>, AliasWeights> coarse_cache, fine_cache;
  auto weights = [&](std::map<std::pair<double, int>, AliasWeights> &cache, double xi, int M,
                     int nf) -> const AliasWeights & {
    auto key = std::make_pair(xi, M);
    auto it = cache.find(key);
    if (it == cache.end()) it = cache.emplace(key, AliasWeights(L, M, xi, a, nf)).first;
    return it->second;
  };
  auto coarse = [&](double xi, int M) -> const AliasWeights & { return weights(coarse_cache, xi, M, 32); };
  double best = 1e300;
  pse_params bp = base;
  pse_tuning_info bi{};
  for (const Cand &cd : cands) {
    const double xi = cd.xi, h = L / cd.M;
    const int M = cd.M, P = cd.P;
    // the Gaussian's width in standard deviations: m = sqrt(pi P) balances
    // the two terms of eps_quad; a smaller m widens the window (sigma =
    // P h / 2m), which cuts the aliasing at the price of the truncation
    // term erfc(m / sqrt 2), down to eta_SE = 1 at m = P h xi; a larger m
    // does the opposite.  The width minimising the window error
    // window_error(eps_quad, eps_alias) on [max(2, P h xi), 1.4 sqrt(pi P)]
    // (golden section) is kept when it meets the budget left by the k-space
    // truncation; sqrt(pi P) when that already does.
    const double m0 = std::sqrt(kPi * P), mlo = std::max(2.0, 1.0001 * P * h * xi), mhi = 1.4 * m0;
    // spreading and interpolation both err for M F; the sample interpolates only
    const double w = (t.deterministic || t.with_forces) ? 2.0 : 1.0;
    const double tw = ts - eps_wave_bound(kPi / h, xi, a);
    // the search runs on a coarser sub-lattice (at most 32 frequencies per
    // axis); the width found is confirmed with the full estimate below
    // the B(k) weights of the coarse estimate, once per (xi, M)
    const AliasWeights &aw = coarse(cd.xi, M);
    auto total = [&](double m, double *e1, double *e2) {
      *e1 = eps_quad_bound(P, m);
      *e2 = w * window_error(*e1, 0.0) > tw ? 1.0 : aw.estimate(P * h / (2 * m));
      return w * window_error(*e1, *e2);
    };
    double e0q, e0a, mk = 0.0, eq = 0.0, al = 0.0;
    if (!(P * h * xi < m0 && 1.0001 * P * h * xi < mhi)) continue;  // eta_SE >= 1 everywhere
    if (total(m0, &e0q, &e0a) <= tw) {
      mk = m0;
      eq = e0q;
      al = e0a;
    } else {
      const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
      double lo = mlo, hi = mhi, x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo), a1, a2, b1, b2;
      double f1 = total(x1, &a1, &b1), f2 = total(x2, &a2, &b2);
      for (int it = 0; it < 14 && std::min(f1, f2) > tw; ++it) {
        if (f1 <= f2) {
          hi = x2;
          x2 = x1;
          f2 = f1;
          a2 = a1;
          b2 = b1;
          x1 = hi - gr * (hi - lo);
          f1 = total(x1, &a1, &b1);
        } else {
          lo = x1;
          x1 = x2;
          f1 = f2;
          a1 = a2;
          b1 = b2;
          x2 = lo + gr * (hi - lo);
          f2 = total(x2, &a2, &b2);
        }
      }
      if (std::min(f1, f2) <= tw) {
        mk = f1 <= f2 ? x1 : x2;
        eq = f1 <= f2 ? a1 : a2;
        al = f1 <= f2 ? b1 : b2;
      }
    }
    if (mk == 0.0) continue;
    al = weights(fine_cache, xi, M, 96).estimate(P * h / (2 * mk));
    if (w * window_error(eq, al) > tw) continue;
    best = cd.cost;
    bp = base;
    bp.xi = xi;
    // the cutoff of the scan, refined on the tail estimate derive_params reports
    {
      const double r1 = rcut_for(ts, xi, a, dens, t.deterministic != 0, std::min(0.499 * L, cd.rc * 1.01 + 0.05));
      bp.rcut = std::isfinite(r1) ? r1 : cd.rc;
    }
    bp.grid = M;
    bp.support = P;
    bp.gauss_m = mk == m0 ? 0.0 : mk;
    bp.lanczos_tol = ts;
    bp.tol = t.tol;
    bi.model_seconds = cd.cost;
    bi.eps_real = std::exp(-xi * xi * bp.rcut * bp.rcut);
    {
      double inc, coh;
      real_tail(bp.rcut, xi, a, dens, &inc, &coh);
      bi.eps_real_tail = t.deterministic ? coh : inc;
    }
    bi.eps_wave = eps_wave_bound(kPi / h, xi, a);
    bi.eps_quad = eq;
    bi.eps_alias = al;
    bi.pairs_per_particle = cd.pairs / n;
    break;
  }
  if (best >= 1e300) return PSE_ERR_PARAMS;
  // eq. (xistar), the large-N asymptote of the optimum for these constants
  // (hard spheres, d_f = 3).  In the form of eq. (work):
  //   pair work  c_pair nprod N dens (4 pi / 3) rc^3 = C_R n_iter N phi xi^-3,
  //              rc = s / xi with s = xi rc at the chosen point (the tail
  //              estimate depends on xi mainly through xi rc),
  //              phi = dens (4 pi / 3) a^3;
  //   FFT work   c_fft M^3 log2 M^3 = C_W xi^3 phi^-1 N ln(...),
  //              M = kc L / pi with kc = kc1 xi (the bound depends on kc / xi
  //              and xi a only weakly; kc1 taken at the chosen xi).
  {
    const double phi = dens * 4.0 / 3.0 * kPi * a * a * a;
    const double nprod = t.n_iter + (t.with_forces ? 1.0 : 0.0) + 2.0;
    const double srx = bp.xi * bp.rcut;
    const double crn = t.c_pair * nprod * srx * srx * srx / (a * a * a);
    const double kc1 = kcut_for(ts, bp.xi, a) / bp.xi;
    const double cw = t.c_fft * kc1 * kc1 * kc1 * (4.0 / 3.0 * kPi) * a * a * a / (kPi * kPi * kPi * std::log(2.0));
    const double df = 3.0;
    bi.xi_star = std::pow(3.0 * cw * std::log(n) / (crn * df * phi * phi), -1.0 / (df + 3.0));
  }
  *out = bp;
  if (info) *info = bi;
  return PSE_OK;
}

}  // namespace pse
