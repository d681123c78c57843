/* Seeded hard-sphere configuration generators for synthetic benchmark inputs.
 *
 * rsa_fill:  random sequential addition of non-overlapping spheres of radius a
 *            into a cubic periodic box (uniform trial positions, rejection on
 *            overlap).
 * mc_relax:  hard-sphere Monte Carlo displacement sweeps (uniform trial moves,
 *            step adapted toward a target acceptance in the first sweeps),
 *            parallelised with an 8-colour checkerboard of cells whose side is
 *            at least 2a + 2*step, so same-colour cells never interact.  Each
 *            (sweep, cell) has its own random stream: results do not depend on
 *            the thread count.
 *
 * These produce inputs only; they contain none of the sampler's arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t splitmix64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static inline double u01(uint64_t *s) { return ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

static inline double wrap(double v, double L) {
  if (v >= 0 && v < L) return v;
  v = fmod(v, L);
  if (v < 0) v += L;
  if (v >= L) v -= L;
  return v;
}
/* minimum image for |d| < 1.5 L (coordinates already wrapped) */
static inline double mind(double d, double L) {
  const double h = 0.5 * L;
  if (d > h) return d - L;
  if (d < -h) return d + L;
  return d;
}

/* ---------------------------------------------------------------- RSA --- */
int rsa_fill(int n, double L, double a, uint64_t seed, double *x, long long max_attempts) {
  const double sig2 = 4.0 * a * a;
  int nc = (int)floor(L / (2.0 * a));
  if (nc < 1) nc = 1;
  const double cs = L / nc;
  int *head = (int *)malloc(sizeof(int) * (size_t)nc * nc * nc);
  int *next = (int *)malloc(sizeof(int) * (size_t)n);
  if (!head || !next) { free(head); free(next); return -1; }
  for (long i = 0; i < (long)nc * nc * nc; ++i) head[i] = -1;
  uint64_t s = seed * 0x2545F4914F6CDD1Dull + 17;
  int placed = 0;
  long long att = 0;
  const int rng = nc >= 3 ? 1 : 0;  /* for nc < 3 scan every cell */
  while (placed < n && att < max_attempts) {
    ++att;
    double p[3] = {u01(&s) * L, u01(&s) * L, u01(&s) * L};
    int c[3];
    for (int d = 0; d < 3; ++d) { c[d] = (int)(p[d] / cs); if (c[d] >= nc) c[d] = nc - 1; }
    int ok = 1;
    if (rng) {
      for (int dx = -1; dx <= 1 && ok; ++dx)
        for (int dy = -1; dy <= 1 && ok; ++dy)
          for (int dz = -1; dz <= 1 && ok; ++dz) {
            int cx = (c[0] + dx + nc) % nc, cy = (c[1] + dy + nc) % nc, cz = (c[2] + dz + nc) % nc;
            for (int j = head[(cx * nc + cy) * nc + cz]; j >= 0; j = next[j]) {
              double ddx = mind(p[0] - x[3 * j], L), ddy = mind(p[1] - x[3 * j + 1], L), ddz = mind(p[2] - x[3 * j + 2], L);
              if (ddx * ddx + ddy * ddy + ddz * ddz < sig2) { ok = 0; break; }
            }
          }
    } else {
      for (int j = 0; j < placed && ok; ++j) {
        double ddx = mind(p[0] - x[3 * j], L), ddy = mind(p[1] - x[3 * j + 1], L), ddz = mind(p[2] - x[3 * j + 2], L);
        if (ddx * ddx + ddy * ddy + ddz * ddz < sig2) ok = 0;
      }
    }
    if (!ok) continue;
    x[3 * placed] = p[0]; x[3 * placed + 1] = p[1]; x[3 * placed + 2] = p[2];
    int cid = (c[0] * nc + c[1]) * nc + c[2];
    next[placed] = head[cid];
    head[cid] = placed;
    ++placed;
  }
  free(head); free(next);
  return placed;
}

/* ------------------------------------------------------------ MC sweeps --- */
/* Returns the number of accepted moves of the last sweep; *step is updated. */
double mc_relax(int n, double L, double a, double *x, int sweeps, uint64_t seed,
                double target_acc, double *step, int adapt_sweeps) {
  const double sig2 = 4.0 * a * a;
  const double step_cap = 0.5 * a;
  int nc = (int)floor(L / (2.0 * a + 2.0 * step_cap));
  if (nc % 2) nc -= 1;
  if (nc < 4) nc = 0; /* too small for a checkerboard: serial sweeps */
  double st = *step > 0 ? (*step < step_cap ? *step : step_cap) : 0.1 * a;
  double acc_frac = 0.0;
  if (nc == 0) {
    uint64_t s = seed ^ 0xA5A5A5A5ull;
    for (int sw = 0; sw < sweeps; ++sw) {
      long acc = 0;
      for (int i = 0; i < n; ++i) {
        double q[3];
        for (int d = 0; d < 3; ++d) q[d] = wrap(x[3 * i + d] + (2 * u01(&s) - 1) * st, L);
        int ok = 1;
        for (int j = 0; j < n && ok; ++j) {
          if (j == i) continue;
          double dx = mind(q[0] - x[3 * j], L), dy = mind(q[1] - x[3 * j + 1], L), dz = mind(q[2] - x[3 * j + 2], L);
          if (dx * dx + dy * dy + dz * dz < sig2) ok = 0;
        }
        if (ok) { memcpy(&x[3 * i], q, sizeof q); ++acc; }
      }
      acc_frac = (double)acc / (n > 0 ? n : 1);
      if (sw < adapt_sweeps) { st *= (acc_frac + 0.05) / (target_acc + 0.05); if (st > step_cap) st = step_cap; if (st < 1e-4 * a) st = 1e-4 * a; }
    }
    *step = st;
    return acc_frac;
  }
  const double cs = L / nc;
  const long ncell = (long)nc * nc * nc;
  int *cnt = (int *)malloc(sizeof(int) * (ncell + 1));
  int *start = (int *)malloc(sizeof(int) * (ncell + 1));
  int *idx = (int *)malloc(sizeof(int) * (size_t)n);
  int *cell_of = (int *)malloc(sizeof(int) * (size_t)n);
  long *acc_cell = (long *)malloc(sizeof(long) * ncell);
  double off[3] = {0, 0, 0};
  for (int sw = 0; sw < sweeps; ++sw) {
    if (sw % 8 == 0) { /* new random grid offset; rebuild membership */
      uint64_t so = seed ^ (0x9E37ull * (uint64_t)(sw + 1));
      for (int d = 0; d < 3; ++d) off[d] = u01(&so) * cs;
    }
    memset(cnt, 0, sizeof(int) * (ncell + 1));
    for (int i = 0; i < n; ++i) {
      int c[3];
      for (int d = 0; d < 3; ++d) { c[d] = (int)(wrap(x[3 * i + d] - off[d], L) / cs); if (c[d] >= nc) c[d] = nc - 1; }
      cell_of[i] = (c[0] * nc + c[1]) * nc + c[2];
      cnt[cell_of[i]]++;
    }
    start[0] = 0;
    for (long c = 0; c < ncell; ++c) start[c + 1] = start[c] + cnt[c];
    for (long c = 0; c < ncell; ++c) cnt[c] = start[c];
    for (int i = 0; i < n; ++i) idx[cnt[cell_of[i]]++] = i;
    memset(acc_cell, 0, sizeof(long) * ncell);
    for (int col = 0; col < 8; ++col) {
      const int px = col & 1, py = (col >> 1) & 1, pz = (col >> 2) & 1;
#pragma omp parallel for schedule(dynamic, 16)
      for (long c = 0; c < ncell; ++c) {
        int cx = (int)(c / ((long)nc * nc)), cy = (int)((c / nc) % nc), cz = (int)(c % nc);
        if ((cx & 1) != px || (cy & 1) != py || (cz & 1) != pz) continue;
        uint64_t s = seed * 0x9E3779B97F4A7C15ull ^ ((uint64_t)sw * 0xD1B54A32D192ED03ull) ^ ((uint64_t)c * 0x8CB92BA72F3D8DD7ull);
        long acc = 0;
        for (int t = start[c]; t < start[c + 1]; ++t) {
          int i = idx[t];
          double q[3];
          int inside = 1;
          for (int d = 0; d < 3; ++d) {
            q[d] = wrap(x[3 * i + d] + (2 * u01(&s) - 1) * st, L);
            int cd = (int)(wrap(q[d] - off[d], L) / cs);
            if (cd >= nc) cd = nc - 1;
            int want = d == 0 ? cx : (d == 1 ? cy : cz);
            if (cd != want) inside = 0;
          }
          if (!inside) continue;
          int ok = 1;
          for (int dx = -1; dx <= 1 && ok; ++dx)
            for (int dy = -1; dy <= 1 && ok; ++dy)
              for (int dz = -1; dz <= 1 && ok; ++dz) {
                long nb = (((cx + dx + nc) % nc) * (long)nc + (cy + dy + nc) % nc) * nc + (cz + dz + nc) % nc;
                for (int u = start[nb]; u < start[nb + 1]; ++u) {
                  int j = idx[u];
                  if (j == i) continue;
                  double ddx = mind(q[0] - x[3 * j], L), ddy = mind(q[1] - x[3 * j + 1], L), ddz = mind(q[2] - x[3 * j + 2], L);
                  if (ddx * ddx + ddy * ddy + ddz * ddz < sig2) { ok = 0; break; }
                }
              }
          if (ok) { x[3 * i] = q[0]; x[3 * i + 1] = q[1]; x[3 * i + 2] = q[2]; ++acc; }
        }
        acc_cell[c] += acc;
      }
    }
    long acc = 0;
    for (long c = 0; c < ncell; ++c) acc += acc_cell[c];
    acc_frac = (double)acc / (n > 0 ? n : 1);
    if (sw < adapt_sweeps) {
      st *= (acc_frac + 0.05) / (target_acc + 0.05);
      if (st > step_cap) st = step_cap;
      if (st < 1e-4 * a) st = 1e-4 * a;
    }
  }
  free(cnt); free(start); free(idx); free(cell_of); free(acc_cell);
  *step = st;
  return acc_frac;
}

/* Smallest pair distance under the minimum image (cell list, side >= 2a):
 * checks that a configuration is overlap-free. */
double min_pair_distance(int n, double L, double a, const double *x) {
  int nc = (int)floor(L / (2.0 * a));
  if (nc < 3) nc = 1;
  const double cs = L / nc;
  const long ncell = (long)nc * nc * nc;
  int *head = (int *)malloc(sizeof(int) * ncell);
  int *next = (int *)malloc(sizeof(int) * (size_t)n);
  for (long c = 0; c < ncell; ++c) head[c] = -1;
  for (int i = 0; i < n; ++i) {
    int c[3];
    for (int d = 0; d < 3; ++d) { c[d] = (int)(wrap(x[3 * i + d], L) / cs); if (c[d] >= nc) c[d] = nc - 1; }
    long cid = ((long)c[0] * nc + c[1]) * nc + c[2];
    next[i] = head[cid];
    head[cid] = i;
  }
  double best = 1e300;
  for (int i = 0; i < n; ++i) {
    int c[3];
    for (int d = 0; d < 3; ++d) { c[d] = (int)(wrap(x[3 * i + d], L) / cs); if (c[d] >= nc) c[d] = nc - 1; }
    int r = nc >= 3 ? 1 : 0;
    for (int dx = -r; dx <= r; ++dx)
      for (int dy = -r; dy <= r; ++dy)
        for (int dz = -r; dz <= r; ++dz) {
          long nb = (((c[0] + dx + nc) % nc) * (long)nc + (c[1] + dy + nc) % nc) * nc + (c[2] + dz + nc) % nc;
          for (int j = head[nb]; j >= 0; j = next[j]) {
            if (j <= i) continue;
            double ddx = mind(x[3 * i] - x[3 * j], L), ddy = mind(x[3 * i + 1] - x[3 * j + 1], L), ddz = mind(x[3 * i + 2] - x[3 * j + 2], L);
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (d2 < best) best = d2;
          }
        }
  }
  free(head); free(next);
  return sqrt(best);
}

/* --------------------------------------------------------- DLCA gel --- */
/* Off-lattice diffusion-limited cluster aggregation in the periodic box.
 * Start: n non-overlapping spheres in x (e.g. RSA), each its own cluster.
 * Each trial picks a live cluster uniformly and accepts its move with
 * probability s^-gamma (s its size: a Stokes-Einstein diffusivity that falls
 * as the cluster grows); an accepted move translates the whole cluster by
 * `step` along a uniformly random direction, stopping at the first contact
 * |x_p - x_q| = 2a with a sphere of another cluster, and the two clusters
 * then merge (they stick for good).  Ends when the largest cluster holds at
 * least stop_frac of the spheres, or after max_moves accepted moves.
 * Cells have side >= 2a + step, so every sphere a move can touch lies in the
 * 27 cells around the moving sphere's cell.
 * stats (may be NULL): [0] accepted moves, [1] clusters left, [2] largest
 * cluster.  Returns 0, or -1 on allocation failure. */
int dlca_gel(int n, double L, double a, uint64_t seed, double step, double gamma, double stop_frac,
             long long max_moves, double *x, int *cluster, double *stats) {
  int nc = (int)floor(L / (2.0 * a + step));
  if (nc < 3) return -2;
  const double cs = L / nc;
  const long ncell = (long)nc * nc * nc;
  int *head = (int *)malloc(sizeof(int) * ncell);
  int *cnext = (int *)malloc(sizeof(int) * (size_t)n), *cprev = (int *)malloc(sizeof(int) * (size_t)n);
  int *cellof = (int *)malloc(sizeof(int) * (size_t)n);
  int *cid = (int *)malloc(sizeof(int) * (size_t)n), *mnext = (int *)malloc(sizeof(int) * (size_t)n);
  int *mtail = (int *)malloc(sizeof(int) * (size_t)n), *msize = (int *)malloc(sizeof(int) * (size_t)n);
  int *live = (int *)malloc(sizeof(int) * (size_t)n), *livepos = (int *)malloc(sizeof(int) * (size_t)n);
  if (!head || !cnext || !cprev || !cellof || !cid || !mnext || !mtail || !msize || !live || !livepos) {
    free(head); free(cnext); free(cprev); free(cellof); free(cid); free(mnext); free(mtail); free(msize);
    free(live); free(livepos);
    return -1;
  }
  for (long c = 0; c < ncell; ++c) head[c] = -1;
  for (int i = 0; i < n; ++i) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
      x[3 * i + d] = wrap(x[3 * i + d], L);
      c[d] = (int)(x[3 * i + d] / cs);
      if (c[d] >= nc) c[d] = nc - 1;
    }
    const int cc = (c[0] * nc + c[1]) * nc + c[2];
    cellof[i] = cc;
    cprev[i] = -1;
    cnext[i] = head[cc];
    if (head[cc] >= 0) cprev[head[cc]] = i;
    head[cc] = i;
    cid[i] = i;
    mnext[i] = -1;
    mtail[i] = i;
    msize[i] = 1;
    live[i] = i;
    livepos[i] = i;
  }
  int nlive = n, largest = 1;
  uint64_t s = seed * 0x9E3779B97F4A7C15ull + 0x243F6A8885A308D3ull;
  long long moves = 0;
  const double sig = 2.0 * a, sig2 = sig * sig;
  while (moves < max_moves && largest < stop_frac * n && nlive > 1) {
    const int r = live[(int)(u01(&s) * nlive) % nlive];
    if (gamma > 0 && u01(&s) > pow((double)msize[r], -gamma)) continue;
    ++moves;
    /* uniform direction on the sphere */
    const double uz = 2.0 * u01(&s) - 1.0, ph = 2.0 * 3.14159265358979323846 * u01(&s);
    const double rho = sqrt(1.0 - uz * uz);
    const double u[3] = {rho * cos(ph), rho * sin(ph), uz};
    double tmin = 1.0;
    int hit = -1;
    for (int p = r; p >= 0; p = mnext[p]) {
      const int cc = cellof[p];
      const int c0 = cc / (nc * nc), c1 = (cc / nc) % nc, c2 = cc % nc;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int nb = (((c0 + dx + nc) % nc) * nc + (c1 + dy + nc) % nc) * nc + (c2 + dz + nc) % nc;
            for (int q = head[nb]; q >= 0; q = cnext[q]) {
              if (cid[q] == r) continue;
              const double d0 = mind(x[3 * q] - x[3 * p], L), d1 = mind(x[3 * q + 1] - x[3 * p + 1], L),
                           d2 = mind(x[3 * q + 2] - x[3 * p + 2], L);
              const double b = d0 * u[0] + d1 * u[1] + d2 * u[2];
              if (b <= 0) continue; /* moving away */
              const double cq = d0 * d0 + d1 * d1 + d2 * d2 - sig2;
              const double disc = b * b - cq;
              if (disc < 0) continue; /* the path passes by */
              double t = (b - sqrt(disc)) / step;
              if (t < 0) t = 0; /* touching already (rounding) */
              if (t < tmin) {
                tmin = t;
                hit = q;
              }
            }
          }
    }
    /* translate the cluster, keeping the cell lists current */
    const double dv[3] = {tmin * step * u[0], tmin * step * u[1], tmin * step * u[2]};
    for (int p = r; p >= 0; p = mnext[p]) {
      int c[3];
      for (int d = 0; d < 3; ++d) {
        x[3 * p + d] = wrap(x[3 * p + d] + dv[d], L);
        c[d] = (int)(x[3 * p + d] / cs);
        if (c[d] >= nc) c[d] = nc - 1;
      }
      const int cc = (c[0] * nc + c[1]) * nc + c[2];
      if (cc != cellof[p]) {
        if (cprev[p] >= 0) cnext[cprev[p]] = cnext[p];
        else head[cellof[p]] = cnext[p];
        if (cnext[p] >= 0) cprev[cnext[p]] = cprev[p];
        cellof[p] = cc;
        cprev[p] = -1;
        cnext[p] = head[cc];
        if (head[cc] >= 0) cprev[head[cc]] = p;
        head[cc] = p;
      }
    }
    if (hit >= 0) {
      /* merge the smaller cluster into the larger: relabel and splice */
      int big = cid[hit], small = r;
      if (msize[small] > msize[big]) { const int t = big; big = small; small = t; }
      for (int p = small; p >= 0; p = mnext[p]) cid[p] = big;
      mnext[mtail[big]] = small;
      mtail[big] = mtail[small];
      msize[big] += msize[small];
      if (msize[big] > largest) largest = msize[big];
      const int ps = livepos[small], last = live[nlive - 1];
      live[ps] = last;
      livepos[last] = ps;
      --nlive;
    }
  }
  if (cluster)
    for (int i = 0; i < n; ++i) cluster[i] = cid[i];
  if (stats) {
    stats[0] = (double)moves;
    stats[1] = nlive;
    stats[2] = largest;
  }
  free(head); free(cnext); free(cprev); free(cellof); free(cid); free(mnext); free(mtail); free(msize);
  free(live); free(livepos);
  return 0;
}
