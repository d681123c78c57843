// Particle-side kernels: wrapping and linked-cell binning, the sorted order,
// the near-field neighbour list, the real-space product w = M_r v
// (eq. Mreal, Appendix A) and the Lanczos square-root iteration (Sec. II B.1).
#include <mutex>
#include <type_traits>
#include <unordered_set>

#include "launch.hpp"

namespace pse {

template <typename T> __device__ __forceinline__ T wrap_coord(T x, T L, T invL) {
  x = x - L * floor(x * invL);
  if (x >= L || x < T(0)) x = T(0);  // x == L (or rounding just past it) maps to 0
  return x;
}

template <typename T> __device__ __forceinline__ T min_image(T d, T L, T invL) { return d - L * rint(d * invL); }

// --------------------------------------------------------------- binning
template <typename T>
__device__ __forceinline__ void wrap_bin_at(const T *__restrict__ pos, int n, T L, T invL, T inv_cs, int nc,
                                            typename vec4<T>::type *__restrict__ pos_w, int *__restrict__ cell_of,
                                            int *__restrict__ slot, int *__restrict__ cell_count,
                                            int *__restrict__ flags, int i) {
  if (i >= n) return;
  T x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
    atomicOr(&flags[0], 1);
    x = y = z = T(0);
  }
  x = wrap_coord(x, L, invL);
  y = wrap_coord(y, L, invL);
  z = wrap_coord(z, L, invL);
  const int cx = min((int)(x * inv_cs), nc - 1);
  const int cy = min((int)(y * inv_cs), nc - 1);
  const int cz = min((int)(z * inv_cs), nc - 1);
  const int c = (cx * nc + cy) * nc + cz;
  cell_of[i] = c;
  // The particle's slot in its cell (arrival order; k_cell_sort fixes the
  // final order).  Lanes holding the same cell as the lane before them join
  // its run, and the first lane of each run reserves the run's slots with
  // one atomic: all runs of the wavefront in a single instruction, one per
  // particle for shuffled callers, a few for spatially ordered ones.  The
  // active lanes are 0 .. k-1 (only the last wavefront is partial).
  const int lane = threadIdx.x & 63;
  const unsigned long long act = __ballot(1);
  const int prev = __shfl_up(c, 1, 64);
  const bool head = lane == 0 || prev != c;
  const unsigned long long H = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0 .. lane
  const int hl = 63 - __clzll((long long)(H & upto));                             // first lane of my run
  const unsigned long long later = H & ~upto;
  const int next = later ? __ffsll((long long)later) - 1 : 64 - __clzll((long long)act);
  int b = 0;
  if (head) b = atomicAdd(&cell_count[c], next - lane);
  slot[i] = __shfl(b, hl, 64) + (lane - hl);
  typename vec4<T>::type q;
  q.x = x; q.y = y; q.z = z; q.w = T(0);
  pos_w[i] = q;
}

template <typename T>
__global__ void k_wrap_bin(const T *__restrict__ pos, int n, T L, T invL, T inv_cs, int nc,
                           typename vec4<T>::type *__restrict__ pos_w, int *__restrict__ cell_of,
                           int *__restrict__ slot, int *__restrict__ cell_count, int *__restrict__ flags) {
  wrap_bin_at<T>(pos, n, L, invL, inv_cs, nc, pos_w, cell_of, slot, cell_count, flags,
                 blockIdx.x * blockDim.x + threadIdx.x);
}

// Exclusive scan of the cell counts in tiles of 4096 cells: k_scan_tiles
// sums each tile, k_scan_apply adds the sums of the tiles before its own
// (a few thousand at most) and scans its tile (16 consecutive cells per
// thread through LDS, the 256 thread sums scanned across wavefronts).
__device__ __forceinline__ int block_sum_i32(int v, int *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  int t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

__device__ __forceinline__ void scan_tiles_at(const int *__restrict__ count, int ncell, int *__restrict__ tile_sum,
                                              int tile) {
  __shared__ int sh[kScanNT / 64];
  const int base = tile * kScanTile;
  int v = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = base + k * kScanNT + (int)threadIdx.x;
    if (i < ncell) v += count[i];
  }
  v = block_sum_i32(v, sh);
  if (threadIdx.x == 0) tile_sum[tile] = v;
}

__global__ __launch_bounds__(kScanNT) void k_scan_tiles(const int *__restrict__ count, int ncell,
                                                        int *__restrict__ tile_sum) {
  scan_tiles_at(count, ncell, tile_sum, blockIdx.x);
}

__device__ __forceinline__ void scan_apply_at(const int *__restrict__ count, const int *__restrict__ tile_sum,
                                              int ncell, int *__restrict__ start, int tb) {
  __shared__ int tile[kScanTile];
  __shared__ int sh[kScanNT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int base = tb * kScanTile;
  int off = 0;
  for (int k = t; k < tb; k += kScanNT) off += tile_sum[k];
  off = block_sum_i32(off, sh);
  for (int k = t; k < kScanTile; k += kScanNT) {
    const int i = base + k;
    tile[k] = i < ncell ? count[i] : 0;
  }
  __syncthreads();
  int loc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) loc += tile[t * kScanPer + k];
  int v = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  __syncthreads();  // sh is reused
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  int wpre = 0;
  for (int w = 0; w < wave; ++w) wpre += sh[w];
  int run = off + wpre + v - loc;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int cnt = tile[t * kScanPer + k];
    tile[t * kScanPer + k] = run;
    run += cnt;
  }
  __syncthreads();
  for (int k = t; k < kScanTile; k += kScanNT) {
    const int i = base + k;
    if (i < ncell) start[i] = tile[k];
  }
  if (t == kScanNT - 1 && base + kScanTile >= ncell) start[ncell] = run;
}

__global__ __launch_bounds__(kScanNT) void k_scan_apply(const int *__restrict__ count, const int *__restrict__ tile_sum,
                                                        int ncell, int *__restrict__ start) {
  scan_apply_at(count, tile_sum, ncell, start, blockIdx.x);
}

__global__ void k_scatter(const int *__restrict__ cell_of, const int *__restrict__ slot, const int *__restrict__ start,
                          int *__restrict__ perm, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[start[cell_of[i]] + slot[i]] = i;
}

// Order each cell's members by caller index: the sorted order (and with it
// every summation order downstream) is then deterministic.  One wavefront
// per cell: with at most 64 members each lane holds one and its rank is the
// number of smaller indices (the indices are distinct); larger cells fall
// back to an insertion sort by lane 0.  The sorted positions are gathered in
// the same pass.
template <typename T4>
__device__ __forceinline__ void cell_sort_at(const int *__restrict__ start, int *__restrict__ perm, int ncell,
                                             const T4 *__restrict__ pos_w, T4 *__restrict__ pos_s, int c) {
  const int lane = threadIdx.x & 63;
  if (c >= ncell) return;
  const int b = start[c], e = start[c + 1], m = e - b;
  if (m <= 64) {
    const int v = lane < m ? perm[b + lane] : 0x7FFFFFFF;
    int rank = 0;
    for (int j = 0; j < m; ++j) rank += __shfl(v, j, 64) < v ? 1 : 0;
    if (lane < m) {
      perm[b + rank] = v;
      pos_s[b + rank] = pos_w[v];
    }
    return;
  }
  if (lane != 0) return;
  for (int i = b + 1; i < e; ++i) {
    const int v = perm[i];
    int j = i - 1;
    while (j >= b && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
  for (int i = b; i < e; ++i) pos_s[i] = pos_w[perm[i]];
}

template <typename T4>
__global__ __launch_bounds__(256) void k_cell_sort(const int *__restrict__ start, int *__restrict__ perm, int ncell,
                                                   const T4 *__restrict__ pos_w, T4 *__restrict__ pos_s) {
  cell_sort_at<T4>(start, perm, ncell, pos_w, pos_s, (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
}

// ------------------------------------------------------- F, G evaluation
// FP32 modes: linear interpolation in an LDS table of (mu0 F, mu0 (G-F)).
struct FGTable {
  const float2 *tab;  // nodes, LDS or global
  float inv_dr;
  __device__ __forceinline__ void eval(float r2, float rinv, float &Fm, float &Dm) const {
    const float u = r2 * rinv * inv_dr;
    int k = (int)u;
    k = min(k, kTableK);
    const float f = u - (float)k;
    const float2 e0 = tab[k], e1 = tab[k + 1];
    Fm = fmaf(f, e1.x - e0.x, e0.x);
    Dm = fmaf(f, e1.y - e0.y, e0.y);
  }
};

// FP64 mode: Appendix A closed forms on the fly (Case 1 / Case 2), with the
// series of the wave complement below the small-r threshold.
struct FGExact {
  const double *ser;  // [2 * kSeriesTerms]: F then G series coefficients
  double xi, a, mu0, small_r2;
  __device__ __forceinline__ void eval(double r2, double rinv, double &Fm, double &Dm) const {
    const double r = r2 * rinv;
    double F, G;
    if (r2 < small_r2) {
      double Ff, Gf;
      if (r > 2.0 * a) {
        const double ci = 0.75 * a / r + 0.5 * a * a * a / (r * r2);
        F = ci;
        G = ci + 0.75 * a / r - 1.5 * a * a * a / (r * r2);
      } else {
        F = 1.0 - 9.0 * r / (32.0 * a);
        G = 1.0 - 3.0 * r / (16.0 * a);
      }
      Ff = 0.0;
      Gf = 0.0;
      for (int n = kSeriesTerms - 1; n >= 0; --n) {
        Ff = Ff * r2 + ser[n];
        Gf = Gf * r2 + ser[kSeriesTerms + n];
      }
      F -= Ff;
      G -= Gf;
    } else {
      const double sp = 1.7724538509055160273;
      const double x = xi, x2 = x * x, x3 = x2 * x, x4 = x2 * x2;
      const double r3 = r2 * r, r4 = r2 * r2, a2 = a * a;
      const double rm = r - 2.0 * a, rp = r + 2.0 * a;
      const double qp = 4.0 * a2 + 4.0 * a * r + 9.0 * r2, qm = 4.0 * a2 - 4.0 * a * r + 9.0 * r2;
      const double e1 = exp(-r2 * x2), e2 = exp(-rm * rm * x2), e3 = exp(-rp * rp * x2);
      const double c1 = erfc(r * x), c2 = erfc(rm * x), c3 = erfc(rp * x);
      const double i64 = 1.0 / (64.0 * sp * a * r3 * x3), i128 = 0.5 * i64;
      const double f1 = (18.0 * r2 * x2 + 3.0) / (64.0 * sp * a * r2 * x3);
      const double f2 = (2.0 * x2 * (2.0 * a - r) * qp - 2.0 * a - 3.0 * r) * i128;
      const double f3 = (-2.0 * x2 * rp * qm + 2.0 * a - 3.0 * r) * i128;
      const double f4 = (3.0 - 36.0 * r4 * x4) / (128.0 * a * r3 * x4);
      const double f5 = (4.0 * x4 * rm * rm * qp - 3.0) / (256.0 * a * r3 * x4);
      const double f6 = (4.0 * x4 * rp * rp * qm - 3.0) / (256.0 * a * r3 * x4);
      const double g1 = (6.0 * r2 * x2 - 3.0) / (32.0 * sp * a * r2 * x3);
      const double g2 = (-2.0 * x2 * rm * rm * (2.0 * a + 3.0 * r) + 2.0 * a + 3.0 * r) * i64;
      const double g3 = (2.0 * x2 * rp * rp * (2.0 * a - 3.0 * r) - 2.0 * a + 3.0 * r) * i64;
      const double g4 = -(3.0 * (4.0 * r4 * x4 + 1.0)) / (64.0 * a * r3 * x4);
      const double tm = 2.0 * a - r;
      const double g5 = (3.0 - 4.0 * x4 * tm * tm * tm * (2.0 * a + 3.0 * r)) / (128.0 * a * r3 * x4);
      const double g6 = (3.0 - 4.0 * x4 * (2.0 * a - 3.0 * r) * rp * rp * rp) / (128.0 * a * r3 * x4);
      double f0 = 0.0, g0 = 0.0;
      if (r <= 2.0 * a) {
        f0 = -rm * rm * qp / (32.0 * a * r3);
        g0 = tm * tm * tm * (2.0 * a + 3.0 * r) / (16.0 * a * r3);
      }
      F = f0 + f1 * e1 + f2 * e2 + f3 * e3 + f4 * c1 + f5 * c2 + f6 * c3;
      G = g0 + g1 * e1 + g2 * e2 + g3 * e3 + g4 * c1 + g5 * c2 + g6 * c3;
    }
    Fm = F * mu0;
    Dm = (G - F) * mu0;
  }
};

// ------------------------------------------ learned-preconditioner features
// 24 geometry features of one particle, accumulated over its near
// neighbours (minimum image, r < 4.5a; d = x_i - x_j, dh = d / r, dh = 0 at
// r = 0) with the dimensionless F, G of Appendix A; f3 alone counts every
// neighbour within rc:
//   0..3   #{r < 2.2a}/4, #{r < 3a}/8, #{r < 4.5a}/16, #{r <= rc}/128
//   4      sum F / 8
//   5..10  sum (G - F) dh dh^T (xx, yy, zz, xy, xz, yz)
//   11..16 sum_{r < 3a} dh dh^T / 4
//   17..19 sum_{r < 3a} dh / 4
//   20     sum (G - F)
//   21     min r / 4.5a (1 without near neighbours)
//   22     sum_{r < 3a} (3a - r) / a / 4
//   23     F_self (eq. self)
template <typename T> struct FeatAcc {
  T f[kNFeat];
  __device__ __forceinline__ void init(T fself) {
#pragma unroll
    for (int k = 0; k < kNFeat; ++k) f[k] = T(0);
    f[21] = T(1);
    f[23] = fself;
  }
  // one near neighbour (r < 4.5a): separation d, r and 1/r (0 at r = 0),
  // dimensionless F and G - F.  The 1/8 of f4 is applied in store(), f3
  // comes from the neighbour count there.
  __device__ __forceinline__ void add(T dx, T dy, T dz, T r, T ir, T Fd, T Dd, T a, T inv_near) {
    const T hx = dx * ir, hy = dy * ir, hz = dz * ir;
    f[0] += r < T(2.2) * a ? T(0.25) : T(0);
    f[2] += T(0.0625);
    f[4] += Fd;
    const T ex = Dd * hx, ey = Dd * hy, ez = Dd * hz;
    f[5] += ex * hx;
    f[6] += ey * hy;
    f[7] += ez * hz;
    f[8] += ex * hy;
    f[9] += ex * hz;
    f[10] += ey * hz;
    f[20] += Dd;
    f[21] = min(f[21], r * inv_near);
    if (r < T(3) * a) {  // close neighbours (a small fraction of the hits)
      f[1] += T(0.125);
      const T qx = T(0.25) * hx, qy = T(0.25) * hy, qz = T(0.25) * hz;
      f[11] += qx * hx;
      f[12] += qy * hy;
      f[13] += qz * hz;
      f[14] += qx * hy;
      f[15] += qx * hz;
      f[16] += qy * hz;
      f[17] += qx;
      f[18] += qy;
      f[19] += qz;
      f[22] += (T(3) * a - r) / a * T(0.25);
    }
  }
  __device__ __forceinline__ void store(uint16_t *__restrict__ out, int count) {
    f[3] = T(count) * T(1.0 / 128);
    f[4] *= T(0.125);
    uint32_t w[kNFeat / 2];
#pragma unroll
    for (int k = 0; k < kNFeat / 2; ++k)
      w[k] = (uint32_t)f32_to_bf16((float)f[2 * k]) | ((uint32_t)f32_to_bf16((float)f[2 * k + 1]) << 16);
    uint4 *o = (uint4 *)out;  // 48 bytes per particle: three 16-byte stores
    o[0] = make_uint4(w[0], w[1], w[2], w[3]);
    o[1] = make_uint4(w[4], w[5], w[6], w[7]);
    o[2] = make_uint4(w[8], w[9], w[10], w[11]);
  }
};

// Near-field neighbour list (ELL layout nbr[k * n + s], sorted indices):
// every t != s with minimum-image distance <= rc, scanning the 27 adjacent
// cells (fewer when a side has < 3 cells, so no cell is visited twice).
// With FEAT the learned-preconditioner features of s are accumulated from
// the same hits (fg gives mu0 F and mu0 (G - F); FeatAcc).
// With REP the overlap repulsion f_s = sum_{t: r < 2a} krep (2a - r) d / r
// (d = x_s - x_t) goes to frep[s].
template <typename T, bool FEAT, typename FG, bool REP = false>
__global__ void k_nbr_build(const typename vec4<T>::type *__restrict__ pos, const int *__restrict__ start, int n,
                            int nc, T L, T invL, T inv_cs, T rc2, int *__restrict__ nbr, int *__restrict__ cnt_out,
                            int cap, int *__restrict__ flags, FG fg, T inv_mu0, T fself, T a, T inv_rc,
                            uint16_t *__restrict__ feat, T krep, typename vec4<T>::type *__restrict__ frep) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (s < n) {
  FeatAcc<T> acc;
  if (FEAT) acc.init(fself);
  T fx = T(0), fy = T(0), fz = T(0);
  const auto p = pos[s];
  const int cx = min((int)(p.x * inv_cs), nc - 1);
  const int cy = min((int)(p.y * inv_cs), nc - 1);
  const int cz = min((int)(p.z * inv_cs), nc - 1);
  const int lo = nc >= 3 ? -1 : 0, hi = nc >= 2 ? 1 : 0;
  for (int dx = lo; dx <= hi; ++dx) {
    const int ax = (cx + dx + nc) % nc;
    for (int dy = lo; dy <= hi; ++dy) {
      const int ay = (cy + dy + nc) % nc;
      for (int dz = lo; dz <= hi; ++dz) {
        const int c = (ax * nc + ay) * nc + (cz + dz + nc) % nc;
        const int e = start[c + 1];
        for (int t = start[c]; t < e; ++t) {
          if (t == s) continue;
          const auto q = pos[t];
          const T ddx = min_image(p.x - q.x, L, invL);
          const T ddy = min_image(p.y - q.y, L, invL);
          const T ddz = min_image(p.z - q.z, L, invL);
          const T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
          if (REP && r2 < T(4) * a * a && r2 > T(0)) {
            const T r = sqrt(r2), m = krep * (T(2) * a - r) / r;
            fx += m * ddx;
            fy += m * ddy;
            fz += m * ddz;
          }
          if (r2 <= rc2) {
            if (cnt < cap) nbr[(size_t)cnt * n + s] = t;
            ++cnt;
            if (FEAT && r2 < T(20.25) * a * a) {  // near shell r < 4.5a
              T Fm = fself / inv_mu0, Dm = T(0), r = T(0), ir = T(0);
              if (r2 > T(1e-24)) {
                r = sqrt(r2);
                ir = T(1) / r;
                fg.eval(r2, ir, Fm, Dm);
              }
              acc.add(ddx, ddy, ddz, r, ir, Fm * inv_mu0, Dm * inv_mu0, a, T(1) / (T(4.5) * a));
            }
          }
        }
      }
    }
  }
  if (FEAT) acc.store(feat + (size_t)s * kNFeat, cnt);
  if (REP) {
    typename vec4<T>::type f;
    f.x = fx;
    f.y = fy;
    f.z = fz;
    f.w = T(0);
    frep[s] = f;
  }
  cnt_out[s] = min(cnt, cap);  // entries stored; flags[1] carries the capacity needed
  }
  // total ordered pairs and the largest count: one set of atomics per wavefront
  const unsigned long long tot = wave_sum((unsigned long long)cnt);
  int mx = cnt;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) {
    if (tot) atomicAdd((unsigned long long *)(flags + 2), tot);
    atomicMax(&flags[1], mx);  // capacity needed
    atomicMax(&flags[5], mx);  // largest neighbour count
  }
}

// --------------------------------------------------- near-field product
// One thread per sorted particle s:
//   out_s = scale * ( self * v_s + sum_{t in nbr(s)} mu0 [F v_t + (G-F)(d.v_t) d / r^2] )
// with v = src (times `scale`).  In the Lanczos variant the scale is the
// device-side 1/beta, the thread also stores the basis vector V_m = scale*src
// and the block reduces V_m . out toward alpha_m (last block finishes it).
template <typename T, typename A, typename FG, bool LZ>
__device__ __forceinline__ void spmv_body(const typename vec4<T>::type *__restrict__ pos, const int *__restrict__ nbr,
                                          const int *__restrict__ cnt, int n, T L, T invL, const FG &fg, T self_r,
                                          const typename vec4<T>::type *__restrict__ src, T scale,
                                          typename vec4<T>::type *__restrict__ out,
                                          typename vec4<T>::type *__restrict__ vm_out, A &dot) {
  using T4 = typename vec4<T>::type;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  dot = A(0);
  if (s >= n) return;
  const T4 p = pos[s];
  const T4 v = src[s];
  T ax = self_r * v.x, ay = self_r * v.y, az = self_r * v.z;
  const int c = cnt[s];
  const int *nb = nbr + s;
#pragma unroll 4
  for (int k = 0; k < c; ++k) {
    const int t = nb[(size_t)k * n];
    const T4 q = pos[t];
    const T4 w = src[t];
    const T dx = min_image(p.x - q.x, L, invL);
    const T dy = min_image(p.y - q.y, L, invL);
    const T dz = min_image(p.z - q.z, L, invL);
    const T r2 = dx * dx + dy * dy + dz * dz;
    T Fm, Dm, rinv;
    if (r2 > T(1e-24)) {
      rinv = T(1) / sqrt(r2);
      fg.eval(r2, rinv, Fm, Dm);
    } else {  // coincident spheres: the r -> 0 limit is isotropic
      Fm = self_r;
      Dm = T(0);
      rinv = T(0);
    }
    const T pr = Dm * rinv * rinv * (dx * w.x + dy * w.y + dz * w.z);
    ax += Fm * w.x + pr * dx;
    ay += Fm * w.y + pr * dy;
    az += Fm * w.z + pr * dz;
  }
  T4 o;
  o.x = ax * scale;
  o.y = ay * scale;
  o.z = az * scale;
  o.w = T(0);
  out[s] = o;
  if (LZ) {
    T4 u;
    u.x = v.x * scale;
    u.y = v.y * scale;
    u.z = v.z * scale;
    u.w = T(0);
    vm_out[s] = u;
    dot = (A)u.x * (A)o.x + (A)u.y * (A)o.y + (A)u.z * (A)o.z;
  }
}

template <typename T, typename A, bool LZ>
__global__ __launch_bounds__(256) void k_spmv_table(const float4 *__restrict__ pos, const int *__restrict__ nbr,
                                                    const int *__restrict__ cnt, int n, float L, float invL,
                                                    const float2 *__restrict__ tab_g, float inv_dr, float self_r,
                                                    const float4 *__restrict__ src, float scale, float4 *__restrict__ out,
                                                    float4 *__restrict__ vm_out, LzState<A> *st, A *partials,
                                                    unsigned *counter) {
  __shared__ float2 tab[kTableN];
  __shared__ A sh[16];
  __shared__ int last;
  if (LZ) {
    if (st->done) return;
    scale = (float)st->inv_beta;
  }
  for (int i = threadIdx.x; i < kTableN; i += blockDim.x) tab[i] = tab_g[i];
  __syncthreads();
  FGTable fg{tab, inv_dr};
  A dot;
  spmv_body<float, A, FGTable, LZ>(pos, nbr, cnt, n, L, invL, fg, self_r, src, scale, out, vm_out, dot);
  if (!LZ) return;
  A bs = block_sum(dot, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = bs;
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (last) {
    __threadfence();
    A v = 0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) v += partials[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) {
      st->alpha[st->m] = v;
      *counter = 0u;
    }
  }
}

template <bool LZ>
__global__ __launch_bounds__(256) void k_spmv_exact(const double4 *__restrict__ pos, const int *__restrict__ nbr,
                                                    const int *__restrict__ cnt, int n, double L, double invL,
                                                    const double *__restrict__ ser, double xi, double a, double mu0,
                                                    double small_r2, double self_r, const double4 *__restrict__ src,
                                                    double scale, double4 *__restrict__ out, double4 *__restrict__ vm_out,
                                                    LzState<double> *st, double *partials, unsigned *counter) {
  __shared__ double sh[16];
  __shared__ int last;
  if (LZ) {
    if (st->done) return;
    scale = st->inv_beta;
  }
  FGExact fg{ser, xi, a, mu0, small_r2};
  double dot;
  spmv_body<double, double, FGExact, LZ>(pos, nbr, cnt, n, L, invL, fg, self_r, src, scale, out, vm_out, dot);
  if (!LZ) return;
  double bs = block_sum(dot, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = bs;
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (last) {
    __threadfence();
    double v = 0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) v += partials[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) {
      st->alpha[st->m] = v;
      *counter = 0u;
    }
  }
}

// ------------------------------------------- LDS-staged near-field kernels
// Target blocks of B x B x B linked cells.  The block's halo, the (B+2)^3
// cells within one cell of its own, is staged in LDS once; the neighbour
// list then holds 16-bit LDS indices, so the product reads neighbours from
// LDS instead of gathering 16-byte records from global memory per pair.
// List layout: chunks of 8 indices, chunk q of sorted particle s at 16-byte
// slot (q * n + s): one coalesced 16-byte load per lane per 8 neighbours.
// The last chunk is padded with the index one past the halo (the product's
// zero source).
// Needs nc >= B + 2 (no halo cell appears twice).  B = 1 ... 4: blocks of
// more cells keep enough targets per workgroup when cells hold few
// particles (small rc).
template <int B> struct Halo {
  static constexpr int HB = B + 2;
  static constexpr int NH = HB * HB * HB;  // 27, 64, 125 or 216 halo cells
  static constexpr int NT = B * B * B;     // target cells
};

template <int B> struct HaloTab {
  int start[Halo<B>::NH];     // global sorted index of each halo cell's first particle
  int base[Halo<B>::NH + 1];  // exclusive prefix of the halo cell counts (LDS offsets)
  int tcell[Halo<B>::NT];     // halo index of each target cell
  int tpre[Halo<B>::NT + 1];  // exclusive prefix of the target cell counts
  int ntc;                    // number of target cells (< B^3 at the partial last block)
};

// blk: the block of B^3 cells this workgroup serves (by default the
// XCD-renumbered workgroup index)
template <int B>
__device__ __forceinline__ void halo_setup(const int *__restrict__ cell_start, int nc, HaloTab<B> &ht, int blk) {
  constexpr int HB = Halo<B>::HB, NH = Halo<B>::NH;
  const int nb = (nc + B - 1) / B;
  const int bz = blk % nb, by = (blk / nb) % nb, bx = blk / (nb * nb);
  if (threadIdx.x < 64) {
    // one wavefront scans the halo cells, 64 at a time, carrying the sum
    const int lane = threadIdx.x;
    int carry = 0;
    for (int h0 = 0; h0 < NH; h0 += 64) {
      const int h = h0 + lane;
      int cnt = 0;
      if (h < NH) {
        const int hx = h / (HB * HB), hy = (h / HB) % HB, hz = h % HB;
        const int gx = (bx * B - 1 + hx + nc) % nc, gy = (by * B - 1 + hy + nc) % nc,
                  gz = (bz * B - 1 + hz + nc) % nc;
        const int c = (gx * nc + gy) * nc + gz;
        const int a = cell_start[c];
        cnt = cell_start[c + 1] - a;
        ht.start[h] = a;
      }
      int v = cnt;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
      }
      if (h < NH) ht.base[h + 1] = carry + v;
      carry += __shfl(v, 63, 64);
    }
    if (lane == 0) ht.base[0] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int k = 0, acc = 0;
    for (int ox = 0; ox < B; ++ox)
      for (int oy = 0; oy < B; ++oy)
        for (int oz = 0; oz < B; ++oz) {
          if (bx * B + ox >= nc || by * B + oy >= nc || bz * B + oz >= nc) continue;
          const int h = ((ox + 1) * HB + (oy + 1)) * HB + (oz + 1);
          ht.tcell[k] = h;
          ht.tpre[k] = acc;
          acc += ht.base[h + 1] - ht.base[h];
          ++k;
        }
    ht.tpre[k] = acc;
    ht.ntc = k;
  }
  __syncthreads();
}

// The staged halo plus the zero-source slot fit the `hcap` records the
// launch reserved.  A launch whose capacity was fixed in advance (a
// captured graph replayed on new positions) may meet a larger halo: the
// workgroup then stages nothing, raises *ovf and returns, and the caller
// redoes that system with capacities sized for it.  Uniform per workgroup.
template <int B> __device__ __forceinline__ bool halo_fits(const HaloTab<B> &ht, int hcap, int *ovf) {
  const bool ok = ht.base[Halo<B>::NH] + 1 <= hcap;
  if (!ok && threadIdx.x == 0) atomicOr(ovf, 1);
  return ok;
}

// LDS index e -> halo cell (largest h with base[h] <= e).
template <int B> __device__ __forceinline__ int halo_cell_of(const HaloTab<B> &ht, int e) {
  int lo = 0, hi = Halo<B>::NH;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ht.base[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// LDS halo records: positions as float4, or as float3 where only the
// coordinates are read (12 bytes: more workgroups per CU)
__device__ __forceinline__ void halo_put(float4 *l, int e, const float4 &q) { l[e] = q; }
__device__ __forceinline__ void halo_put(float3 *l, int e, const float4 &q) { l[e] = make_float3(q.x, q.y, q.z); }

template <int B, typename LT>
__device__ __forceinline__ void halo_stage(const float4 *__restrict__ g, LT *l, const HaloTab<B> &ht) {
  const int total = ht.base[Halo<B>::NH];
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int h = halo_cell_of<B>(ht, e);
    halo_put(l, e, g[ht.start[h] + (e - ht.base[h])]);
  }
}

// Stage positions relative to the block centre c, each at its periodic image
// nearest to c: pairs then need no minimum-image correction (valid when the
// block half-width plus rc stays below L/2, i.e. nc >= B + 3), and the
// staged coordinates are small (a few cells), so that their differences
// keep the precision of the relative position rather than of the box size.
template <int B, typename LT>
__device__ __forceinline__ void halo_stage_unwrapped(const float4 *__restrict__ g, LT *l, const HaloTab<B> &ht,
                                                     float cx, float cy, float cz, float L, float invL) {
  const int total = ht.base[Halo<B>::NH];
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int h = halo_cell_of<B>(ht, e);
    float4 q = g[ht.start[h] + (e - ht.base[h])];
    q.x = min_image(q.x - cx, L, invL);
    q.y = min_image(q.y - cy, L, invL);
    q.z = min_image(q.z - cz, L, invL);
    halo_put(l, e, q);
  }
}

// target i of the block -> (halo cell index, LDS index, global sorted index)
template <int B> __device__ __forceinline__ void target_of(const HaloTab<B> &ht, int i, int &h, int &li, int &s) {
  // largest target cell j with tpre[j] <= i
  int j = 0, hi = ht.ntc;
  while (hi - j > 1) {
    const int mid = (j + hi) >> 1;
    if (ht.tpre[mid] <= i) j = mid;
    else hi = mid;
  }
  h = ht.tcell[j];
  const int off = i - ht.tpre[j];
  li = ht.base[h] + off;
  s = ht.start[h] + off;
}

// Per-block halo sizes (largest goes to flags[4]) for sizing the LDS: one
// wavefront per block, lane (hx, hy) sums its column of HB halo cells.
template <int B>
__global__ __launch_bounds__(256) void k_halo_size(const int *__restrict__ cell_start, int nc, int *__restrict__ flags) {
  constexpr int HB = Halo<B>::HB;
  static_assert(HB * HB <= 64, "one lane per halo column");
  const int nb = (nc + B - 1) / B;
  const int blk = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (blk >= nb * nb * nb) return;  // uniform across the wavefront
  const int bz = blk % nb, by = (blk / nb) % nb, bx = blk / (nb * nb);
  int tot = 0;
  if (lane < HB * HB) {
    const int hx = lane / HB, hy = lane % HB;
    const int gx = (bx * B - 1 + hx + nc) % nc, gy = (by * B - 1 + hy + nc) % nc;
    const int row = (gx * nc + gy) * nc;
    for (int hz = 0; hz < HB; ++hz) {
      const int gz = (bz * B - 1 + hz + nc) % nc;
      tot += cell_start[row + gz + 1] - cell_start[row + gz];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
  if (lane == 0) atomicMax(&flags[4], tot);
}

// flags[1]: list capacity needed; flags[5]: largest count.  With REP the
// same scan accumulates the overlap repulsion of each target,
//   f_s = sum_{t: r < 2a} krep (2a - r) d / r,  d = x_s - x_t,
// into frep[s] (the candidates' distances are at hand; overlapping pairs
// are rare, so the branch is almost never taken).
template <int B, bool UNWRAP, bool REP>
__device__ __forceinline__ void nbr_lds_block(const float4 *__restrict__ pos, const int *__restrict__ cell_start,
                                              int nc, float cs, int n, float L, float invL, float rc2,
                                              uint16_t *__restrict__ nbr, int *__restrict__ cnt_out, int cap,
                                              int *__restrict__ flags, float contact, float krep,
                                              float4 *__restrict__ frep, int hcap, int blk) {
  constexpr int HB = Halo<B>::HB, NH = Halo<B>::NH;
  extern __shared__ float3 hpos3[];  // coordinates only
  __shared__ HaloTab<B> ht;
  // for each 4-bit hit mask: (offsets of the set bits in 16-bit fields, low
  // and high word; 0xFFFF in each used field, low and high word)
  __shared__ uint4 pack_tab[16];
  if (threadIdx.x < 16) {
    uint64_t pat = 0, msk = 0;
    int f = 0;
    for (int u = 0; u < 4; ++u)
      if (threadIdx.x & (1 << u)) {
        pat |= (uint64_t)u << (16 * f);
        msk |= 0xFFFFull << (16 * f);
        ++f;
      }
    pack_tab[threadIdx.x] = make_uint4((uint32_t)pat, (uint32_t)(pat >> 32), (uint32_t)msk, (uint32_t)(msk >> 32));
  }
  halo_setup<B>(cell_start, nc, ht, blk);
  if (!halo_fits<B>(ht, hcap, flags + 7)) return;
  if (UNWRAP) {
    const int nb = (nc + B - 1) / B;
    const int bz = blk % nb, by = (blk / nb) % nb, bx = blk / (nb * nb);
    const float c0 = 0.5f * B * cs;
    halo_stage_unwrapped<B>(pos, hpos3, ht, bx * B * cs + c0, by * B * cs + c0, bz * B * cs + c0, L, invL);
  } else {
    halo_stage<B>(pos, hpos3, ht);
  }
  __syncthreads();
  const int ntarg = ht.tpre[ht.ntc];
  unsigned long long mine = 0;
  int mx = 0;
  uint4 *row = (uint4 *)nbr;
  for (int i = threadIdx.x; i < ntarg; i += blockDim.x) {
    int h, li, s;
    target_of(ht, i, h, li, s);
    const int ox = h / (HB * HB) - 1, oy = (h / HB) % HB - 1, oz = h % HB - 1;
    const float3 p = hpos3[li];
    int k = 0;
    float fx = 0.f, fy = 0.f, fz = 0.f;  // overlap repulsion (REP)
    uint64_t lo = 0, hi = 0;  // the current chunk of 8 packed 16-bit indices
    // the three cells dz = -1, 0, 1 of a (dx, dy) column are consecutive
    // halo cells, staged contiguously: one run of candidates per column, in
    // the same order as cell by cell
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        const int hh = ((ox + 1 + dx) * HB + (oy + 1 + dy)) * HB + oz;
        const int e = ht.base[hh + 3];
        // four candidates per step: their LDS reads are in flight together
        // (up to 3 past the run, into the next cell or the 3 padding slots
        // after the halo; masked out below)
        for (int j0 = ht.base[hh]; j0 < e; j0 += 4) {
          float3 q[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) q[u] = hpos3[j0 + u];
          unsigned hit = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float ddx = p.x - q[u].x, ddy = p.y - q[u].y, ddz = p.z - q[u].z;
            if (!UNWRAP) {
              ddx = min_image(ddx, L, invL);
              ddy = min_image(ddy, L, invL);
              ddz = min_image(ddz, L, invL);
            }
            const float r2 = ddx * ddx + ddy * ddy + ddz * ddz;
            const int j = j0 + u;
            hit |= (j < e && j != li && r2 <= rc2) ? 1u << u : 0u;
            if (REP && j < e && j != li && r2 < contact * contact && r2 > 0.f) {
              const float r = sqrtf(r2), m = krep * (contact - r) / r;
              fx += m * ddx;
              fy += m * ddy;
              fz += m * ddz;
            }
          }
          // the hits of the step, compacted: field f of V is j0 plus the
          // offset of the f-th set bit (pattern table), then V is
          // shifted into the chunk at field k & 7; fields past 8 carry
          // into the next chunk
          const uint4 tb = pack_tab[hit];
          const uint32_t X = (uint32_t)j0 * 0x10001u;
          const uint64_t V = ((uint64_t)((X & tb.w) + tb.y) << 32) | (uint64_t)((X & tb.z) + tb.x);
          const int sh = 16 * (k & 7);
          const bool upper = sh >= 64;
          const int s2 = upper ? sh - 64 : sh;
          const uint64_t vs = V << s2, spill = s2 ? V >> (64 - s2) : 0ull;
          lo |= upper ? 0ull : vs;
          hi |= upper ? vs : spill;
          const int k1 = k + __builtin_popcount(hit);
          if ((k1 >> 3) != (k >> 3)) {
            if ((k >> 3) < (cap >> 3))
              row[(size_t)(k >> 3) * n + s] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi,
                                                         (uint32_t)(hi >> 32));
            lo = upper ? spill : 0ull;
            hi = 0;
          }
          k = k1;
        }
      }
    if ((k & 7) && (k >> 3) < (cap >> 3)) {
      // the rest of the last chunk points at the zero-source slot the
      // product stages after the halo (index = halo size)
      const uint64_t sent = (uint64_t)ht.base[NH];
#pragma unroll
      for (int sl = 1; sl < 8; ++sl) {
        if (sl < (k & 7)) continue;
        const uint64_t v = sent << (16 * (sl & 3));
        if (sl < 4) lo |= v;
        else hi |= v;
      }
      row[(size_t)(k >> 3) * n + s] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    }
    cnt_out[s] = min(k, cap);  // entries stored; flags[1] carries the capacity needed
    if (REP) frep[s] = make_float4(fx, fy, fz, 0.f);
    mine += (unsigned long long)k;
    mx = max(mx, k);
  }
  // one set of atomics per workgroup: every wavefront hitting the same
  // flags serialises at the L2
  const unsigned long long tot = wave_sum(mine);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
  __shared__ unsigned long long wtot[8];
  __shared__ int wmx[8];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wtot[wave] = tot;
    wmx[wave] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    int m = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      t += wtot[w];
      m = max(m, wmx[w]);
    }
    if (t) atomicAdd((unsigned long long *)(flags + 2), t);
    atomicMax(&flags[1], m);
    atomicMax(&flags[5], m);
  }
}

template <int B, bool UNWRAP, bool REP = false>
__global__ __launch_bounds__(512) void k_nbr_lds(const float4 *__restrict__ pos, const int *__restrict__ cell_start,
                                                 int nc, float cs, int n, float L, float invL, float rc2,
                                                 uint16_t *__restrict__ nbr, int *__restrict__ cnt_out, int cap,
                                                 int *__restrict__ flags, float contact, float krep,
                                                 float4 *__restrict__ frep, int hcap) {
  nbr_lds_block<B, UNWRAP, REP>(pos, cell_start, nc, cs, n, L, invL, rc2, nbr, cnt_out, cap, flags, contact, krep,
                                frep, hcap, xcd_block(blockIdx.x, gridDim.x));
}

// The neighbour build of many systems (a batch of replicas) in one launch:
// pmap lists (system, block of that system) per workgroup.
template <int B, bool UNWRAP>
__global__ __launch_bounds__(512) void k_nbr_lds_batch(const NbrRep *__restrict__ reps, const int2 *__restrict__ pmap) {
  const int2 rb = pmap[blockIdx.x];
  const NbrRep &r = reps[rb.x];
  nbr_lds_block<B, UNWRAP, false>(r.pos, r.cell_start, r.nc, r.cs, r.n, r.L, r.invL, r.rc2, r.nbr, r.cnt, r.cap,
                                  r.flags, 0.0f, 0.0f, nullptr, r.hcap, rb.y);
}

// Preconditioner features (FeatAcc; F, G from the LDS table).  Three lanes
// per target, as in the product:
// lane q of a group scans neighbour chunks q, q + 3, ... against the staged
// halo and queues every entry closer than 4.5a in its column of an LDS
// queue.  The queue is drained (one FeatAcc.add per entry) when some lane of
// the wavefront could overflow it, and at the end, so a wavefront spends on
// the features about its largest near count rather than the largest per
// chunk summed over chunks.  The three partial sums are then combined with
// lane shuffles (the minimum for f21).
constexpr int kFeatQ = 16;    // queue entries per lane
constexpr int kFeatNT = 512;  // lanes per workgroup (two workgroups per CU)
template <int B, bool UNWRAP>
__global__ __launch_bounds__(kFeatNT) void k_feat_lds(const float4 *__restrict__ pos, const int *__restrict__ cell_start,
                                                   int nc, float cs, int n, float L, float invL,
                                                   const uint16_t *__restrict__ nbr, const int *__restrict__ cnt,
                                                   const float2 *__restrict__ tab, float inv_dr, float inv_mu0,
                                                   float fself, float a, float near2, uint16_t *__restrict__ feat,
                                                   int hcap, int *__restrict__ ovf) {
  constexpr int NH = Halo<B>::NH;
  constexpr int G = 3, GPW = 64 / G;
  extern __shared__ float4 hpos[];
  __shared__ HaloTab<B> ht;
  __shared__ uint16_t queue[kFeatQ * kFeatNT];
  __shared__ float2 ftab[kTableN];
  for (int k = threadIdx.x; k < kTableN; k += blockDim.x) ftab[k] = tab[k];
  halo_setup<B>(cell_start, nc, ht, xcd_block(blockIdx.x, gridDim.x));
  if (!halo_fits<B>(ht, hcap, ovf)) return;
  if (UNWRAP) {
    const int nb = (nc + B - 1) / B;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int bz = blk % nb, by = (blk / nb) % nb, bx = blk / (nb * nb);
    const float c0 = 0.5f * B * cs;
    halo_stage_unwrapped<B>(pos, hpos, ht, bx * B * cs + c0, by * B * cs + c0, bz * B * cs + c0, L, invL);
  } else {
    halo_stage<B>(pos, hpos, ht);
  }
  __syncthreads();
  const FGTable fg{ftab, inv_dr};
  const int ntarg = ht.tpre[ht.ntc];
  const uint4 *row = (const uint4 *)nbr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, g = lane - grp * G;
  const bool ingrp = grp < GPW;
  uint16_t *myq = queue + threadIdx.x;  // entry t at myq[kFeatNT t]
  for (int i0 = 0; i0 < ntarg; i0 += (int)(blockDim.x >> 6) * GPW) {
    const int i = i0 + wave * GPW + grp;
    const bool act = ingrp && i < ntarg;
    int h = 0, li = 0, s = 0;
    if (act) target_of(ht, i, h, li, s);
    const float4 p = hpos[li];
    FeatAcc<float> acc;
    acc.init(0.0f);
    int nq = 0;
    // one near pair into the sums (F, G - F from the LDS table)
    auto add = [&](const float4 &q) {
      float ddx = p.x - q.x, ddy = p.y - q.y, ddz = p.z - q.z;
      if (!UNWRAP) {
        ddx = min_image(ddx, L, invL);
        ddy = min_image(ddy, L, invL);
        ddz = min_image(ddz, L, invL);
      }
      const float r2 = ddx * ddx + ddy * ddy + ddz * ddz;
      const bool nz = r2 > 1e-24f;
      const float ir = nz ? __frsqrt_rn(r2) : 0.0f;
      float Fm = fself / inv_mu0, Dm = 0.0f;
      if (nz) fg.eval(r2, ir, Fm, Dm);
      acc.add(ddx, ddy, ddz, r2 * ir, ir, Fm * inv_mu0, Dm * inv_mu0, a, 1.0f / (4.5f * a));
    };
    // two queue entries per pass: their LDS reads are in flight together
    auto drain = [&]() {
      for (int t = 0; t < nq; t += 2) {
        const bool two = t + 1 < nq;
        const int j0 = myq[kFeatNT * t], j1 = myq[kFeatNT * (two ? t + 1 : t)];
        const float4 q0 = hpos[j0], q1 = hpos[j1];
        add(q0);
        if (two) add(q1);
      }
      nq = 0;
    };
    const int c = act ? cnt[s] : 0;
    uint4 nxt = 8 * g < c ? row[(size_t)g * n + s] : make_uint4(0, 0, 0, 0);
    for (int kb = 8 * g; kb < c; kb += 8 * G) {
      const uint4 pk = nxt;
      if (kb + 8 * G < c) nxt = row[(size_t)((kb >> 3) + G) * n + s];
      const uint32_t wd[4] = {pk.x, pk.y, pk.z, pk.w};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = (wd[u >> 1] >> (16 * (u & 1))) & 0xFFFF;
        const float4 q = hpos[kb + u < c ? j : li];
        float ddx = p.x - q.x, ddy = p.y - q.y, ddz = p.z - q.z;
        if (!UNWRAP) {
          ddx = min_image(ddx, L, invL);
          ddy = min_image(ddy, L, invL);
          ddz = min_image(ddz, L, invL);
        }
        const float r2 = ddx * ddx + ddy * ddy + ddz * ddz;
        if (kb + u < c && r2 < near2) {
          myq[kFeatNT * nq] = (uint16_t)j;
          ++nq;
        }
      }
      // the next chunk adds at most 8 entries
      if (__any(nq > kFeatQ - 8)) drain();
    }
    drain();
    // combine the G lanes of the target (lanes G grp .. G grp + G - 1)
    const int base_lane = (lane / G) * G;
#pragma unroll
    for (int k = 0; k < kNFeat; ++k) {
      if (k == 3 || k == 23) continue;  // set by store() / the self value
      float v = acc.f[k];
#pragma unroll
      for (int o = 1; o < G; ++o) {
        const int srcl = base_lane + o < 64 ? base_lane + o : lane;
        const float t = __shfl(acc.f[k], srcl, 64);
        v = k == 21 ? fminf(v, t) : v + t;
      }
      acc.f[k] = v;
    }
    acc.f[23] = fself;
    if (act && g == 0) acc.store(feat + (size_t)s * kNFeat, c);
  }
}

// Near-field product from the staged halo.  The halo is packed as
// (x, y, z, v_x) + (v_y, v_z) (24 bytes per particle) together with the F/G
// table (mu0 F, mu0 (G - F) at nodes rc / 2048 apart; two 8-byte reads per
// pair for the linear interpolation).  G lanes per target (lane q of the group takes neighbour chunks
// q, q + G, ...; 64 / G groups per wavefront; 3 unless pse_autotune picks 2
// or 4) are combined with lane shuffles; each chunk of 8 neighbours is processed branch-free in two
// halves of 4 (padding entries read the zero source), the LDS reads of a half
// in flight together.  Registers are held to 64 so that two 1024-lane
// workgroups share a compute unit: one stages its halo while the other
// computes.  With UNWRAP the staged positions are the images nearest the
// block centre.
// With LZ (a Lanczos step) the epilogue scales by 1 / beta_m and stores the
// basis vector v_m; alpha_m = <v_m, out> is formed by the update step.
// With PC (Lanczos on A = P M_r P^T): src holds u = P^T r, and the
// epilogue forms out = P (M_r u) / beta and v_m = r / beta (r from rsrc);
// Pm holds the rows of P_i as (x, y, z, 0).
template <int B, bool UNWRAP, typename A, bool LZ, bool PC, int G>
__device__ __forceinline__ void spmv_lds_block(const float4 *__restrict__ pos, const float4 *__restrict__ src,
                                               const int *__restrict__ cell_start, int nc, float cs, int n, int hcap,
                                               float L, float invL, const uint16_t *__restrict__ nbr,
                                               const int *__restrict__ cnt, const float2 *__restrict__ tab,
                                               float inv_dr, float self_r, float scale, float4 *__restrict__ out,
                                               float4 *__restrict__ vm_out, const LzState<A> *st,
                                               int *__restrict__ ovf, const float4 *__restrict__ Pm,
                                               const float4 *__restrict__ rsrc, int blk) {
  constexpr int NH = Halo<B>::NH;
  static_assert(G >= 2 && G <= 4, "lanes per target");
  constexpr int GPW = 64 / G;               // groups per wavefront (lane 63 idle at G = 3)
  extern __shared__ float4 smem[];
  float4 *hA = smem;                        // (x, y, z, v_x)
  float2 *hB = (float2 *)(smem + hcap);     // (v_y, v_z)
  __shared__ float2 tabs[kTableN];
  __shared__ HaloTab<B> ht;
  if (LZ) {
    if (st->done) return;
    scale = (float)st->inv_beta;
  }
  for (int k = threadIdx.x; k < kTableN; k += blockDim.x) tabs[k] = tab[k];
  halo_setup<B>(cell_start, nc, ht, blk);
  // a halo past the capacity stages nothing and computes no target
  const bool fits = halo_fits<B>(ht, hcap, ovf);
  if (fits) {
    const int nb = (nc + B - 1) / B;
    const int bz = blk % nb, by = (blk / nb) % nb, bx = blk / (nb * nb);
    const float c0 = 0.5f * B * cs;
    const float cx = bx * B * cs + c0, cy = by * B * cs + c0, cz = bz * B * cs + c0;
    const int total = ht.base[NH];
    // slot `total`: a source with zero vector at the block centre, read by
    // the padding entries of the neighbour chunks (contributes exactly 0)
    // coordinates are staged in units of the table spacing rc / kTableK:
    // r is then the table coordinate itself (the (G - F) term is invariant)
    if (threadIdx.x == 0) {
      // (UNWRAP: coordinates relative to the block centre)
      hA[total] = UNWRAP ? make_float4(0.0f, 0.0f, 0.0f, 0.0f)
                         : make_float4(cx * inv_dr, cy * inv_dr, cz * inv_dr, 0.0f);
      hB[total] = make_float2(0.0f, 0.0f);
    }
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int h = halo_cell_of<B>(ht, e);
      const int gi = ht.start[h] + (e - ht.base[h]);
      float4 q = pos[gi];
      const float4 v = src[gi];
      if (UNWRAP) {
        q.x = min_image(q.x - cx, L, invL);
        q.y = min_image(q.y - cy, L, invL);
        q.z = min_image(q.z - cz, L, invL);
      }
      q.x *= inv_dr;
      q.y *= inv_dr;
      q.z *= inv_dr;
      q.w = v.x;
      hA[e] = q;
      hB[e] = make_float2(v.y, v.z);
    }
  }
  __syncthreads();
  const int ntarg = fits ? ht.tpre[ht.ntc] : 0;
  const float Ls = L * inv_dr, invLs = invL / inv_dr;  // box in table units
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, g = lane - grp * G;
  const bool ingrp = grp < GPW;
  
  for (int i0 = 0; i0 < ntarg; i0 += (int)(blockDim.x >> 6) * GPW) {
    const int i = i0 + wave * GPW + grp;
    const bool act = ingrp && i < ntarg;
    int h = 0, li = 0, s = 0;
    if (act) target_of(ht, i, h, li, s);
    const float4 pa = hA[li];
    const float2 pb = hB[li];
    float ax = 0.f, ay = 0.f, az = 0.f;
    const int c = act ? cnt[s] : 0;
    const uint4 *row = (const uint4 *)nbr + s;
    // the next chunk of indices is loaded while the current one is used
    uint4 nxt = 8 * g < c ? row[(size_t)g * n] : make_uint4(0, 0, 0, 0);
    for (int kb = 8 * g; kb < c; kb += 8 * G) {
      const uint4 pk = nxt;
      if (kb + 8 * G < c) nxt = row[(size_t)((kb >> 3) + G) * n];
      const uint32_t wd[4] = {pk.x, pk.y, pk.z, pk.w};
      // entries past the count in the last chunk hold the zero-source slot;
      // two halves of 4: all halo reads of a half first, then its table reads
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        int jj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) jj[u] = (wd[2 * hf + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
        float4 q[4];
        float2 wb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          q[u] = hA[jj[u]];
          wb[u] = hB[jj[u]];
        }
        float dx[4], dy[4], dz[4], rinv[4], fr[4];
        int kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          dx[u] = pa.x - q[u].x;
          dy[u] = pa.y - q[u].y;
          dz[u] = pa.z - q[u].z;
          if (!UNWRAP) {
            dx[u] = min_image(dx[u], Ls, invLs);
            dy[u] = min_image(dy[u], Ls, invLs);
            dz[u] = min_image(dz[u], Ls, invLs);
          }
          const float r2 = fmaxf(dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u], 1e-20f);
          rinv[u] = __frsqrt_rn(r2);
          const float uu = r2 * rinv[u];
          kk[u] = min((int)uu, kTableK);
          fr[u] = __builtin_amdgcn_fractf(uu);
        }
        float2 e0[4], e1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          e0[u] = tabs[kk[u]];
          e1[u] = tabs[kk[u] + 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float wx = q[u].w, wy = wb[u].x, wz = wb[u].y;
          const float Fm = fmaf(fr[u], e1[u].x - e0[u].x, e0[u].x);
          const float Dm = fmaf(fr[u], e1[u].y - e0[u].y, e0[u].y);
          const float pr = Dm * rinv[u] * rinv[u] * (dx[u] * wx + dy[u] * wy + dz[u] * wz);
          ax = fmaf(pr, dx[u], fmaf(Fm, wx, ax));
          ay = fmaf(pr, dy[u], fmaf(Fm, wy, ay));
          az = fmaf(pr, dz[u], fmaf(Fm, wz, az));
        }
      }
    }
    // combine the G lanes of the target (lanes G grp .. G grp + G - 1)
    const int base_lane = (lane / G) * G;
    float sx = ax, sy = ay, sz = az;
#pragma unroll
    for (int o = 1; o < G; ++o) {
      const int srcl = base_lane + o < 64 ? base_lane + o : lane;
      const float tx = __shfl(ax, srcl, 64), ty = __shfl(ay, srcl, 64), tz = __shfl(az, srcl, 64);
      sx += tx;
      sy += ty;
      sz += tz;
    }
    if (act && g == 0) {
      const float vx = pa.w, vy = pb.x, vz = pb.y;
      float4 u4;
      if (PC) {
        const float tx = sx + self_r * vx, ty = sy + self_r * vy, tz = sz + self_r * vz;
        const float4 p0 = Pm[3 * (size_t)s], p1 = Pm[3 * (size_t)s + 1], p2 = Pm[3 * (size_t)s + 2];
        sx = (p0.x * tx + p0.y * ty + p0.z * tz) * scale;
        sy = (p1.x * tx + p1.y * ty + p1.z * tz) * scale;
        sz = (p2.x * tx + p2.y * ty + p2.z * tz) * scale;
        const float4 r = rsrc[s];
        u4 = make_float4(r.x * scale, r.y * scale, r.z * scale, 0.0f);
      } else {
        sx = (sx + self_r * vx) * scale;
        sy = (sy + self_r * vy) * scale;
        sz = (sz + self_r * vz) * scale;
        u4 = make_float4(vx * scale, vy * scale, vz * scale, 0.0f);
      }
      out[s] = make_float4(sx, sy, sz, 0.0f);
      if (LZ) vm_out[s] = u4;
    }
  }
}

template <int B, bool UNWRAP, typename A, bool LZ, bool PC = false, int G = 3>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spmv_lds(
    const float4 *__restrict__ pos, const float4 *__restrict__ src, const int *__restrict__ cell_start, int nc, float cs,
    int n, int hcap, float L, float invL, const uint16_t *__restrict__ nbr, const int *__restrict__ cnt,
    const float2 *__restrict__ tab, float inv_dr, float self_r, float scale, float4 *__restrict__ out,
    float4 *__restrict__ vm_out, const LzState<A> *st, int *__restrict__ ovf, const float4 *__restrict__ Pm = nullptr,
    const float4 *__restrict__ rsrc = nullptr) {
  spmv_lds_block<B, UNWRAP, A, LZ, PC, G>(pos, src, cell_start, nc, cs, n, hcap, L, invL, nbr, cnt, tab, inv_dr,
                                          self_r, scale, out, vm_out, st, ovf, Pm, rsrc,
                                          xcd_block(blockIdx.x, gridDim.x));
}

// ------------------------------------------------------------- Lanczos
// Block partial sums of |z|^2 (sorted order vector of length 3n).
template <typename T, typename A>
__global__ void k_norm2_partial(const T *__restrict__ z, int len, A *__restrict__ partials) {
  __shared__ A sh[16];
  A v = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) v += (A)z[i] * (A)z[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

template <typename A>
__device__ __forceinline__ void lz_init_body(const A *__restrict__ partials, int nparts, LzState<A> *st) {
  __shared__ A sh[16];
  A v = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += partials[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const A b0 = sqrt(v);
    st->beta[0] = b0;
    st->m = 0;
    st->rel_change = A(1);
    st->converged = 0;
    st->nonfinite = !isfinite(b0);
    st->done = (b0 == A(0)) || !isfinite(b0);
    if (b0 == A(0)) st->converged = 1;
    st->inv_beta = b0 > A(0) ? A(1) / b0 : A(0);
  }
}

template <typename A>
__global__ void k_lz_init(const A *__restrict__ partials, int nparts, LzState<A> *st) {
  lz_init_body<A>(partials, nparts, st);
}

// w = t - alpha_m v_m - beta_m v_{m-1}, one particle (x, y, z, 0) per
// step; block partials of |w|^2.
// alpha_m = <v_m, t> of the step.  k_lz_alpha_part writes block partial
// sums; lz_alpha (inside the update kernels) adds them in a fixed order in
// every block, and block 0 stores alpha_m.  Computed here rather than in
// the LDS product's epilogue: without the reduction the product needs no
// register spills (64 VGPRs), which costs far more than this extra pass
// over two vectors.
template <typename T, typename A>
__global__ void k_lz_alpha_part(const typename vec4<T>::type *__restrict__ t,
                                const typename vec4<T>::type *__restrict__ vm, int n, const LzState<A> *st,
                                A *__restrict__ partials) {
  __shared__ A sh[16];
  if (st->done) return;
  A v = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const auto a = t[i], b = vm[i];
    v += (A)a.x * (A)b.x + (A)a.y * (A)b.y + (A)a.z * (A)b.z;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

template <typename A> __device__ A lz_alpha(LzState<A> *st, const A *apart, int napart, A *sh, bool store) {
  __shared__ A alpha_s;
  if (!apart) return st->alpha[st->m];
  A v = 0;
  for (int i = threadIdx.x; i < napart; i += blockDim.x) v += apart[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) {
    alpha_s = v;
    if (store) st->alpha[st->m] = v;
  }
  __syncthreads();
  return alpha_s;
}

template <typename T, typename A>
__global__ void k_lz_update(const typename vec4<T>::type *__restrict__ t, const typename vec4<T>::type *__restrict__ vm,
                            const typename vec4<T>::type *__restrict__ vprev, typename vec4<T>::type *__restrict__ w,
                            int n, LzState<A> *st, A *__restrict__ partials, const A *__restrict__ apart = nullptr,
                            int napart = 0) {
  __shared__ A sh[16];
  if (st->done) return;
  const int m = st->m;
  const T al = (T)lz_alpha(st, apart, napart, sh, blockIdx.x == 0);
  const T be = m > 0 ? (T)st->beta[m] : T(0);
  A v = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const auto a = t[i], b = vm[i];
    typename vec4<T>::type x;
    x.x = a.x - al * b.x;
    x.y = a.y - al * b.y;
    x.z = a.z - al * b.z;
    if (m > 0) {
      const auto c = vprev[i];
      x.x -= be * c.x;
      x.y -= be * c.y;
      x.z -= be * c.z;
    }
    x.w = T(0);
    w[i] = x;
    v += (A)x.x * (A)x.x + (A)x.y * (A)x.y + (A)x.z * (A)x.z;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// Preconditioned variant, per particle: w as above, and u = P^T w, the
// source of the next product (P rows as (x, y, z, 0), 12 values each).
template <typename T, typename A>
__global__ void k_lz_update_pc(const typename vec4<T>::type *__restrict__ t,
                               const typename vec4<T>::type *__restrict__ vm,
                               const typename vec4<T>::type *__restrict__ vprev, typename vec4<T>::type *__restrict__ w,
                               const T *__restrict__ P, typename vec4<T>::type *__restrict__ u, int n,
                               LzState<A> *st, A *__restrict__ partials, const A *__restrict__ apart = nullptr,
                               int napart = 0) {
  __shared__ A sh[16];
  if (st->done) return;
  const int m = st->m;
  const T al = (T)lz_alpha(st, apart, napart, sh, blockIdx.x == 0);
  const T be = m > 0 ? (T)st->beta[m] : T(0);
  A v = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const auto a = t[i], b = vm[i];
    typename vec4<T>::type x;
    x.x = a.x - al * b.x;
    x.y = a.y - al * b.y;
    x.z = a.z - al * b.z;
    if (m > 0) {
      const auto c = vprev[i];
      x.x -= be * c.x;
      x.y -= be * c.y;
      x.z -= be * c.z;
    }
    x.w = T(0);
    w[i] = x;
    v += (A)x.x * (A)x.x + (A)x.y * (A)x.y + (A)x.z * (A)x.z;
    const auto *pr = (const typename vec4<T>::type *)(P + (size_t)i * 12);  // rows of P_i
    const auto r0 = pr[0], r1 = pr[1], r2 = pr[2];
    typename vec4<T>::type o;
    o.x = r0.x * x.x + r1.x * x.y + r2.x * x.z;
    o.y = r0.y * x.x + r1.y * x.y + r2.y * x.z;
    o.z = r0.z * x.x + r1.z * x.y + r2.z * x.z;
    o.w = T(0);
    u[i] = o;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// s = T^{1/2} e_1 for the n x n tridiagonal T (diag d, off-diagonal e with
// e[i] coupling i, i+1), by implicit QL with Wilkinson-type shifts.  One
// wavefront: lane j holds d[j], e[j]; lane k owns row k of the eigenvector
// matrix Q (stored column-major in LDS).  Returns s_k in lane k.
template <typename A>
__device__ A tridiag_sqrt_e1(int n, A d, A e, A *Q, int &ok) {
  const int lane = threadIdx.x & 63;
  const A eps = sizeof(A) == 8 ? A(2.2e-16) : A(1.2e-7);
  for (int j = 0; j < n; ++j) Q[j * 64 + lane] = (lane == j) ? A(1) : A(0);
  auto gd = [&](int i) { return __shfl(d, i, 64); };
  auto ge = [&](int i) { return __shfl(e, i, 64); };
  ok = 1;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int mm;
      for (mm = l; mm < n - 1; ++mm) {
        const A dd = fabs(gd(mm)) + fabs(gd(mm + 1));
        if (fabs(ge(mm)) <= eps * dd) break;
      }
      if (mm == l) break;
      if (++iter > 60) {
        ok = 0;
        break;
      }
      A g = (gd(l + 1) - gd(l)) / (A(2) * ge(l));
      A r = hypot(g, A(1));
      g = gd(mm) - gd(l) + ge(l) / (g + copysign(r, g));
      A s = 1, c = 1, p = 0;
      bool early = false;
      for (int i = mm - 1; i >= l; --i) {
        const A f = s * ge(i), b = c * ge(i);
        r = hypot(f, g);
        if (lane == i + 1) e = r;
        if (r == A(0)) {
          const A v = gd(i + 1) - p;
          if (lane == i + 1) d = v;
          if (lane == mm) e = A(0);
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = gd(i + 1) - p;
        r = (gd(i) - g) * s + A(2) * c * b;
        p = s * r;
        const A nd = g + p;
        if (lane == i + 1) d = nd;
        g = c * r - b;
        const A qi1 = Q[(i + 1) * 64 + lane], qi = Q[i * 64 + lane];
        Q[(i + 1) * 64 + lane] = s * qi + c * qi1;
        Q[i * 64 + lane] = c * qi - s * qi1;
      }
      if (early) continue;
      const A nl = gd(l) - p;
      if (lane == l) {
        d = nl;
        e = g;
      }
      if (lane == mm) e = A(0);
    }
    if (!ok) break;
  }
  __builtin_amdgcn_wave_barrier();
  A acc = 0;
  for (int j = 0; j < n; ++j) {
    const A lam = gd(j);
    acc += Q[j * 64 + lane] * sqrt(lam > A(0) ? lam : A(0)) * Q[j * 64];
  }
  return acc;
}

// After iteration m: beta_{m+1} = |w|, s = T_{m+1}^{1/2} e_1, convergence test
// |s_{m+1} - s_m| <= tol |s_{m+1}| (successive iterates; V orthonormal), and
// the scale 1/beta_{m+1} of the next Lanczos vector.  One wavefront.
template <typename A>
__device__ __forceinline__ void lz_check_body(const A *__restrict__ partials, int nparts, LzState<A> *st, A tol,
                                              int max_iter) {
  __shared__ A Q[kMaxIter * 64];
  if (st->done) return;
  const int lane = threadIdx.x;
  // eight interleaved sums keep eight loads in flight (fixed order)
  A vs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = lane;
  for (; i + 7 * 64 < nparts; i += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) vs[u] += partials[i + u * 64];
  }
  for (; i < nparts; i += 64) vs[0] += partials[i];
  A v = ((vs[0] + vs[1]) + (vs[2] + vs[3])) + ((vs[4] + vs[5]) + (vs[6] + vs[7]));
  v = wave_sum(v);
  const A bb = sqrt(v);
  const int m = st->m;
  const int nn = m + 1;
  A d = lane < nn ? st->alpha[lane] : A(0);
  A e = lane < nn - 1 ? st->beta[lane + 1] : A(0);
  int ok;
  const A sk = tridiag_sqrt_e1<A>(nn, d, e, Q, ok);
  const A sold = (lane < m) ? st->s[lane] : A(0);
  const A dif = lane < nn ? (sk - sold) : A(0);
  const A num = wave_sum(dif * dif);
  const A den = wave_sum(lane < nn ? sk * sk : A(0));
  const A rel = den > A(0) ? sqrt(num / den) : A(0);
  A scale2 = 0;
  for (int j = 0; j < nn; ++j) {
    const A aj = __shfl(d, j, 64);
    scale2 += aj * aj;
  }
  const A bdn = (sizeof(A) == 8 ? A(1e-11) : A(1e-6)) * sqrt(scale2 + bb * bb);
  const bool finite = isfinite(bb) && isfinite(den) && ok;
  if (lane < nn) st->s[lane] = sk;
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
    st->beta[nn] = bb;
    st->rel_change = m > 0 ? rel : A(1);
    st->m = nn;
    const bool conv = (m > 0 && rel <= tol) || (bb <= bdn);
    st->converged = conv && finite;
    st->nonfinite = !finite;
    st->done = conv || !finite || nn >= max_iter;
    st->inv_beta = bb > A(0) ? A(1) / bb : A(0);
  }
}

template <typename A>
__global__ __launch_bounds__(64) void k_lz_check(const A *__restrict__ partials, int nparts, LzState<A> *st, A tol,
                                                 int max_iter) {
  lz_check_body<A>(partials, nparts, st, tol, max_iter);
}

// ------------------------------------------------- batched Krylov loop
// Iteration m of the Lanczos process on many systems at once (a batch of
// replicas): the same arithmetic, in the same order, as the single-system
// kernels above, so that every system's iterate is bit-identical to its own
// run.  pmap / vmap list (system, block of that system) per workgroup: the
// product's blocks of B^3 cells, and the vector kernels' blocks of 256
// particles (n <= kRedBlock 256 per system, so that each thread owns at most
// one particle, as in the single-system kernels).
template <int B, bool UNWRAP, typename A, int G>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spmv_lds_batch(
    const LzRep<A> *__restrict__ reps, const int2 *__restrict__ pmap, int m) {
  const int2 rb = pmap[blockIdx.x];
  const LzRep<A> &r = reps[rb.x];
  spmv_lds_block<B, UNWRAP, A, true, false, G>(r.pos, m == 0 ? r.z : r.w, r.cell_start, r.nc, r.cs, r.n, r.hcap,
                                               r.L, r.invL, r.nbr, r.cnt, r.tab, r.inv_dr, r.self_r, 1.0f, r.t,
                                               r.V + (size_t)m * r.n, r.st, r.ovf, nullptr, nullptr, rb.y);
}

// M_r F of the systems whose record carries forces (the others' blocks exit)
template <int B, bool UNWRAP, typename A, int G>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spmv_lds_batch_plain(
    const LzRep<A> *__restrict__ reps, const int2 *__restrict__ pmap) {
  const int2 rb = pmap[blockIdx.x];
  const LzRep<A> &r = reps[rb.x];
  if (!r.fs) return;
  spmv_lds_block<B, UNWRAP, A, false, false, G>(r.pos, r.fs, r.cell_start, r.nc, r.cs, r.n, r.hcap, r.L, r.invL,
                                                r.nbr, r.cnt, r.tab, r.inv_dr, r.self_r, 1.0f, r.ur, nullptr, nullptr,
                                                r.ovf, nullptr, nullptr, rb.y);
}

template <typename A>
__global__ __launch_bounds__(256) void k_lz_alpha_batch(const LzRep<A> *__restrict__ reps,
                                                        const int2 *__restrict__ vmap, int m) {
  __shared__ A sh[16];
  const int2 rb = vmap[blockIdx.x];
  const LzRep<A> &r = reps[rb.x];
  if (r.st->done) return;
  const float4 *vm = r.V + (size_t)m * r.n;
  A *part = r.partials + kRedBlock;
  A v = 0;
  const int i = rb.y * 256 + (int)threadIdx.x;
  if (i < r.n) {
    const float4 a = r.t[i], b = vm[i];
    v += (A)a.x * (A)b.x + (A)a.y * (A)b.y + (A)a.z * (A)b.z;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[rb.y] = v;
  if (rb.y == 0)  // the blocks past the system's particles hold 0, as a single-system launch writes them
    for (int k = (r.n + 255) / 256 + (int)threadIdx.x; k < kRedBlock; k += 256) part[k] = A(0);
}

template <typename A>
__global__ __launch_bounds__(256) void k_lz_update_batch(const LzRep<A> *__restrict__ reps,
                                                         const int2 *__restrict__ vmap, int m) {
  __shared__ A sh[16];
  const int2 rb = vmap[blockIdx.x];
  const LzRep<A> &r = reps[rb.x];
  LzState<A> *st = r.st;
  if (st->done) return;
  const int mm = st->m;
  const float al = (float)lz_alpha(st, r.partials + kRedBlock, kRedBlock, sh, rb.y == 0);
  const float be = mm > 0 ? (float)st->beta[mm] : 0.0f;
  const float4 *vm = r.V + (size_t)m * r.n;
  const float4 *vprev = m > 0 ? r.V + (size_t)(m - 1) * r.n : r.V;
  A v = 0;
  const int i = rb.y * 256 + (int)threadIdx.x;
  if (i < r.n) {
    const float4 a = r.t[i], b = vm[i];
    float4 x;
    x.x = a.x - al * b.x;
    x.y = a.y - al * b.y;
    x.z = a.z - al * b.z;
    if (mm > 0) {
      const float4 c = vprev[i];
      x.x -= be * c.x;
      x.y -= be * c.y;
      x.z -= be * c.z;
    }
    x.w = 0.0f;
    r.w[i] = x;
    v += (A)x.x * (A)x.x + (A)x.y * (A)x.y + (A)x.z * (A)x.z;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) r.partials[rb.y] = v;
  if (rb.y == 0)
    for (int k = (r.n + 255) / 256 + (int)threadIdx.x; k < kRedBlock; k += 256) r.partials[k] = A(0);
}

// one wavefront per system
template <typename A>
__global__ __launch_bounds__(64) void k_lz_check_batch(const LzRep<A> *__restrict__ reps) {
  const LzRep<A> &r = reps[blockIdx.x];
  lz_check_body<A>(r.partials, kRedBlock, r.st, r.tol, r.maxit);
}

// y = beta_0 sum_{j < m} V_j s_j  (sorted order, length 3n)
// one element of y from the coefficients sc[0 .. m)
template <typename T, typename A>
__device__ __forceinline__ T lz_combine_at(const T *__restrict__ V, size_t ld, const A *sc, int m, int i) {
  A acc = 0;
  for (int j = 0; j < m; ++j) acc += sc[j] * (A)V[(size_t)j * ld + i];
  return (T)acc;
}

template <typename T, typename A>
__global__ void k_lz_combine(const T *__restrict__ V, size_t ld, int len, const LzState<A> *st, T *__restrict__ y) {
  __shared__ A sc[kMaxIter];
  const int m = st->m;
  if (threadIdx.x < (unsigned)m) sc[threadIdx.x] = st->beta[0] * st->s[threadIdx.x];
  __syncthreads();
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x)
    y[i] = lz_combine_at<T, A>(V, ld, sc, m, i);
}

// ------------------------------------------------------------- vectors
// Caller-order n x 3 -> sorted (x, y, z, 0).
template <typename T>
__global__ void k_gather3(const T *__restrict__ in, const int *__restrict__ perm, typename vec4<T>::type *__restrict__ out,
                          int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  typename vec4<T>::type v;
  v.x = in[3 * i];
  v.y = in[3 * i + 1];
  v.z = in[3 * i + 2];
  v.w = T(0);
  out[s] = v;
}

// Caller-order n x 3 (or none) -> sorted (x, y, z, 0), plus a sorted
// vector `add` (or none).
template <typename T>
__global__ void k_gather3_add(const T *__restrict__ in, const int *__restrict__ perm,
                              const typename vec4<T>::type *__restrict__ add, typename vec4<T>::type *__restrict__ out,
                              int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  typename vec4<T>::type v;
  v.x = v.y = v.z = v.w = T(0);
  if (in) {
    const int i = perm[s];
    v.x = in[3 * i];
    v.y = in[3 * i + 1];
    v.z = in[3 * i + 2];
  }
  if (add) {
    const auto a = add[s];
    v.x += a.x;
    v.y += a.y;
    v.z += a.z;
  }
  out[s] = v;
}

// x += dx over len scalars (caller order, the Euler-Maruyama update).
template <typename T> __global__ void k_advance(T *__restrict__ x, const T *__restrict__ dx, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) x[i] += dx[i];
}

// out[perm[s]] = cr * yr[s] + dt * ur[s] + wv[s]   (null terms omitted;
// sorted inputs are (x, y, z, 0), the output is caller-order n x 3)
template <typename T>
__device__ __forceinline__ void finalize_at(const int *__restrict__ perm, const typename vec4<T>::type *__restrict__ yr,
                                            T cr, const typename vec4<T>::type *__restrict__ ur, T dt,
                                            const typename vec4<T>::type *__restrict__ wv, T *__restrict__ out, int n,
                                            int s) {
  if (s >= n) return;
  const int i = perm[s];
  T x = 0, y = 0, z = 0;
  if (yr) {
    const auto a = yr[s];
    x += cr * a.x;
    y += cr * a.y;
    z += cr * a.z;
  }
  if (ur) {
    const auto a = ur[s];
    x += dt * a.x;
    y += dt * a.y;
    z += dt * a.z;
  }
  if (wv) {
    const auto a = wv[s];
    x += a.x;
    y += a.y;
    z += a.z;
  }
  out[3 * i] = x;
  out[3 * i + 1] = y;
  out[3 * i + 2] = z;
}

template <typename T>
__global__ void k_finalize(const int *__restrict__ perm, const typename vec4<T>::type *__restrict__ yr, T cr,
                           const typename vec4<T>::type *__restrict__ ur, T dt,
                           const typename vec4<T>::type *__restrict__ wv, T *__restrict__ out, int n) {
  finalize_at<T>(perm, yr, cr, ur, dt, wv, out, n, blockIdx.x * blockDim.x + threadIdx.x);
}

// ------------------------------------------------ Philox noise for z1
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t lo0 = 0xD2E7470EE14C6C93ull * c[0], hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c[0]);
    const uint64_t lo1 = 0xCA5A826395121157ull * c[2], hi1 = __umul64hi(0xCA5A826395121157ull, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

template <typename T> __device__ __forceinline__ void box_muller(uint64_t wa, uint64_t wb, T &na, T &nb);
template <> __device__ __forceinline__ void box_muller<double>(uint64_t wa, uint64_t wb, double &na, double &nb) {
  const double ua = ((double)(wa >> 11) + 0.5) * 0x1.0p-53;
  const double ub = ((double)(wb >> 11) + 0.5) * 0x1.0p-53;
  const double rho = sqrt(-2.0 * log(ua));
  double sn, cs;
  sincospi(2.0 * ub, &sn, &cs);
  na = rho * cs;
  nb = rho * sn;
}
template <> __device__ __forceinline__ void box_muller<float>(uint64_t wa, uint64_t wb, float &na, float &nb) {
  const float ua = ((float)(uint32_t)(wa >> 40) + 0.5f) * 0x1.0p-24f;
  const float ub = ((float)(uint32_t)(wb >> 40) + 0.5f) * 0x1.0p-24f;
  const float rho = sqrtf(-2.0f * logf(ua));
  float sn, cs;
  sincospif(2.0f * ub, &sn, &cs);
  na = rho * cs;
  nb = rho * sn;
}

// z1 is defined in caller order: Philox block b (key (seed, 0), counter
// (b, sample)) gives elements 4b .. 4b+3 of the 3n vector.  It is written
// straight into sorted order: sorted particle s (caller index i = perm[s])
// takes elements 3i .. 3i+2, i.e. the normals of block (3i) >> 2 and, when
// they straddle, of the next.
template <typename T>
__device__ __forceinline__ void real_noise_at(const int *__restrict__ perm, int n, uint64_t seed, uint64_t sample,
                                              typename vec4<T>::type *__restrict__ z, const uint64_t *__restrict__ rng,
                                              int s) {
  if (s >= n) return;
  if (rng) {
    // key and counter from device memory (a graph replayed per step)
    seed = rng[0];
    sample = rng[1];
  }
  const uint64_t e0 = 3ull * (uint64_t)perm[s];
  const uint64_t b0 = e0 >> 2;
  const int off = (int)(e0 & 3);
  T v[8];
  {
    uint64_t c[4] = {b0, sample, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    box_muller<T>(c[0], c[1], v[0], v[1]);
    box_muller<T>(c[2], c[3], v[2], v[3]);
  }
  if (off >= 2) {
    uint64_t c[4] = {b0 + 1, sample, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    box_muller<T>(c[0], c[1], v[4], v[5]);
    box_muller<T>(c[2], c[3], v[6], v[7]);
  }
  typename vec4<T>::type o;
  o.x = off == 0 ? v[0] : (off == 1 ? v[1] : (off == 2 ? v[2] : v[3]));
  o.y = off == 0 ? v[1] : (off == 1 ? v[2] : (off == 2 ? v[3] : v[4]));
  o.z = off == 0 ? v[2] : (off == 1 ? v[3] : (off == 2 ? v[4] : v[5]));
  o.w = T(0);
  z[s] = o;
}

template <typename T>
__global__ void k_real_noise_sorted(const int *__restrict__ perm, int n, uint64_t seed, uint64_t sample,
                                    typename vec4<T>::type *__restrict__ z, const uint64_t *__restrict__ rng) {
  real_noise_at<T>(perm, n, seed, sample, z, rng, blockIdx.x * blockDim.x + threadIdx.x);
}

// ----------------------------------------------------------- launchers
static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

__global__ void k_zero_words(uint32_t *__restrict__ p, size_t nw) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

void launch_zero_words(hipStream_t s, void *p, size_t nwords) {
  if (!nwords) return;
  const size_t b = (nwords + 255) / 256;
  k_zero_words<<<(int)(b < 4096 ? b : 4096), 256, 0, s>>>((uint32_t *)p, nwords);
}

// a[0 .. na) = 0 and b[0 .. nb) = 0.
__global__ void k_zero_i32(int *__restrict__ a, int na, int *__restrict__ b, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) a[i] = 0;
  else if (i - na < nb) b[i - na] = 0;
}

template <typename T>
void launch_bin(pse_ctx *c, const void *pos) {
  using T4 = typename vec4<T>::type;
  const int n = c->n;
  const T L = (T)c->d.L, invL = (T)(1.0 / c->d.L), inv_cs = (T)(1.0 / c->d.cs);
  ProfScope ps(c, PSE_STAGE_BIN);
  // a fill kernel rather than a memset: the same code runs under graph capture
  k_zero_i32<<<nblk(c->ncell + 8, 256), 256, 0, c->stream>>>(c->cell_count, c->ncell, c->flags, 8);
  // cell_of holds the cells [0, n) and the slots [n, 2n); cell_count the
  // counts [0, ncell) and the tile sums of the scan after them
  k_wrap_bin<T><<<nblk(n, 256), 256, 0, c->stream>>>((const T *)pos, n, L, invL, inv_cs, c->d.nc, (T4 *)c->pos_w,
                                                     c->cell_of, c->cell_of + n, c->cell_count, c->flags);
  const int ntiles = nblk(c->ncell, kScanTile);
  k_scan_tiles<<<ntiles, kScanNT, 0, c->stream>>>(c->cell_count, c->ncell, c->cell_count + c->ncell);
  k_scan_apply<<<ntiles, kScanNT, 0, c->stream>>>(c->cell_count, c->cell_count + c->ncell, c->ncell, c->cell_start);
  k_scatter<<<nblk(n, 256), 256, 0, c->stream>>>(c->cell_of, c->cell_of + n, c->cell_start, c->perm, n);
  k_cell_sort<T4><<<nblk(c->ncell, 4), 256, 0, c->stream>>>(c->cell_start, c->perm, c->ncell, (const T4 *)c->pos_w,
                                                           (T4 *)c->pos_s);
}

template <typename T>
void launch_nbr(pse_ctx *c) {
  using T4 = typename vec4<T>::type;
  const int n = c->n;
  const T L = (T)c->d.L, invL = (T)(1.0 / c->d.L), inv_cs = (T)(1.0 / c->d.cs);
  const T rc2 = (T)(c->p.rcut * c->p.rcut);
  ProfScope ps(c, PSE_STAGE_NBR);
  const T inv_mu0 = (T)(1.0 / c->d.mu0), fself = (T)(c->d.self_r / c->d.mu0), a = (T)c->p.a,
          inv_rc = (T)(1.0 / c->p.rcut);
  const bool rep = c->rep_k > 0;
  auto go = [&](auto kern, auto fg) {
    kern<<<nblk(n, 128), 128, 0, c->stream>>>((const T4 *)c->pos_s, c->cell_start, n, c->d.nc, L, invL, inv_cs, rc2,
                                              c->nbr, c->nbr_cnt, c->nbr_cap, c->flags, fg, inv_mu0, fself, a, inv_rc,
                                              c->pc_feat, (T)c->rep_k, (T4 *)c->vbuf[kRepBuf]);
  };
  if constexpr (sizeof(T) == 8) {
    const FGExact fg{c->series, c->p.xi, c->p.a, c->d.mu0, c->small_r2};
    if (c->pc_on) rep ? go(k_nbr_build<double, true, FGExact, true>, fg) : go(k_nbr_build<double, true, FGExact>, fg);
    else rep ? go(k_nbr_build<double, false, FGExact, true>, fg) : go(k_nbr_build<double, false, FGExact>, fg);
  } else {
    const FGTable fg{c->table, (float)(kTableK / c->p.rcut)};
    if (c->pc_on) rep ? go(k_nbr_build<float, true, FGTable, true>, fg) : go(k_nbr_build<float, true, FGTable>, fg);
    else rep ? go(k_nbr_build<float, false, FGTable, true>, fg) : go(k_nbr_build<float, false, FGTable>, fg);
  }
}

static int lds_nblocks(int nc, int B) {
  const int nb = (nc + B - 1) / B;
  return nb * nb * nb;
}

// f(std::integral_constant<int, B>) for the block edge B = 1 ... 4.
template <typename F> static void with_block_edge(int B, F f) {
  switch (B) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

void launch_halo_size(pse_ctx *c, int B) {
  ProfScope ps(c, PSE_STAGE_NBR);
  const int nblocks = lds_nblocks(c->d.nc, B);
  with_block_edge(B, [&](auto b) {
    constexpr int BE = decltype(b)::value;
    k_halo_size<BE><<<nblk(64L * nblocks, 256), 256, 0, c->stream>>>(c->cell_start, c->d.nc, c->flags);
  });
}

// Dynamic LDS above 64 KB needs a per-kernel attribute.  It is set once per
// kernel, to everything the CU's LDS leaves beside the kernel's static LDS,
// so that launches from several host threads (batches) with different halo
// sizes never lower it under one another.
template <typename K> static void allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return;
  static std::mutex mu;
  static std::unordered_set<const void *> done;
  const void *k = reinterpret_cast<const void *>(kernel);
  std::lock_guard<std::mutex> lock(mu);
  if (!done.insert(k).second) return;
  hipFuncAttributes fa{};
  const size_t stat = hipFuncGetAttributes(&fa, k) == hipSuccess ? fa.sharedSizeBytes : 32 * 1024;
  (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsPerCU - stat));
}

void launch_nbr_lds(pse_ctx *c) {
  ProfScope ps(c, PSE_STAGE_NBR);
  const size_t smem = sizeof(float3) * (size_t)(c->hcap + 3);  // 3 slots read past the last cell
  const float L = (float)c->d.L, invL = (float)(1.0 / c->d.L), rc2 = (float)(c->p.rcut * c->p.rcut);
  auto *nb = (uint16_t *)c->nbr;
  const bool unwrap = c->d.nc >= c->lds_B + 3;
  auto go = [&](auto kern) {
    allow_lds(kern, smem);
    kern<<<c->lds_blocks, 512, smem, c->stream>>>((const float4 *)c->pos_s, c->cell_start, c->d.nc, (float)c->d.cs,
                                                  c->n, L, invL, rc2, nb, c->nbr_cnt, c->nbr_cap, c->flags,
                                                  (float)(2.0 * c->p.a), (float)c->rep_k, (float4 *)c->vbuf[kRepBuf],
                                                  c->hcap);
  };
  const bool rep = c->rep_k > 0;
  with_block_edge(c->lds_B, [&](auto b) {
    constexpr int BE = decltype(b)::value;
    if (rep) {
      if (unwrap) go(k_nbr_lds<BE, true, true>);
      else go(k_nbr_lds<BE, false, true>);
    } else {
      if (unwrap) go(k_nbr_lds<BE, true>);
      else go(k_nbr_lds<BE, false>);
    }
  });
}

void launch_nbr_batch(hipStream_t s, const NbrRep *reps, const NbrGroup *groups, int ngroups) {
  for (int g = 0; g < ngroups; ++g) {
    const NbrGroup &gr = groups[g];
    with_block_edge(gr.B, [&](auto b) {
      constexpr int BE = decltype(b)::value;
      auto go = [&](auto kern) {
        allow_lds(kern, gr.smem);
        kern<<<gr.nblk, 512, gr.smem, s>>>(reps, gr.pmap);
      };
      if (gr.unwrap) go(k_nbr_lds_batch<BE, true>);
      else go(k_nbr_lds_batch<BE, false>);
    });
  }
}

// Preconditioner features on the LDS path, from the list and the staged halo.
void launch_feat_lds(pse_ctx *c) {
  ProfScope ps(c, PSE_STAGE_PRECOND);
  const size_t smem = sizeof(float4) * (size_t)c->hcap;
  const float L = (float)c->d.L, invL = (float)(1.0 / c->d.L);
  const bool unwrap = c->d.nc >= c->lds_B + 3;
  const float inv_mu0 = (float)(1.0 / c->d.mu0), fself = (float)(c->d.self_r / c->d.mu0);
  const float near2 = (float)(20.25 * c->p.a * c->p.a);  // r < 4.5a
  auto go = [&](auto kern) {
    allow_lds(kern, smem);
    kern<<<c->lds_blocks, kFeatNT, smem, c->stream>>>((const float4 *)c->pos_s, c->cell_start, c->d.nc,
                                                     (float)c->d.cs, c->n, L, invL, (const uint16_t *)c->nbr, c->nbr_cnt,
                                                  (const float2 *)c->table, (float)(kTableK / c->p.rcut), inv_mu0,
                                                  fself, (float)c->p.a, near2, c->pc_feat, c->hcap, c->flags + 7);
  };
  with_block_edge(c->lds_B, [&](auto b) {
    constexpr int BE = decltype(b)::value;
    if (unwrap) go(k_feat_lds<BE, true>);
    else go(k_feat_lds<BE, false>);
  });
}

template <typename A, bool LZ, bool PC = false>
static void spmv_lds(pse_ctx *c, const float4 *src, float4 *out, float4 *vm_out, LzState<A> *st,
                     const float4 *rsrc = nullptr) {
  const size_t smem = (sizeof(float4) + sizeof(float2)) * (size_t)c->hcap;
  const float L = (float)c->d.L, invL = (float)(1.0 / c->d.L);
  const auto *nb = (const uint16_t *)c->nbr;
  const float inv_dr = (float)(kTableK / c->p.rcut), self_r = (float)c->d.self_r;
  const bool unwrap = c->d.nc >= c->lds_B + 3;
  auto go = [&](auto kernel) {
    allow_lds(kernel, smem);
    kernel<<<c->lds_blocks, 1024, smem, c->stream>>>((const float4 *)c->pos_s, src, c->cell_start, c->d.nc,
                                                      (float)c->d.cs, c->n, c->hcap, L, invL, nb, c->nbr_cnt,
                                                      c->table, inv_dr, self_r, 1.0f, out, vm_out, st,
                                                      c->flags + 7, (const float4 *)c->pc_P, rsrc);
  };
  auto pick = [&](auto g) {
    constexpr int G = decltype(g)::value;
    with_block_edge(c->lds_B, [&](auto b) {
      constexpr int BE = decltype(b)::value;
      if (unwrap) go(k_spmv_lds<BE, true, A, LZ, PC, G>);
      else go(k_spmv_lds<BE, false, A, LZ, PC, G>);
    });
  };
  // lanes per target: 3 built in (the best measured at phi = 0.3 with
  // r_c = 8a), 2 or 4 when pse_autotune found them faster
  if (c->tune_spmv_lanes == 2) pick(std::integral_constant<int, 2>{});
  else if (c->tune_spmv_lanes == 4) pick(std::integral_constant<int, 4>{});
  else pick(std::integral_constant<int, 3>{});
}

// The fused Lanczos product (5 of the 6 product launches of a sample) is
// timed: the Krylov state is initialised from the sorted positions as the
// start vector (finite, nonzero), so every trial is iteration 0 and writes
// alpha_0, the basis slot 0 and vbuf[5], scratch that every sample
// re-initialises or rewrites.
template <typename A> static pse_status autotune_spmv_impl(pse_ctx *c) {
  launch_lz_init<float, A>(c, c->pos_s);
  auto *st = (LzState<A> *)c->lz;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PSE_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PSE_ERR_HIP;
  }
  const int keep = c->tune_spmv_lanes;
  int best = 0;
  float tbest = 1e30f, t3 = 1e30f;
  for (int g : {3, 2, 4}) {
    c->tune_spmv_lanes = g;
    auto launch = [&] {
      spmv_lds<A, true>(c, (const float4 *)c->pos_s, (float4 *)c->vbuf[5], (float4 *)c->V, st);
    };
    launch();  // warm-up
    float t = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      float ms = 1e30f;
      if (hipEventRecord(e0, c->stream) != hipSuccess) break;
      launch();
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        break;
      t = ms < t ? ms : t;
    }
    if (g == 3) t3 = t;
    // another lane count replaces the built-in 3 only when it is faster by
    // more than the timing noise (3 %), so that the choice is stable
    if (g == 3 ? t < tbest : t < tbest && t < 0.97f * t3) {
      tbest = t;
      best = g;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const pse_status st_ = hipGetLastError() == hipSuccess ? PSE_OK : PSE_ERR_HIP;
  c->tune_spmv_lanes = st_ == PSE_OK && best ? best : keep;
  return st_;
}

pse_status autotune_spmv(pse_ctx *c, int32_t *lanes) {
  if (lanes) *lanes = 0;
  if (c->dbl || !c->lds_B) return PSE_OK;
  const uint32_t mask = c->prof_mask;
  c->prof_mask = 0;  // the trial launches are not stage time
  const pse_status st = c->acc_dbl ? autotune_spmv_impl<double>(c) : autotune_spmv_impl<float>(c);
  c->prof_mask = mask;
  if (lanes) *lanes = c->tune_spmv_lanes ? c->tune_spmv_lanes : 3;
  return st;
}

template <typename T, typename A>
void launch_spmv(pse_ctx *c, const void *src, void *out, bool lz, void *vm_out) {
  const int n = c->n;
  const int nb = nblk(n, 256);
  (void)lz;
  (void)vm_out;
  ProfScope ps(c, PSE_STAGE_SPMV);
  if constexpr (sizeof(T) == 4) {
    if (c->lds_B) {
      spmv_lds<A, false>(c, (const float4 *)src, (float4 *)out, nullptr, nullptr);
      return;
    }
  }
  if constexpr (sizeof(T) == 8) {
    k_spmv_exact<false><<<nb, 256, 0, c->stream>>>(
        (const double4 *)c->pos_s, c->nbr, c->nbr_cnt, n, c->d.L, 1.0 / c->d.L, c->series, c->p.xi, c->p.a, c->d.mu0,
        c->small_r2, c->d.self_r, (const double4 *)src, 1.0, (double4 *)out, nullptr, nullptr, nullptr, nullptr);
  } else {
    k_spmv_table<float, A, false><<<nb, 256, 0, c->stream>>>(
        (const float4 *)c->pos_s, c->nbr, c->nbr_cnt, n, (float)c->d.L, (float)(1.0 / c->d.L), c->table,
        (float)(kTableK / c->p.rcut), (float)c->d.self_r, (const float4 *)src, 1.0f, (float4 *)out, nullptr, nullptr,
        nullptr, nullptr);
  }
}

// Sorted particle vectors are (x, y, z, 0): the reductions and updates run
// over the flat 4n scalars (the zero lanes stay zero).
template <typename T, typename A>
void launch_lz_init(pse_ctx *c, const void *z) {
  const int len = 4 * c->n;
  ProfScope ps(c, PSE_STAGE_LANCZOS);
  k_norm2_partial<T, A><<<kRedBlock, 256, 0, c->stream>>>((const T *)z, len, (A *)c->partials);
  k_lz_init<A><<<1, 256, 0, c->stream>>>((const A *)c->partials, kRedBlock, (LzState<A> *)c->lz);
}

// One Lanczos iteration: SpMV (+alpha), update (+|w|^2 partials), check.
// src = z (m = 0) or the previous residual w.
template <typename T, typename A>
void launch_lz_iter(pse_ctx *c, int m, const void *z) {
  using T4 = typename vec4<T>::type;
  const int n = c->n, len = 4 * n;
  T4 *V = (T4 *)c->V;
  T4 *t = (T4 *)c->vbuf[2];
  T4 *w = (T4 *)c->vbuf[3];
  const T4 *src = m == 0 ? (const T4 *)z : w;
  const int nb = nblk(n, 256);
  auto *st = (LzState<A> *)c->lz;
  prof_begin(c, PSE_STAGE_SPMV);
  if constexpr (sizeof(T) == 8) {
    k_spmv_exact<true><<<nb, 256, 0, c->stream>>>((const double4 *)c->pos_s, c->nbr, c->nbr_cnt, n, c->d.L,
                                                   1.0 / c->d.L, c->series, c->p.xi, c->p.a, c->d.mu0, c->small_r2,
                                                   c->d.self_r, src, 1.0, t, V + (size_t)m * n, st,
                                                   (double *)c->partials, c->counter);
  } else if (c->lds_B) {
    spmv_lds<A, true>(c, src, t, V + (size_t)m * n, st);
  } else {
    k_spmv_table<float, A, true><<<nb, 256, 0, c->stream>>>(
        (const float4 *)c->pos_s, c->nbr, c->nbr_cnt, n, (float)c->d.L, (float)(1.0 / c->d.L), c->table,
        (float)(kTableK / c->p.rcut), (float)c->d.self_r, src, 1.0f, t, V + (size_t)m * n, st, (A *)c->partials,
        c->counter);
  }
  prof_end(c, PSE_STAGE_SPMV);
  const T4 *vprev = m > 0 ? V + (size_t)(m - 1) * n : V;
  ProfScope ps(c, PSE_STAGE_LANCZOS);
  if (sizeof(T) == 4 && c->lds_B) {
    // the LDS product leaves alpha_m to its own pass
    A *ap = (A *)c->partials + kRedBlock;
    k_lz_alpha_part<T, A><<<kRedBlock, 256, 0, c->stream>>>(t, V + (size_t)m * n, n, st, ap);
    k_lz_update<T, A><<<kRedBlock, 256, 0, c->stream>>>(t, V + (size_t)m * n, vprev, w, n, st, (A *)c->partials,
                                                        ap, kRedBlock);
  } else {
    k_lz_update<T, A><<<kRedBlock, 256, 0, c->stream>>>(t, V + (size_t)m * n, vprev, w, n, st, (A *)c->partials);
  }
  k_lz_check<A><<<1, 64, 0, c->stream>>>((const A *)c->partials, kRedBlock, st, (A)c->p.lanczos_tol,
                                         c->lz_maxit);
}

// Lanczos step on A = P M_r P^T: u = P^T r, t' = M_r u, then the basis
// vector, A v_m and alpha_m from t' (k_pc_post), then the usual update and
// check.  The product runs unconditionally; the other kernels skip once the
// iteration is done.
template <typename T, typename A>
void launch_lz_iter_pc(pse_ctx *c, int m, const void *z) {
  using T4 = typename vec4<T>::type;
  T4 *V = (T4 *)c->V;
  T4 *t = (T4 *)c->vbuf[2];
  T4 *w = (T4 *)c->vbuf[3];
  T4 *u = (T4 *)c->vbuf[8];
  T4 *tp = (T4 *)c->vbuf[9];
  const T4 *src = m == 0 ? (const T4 *)z : w;
  if constexpr (sizeof(T) == 4) {
    if (c->lds_B) {
      // u = P^T r comes from the previous update (from z at m = 0); P and
      // alpha_m are applied in the product's epilogue
      if (m == 0) {
        ProfScope ps(c, PSE_STAGE_PRECOND);
        launch_pc_pre<T, A>(c, src, u);
      }
      {
        ProfScope ps(c, PSE_STAGE_SPMV);
        spmv_lds<A, true, true>(c, (const float4 *)u, (float4 *)t, (float4 *)(V + (size_t)m * c->n),
                                (LzState<A> *)c->lz, (const float4 *)src);
      }
      ProfScope ps(c, PSE_STAGE_LANCZOS);
      const T4 *vprev = m > 0 ? V + (size_t)(m - 1) * c->n : V;
      A *ap = (A *)c->partials + kRedBlock;
      k_lz_alpha_part<T, A><<<kRedBlock, 256, 0, c->stream>>>(t, V + (size_t)m * c->n, c->n, (LzState<A> *)c->lz, ap);
      k_lz_update_pc<T, A><<<kRedBlock, 256, 0, c->stream>>>(t, V + (size_t)m * c->n, vprev, w, (const T *)c->pc_P,
                                                             u, c->n, (LzState<A> *)c->lz, (A *)c->partials, ap,
                                                             kRedBlock);
      k_lz_check<A><<<1, 64, 0, c->stream>>>((const A *)c->partials, kRedBlock, (LzState<A> *)c->lz,
                                             (A)c->p.lanczos_tol, c->lz_maxit);
      return;
    }
  }
  {
    ProfScope ps(c, PSE_STAGE_PRECOND);
    launch_pc_pre<T, A>(c, src, u);
  }
  launch_spmv<T, A>(c, u, tp, false, nullptr);
  ProfScope ps(c, PSE_STAGE_LANCZOS);
  launch_pc_post<T, A>(c, tp, src, t, V + (size_t)m * c->n);
  const T4 *vprev = m > 0 ? V + (size_t)(m - 1) * c->n : V;
  k_lz_update<T, A><<<kRedBlock, 256, 0, c->stream>>>(t, V + (size_t)m * c->n, vprev, w, c->n, (LzState<A> *)c->lz,
                                                      (A *)c->partials);
  k_lz_check<A><<<1, 64, 0, c->stream>>>((const A *)c->partials, kRedBlock, (LzState<A> *)c->lz,
                                         (A)c->p.lanczos_tol, c->lz_maxit);
}

// One iteration of the batched Krylov loop: the product of every group of
// systems sharing a block edge, halo form and lanes per target, then the
// vector kernels and the checks of all systems.
template <typename A>
void launch_lz_batch_iter(hipStream_t s, const LzRep<A> *reps, int nrep, const LzGroup *groups, int ngroups,
                          const int2 *vmap, int nvblk, int m) {
  for (int g = 0; g < ngroups; ++g) {
    const LzGroup &gr = groups[g];
    with_block_edge(gr.B, [&](auto b) {
      constexpr int BE = decltype(b)::value;
      auto go = [&](auto kernel) {
        allow_lds(kernel, gr.smem);
        kernel<<<gr.nblk, 1024, gr.smem, s>>>(reps, gr.pmap, m);
      };
      auto pick = [&](auto gl) {
        constexpr int GL = decltype(gl)::value;
        if (gr.unwrap) go(k_spmv_lds_batch<BE, true, A, GL>);
        else go(k_spmv_lds_batch<BE, false, A, GL>);
      };
      if (gr.G == 2) pick(std::integral_constant<int, 2>{});
      else if (gr.G == 4) pick(std::integral_constant<int, 4>{});
      else pick(std::integral_constant<int, 3>{});
    });
  }
  k_lz_alpha_batch<A><<<nvblk, 256, 0, s>>>(reps, vmap, m);
  k_lz_update_batch<A><<<nvblk, 256, 0, s>>>(reps, vmap, m);
  k_lz_check_batch<A><<<nrep, 64, 0, s>>>(reps);
}
__global__ void k_batch_status(const RepStatusSrc *__restrict__ src, int nrep, RepStatus *__restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrep) return;
  const RepStatusSrc q = src[r];
  RepStatus o;
  for (int k = 0; k < 8; ++k) o.flags[k] = q.flags[k];
  if (q.acc_dbl) {
    const auto *st = (const LzState<double> *)q.lz;
    o.m = st->m;
    o.done = st->done;
    o.converged = st->converged;
    o.nonfinite = st->nonfinite;
    o.rel_change = st->rel_change;
  } else {
    const auto *st = (const LzState<float> *)q.lz;
    o.m = st->m;
    o.done = st->done;
    o.converged = st->converged;
    o.nonfinite = st->nonfinite;
    o.rel_change = (double)st->rel_change;
  }
  out[r] = o;
}

void launch_batch_status(hipStream_t s, const RepStatusSrc *src, int nrep, RepStatus *out) {
  k_batch_status<<<(nrep + 63) / 64, 64, 0, s>>>(src, nrep, out);
}

// ------------------------------------------ fully batched systems
// The per-system kernels of a captured step (binning, noise, Krylov start,
// combination, final sum) for many systems in one launch each: the same
// bodies as the single-system kernels, the system and block from a map.
__global__ __launch_bounds__(256) void k_zero_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  const int i = rb.y * 256 + (int)threadIdx.x;
  if (i < r.ncell) r.cell_count[i] = 0;
  else if (i - r.ncell < 8) r.flags[i - r.ncell] = 0;
}
__global__ __launch_bounds__(256) void k_wrap_bin_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  wrap_bin_at<float>(r.pos_in, r.n, r.L, r.invL, r.inv_cs, r.nc, r.pos_w, r.cell_of, r.slot, r.cell_count, r.flags,
                     rb.y * 256 + (int)threadIdx.x);
}
__global__ __launch_bounds__(kScanNT) void k_scan_tiles_batch(const SampRep *__restrict__ reps,
                                                              const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  scan_tiles_at(r.cell_count, r.ncell, r.tile_sum, rb.y);
}
__global__ __launch_bounds__(kScanNT) void k_scan_apply_batch(const SampRep *__restrict__ reps,
                                                              const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  scan_apply_at(r.cell_count, r.tile_sum, r.ncell, r.cell_start, rb.y);
}
__global__ __launch_bounds__(256) void k_scatter_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  const int i = rb.y * 256 + (int)threadIdx.x;
  if (i < r.n) r.perm[r.cell_start[r.cell_of[i]] + r.slot[i]] = i;
}
__global__ __launch_bounds__(256) void k_cell_sort_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  cell_sort_at<float4>(r.cell_start, r.perm, r.ncell, r.pos_w, r.pos_s, rb.y * 4 + (int)(threadIdx.x >> 6));
}
__global__ __launch_bounds__(256) void k_noise_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  real_noise_at<float>(r.perm, r.n, 0ull, 0ull, r.z, r.rng, rb.y * 256 + (int)threadIdx.x);
}
template <typename A>
__global__ __launch_bounds__(256) void k_norm2_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  __shared__ A sh[16];
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  const float *zf = (const float *)r.z;
  A *part = (A *)r.partials;
  const int len = 4 * r.n, i = rb.y * 256 + (int)threadIdx.x;
  A v = 0;
  if (i < len) v += (A)zf[i] * (A)zf[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[rb.y] = v;
  if (rb.y == 0)
    for (int k = (len + 255) / 256 + (int)threadIdx.x; k < kRedBlock; k += 256) part[k] = A(0);
}
template <typename A>
__global__ __launch_bounds__(256) void k_lz_init_batch(const SampRep *__restrict__ reps) {
  const SampRep &r = reps[blockIdx.x];
  lz_init_body<A>((const A *)r.partials, kRedBlock, (LzState<A> *)r.st);
}
template <typename A>
__global__ __launch_bounds__(256) void k_combine_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  __shared__ A sc[kMaxIter];
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  const LzState<A> *st = (const LzState<A> *)r.st;
  const int m = st->m;
  if (threadIdx.x < (unsigned)m) sc[threadIdx.x] = st->beta[0] * st->s[threadIdx.x];
  __syncthreads();
  const int len = 4 * r.n, i = rb.y * 256 + (int)threadIdx.x;
  if (i < len) ((float *)r.yr)[i] = lz_combine_at<float, A>((const float *)r.V, (size_t)len, sc, m, i);
}
__global__ __launch_bounds__(256) void k_finalize_batch(const SampRep *__restrict__ reps, const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  finalize_at<float>(r.perm, r.yr, r.cr, r.f_in ? r.ur : nullptr, r.dt, r.wave, r.out, r.n,
                     rb.y * 256 + (int)threadIdx.x);
}
__global__ __launch_bounds__(256) void k_gather_forces_batch(const SampRep *__restrict__ reps,
                                                             const int2 *__restrict__ map) {
  const int2 rb = map[blockIdx.x];
  const SampRep &r = reps[rb.x];
  const int s = rb.y * 256 + (int)threadIdx.x;
  if (!r.f_in || s >= r.n) return;
  const int i = r.perm[s];
  float4 v;
  v.x = r.f_in[3 * i];
  v.y = r.f_in[3 * i + 1];
  v.z = r.f_in[3 * i + 2];
  v.w = 0.0f;
  r.f_s[s] = v;
}

void launch_samp_batch_bin(hipStream_t s, const SampRep *reps, const SampMaps &m) {
  k_zero_batch<<<m.nzero, 256, 0, s>>>(reps, m.zero);
  k_wrap_bin_batch<<<m.npart, 256, 0, s>>>(reps, m.part);
  k_scan_tiles_batch<<<m.ntile, kScanNT, 0, s>>>(reps, m.tile);
  k_scan_apply_batch<<<m.ntile, kScanNT, 0, s>>>(reps, m.tile);
  k_scatter_batch<<<m.npart, 256, 0, s>>>(reps, m.part);
  k_cell_sort_batch<<<m.ncell, 256, 0, s>>>(reps, m.cell);
}
void launch_samp_batch_forces(hipStream_t s, const SampRep *reps, const SampMaps &m) {
  k_gather_forces_batch<<<m.npart, 256, 0, s>>>(reps, m.part);
}
template <typename A> void launch_samp_batch_start(hipStream_t s, const SampRep *reps, const SampMaps &m) {
  k_noise_batch<<<m.npart, 256, 0, s>>>(reps, m.part);
  k_norm2_batch<A><<<m.nflat, 256, 0, s>>>(reps, m.flat);
  k_lz_init_batch<A><<<m.nrep, 256, 0, s>>>(reps);
}
template <typename A> void launch_samp_batch_end(hipStream_t s, const SampRep *reps, const SampMaps &m) {
  k_combine_batch<A><<<m.nflat, 256, 0, s>>>(reps, m.flat);
  k_finalize_batch<<<m.npart, 256, 0, s>>>(reps, m.part);
}
template void launch_samp_batch_start<float>(hipStream_t, const SampRep *, const SampMaps &);
template void launch_samp_batch_start<double>(hipStream_t, const SampRep *, const SampMaps &);
template void launch_samp_batch_end<float>(hipStream_t, const SampRep *, const SampMaps &);
template void launch_samp_batch_end<double>(hipStream_t, const SampRep *, const SampMaps &);

template <typename A>
void launch_lz_batch_plain(hipStream_t s, const LzRep<A> *reps, const LzGroup *groups, int ngroups) {
  for (int g = 0; g < ngroups; ++g) {
    const LzGroup &gr = groups[g];
    with_block_edge(gr.B, [&](auto b) {
      constexpr int BE = decltype(b)::value;
      auto go = [&](auto kernel) {
        allow_lds(kernel, gr.smem);
        kernel<<<gr.nblk, 1024, gr.smem, s>>>(reps, gr.pmap);
      };
      auto pick = [&](auto gl) {
        constexpr int GL = decltype(gl)::value;
        if (gr.unwrap) go(k_spmv_lds_batch_plain<BE, true, A, GL>);
        else go(k_spmv_lds_batch_plain<BE, false, A, GL>);
      };
      if (gr.G == 2) pick(std::integral_constant<int, 2>{});
      else if (gr.G == 4) pick(std::integral_constant<int, 4>{});
      else pick(std::integral_constant<int, 3>{});
    });
  }
}
template void launch_lz_batch_plain<float>(hipStream_t, const LzRep<float> *, const LzGroup *, int);
template void launch_lz_batch_plain<double>(hipStream_t, const LzRep<double> *, const LzGroup *, int);

template void launch_lz_batch_iter<float>(hipStream_t, const LzRep<float> *, int, const LzGroup *, int, const int2 *,
                                          int, int);
template void launch_lz_batch_iter<double>(hipStream_t, const LzRep<double> *, int, const LzGroup *, int,
                                           const int2 *, int, int);


template <typename T, typename A>
void launch_lz_combine(pse_ctx *c, void *y) {
  const int len = 4 * c->n;
  ProfScope ps(c, PSE_STAGE_LANCZOS);
  k_lz_combine<T, A><<<nblk(len, 256) < 2048 ? nblk(len, 256) : 2048, 256, 0, c->stream>>>(
      (const T *)c->V, (size_t)len, len, (const LzState<A> *)c->lz, (T *)y);
}

template <typename T>
void launch_gather3(pse_ctx *c, const void *in, void *out) {
  ProfScope ps(c, PSE_STAGE_OTHER);
  k_gather3<T><<<nblk(c->n, 256), 256, 0, c->stream>>>((const T *)in, c->perm, (typename vec4<T>::type *)out, c->n);
}

template <typename T> void launch_gather3_add(pse_ctx *c, const void *in, const void *add, void *out) {
  ProfScope ps(c, PSE_STAGE_OTHER);
  using T4 = typename vec4<T>::type;
  k_gather3_add<T><<<nblk(c->n, 256), 256, 0, c->stream>>>((const T *)in, c->perm, (const T4 *)add, (T4 *)out, c->n);
}

template <typename T> void launch_advance(pse_ctx *c, void *x, const void *dx) {
  ProfScope ps(c, PSE_STAGE_OTHER);
  k_advance<T><<<nblk(3 * (long)c->n, 256), 256, 0, c->stream>>>((T *)x, (const T *)dx, 3 * c->n);
}

template <typename T>
void launch_finalize(pse_ctx *c, const void *yr, double cr, const void *ur, double dt, const void *wv, void *out) {
  using T4 = typename vec4<T>::type;
  ProfScope ps(c, PSE_STAGE_OTHER);
  k_finalize<T><<<nblk(c->n, 256), 256, 0, c->stream>>>(c->perm, (const T4 *)yr, (T)cr, (const T4 *)ur, (T)dt,
                                                        (const T4 *)wv, (T *)out, c->n);
}

template <typename T>
void launch_real_noise(pse_ctx *c, void *z_sorted, uint64_t seed, uint64_t sample) {
  ProfScope ps(c, PSE_STAGE_NOISE);
  k_real_noise_sorted<T><<<nblk(c->n, 256), 256, 0, c->stream>>>(c->perm, c->n, seed, sample,
                                                                  (typename vec4<T>::type *)z_sorted, c->rng_dev);
}

#define INST_T(T)                                                                                  \
  template void launch_bin<T>(pse_ctx *, const void *);                                            \
  template void launch_nbr<T>(pse_ctx *);                                                          \
  template void launch_gather3<T>(pse_ctx *, const void *, void *);                                \
  template void launch_gather3_add<T>(pse_ctx *, const void *, const void *, void *);              \
  template void launch_advance<T>(pse_ctx *, void *, const void *);                                \
  template void launch_finalize<T>(pse_ctx *, const void *, double, const void *, double, const void *, void *); \
  template void launch_real_noise<T>(pse_ctx *, void *, uint64_t, uint64_t);
INST_T(float)
INST_T(double)
#define INST_TA(T, A)                                                           \
  template void launch_spmv<T, A>(pse_ctx *, const void *, void *, bool, void *); \
  template void launch_lz_init<T, A>(pse_ctx *, const void *);                  \
  template void launch_lz_iter<T, A>(pse_ctx *, int, const void *);             \
  template void launch_lz_iter_pc<T, A>(pse_ctx *, int, const void *);          \
  template void launch_lz_combine<T, A>(pse_ctx *, void *);
INST_TA(float, float)
INST_TA(float, double)
INST_TA(double, double)

}  // namespace pse
