// Grid-side kernels of the wave-space part (Sec. II B.2, Spectral Ewald):
// Gaussian spreading S and interpolation S^T (truncated to P^3 nodes), the 3D
// FFT as three 1D passes (z: real <-> half complex, then y and x strided), and
// the fused x pass that applies the split kernel B(k) (eq. Mwave), the
// projector (I - kk), the Gaussian deconvolution and draws the k-space noise.
//
// Grid layout (per component c, planar): real u[c][ix][iy][iz], z fastest.
// Spectrum in place of it: S[c][jx][jy][jz], jz < M/2 (the Nyquist plane
// jz = M/2 is never used: Nyquist modes are outside the k-set).
#include <type_traits>

#include "launch.hpp"

namespace pse {

template <typename T> using C = typename vec2<T>::type;
#define DI __device__ __forceinline__

template <typename T> DI C<T> cmk(T x, T y) {
  C<T> r;
  r.x = x;
  r.y = y;
  return r;
}
#define PSE_COMPLEX_OPS(CT, RT)                                                                     \
  DI CT cadd(CT a, CT b) { return cmk<RT>(a.x + b.x, a.y + b.y); }                                   \
  DI CT csub(CT a, CT b) { return cmk<RT>(a.x - b.x, a.y - b.y); }                                   \
  DI CT cmul(CT a, CT b) { return cmk<RT>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }           \
  DI CT cconj(CT a) { return cmk<RT>(a.x, -a.y); }                                                   \
  DI CT cscale(CT a, RT s) { return cmk<RT>(a.x * s, a.y * s); }
PSE_COMPLEX_OPS(float2, float)
PSE_COMPLEX_OPS(double2, double)

// ------------------------------------------------ compile-time twiddles
constexpr double kPiC = 3.14159265358979323846;
constexpr double ct_sin(double x) {
  while (x > kPiC) x -= 2 * kPiC;
  while (x < -kPiC) x += 2 * kPiC;
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos(double x) {
  while (x > kPiC) x -= 2 * kPiC;
  while (x < -kPiC) x += 2 * kPiC;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
template <int R> struct RegTw {
  double c[R / 2 > 0 ? R / 2 : 1], s[R / 2 > 0 ? R / 2 : 1];
  constexpr RegTw() : c(), s() {
    for (int k = 0; k < R / 2; ++k) {
      c[k] = ct_cos(2.0 * kPiC * k / R);
      s[k] = ct_sin(2.0 * kPiC * k / R);
    }
  }
};

// DFT of R points held in registers, natural order in and out.
// DIR = -1: X_k = sum x_n e^{-2 pi i nk/R};  DIR = +1: e^{+2 pi i nk/R}.
template <typename T, int R, int DIR> struct DFT {
  static DI void run(C<T> *v) {
    static_assert((R & (R - 1)) == 0, "power of two");
    C<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    DFT<T, R / 2, DIR>::run(e);
    DFT<T, R / 2, DIR>::run(o);
    constexpr RegTw<R> tw{};
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const T c = (T)tw.c[k], s = (T)(DIR * tw.s[k]);
      const C<T> t = cmk<T>(o[k].x * c - o[k].y * s, o[k].x * s + o[k].y * c);
      v[k] = cadd(e[k], t);
      v[k + R / 2] = csub(e[k], t);
    }
  }
};
template <typename T, int DIR> struct DFT<T, 1, DIR> {
  static DI void run(C<T> *) {}
};
template <typename T, int DIR> struct DFT<T, 2, DIR> {
  static DI void run(C<T> *v) {
    const C<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <typename T, int DIR> struct DFT<T, 3, DIR> {
  static DI void run(C<T> *v) {
    const T h = (T)0.86602540378443864676 * (T)DIR;  // DIR sqrt(3)/2
    const C<T> a = v[0], b = v[1], c = v[2];
    const C<T> t1 = cadd(b, c);
    const C<T> t2 = cmk<T>(a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y);
    const C<T> dbc = csub(b, c);
    const C<T> t3 = cmk<T>(-h * dbc.y, h * dbc.x);  // i DIR sqrt3/2 (b - c)
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

// One Stockham autosort stage of radix R on NCOLS columns of length N held
// in LDS as buf[n * NCOLS + col].  Ns = product of the radices already done.
// tw[k] = exp(-2 pi i k / N) (conjugated for DIR = +1).
template <typename T, int N, int R, int DIR, int NCOLS, int BLOCK>
DI void stockham_stage(C<T> *buf, const C<T> *tw, int Ns) {
  constexpr int NB = (N / R) * NCOLS;
  constexpr int BPT = (NB + BLOCK - 1) / BLOCK;
  C<T> v[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * BLOCK;
    if (b < NB) {
      const int col = b % NCOLS, j = b / NCOLS;
      const int jm = j % Ns;
      const int tstep = jm * (N / (Ns * R));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C<T> x = buf[(j + r * (N / R)) * NCOLS + col];
        if (r > 0) {
          C<T> w = tw[tstep * r];
          if (DIR > 0) w.y = -w.y;
          x = cmul(x, w);
        }
        v[q][r] = x;
      }
      DFT<T, R, DIR>::run(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * BLOCK;
    if (b < NB) {
      const int col = b % NCOLS, j = b / NCOLS;
      const int jm = j % Ns;
      const int idxD = (j / Ns) * Ns * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(idxD + r * Ns) * NCOLS + col] = v[q][r];
    }
  }
  __syncthreads();
}

// Radix plans (product = N).
template <int N> struct Plan;
template <> struct Plan<4> { static constexpr int n = 1, r[3] = {4, 1, 1}; };
template <> struct Plan<8> { static constexpr int n = 1, r[3] = {8, 1, 1}; };
template <> struct Plan<16> { static constexpr int n = 1, r[3] = {16, 1, 1}; };
template <> struct Plan<32> { static constexpr int n = 2, r[3] = {8, 4, 1}; };
template <> struct Plan<64> { static constexpr int n = 2, r[3] = {8, 8, 1}; };
template <> struct Plan<128> { static constexpr int n = 2, r[3] = {16, 8, 1}; };
template <> struct Plan<256> { static constexpr int n = 2, r[3] = {16, 16, 1}; };
template <> struct Plan<512> { static constexpr int n = 3, r[3] = {8, 8, 8}; };
// 3 x 2^k lengths (grids 24, 48, 96, 192, 384 and their half lengths)
template <> struct Plan<12> { static constexpr int n = 2, r[3] = {4, 3, 1}; };
template <> struct Plan<24> { static constexpr int n = 2, r[3] = {8, 3, 1}; };
template <> struct Plan<48> { static constexpr int n = 2, r[3] = {16, 3, 1}; };
template <> struct Plan<96> { static constexpr int n = 3, r[3] = {8, 4, 3}; };
template <> struct Plan<192> { static constexpr int n = 3, r[3] = {16, 4, 3}; };
template <> struct Plan<384> { static constexpr int n = 3, r[3] = {16, 8, 3}; };

template <typename T, int N, int DIR, int NCOLS, int BLOCK>
DI void fft_lds(C<T> *buf, const C<T> *tw) {
  using PL = Plan<N>;
  stockham_stage<T, N, PL::r[0], DIR, NCOLS, BLOCK>(buf, tw, 1);
  if constexpr (PL::n > 1) stockham_stage<T, N, PL::r[1], DIR, NCOLS, BLOCK>(buf, tw, PL::r[0]);
  if constexpr (PL::n > 2) stockham_stage<T, N, PL::r[2], DIR, NCOLS, BLOCK>(buf, tw, PL::r[0] * PL::r[1]);
}

// ------------------------------------------------------------- z pass
// Lines of M reals (= M/2 complex), contiguous.  Forward: real -> half
// spectrum jz = 0 .. M/2-1 (packing the real line as M/2 complex pairs,
// one M/2-point FFT, then the split into even/odd parts).  Inverse: the
// adjoint route, unnormalised, with the Nyquist value taken as 0 and the
// jz = 0 value as real.  In place or out of place (src -> dst).
template <typename T, int M, int DIR, int NL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fft_z(const C<T> *__restrict__ src, C<T> *__restrict__ dst,
                                                 const C<T> *__restrict__ twH_g, const C<T> *__restrict__ twM_g) {
  constexpr int H = M / 2;
  __shared__ C<T> buf[H * NL];
  __shared__ C<T> twH[H];
  __shared__ C<T> twM[H];
  for (int i = threadIdx.x; i < H; i += BLOCK) {
    twH[i] = twH_g[i];
    twM[i] = twM_g[i];
  }
  const size_t line0 = (size_t)blockIdx.x * NL;
  __syncthreads();
  for (int e = threadIdx.x; e < H * NL; e += BLOCK) {
    const int k = e % H, l = e / H;
    const C<T> *ln = src + (line0 + l) * H;
    if (DIR < 0) {
      buf[k * NL + l] = ln[k];
    } else {
      C<T> xk = ln[k];
      C<T> xm = k == 0 ? cmk<T>(T(0), T(0)) : ln[H - k];
      if (k == 0) xk.y = T(0);
      const C<T> s = cadd(xk, cconj(xm));
      const C<T> dd = csub(xk, cconj(xm));
      const C<T> w = cconj(twM[k]);  // e^{+2 pi i k / M}
      const C<T> t = cmul(w, dd);
      buf[k * NL + l] = cmk<T>(s.x - t.y, s.y + t.x);  // s + i t
    }
  }
  __syncthreads();
  fft_lds<T, H, DIR, NL, BLOCK>(buf, twH);
  for (int e = threadIdx.x; e < H * NL; e += BLOCK) {
    const int k = e % H, l = e / H;
    C<T> *ln = dst + (line0 + l) * H;
    if (DIR < 0) {
      const C<T> zk = buf[k * NL + l];
      const C<T> zm = cconj(buf[((H - k) % H) * NL + l]);
      const C<T> s = cadd(zk, zm);
      const C<T> dd = csub(zk, zm);
      const C<T> t = cmul(twM[k], dd);                              // w^k (Z_k - conj Z_{H-k})
      ln[k] = cmk<T>((T)0.5 * (s.x + t.y), (T)0.5 * (s.y - t.x));  // (s - i t)/2
    } else {
      ln[k] = buf[k * NL + l];
    }
  }
}

// z pass between the real grid (nodes [x][y][z], packed: c0, c1, c2 per
// node, no padding) and the planar half spectrum: the three component lines
// of NXY (x, y) columns are transformed together, so every node is read or
// written once, whole.  Forward (DIR < 0): real -> spectrum, from the grid
// that spreading writes; inverse (DIR > 0): spectrum -> real, into the grid
// that interpolation reads.  Same packing of the half spectrum as k_fft_z.
template <typename T, int M, int DIR, int NXY, int BLOCK>
DI void fft_z_aos_block(const void *__restrict__ src, void *__restrict__ dst, const C<T> *__restrict__ twH_g,
                        const C<T> *__restrict__ twM_g, int bx) {
  constexpr int H = M / 2, NL = 3 * NXY;
  __shared__ C<T> buf[H * NL];
  __shared__ C<T> twH[H];
  __shared__ C<T> twM[H];
  for (int i = threadIdx.x; i < H; i += BLOCK) {
    twH[i] = twH_g[i];
    twM[i] = twM_g[i];
  }
  const size_t xy0 = (size_t)bx * NXY;
  const size_t s_comp = (size_t)M * M;  // spectrum lines per component
  __syncthreads();
  if (DIR < 0) {
    // packed input: nodes 2k and 2k + 1 are six consecutive values
    // (c0, c1, c2, c0, c1, c2), read as three pairs
    for (int e = threadIdx.x; e < H * NXY; e += BLOCK) {
      const int k = e % H, l = e / H;
      const C<T> *ln = (const C<T> *)src + (xy0 + l) * (3 * H) + 3 * k;
      const C<T> p0 = ln[0], p1 = ln[1], p2 = ln[2];
      buf[k * NL + l] = cmk<T>(p0.x, p1.y);
      buf[k * NL + NXY + l] = cmk<T>(p0.y, p2.x);
      buf[k * NL + 2 * NXY + l] = cmk<T>(p1.x, p2.y);
    }
  } else {
    for (int e = threadIdx.x; e < H * NL; e += BLOCK) {
      const int k = e % H, l = e / H, cc = l / NXY, lxy = l % NXY;
      const C<T> *ln = (const C<T> *)src + (cc * s_comp + xy0 + lxy) * H;
      C<T> xk = ln[k];
      C<T> xm = k == 0 ? cmk<T>(T(0), T(0)) : ln[H - k];
      if (k == 0) xk.y = T(0);
      const C<T> sm = cadd(xk, cconj(xm));
      const C<T> dd = csub(xk, cconj(xm));
      const C<T> w = cconj(twM[k]);  // e^{+2 pi i k / M}
      const C<T> t = cmul(w, dd);
      buf[k * NL + l] = cmk<T>(sm.x - t.y, sm.y + t.x);  // s + i t
    }
  }
  __syncthreads();
  fft_lds<T, H, DIR, NL, BLOCK>(buf, twH);
  if (DIR < 0) {
    for (int e = threadIdx.x; e < H * NL; e += BLOCK) {
      const int k = e % H, l = e / H, cc = l / NXY, lxy = l % NXY;
      const C<T> zk = buf[k * NL + l];
      const C<T> zm = cconj(buf[((H - k) % H) * NL + l]);
      const C<T> sm = cadd(zk, zm);
      const C<T> dd = csub(zk, zm);
      const C<T> t = cmul(twM[k], dd);
      C<T> *ln = (C<T> *)dst + (cc * s_comp + xy0 + lxy) * H;
      ln[k] = cmk<T>((T)0.5 * (sm.x + t.y), (T)0.5 * (sm.y - t.x));
    }
  } else {
    // packed output: nodes 2k and 2k + 1 are six consecutive values
    // (c0, c1, c2, c0, c1, c2), written as three pairs
    for (int e = threadIdx.x; e < H * NXY; e += BLOCK) {
      const int k = e % H, l = e / H;
      const C<T> u0 = buf[k * NL + l], u1 = buf[k * NL + NXY + l], u2 = buf[k * NL + 2 * NXY + l];
      C<T> *ln = (C<T> *)dst + (xy0 + l) * (3 * H) + 3 * k;
      ln[0] = cmk<T>(u0.x, u1.x);
      ln[1] = cmk<T>(u2.x, u0.y);
      ln[2] = cmk<T>(u1.y, u2.y);
    }
  }
}

template <typename T, int M, int DIR, int NXY, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fft_z_aos(const void *__restrict__ src, void *__restrict__ dst,
                                                     const C<T> *__restrict__ twH_g, const C<T> *__restrict__ twM_g) {
  fft_z_aos_block<T, M, DIR, NXY, BLOCK>(src, dst, twH_g, twM_g, blockIdx.x);
}

// ------------------------------------------------------- strided passes
// 1D FFTs of length N along a strided axis for a tile of TZ consecutive jz
// columns and NCOMP components: element n of column (comp, col) is at
// data[(comp0+comp)*s_comp + o*s_outer + n*s_fft + z0 + col].
template <typename T, int N, int TZ, int NCOMP>
DI void tile_load(C<T> *buf, const C<T> *data, size_t base, size_t s_fft, size_t s_comp, int block) {
  constexpr int NCOLS = TZ * NCOMP;
  for (int e = threadIdx.x; e < N * NCOLS; e += block) {
    const int col = e % TZ, rest = e / TZ, cc = rest % NCOMP, nn = rest / NCOMP;
    buf[nn * NCOLS + cc * TZ + col] = data[base + cc * s_comp + (size_t)nn * s_fft + col];
  }
}
template <typename T, int N, int TZ, int NCOMP>
DI void tile_store(const C<T> *buf, C<T> *data, size_t base, size_t s_fft, size_t s_comp, int block) {
  constexpr int NCOLS = TZ * NCOMP;
  for (int e = threadIdx.x; e < N * NCOLS; e += block) {
    const int col = e % TZ, rest = e / TZ, cc = rest % NCOMP, nn = rest / NCOMP;
    data[base + cc * s_comp + (size_t)nn * s_fft + col] = buf[nn * NCOLS + cc * TZ + col];
  }
}

template <typename T, int N, int DIR, int TZ, int BLOCK>
DI void fft_strided_block(C<T> *__restrict__ data, size_t s_fft, size_t s_outer, size_t s_comp,
                          const C<T> *__restrict__ tw_g, int bx, int by, int bz) {
  __shared__ C<T> buf[N * TZ];
  __shared__ C<T> tw[N];
  for (int i = threadIdx.x; i < N; i += BLOCK) tw[i] = tw_g[i];
  const size_t base = (size_t)bz * s_comp + (size_t)by * s_outer + (size_t)bx * TZ;
  tile_load<T, N, TZ, 1>(buf, data, base, s_fft, s_comp, BLOCK);
  __syncthreads();
  fft_lds<T, N, DIR, TZ, BLOCK>(buf, tw);
  tile_store<T, N, TZ, 1>(buf, data, base, s_fft, s_comp, BLOCK);
}

template <typename T, int N, int DIR, int TZ, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fft_strided(C<T> *__restrict__ data, size_t s_fft, size_t s_outer,
                                                       size_t s_comp, const C<T> *__restrict__ tw_g) {
  fft_strided_block<T, N, DIR, TZ, BLOCK>(data, s_fft, s_outer, s_comp, tw_g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// --------------------------------------------------- Philox k-space noise
DI void philox4x64_10g(uint64_t c[4], uint64_t k0, uint64_t k1) {
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
// Box-Muller of one 64-bit pair (the precision's uniform construction)
template <typename T> DI C<T> zeta_from(uint64_t wa, uint64_t wb);
template <> DI C<double> zeta_from<double>(uint64_t wa, uint64_t wb) {
  const double ua = ((double)(wa >> 11) + 0.5) * 0x1.0p-53;
  const double ub = ((double)(wb >> 11) + 0.5) * 0x1.0p-53;
  const double rho = sqrt(-2.0 * log(ua)) * 0.70710678118654752440;
  double sn, cs;
  sincospi(2.0 * ub, &sn, &cs);
  return cmk<double>(rho * cs, rho * sn);
}
template <> DI C<float> zeta_from<float>(uint64_t wa, uint64_t wb) {
  const float ua = ((float)(uint32_t)(wa >> 40) + 0.5f) * 0x1.0p-24f;
  const float ub = ((float)(uint32_t)(wb >> 40) + 0.5f) * 0x1.0p-24f;
  const float rho = sqrtf(-2.0f * logf(ua)) * 0.70710678f;
  float sn, cs;
  sincospif(2.0f * ub, &sn, &cs);
  return cmk<float>(rho * cs, rho * sn);
}
// zeta of the even element 2q and the odd element 2q + 1 from one block
template <typename T> DI void zeta_pair(uint64_t e_even, uint64_t seed, uint64_t sample, C<T> &z0, C<T> &z1) {
  uint64_t c[4] = {e_even >> 1, sample, 0ull, 0ull};
  philox4x64_10g(c, seed, 1ull);
  z0 = zeta_from<T>(c[0], c[1]);
  z1 = zeta_from<T>(c[2], c[3]);
}
template <typename T> DI C<T> zeta_at(uint64_t e, uint64_t seed, uint64_t sample) {
  uint64_t c[4] = {e >> 1, sample, 0ull, 0ull};
  philox4x64_10g(c, seed, 1ull);
  return (e & 1) ? zeta_from<T>(c[2], c[3]) : zeta_from<T>(c[0], c[1]);
}

// ------------------------------------------------------ fused x pass
// For a tile (one jy, jz in [z0, z0+TZ)) and all jx:
//   [FORCES] forward x-FFT of the spread-force spectrum (z, y already done);
//   Uhat(k) = (I - kk/k^2) [ det_scale B ghat^-2 Fhat + sto_scale sqrt(B) ghat^-1 zeta ]
//   with B = sinc^2(ka) H(k, xi) / k^2 (eq. Mwave), ghat = exp(-k^2 sigma^2 / 2);
//   inverse x-FFT; store.  zeta: Philox (NOISE = 1) or the transformed grid
//   noise times M^{-3/2} (NOISE = 2).  k = 0 and Nyquist indices give 0.
// k-space scaling functions: FP64 takes the library's exponential and
// division; FP32 the hardware base-2 exponential (exponents <= 0) and
// reciprocal, each within about an ulp, far below the window's error
template <typename T> DI T ks_exp(T x) { return exp(x); }
template <typename T> DI T ks_rcp(T x) { return T(1) / x; }
template <> DI float ks_exp<float>(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
template <> DI float ks_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T, int M, int TZ, int BLOCK, bool FORCES, int NOISE>
DI void xpass_block(C<T> *__restrict__ data, const C<T> *__restrict__ specW, WaveCoef wc,
                    const C<T> *__restrict__ tw_g, int bx, int by, int gx, int gy) {
  constexpr int H = M / 2;
  constexpr int NCOLS = 3 * TZ;
  __shared__ C<T> buf[M * NCOLS];
  __shared__ C<T> tw[M];
  if (NOISE == 1 && wc.rng) {
    // key and counter from device memory (a graph replayed per step)
    wc.seed = wc.rng[0];
    wc.counter = wc.rng[1];
  }
  for (int i = threadIdx.x; i < M; i += BLOCK) tw[i] = tw_g[i];
  const size_t s_fft = (size_t)M * H, s_comp = (size_t)M * M * H;
  // adjacent z tiles share cache lines: keep them on one XCD
  const int lin = xcd_block(bx + by * gx, gx * gy);
  const int jy = lin / gx, z0 = (lin % gx) * TZ;
  const size_t base = (size_t)jy * H + z0;
  if (FORCES) {
    tile_load<T, M, TZ, 3>(buf, data, base, s_fft, s_comp, BLOCK);
    __syncthreads();
    fft_lds<T, M, -1, NCOLS, BLOCK>(buf, tw);
  } else {
    __syncthreads();
  }
  const T tpl = (T)wc.two_pi_over_L;
  const int sy = jy < H ? jy : jy - M;
  // two adjacent jz per thread: one Philox block gives the noise of both
  // (its elements 2q, 2q + 1; z0 and TZ are even)
  for (int e = threadIdx.x; e < M * (TZ / 2); e += BLOCK) {
    const int col0 = 2 * (e % (TZ / 2)), jx = e / (TZ / 2);
    const int sx = jx < H ? jx : jx - M;
    const bool nyq = (jx == H) || (jy == H);
    C<T> zeta[2][3];
    if (NOISE == 1 && !nyq) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        zeta_pair<T>((((uint64_t)c * M + jx) * M + jy) * H + z0 + col0, wc.seed, wc.counter, zeta[0][c], zeta[1][c]);
      if (z0 + col0 == 0 && !(sy > 0 || (sy == 0 && sx > 0))) {
        // jz = 0 outside the canonical half: the conjugate of the partner
        const int px = (M - jx) % M, py = (M - jy) % M;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          zeta[0][c] = cconj(zeta_at<T>((((uint64_t)c * M + px) * M + py) * H + 0, wc.seed, wc.counter));
      }
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int col = col0 + hh;
      const int jz = z0 + col;
      C<T> out[3] = {cmk<T>(0, 0), cmk<T>(0, 0), cmk<T>(0, 0)};
      if (!nyq && (sx | sy | jz)) {
        const T kx = tpl * sx, ky = tpl * sy, kz = tpl * jz;
        const T k2 = kx * kx + ky * ky + kz * kz;
        const T kk = sqrt(k2);
        const T ka = kk * (T)wc.a;
        const T sinc = sin(ka) * ks_rcp(ka);
        const T q = k2 * (T)wc.inv_4xi2;
        const T gs = k2 * (T)wc.sigma2;
        // e^{(gs - q) / 2}: its square scales the deterministic term
        const T eh = ks_exp(T(0.5) * (gs - q));
        C<T> v[3];
        for (int c = 0; c < 3; ++c) v[c] = cmk<T>(0, 0);
        if (FORCES) {
          const T det = (T)wc.det_scale * sinc * sinc * (T(1) + q) * ks_rcp(k2) * (eh * eh);
#pragma unroll
          for (int c = 0; c < 3; ++c) v[c] = cscale(buf[jx * NCOLS + c * TZ + col], det);
        }
        if (NOISE) {
          // B^{1/2} is the non-negative root: |sinc(ka)| (sinc changes sign for ka > pi)
          const T sto = (T)wc.sto_scale * fabs(sinc) * sqrt(T(1) + q) * ks_rcp(kk) * eh;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            C<T> z;
            if (NOISE == 1) z = zeta[hh][c];
            else if (jz == 0 && !(sy > 0 || (sy == 0 && sx > 0)))
              // jz = 0 outside the canonical half: the conjugate of the
              // partner -k (exact Hermitian symmetry for any input spectrum)
              z = cscale(cconj(specW[c * s_comp + (size_t)((M - jx) % M) * s_fft + (size_t)((M - jy) % M) * H]),
                         (T)wc.w_scale);
            else z = cscale(specW[c * s_comp + (size_t)jx * s_fft + base + col], (T)wc.w_scale);
            v[c] = cadd(v[c], cscale(z, sto));
          }
        }
        const C<T> kdv = cmk<T>(kx * v[0].x + ky * v[1].x + kz * v[2].x, kx * v[0].y + ky * v[1].y + kz * v[2].y);
        const T ik2 = T(1) / k2;
        out[0] = csub(v[0], cscale(kdv, kx * ik2));
        out[1] = csub(v[1], cscale(kdv, ky * ik2));
        out[2] = csub(v[2], cscale(kdv, kz * ik2));
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) buf[jx * NCOLS + c * TZ + col] = out[c];
    }
  }
  __syncthreads();
  fft_lds<T, M, +1, NCOLS, BLOCK>(buf, tw);
  tile_store<T, M, TZ, 3>(buf, data, base, s_fft, s_comp, BLOCK);
}

template <typename T, int M, int TZ, int BLOCK, bool FORCES, int NOISE>
__global__ __launch_bounds__(BLOCK) void k_xpass_fused(C<T> *__restrict__ data, const C<T> *__restrict__ specW,
                                                       WaveCoef wc, const C<T> *__restrict__ tw_g) {
  xpass_block<T, M, TZ, BLOCK, FORCES, NOISE>(data, specW, wc, tw_g, blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
}

// e^x for the Gaussian weights (x <= 0).  FP32: the hardware base-2
// exponential of x log2(e); the scaling adds a relative error of about
// |x| 2^-24, below 1e-6 over a support (|x| <= pi P / 2).
template <typename T> __device__ __forceinline__ T gauss_exp(T x) { return exp(x); }
template <> __device__ __forceinline__ float gauss_exp<float>(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}

// --------------------------------------------------- spread / interpolate
// One wavefront per (sorted) particle; lane -> (ix, iy) pairs of the P x P
// support columns, loop over the P z-nodes.  Support nodes along each axis:
// g = floor(x/h) - P/2 + 1 ... floor(x/h) + P/2 (wrapped mod M); weight
// = normalised Gaussian of standard deviation sigma (separable).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_spread(const typename vec4<T>::type *__restrict__ pos,
                                                const typename vec4<T>::type *__restrict__ f, int n, T *__restrict__ grid, int M, T h,
                                                T invh, T inv2s2, T norm) {
  // particles are in cell order: XCD-contiguous ranges keep the grid
  // nodes of neighbouring particles within one L2
  const int s = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (s >= n) return;
  const auto p = pos[s];
  const int bx = min((int)(p.x * invh), M - 1), by = min((int)(p.y * invh), M - 1), bz = min((int)(p.z * invh), M - 1);
  const int gx0 = bx - P / 2 + 1, gy0 = by - P / 2 + 1, gz0 = bz - P / 2 + 1;
  const auto fv = f[s];
  const T fx = fv.x, fy = fv.y, fz = fv.z;
  const size_t M3 = (size_t)M * M * M;
  T wz[P];
  int iz_m[P];
#pragma unroll
  for (int iz = 0; iz < P; ++iz) {
    const int gz = gz0 + iz;
    const T dz = (T)gz * h - p.z;
    wz[iz] = exp(-dz * dz * inv2s2);
    iz_m[iz] = (gz + M) % M;
  }
  for (int pr = lane; pr < P * P; pr += 64) {
    const int ix = pr / P, iy = pr % P;
    const int gx = gx0 + ix, gy = gy0 + iy;
    const T dx = (T)gx * h - p.x, dy = (T)gy * h - p.y;
    const T wxy = norm * exp(-(dx * dx + dy * dy) * inv2s2);
    const size_t row = ((size_t)((gx + M) % M) * M + (size_t)((gy + M) % M)) * M;
#pragma unroll
    for (int iz = 0; iz < P; ++iz) {
      const T w = wxy * wz[iz];
      const size_t g = row + iz_m[iz];
      unsafeAtomicAdd(&grid[3 * g], w * fx);  // packed nodes (c0, c1, c2)
      unsafeAtomicAdd(&grid[3 * g + 1], w * fy);
      unsafeAtomicAdd(&grid[3 * g + 2], w * fz);
    }
  }
}

// Sum of v over the 64 lanes of the wavefront, valid in lane 63: quad sums
// by quad permutes, row sums by row shifts (4, 8), then the row totals by
// the row-15 and row-31 broadcasts; disabled lanes contribute 0.
__device__ __forceinline__ float wave_sum_lane63(float v) {
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1, 0, 3, 2]
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2, 3, 0, 1]
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0x114, 0xF, 0xF, true);  // row_shr 4
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0x118, 0xF, 0xF, true);  // row_shr 8
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0x142, 0xA, 0xF, true);  // row_bcast 15 -> rows 1, 3
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0x143, 0xC, 0xF, true);  // row_bcast 31 -> rows 2, 3
  return v;
}

// Interpolation: one wavefront per particle (16 per workgroup, neighbours in
// cell order, so their support rows are shared in the L1); lane -> (iz, ix) of the support
// (consecutive lanes read consecutive z nodes of one grid row, one packed
// (c0, c1, c2) vector per node), loop over iy.
template <typename T, int P>
DI void interp_particle(const typename vec4<T>::type *__restrict__ pos, const T *__restrict__ grid, int n,
                        typename vec4<T>::type *__restrict__ out, int M, T h, T invh, T inv2s2, T norm_h3, int s) {
  const int lane = threadIdx.x & 63;
  if (s >= n) return;
  const auto p = pos[s];
  const int bx = __builtin_amdgcn_readfirstlane(min((int)(p.x * invh), M - 1));
  const int by = __builtin_amdgcn_readfirstlane(min((int)(p.y * invh), M - 1));
  const int bz = __builtin_amdgcn_readfirstlane(min((int)(p.z * invh), M - 1));
  const int gx0 = bx - P / 2 + 1, gy0 = by - P / 2 + 1, gz0 = bz - P / 2 + 1;
  // support nodes lie within one period of the grid: one conditional wrap
  auto wrapi = [M](int g) { return g < 0 ? g + M : (g >= M ? g - M : g); };
  struct P3 {
    T x, y, z;
  };
  auto *g3 = (const P3 *)grid;  // packed nodes (c0, c1, c2)
  unsigned ym[P];  // y offset of the node index, (y mod M) M
#pragma unroll
  for (int iy = 0; iy < P; ++iy) ym[iy] = (unsigned)wrapi(gy0 + iy) * (unsigned)M;
  T ax = 0, ay = 0, az = 0;
  if constexpr (std::is_same<T, float>::value) {
    // y weights: lane iy evaluates the weight of support row iy, and every
    // lane reads the P values as scalars
    static_assert(P <= 64, "one lane per support row");
    const float dyl = (float)(gy0 + lane % P) * h - p.y;
    const float wl = gauss_exp(-dyl * dyl * inv2s2);
    float wy[P];
#pragma unroll
    for (int iy = 0; iy < P; ++iy) wy[iy] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wl), iy));
    // buffer loads: the lane's (x, z) offset in the address register and
    // the row's y offset (a scalar) in the scalar offset; the grid's byte
    // size bounds every access
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)grid, 0, (int)(12u * (unsigned)M * M * M), 0x00020000);
    for (int pr = lane; pr < P * P; pr += 64) {
      const int iz = pr % P, ix = pr / P;
      const int gx = gx0 + ix, gz = gz0 + iz;
      const float dx = (float)gx * h - p.x, dz = (float)gz * h - p.z;
      const float wxz = gauss_exp(-(dx * dx + dz * dz) * inv2s2);
      const unsigned xz = (unsigned)wrapi(gx) * (unsigned)(M * M) + (unsigned)wrapi(gz);
      float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
      for (int iy = 0; iy < P; ++iy) {
        typedef unsigned u32x3 __attribute__((ext_vector_type(3)));
        const u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(rs, (int)(12u * xz), (int)(12u * ym[iy]), 0);
        sx = fmaf(wy[iy], __uint_as_float(v.x), sx);
        sy = fmaf(wy[iy], __uint_as_float(v.y), sy);
        sz = fmaf(wy[iy], __uint_as_float(v.z), sz);
      }
      ax = fmaf(wxz, sx, ax);
      ay = fmaf(wxz, sy, ay);
      az = fmaf(wxz, sz, az);
    }
    ax = wave_sum_lane63(ax);
    ay = wave_sum_lane63(ay);
    az = wave_sum_lane63(az);
  } else {
    // y weights of the equally spaced support nodes by the Gaussian
    // recurrence w_{k+1} = w_k r_k, r_{k+1} = r_k q (r_0 = e^{-(2 d_0 h + h^2) c},
    // q = e^{-2 h^2 c}, c = 1 / 2 sigma^2): three exponentials instead of P
    T wy[P];
    {
      const T dy0 = (T)gy0 * h - p.y;
      T w = gauss_exp(-dy0 * dy0 * inv2s2), r = gauss_exp(-(T(2) * dy0 + h) * h * inv2s2);
      const T q = gauss_exp(T(-2) * h * h * inv2s2);
#pragma unroll
      for (int iy = 0; iy < P; ++iy) {
        wy[iy] = w;
        w *= r;
        r *= q;
      }
    }
    for (int pr = lane; pr < P * P; pr += 64) {
      const int iz = pr % P, ix = pr / P;
      const int gx = gx0 + ix, gz = gz0 + iz;
      const T dx = (T)gx * h - p.x, dz = (T)gz * h - p.z;
      const T wxz = gauss_exp(-(dx * dx + dz * dz) * inv2s2);
      const unsigned xz = (unsigned)wrapi(gx) * (unsigned)(M * M) + (unsigned)wrapi(gz);
#pragma unroll
      for (int iy = 0; iy < P; ++iy) {
        const T w = wxz * wy[iy];
        const P3 v = g3[xz + ym[iy]];
        ax += w * v.x;
        ay += w * v.y;
        az += w * v.z;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ax += __shfl_xor(ax, off, 64);
      ay += __shfl_xor(ay, off, 64);
      az += __shfl_xor(az, off, 64);
    }
  }
  if (lane == (std::is_same<T, float>::value ? 63 : 0)) {
    typename vec4<T>::type o;
    o.x = norm_h3 * ax;
    o.y = norm_h3 * ay;
    o.z = norm_h3 * az;
    o.w = T(0);
    out[s] = o;
  }
}

template <typename T, int P>
__global__ __launch_bounds__(1024) void k_interp(const typename vec4<T>::type *__restrict__ pos,
                                                const T *__restrict__ grid, int n,
                                                typename vec4<T>::type *__restrict__ out, int M, T h,
                                                T invh, T inv2s2, T norm_h3) {
  // particles are in cell order: XCD-contiguous ranges keep the grid
  // nodes of neighbouring particles within one L2.  The particle is the
  // wavefront's: its index and support origin are scalar values.
  const int s = __builtin_amdgcn_readfirstlane((xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6);
  interp_particle<T, P>(pos, grid, n, out, M, h, invh, inv2s2, norm_h3, s);
}

// Spreading, owner computes, no atomics: one workgroup owns a tile of
// 8 x 8 x (8 NW) grid nodes; wavefront w owns the 8 x 8 x 8 sub-tile of z
// nodes [8w, 8w + 8), lane (lx, ly) one column of it, and accumulates its
// 8 nodes x 3 components in registers.  Particles whose P^3 support overlaps
// the tile are found from the linked cells covering the tile plus the
// support reach, one (x, y) cell column at a time (one candidate per thread,
// hits compacted into an LDS list).  For each listed particle every lane
// evaluates its own weights: the (x, y) factor with one exponential, the z
// factors of the wavefront's overlapping nodes by the Gaussian recurrence
// (two exponentials); no cross-lane reads.  Every node is written once, deterministically
// (fixed particle order), with no grid clear.  Needs M >= 2 max(8, 8 NW) + P
// so that the nearest periodic image of a base node relative to the tile is
// unique.
// lin: the tile (XCD-renumbered linear index over the gx x gy x gz tiles)
template <typename T, int P, int NW>
DI void spread_tile_block(const typename vec4<T>::type *__restrict__ pos, const typename vec4<T>::type *__restrict__ f,
                          const int *__restrict__ cell_start, int nc, T cs, int M, T h, T invh, T inv2s2, T norm,
                          T *__restrict__ grid, int lin, int gx, int gy) {
  constexpr int TX = 8, TY = 8, TZ = 8 * NW;
  constexpr int NT = 64 * NW;
  using T4 = typename vec4<T>::type;
  __shared__ T4 lpu[NT];  // image coordinate of the particle nearest the tile
  __shared__ T4 lf[NT];   // its force
  __shared__ int ls0[NT];  // first support node per axis (tile-local) + 64, 8 bits each
  __shared__ uint16_t sidx[NW][NT];  // per z slab: list entries whose support reaches it
  __shared__ int scnt[NW][NW];       // [slab][wavefront that listed them]
  const int t0x = (lin / (gx * gy)) * TX, t0y = ((lin / gx) % gy) * TY, t0z = (lin % gx) * TZ;
  const int t0[3] = {t0x, t0y, t0z}, tt[3] = {TX, TY, TZ};
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lx = lane >> 3, ly = lane & 7;
  const int zw = wave * 8;  // first z node (tile-local) of this wavefront
  const int half = M / 2;
  const T qz = gauss_exp(T(-2) * h * h * inv2s2);  // ratio step of the z-weight recurrence
  T acc[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[c][q] = T(0);
  // cell ranges holding every base node b in [t0 - P/2, t0 + T - 2 + P/2]
  int cl[3], cn[3];
  {
    const T inv_cs = T(1) / cs;
    for (int d = 0; d < 3; ++d) {
      const T lo = (T)(t0[d] - P / 2) * h, hi = (T)(t0[d] + tt[d] - 1 + P / 2) * h;
      const int a = (int)floor(lo * inv_cs - T(1e-4)), b = (int)floor(hi * inv_cs + T(1e-4));
      if (b - a + 1 >= nc) {
        cl[d] = 0;
        cn[d] = nc;
      } else {
        cl[d] = ((a % nc) + nc) % nc;
        cn[d] = b - a + 1;
      }
    }
  }
  for (int kx = 0; kx < cn[0]; ++kx) {
    const int cx = (cl[0] + kx) % nc;
    for (int ky = 0; ky < cn[1]; ++ky) {
      const int cy = (cl[1] + ky) % nc;
      const int base = (cx * nc + cy) * nc;
      // z cells cl[2] .. cl[2]+cn[2]-1 (mod nc): one or two contiguous runs
      const int z1 = cl[2] + cn[2] - 1;
      const int a1 = cell_start[base + cl[2]];
      const int b1 = cell_start[base + (z1 >= nc ? nc - 1 : z1) + 1];
      const int a2 = cell_start[base];
      const int b2 = z1 >= nc ? cell_start[base + (z1 - nc) + 1] : a2;
      const int n1 = b1 - a1, ntot = n1 + (b2 - a2);
      for (int c0 = 0; c0 < ntot; c0 += NT) {
        const int ci = c0 + (int)threadIdx.x;
        int t = 0, s0[3] = {0, 0, 0};
        T pu[3] = {T(0), T(0), T(0)};
        bool hit = false;
        if (ci < ntot) {
          t = ci < n1 ? a1 + ci : a2 + (ci - n1);
          const auto q = pos[t];
          const T qc[3] = {q.x, q.y, q.z};
          hit = true;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int b = min((int)(qc[d] * invh), M - 1);
            const int dd = ((b - t0[d] + half + M) % M) - half;  // nearest image, in [-M/2, M/2)
            s0[d] = dd - P / 2 + 1;                              // first support node, tile-local
            pu[d] = qc[d] + (T)(t0[d] + dd - b) * h;             // coordinate of that image
            hit = hit && (s0[d] <= tt[d] - 1) && (s0[d] + P - 1 >= 0);
          }
        }
        // ordered compaction: wavefront w packs its hits (ballot + lane
        // prefix) into list slots [64 w, 64 w + count), and every z slab
        // gets the indices of the entries whose support reaches it (at most
        // ceil((P + 7) / 8) slabs each); lists and summation orders follow
        // the candidates' order
        const unsigned long long below = (1ull << lane) - 1ull;
        const unsigned long long bal = __ballot(hit);
        const int e = 64 * wave + __popcll(bal & below);
        const int slo = s0[2] > 0 ? s0[2] >> 3 : 0, shi = min(NW - 1, (s0[2] + P - 1) >> 3);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const bool inw = hit && w >= slo && w <= shi;
          const unsigned long long bw = __ballot(inw);
          if (lane == 0) scnt[w][wave] = __popcll(bw);
          if (inw) sidx[w][64 * wave + __popcll(bw & below)] = (uint16_t)e;
        }
        if (hit) {
          T4 pv, fv = f[t];
          pv.x = pu[0];
          pv.y = pu[1];
          pv.z = pu[2];
          pv.w = T(0);
          fv.w = T(0);
          lpu[e] = pv;
          lf[e] = fv;
          ls0[e] = (s0[0] + 64) | ((s0[1] + 64) << 8) | ((s0[2] + 64) << 16);
        }
        __syncthreads();
        for (int from = 0; from < NW; ++from) {
        const int nf = scnt[wave][from];
        for (int k = 0; k < nf; ++k) {
          // the entry and its support offsets are the same for the whole
          // wavefront: scalar values, so the z tests below are scalar branches
          const int e = __builtin_amdgcn_readfirstlane(sidx[wave][64 * from + k]);
          const int sp = __builtin_amdgcn_readfirstlane(ls0[e]);
          const T4 pv = lpu[e], fv = lf[e];
          const int sx = (sp & 255) - 64, sy = ((sp >> 8) & 255) - 64, sz = ((sp >> 16) & 255) - 64;
          const int ix = lx - sx, iy = ly - sy;
          const bool in = ix >= 0 && ix < P && iy >= 0 && iy < P;
          const T dx = (T)(t0x + lx) * h - pv.x, dy = (T)(t0y + ly) * h - pv.y;
          const T wxy = in ? norm * gauss_exp(-(dx * dx + dy * dy) * inv2s2) : T(0);
          // z weights from the wavefront's first node inside the support
          // (uniform): w_{q+1} = w_q r_q, r_{q+1} = r_q qz
          const int q0 = max(0, sz - zw);
          const T dz0 = (T)(t0z + zw + q0) * h - pv.z;
          T wz = gauss_exp(-dz0 * dz0 * inv2s2), rz = gauss_exp(-(T(2) * dz0 + h) * h * inv2s2);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int iz = zw + q - sz;  // uniform across the wavefront
            if (iz >= 0 && iz < P) {
              const T w = wxy * wz;
              acc[0][q] += w * fv.x;
              acc[1][q] += w * fv.y;
              acc[2][q] += w * fv.z;
              wz *= rz;
              rz *= qz;
            }
          }
        }
        }
        __syncthreads();  // the list and the counts are rewritten next
      }
    }
  }
  const size_t col = ((size_t)(t0x + lx) * M + (t0y + ly)) * M + t0z + zw;
  // packed nodes (c0, c1, c2): the column's 8 nodes are 24 consecutive values
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    grid[3 * (col + q)] = acc[0][q];
    grid[3 * (col + q) + 1] = acc[1][q];
    grid[3 * (col + q) + 2] = acc[2][q];
  }
}

// Spreading as a contraction on the matrix cores (FP32).  The window is a
// product of one-dimensional Gaussians, so over a block of nodes the spread
// grid is
//   G_c[x][(y, z)] = sum_p wx_p(x) * (wy_p(y) wz_p(z) f_p,c),
// a product of a (16 x K) matrix of x weights with a (K x 16) matrix of
// per-particle (y, z) terms, K the particles whose support reaches the
// block.  One workgroup owns a tile of 16 x 8 x (8 NW) nodes and lists the
// particles overlapping it (from the linked cells, as the VALU form does);
// each of its 4 NW wavefronts owns a 16 x 4 x 4 sub-tile, keeps its own list
// of the particles that reach it (contiguous, in candidate order) and runs
// three v_mfma_f32_16x16x4_f32 (one per component) per four listed
// particles.  Operand layout: lane l holds A[x = l % 16][particle l / 16]
// and B[particle l / 16][column l % 16], column = 4 y + z; the result gives
// lane l rows 4 (l / 16) .. + 3 of column l % 16.  Weights outside a
// particle's P-node support along an axis are exactly zero, so every
// product outside the P^3 support adds +0.  The particle order, and with it
// the result, is fixed: no atomics, every node written once.  Needs M a
// multiple of 16 and 8 NW, M >= 2 max(16, 8 NW) + P.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
template <int P, int NW>
DI void spread_mfma_block(const float4 *__restrict__ pos, const float4 *__restrict__ f,
                          const int *__restrict__ cell_start, int nc, float cs, int M, float h, float invh,
                          float inv2s2, float norm, float *__restrict__ grid, int lin, int gx, int gy) {
  constexpr int TX = 16, TY = 8, TZ = 8 * NW;
  constexpr int NV = 4 * NW;  // wavefronts = sub-tiles: 2 along y, 2 NW along z
  constexpr int NT = 64 * NV;
  __shared__ float4 lpu[NT + 1];     // image coordinate of the particle nearest the tile
  __shared__ float4 lf[NT + 1];      // its force
  __shared__ int ls0[NT + 1];        // first support node per axis (tile-local) + 64, 8 bits each
  __shared__ uint16_t sidx[NV][NT];  // per sub-tile, contiguous over the listing wavefronts
  __shared__ int scnt[NV][NV];       // [sub-tile][wavefront that listed them]
  // the cell columns of one batch: start and length of the first z run,
  // start of the wrapped second run, inclusive prefix of the run lengths
  __shared__ int colA1[64], colN1[64], colA2[64], colEnd[64];
  const int t0x = (lin / (gx * gy)) * TX, t0y = ((lin / gx) % gy) * TY, t0z = (lin % gx) * TZ;
  const int t0[3] = {t0x, t0y, t0z}, tt[3] = {TX, TY, TZ};
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int y0 = 4 * (wave & 1), z0 = 4 * (wave >> 1);  // this wavefront's sub-tile (tile-local)
  const int half = M / 2;
  // operand coordinates: particle slot kp of a step; x row (A); column
  // (B) = node (y0 + yc, z0 + zc)
  const int kp = lane >> 4, col = lane & 15, yc = col >> 2, zc = col & 3;
  f32x4_t acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  if (threadIdx.x == 0) {  // the empty entry: support offsets -64 reach no node of the tile
    lpu[NT] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    lf[NT] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    ls0[NT] = 0;
  }
  int cl[3], cn[3];
  {
    const float inv_cs = 1.0f / cs;
    for (int d = 0; d < 3; ++d) {
      const float lo = (float)(t0[d] - P / 2) * h, hi = (float)(t0[d] + tt[d] - 1 + P / 2) * h;
      const int a = (int)floorf(lo * inv_cs - 1e-4f), b = (int)floorf(hi * inv_cs + 1e-4f);
      if (b - a + 1 >= nc) {
        cl[d] = 0;
        cn[d] = nc;
      } else {
        cl[d] = ((a % nc) + nc) % nc;
        cn[d] = b - a + 1;
      }
    }
  }
  // the (x, y) cell columns covering the tile, taken 64 at a time; their
  // z runs are concatenated so that each listing round takes NT candidates
  const int ncol = cn[0] * cn[1];
  for (int cb = 0; cb < ncol; cb += 64) {
    const int nb = min(64, ncol - cb);
    __syncthreads();  // the previous batch's columns are no longer read
    if (threadIdx.x < 64) {
      int a1 = 0, n1 = 0, a2 = 0, nt = 0;
      if ((int)threadIdx.x < nb) {
        const int cidx = cb + (int)threadIdx.x;
        const int cx = (cl[0] + cidx / cn[1]) % nc, cy = (cl[1] + cidx % cn[1]) % nc;
        const int base = (cx * nc + cy) * nc;
        // z cells cl[2] .. cl[2]+cn[2]-1 (mod nc): one or two contiguous runs
        const int z1 = cl[2] + cn[2] - 1;
        a1 = cell_start[base + cl[2]];
        const int b1 = cell_start[base + (z1 >= nc ? nc - 1 : z1) + 1];
        a2 = cell_start[base];
        const int b2 = z1 >= nc ? cell_start[base + (z1 - nc) + 1] : a2;
        n1 = b1 - a1;
        nt = n1 + (b2 - a2);
      }
      // inclusive prefix of the run lengths over the 64 lanes
      int pre = nt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(pre, o, 64);
        if (lane >= o) pre += v;
      }
      colA1[lane] = a1;
      colN1[lane] = n1;
      colA2[lane] = a2;
      colEnd[lane] = pre;
    }
    __syncthreads();
    const int ntot = colEnd[63];
    {
      for (int c0 = 0; c0 < ntot; c0 += NT) {
        const int ci = c0 + (int)threadIdx.x;
        int t = 0, s0[3] = {0, 0, 0};
        float pu[3] = {0.0f, 0.0f, 0.0f};
        bool hit = false;
        if (ci < ntot) {
          // the column holding candidate ci: the first with colEnd > ci
          int j = 0;
#pragma unroll
          for (int st = 32; st > 0; st >>= 1)
            if (colEnd[j + st - 1] <= ci) j += st;
          const int loc = ci - (j > 0 ? colEnd[j - 1] : 0);
          t = loc < colN1[j] ? colA1[j] + loc : colA2[j] + (loc - colN1[j]);
          const float4 q = pos[t];
          const float qc[3] = {q.x, q.y, q.z};
          hit = true;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int b = min((int)(qc[d] * invh), M - 1);
            // nearest image in [-M/2, M/2): b - t0 + M/2 lies in (-M/2, 3M/2)
            int r = b - t0[d] + half;
            r += r < 0 ? M : 0;
            r -= r >= M ? M : 0;
            const int dd = r - half;
            s0[d] = dd - P / 2 + 1;
            pu[d] = qc[d] + (float)(t0[d] + dd - b) * h;
            hit = hit && (s0[d] <= tt[d] - 1) && (s0[d] + P - 1 >= 0);
          }
        }
        const unsigned long long below = (1ull << lane) - 1ull;
        const unsigned long long bal = __ballot(hit);
        const int e = 64 * wave + __popcll(bal & below);
        // sub-tiles reached: y quarters ylo..yhi, z quarters zlo..zhi
        const int ylo = s0[1] > 0 ? s0[1] >> 2 : 0, yhi = min(1, (s0[1] + P - 1) >> 2);
        const int zlo = s0[2] > 0 ? s0[2] >> 2 : 0, zhi = min(2 * NW - 1, (s0[2] + P - 1) >> 2);
        unsigned long long bw[NV];
#pragma unroll
        for (int w = 0; w < NV; ++w) {
          const int qy = w & 1, qz = w >> 1;
          bw[w] = __ballot(hit && qy >= ylo && qy <= yhi && qz >= zlo && qz <= zhi);
          if (lane == 0) scnt[w][wave] = __popcll(bw[w]);
        }
        if (hit) {
          lpu[e] = make_float4(pu[0], pu[1], pu[2], 0.0f);
          const float4 fv = f[t];
          lf[e] = make_float4(fv.x, fv.y, fv.z, 0.0f);
          ls0[e] = (s0[0] + 64) | ((s0[1] + 64) << 8) | ((s0[2] + 64) << 16);
        }
        __syncthreads();
        // sub-tile lists in listing-wavefront order: lane w < NV sums the
        // counts of sub-tile w (its offset for this wavefront and its total)
        int offl = 0, totl = 0;
        if (lane < NV) {
#pragma unroll
          for (int from = 0; from < NV; ++from) {
            const int cw = scnt[lane][from];
            totl += cw;
            offl += from < wave ? cw : 0;
          }
        }
#pragma unroll
        for (int w = 0; w < NV; ++w) {
          const int off = __builtin_amdgcn_readlane(offl, w);
          if ((bw[w] >> lane) & 1ull) sidx[w][off + __popcll(bw[w] & below)] = (uint16_t)e;
        }
        const int total = __builtin_amdgcn_readlane(totl, wave);
        __syncthreads();
        // steps of four list entries; slots past the end read the empty
        // entry NT (zero force, support out of reach), so the loop is
        // branch-free.  The next step's entry is read while this one runs.
        auto entry = [&](int k) {
          const int idx = k + kp;
          const int ee = sidx[wave][min(idx, total - 1)];
          return idx < total ? ee : NT;
        };
        int ee_n = entry(0);
        float4 pv_n = lpu[ee_n], fv_n = lf[ee_n];
        int sp_n = ls0[ee_n];
        for (int k = 0; k < total; k += 4) {
          const float4 pv = pv_n, fv = fv_n;
          const int sp = sp_n;
          ee_n = entry(k + 4);
          pv_n = lpu[ee_n];
          fv_n = lf[ee_n];
          sp_n = ls0[ee_n];
          const int ix = col - ((sp & 255) - 64), iy = y0 + yc - (((sp >> 8) & 255) - 64),
                    iz = z0 + zc - (((sp >> 16) & 255) - 64);
          const float dx = (float)(t0x + col) * h - pv.x, dy = (float)(t0y + y0 + yc) * h - pv.y,
                      dz = (float)(t0z + z0 + zc) * h - pv.z;
          const float ex = norm * gauss_exp(-dx * dx * inv2s2), eyz = gauss_exp(-(dy * dy + dz * dz) * inv2s2);
          const float wx = (unsigned)ix < (unsigned)P ? ex : 0.0f;
          const float wyz = ((unsigned)iy < (unsigned)P && (unsigned)iz < (unsigned)P) ? eyz : 0.0f;
          acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx, wyz * fv.x, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx, wyz * fv.y, acc[1], 0, 0, 0);
          acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx, wyz * fv.z, acc[2], 0, 0, 0);
        }
        __syncthreads();  // the list and the counts are rewritten next
      }
    }
  }
  // packed nodes (c0, c1, c2)
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const size_t node = ((size_t)(t0x + 4 * kp + v) * M + (t0y + y0 + yc)) * M + t0z + z0 + zc;
    grid[3 * node] = acc[0][v];
    grid[3 * node + 1] = acc[1][v];
    grid[3 * node + 2] = acc[2][v];
  }
}

template <int P, int NW>
__global__ __launch_bounds__(256 * NW) void k_spread_mfma(const float4 *__restrict__ pos,
                                                          const float4 *__restrict__ f,
                                                          const int *__restrict__ cell_start, int nc, float cs, int M,
                                                          float h, float invh, float inv2s2, float norm,
                                                          float *__restrict__ grid) {
  const int lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            gridDim.x * gridDim.y * gridDim.z);
  spread_mfma_block<P, NW>(pos, f, cell_start, nc, cs, M, h, invh, inv2s2, norm, grid, lin, gridDim.x, gridDim.y);
}

template <typename T, int P, int NW>
__global__ __launch_bounds__(64 * NW) void k_spread_tile(const typename vec4<T>::type *__restrict__ pos,
                                                         const typename vec4<T>::type *__restrict__ f,
                                                         const int *__restrict__ cell_start, int nc, T cs, int M,
                                                         T h, T invh, T inv2s2, T norm, T *__restrict__ grid) {
  // neighbouring tiles read the same cells: keep them on one XCD
  const int lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            gridDim.x * gridDim.y * gridDim.z);
  spread_tile_block<T, P, NW>(pos, f, cell_start, nc, cs, M, h, invh, inv2s2, norm, grid, lin, gridDim.x, gridDim.y);
}

// ----------------------------------------------------------- launchers
// Largest divisor of n (a multiple of `step`) that is at most lim (at least step).
constexpr int div_at_most(int n, int lim, int step) {
  int best = step;
  for (int d = step; d <= n && d <= lim; d += step)
    if (n % d == 0) best = d;
  return best;
}
constexpr int pow2_at_most(int lim) {
  int p = 1;
  while (2 * p <= lim) p *= 2;
  return p;
}
template <typename T, int M> struct GridCfg {
  // fused x pass holds 3 components: TZ columns x M x 3 complex in LDS
  // (24 KB at M = 256 FP32; at least 4 columns, 32-byte row segments: at
  // 512^3 4 columns beat 2, 2.1 against 2.6 ms); TZ divides M/2 and is even
  static constexpr int TZ = (sizeof(T) == 4) ? div_at_most(M / 2, (1024 / M) > 4 ? (1024 / M) : 4, 2)
                                             : div_at_most(M / 2, (1024 / M) > 2 ? (1024 / M) : 2, 2);
  // strided y pass: TZ1 columns x M complex in LDS (32 KB at M = 256 FP32:
  // four workgroups per CU keep enough loads in flight); TZ1 divides M/2
  static constexpr int TZ1 = div_at_most(M / 2, (sizeof(T) == 4) ? 4096 / M : 2048 / M, 1);
  // z pass: NL lines per workgroup, a power of two (divides 3 M^2)
  static constexpr int NL = pow2_at_most(((sizeof(T) == 4) ? 8192 / M : 4096 / M) < 64
                                             ? ((sizeof(T) == 4) ? 8192 / M : 4096 / M) : 64);
  static_assert((M / 2) % TZ == 0 && TZ % 2 == 0 && (M / 2) % TZ1 == 0 && (3 * M * M) % NL == 0, "tiles");
};

template <typename T, int M>
static void fft_z(pse_ctx *c, const void *src, void *dst, int dir) {
  using CT = C<T>;
  constexpr int NL = GridCfg<T, M>::NL;
  const int nlines = 3 * M * M;
  const dim3 g(nlines / NL);
  ProfScope ps(c, PSE_STAGE_FFT);
  if (dir < 0)
    k_fft_z<T, M, -1, NL, 256><<<g, 256, 0, c->stream>>>((const CT *)src, (CT *)dst, (const CT *)c->tw_H,
                                                         (const CT *)c->tw_M);
  else
    k_fft_z<T, M, +1, NL, 256><<<g, 256, 0, c->stream>>>((const CT *)src, (CT *)dst, (const CT *)c->tw_H,
                                                         (const CT *)c->tw_M);
}

// z pass on the packed real grid: NXY (x, y) columns (3 NXY lines) per
// workgroup, at most 24 KB of LDS (six workgroups per CU)
template <typename T, int M>
static void fft_z_aos(pse_ctx *c, const void *src, void *dst, int dir) {
  using CT = C<T>;
  constexpr int NX0 = 24576 / (3 * M * (int)sizeof(T));
  constexpr int NXY = NX0 >= 16 ? 16 : (NX0 >= 8 ? 8 : (NX0 >= 4 ? 4 : (NX0 >= 2 ? 2 : 1)));
  const dim3 g(M * M / NXY);
  ProfScope ps(c, PSE_STAGE_FFT);
  if (dir < 0)
    k_fft_z_aos<T, M, -1, NXY, 256><<<g, 256, 0, c->stream>>>(src, dst, (const CT *)c->tw_H, (const CT *)c->tw_M);
  else
    k_fft_z_aos<T, M, +1, NXY, 256><<<g, 256, 0, c->stream>>>(src, dst, (const CT *)c->tw_H, (const CT *)c->tw_M);
}

template <typename T, int M>
static void fft_strided(pse_ctx *c, void *data, int axis, int dir) {
  using CT = C<T>;
  constexpr int H = M / 2;
  constexpr int TZ = GridCfg<T, M>::TZ1;
  const size_t s_comp = (size_t)M * M * H;
  const size_t s_fft = axis == 0 ? (size_t)M * H : (size_t)H;
  const size_t s_outer = axis == 0 ? (size_t)H : (size_t)M * H;
  const dim3 g(H / TZ, M, 3);
  ProfScope ps(c, PSE_STAGE_FFT);
  if (dir < 0)
    k_fft_strided<T, M, -1, TZ, 256><<<g, 256, 0, c->stream>>>((CT *)data, s_fft, s_outer, s_comp, (const CT *)c->tw_M);
  else
    k_fft_strided<T, M, +1, TZ, 256><<<g, 256, 0, c->stream>>>((CT *)data, s_fft, s_outer, s_comp, (const CT *)c->tw_M);
}

template <typename T, int M>
static void xpass(pse_ctx *c, void *data, const void *specW, const WaveCoef &wc, bool forces, int noise) {
  using CT = C<T>;
  constexpr int H = M / 2;
  constexpr int TZ = GridCfg<T, M>::TZ;
  const dim3 g(H / TZ, M);
  auto *d = (CT *)data;
  auto *w = (const CT *)specW;
  auto *tw = (const CT *)c->tw_M;
  ProfScope ps(c, PSE_STAGE_XFUSED);
  if (forces) {
    if (noise == 1) k_xpass_fused<T, M, TZ, 256, true, 1><<<g, 256, 0, c->stream>>>(d, w, wc, tw);
    else if (noise == 2) k_xpass_fused<T, M, TZ, 256, true, 2><<<g, 256, 0, c->stream>>>(d, w, wc, tw);
    else k_xpass_fused<T, M, TZ, 256, true, 0><<<g, 256, 0, c->stream>>>(d, w, wc, tw);
  } else {
    if (noise == 1) k_xpass_fused<T, M, TZ, 256, false, 1><<<g, 256, 0, c->stream>>>(d, w, wc, tw);
    else if (noise == 2) k_xpass_fused<T, M, TZ, 256, false, 2><<<g, 256, 0, c->stream>>>(d, w, wc, tw);
    else k_xpass_fused<T, M, TZ, 256, false, 0><<<g, 256, 0, c->stream>>>(d, w, wc, tw);
  }
}

template <typename T, int M>
static void dispatch_grid_op(pse_ctx *c, GridOp op, const void *a, void *b, const WaveCoef *wc, int x, int y) {
  switch (op) {
    case GridOp::FftZ: fft_z<T, M>(c, a, b, x); break;
    case GridOp::FftZAos: fft_z_aos<T, M>(c, a, b, x); break;
    case GridOp::FftStrided: fft_strided<T, M>(c, b, x, y); break;
    case GridOp::XFused: xpass<T, M>(c, b, a, *wc, x != 0, y); break;
  }
}

template <typename T>
void launch_grid_op(pse_ctx *c, GridOp op, const void *a, void *b, const WaveCoef *wc, int x, int y) {
  switch (c->p.grid) {
    case 16: dispatch_grid_op<T, 16>(c, op, a, b, wc, x, y); break;
    case 24: dispatch_grid_op<T, 24>(c, op, a, b, wc, x, y); break;
    case 48: dispatch_grid_op<T, 48>(c, op, a, b, wc, x, y); break;
    case 96: dispatch_grid_op<T, 96>(c, op, a, b, wc, x, y); break;
    case 192: dispatch_grid_op<T, 192>(c, op, a, b, wc, x, y); break;
    case 384: dispatch_grid_op<T, 384>(c, op, a, b, wc, x, y); break;
    case 32: dispatch_grid_op<T, 32>(c, op, a, b, wc, x, y); break;
    case 64: dispatch_grid_op<T, 64>(c, op, a, b, wc, x, y); break;
    case 128: dispatch_grid_op<T, 128>(c, op, a, b, wc, x, y); break;
    case 256: dispatch_grid_op<T, 256>(c, op, a, b, wc, x, y); break;
    case 512: dispatch_grid_op<T, 512>(c, op, a, b, wc, x, y); break;
    default: break;
  }
}

// Tiled spreading needs M >= 2 max(TX, TY, TZ) + P (unique nearest image):
// the smallest tiles, 8 x 8 x 8 nodes, need M >= 16 + P; smaller grids
// spread with atomics.
static bool spread_tiled(int M, int P) { return M % 8 == 0 && M >= 16 + P; }
bool spread_writes_whole_grid(int M, int P) { return spread_tiled(M, P); }

// Spreading tile depth nw is valid when the tile (8 x 8 x 8 nw) divides the
// grid and the nearest periodic image stays unique: M >= 2 max(8, 8 nw) + P.
static bool spread_nw_valid(int M, int P, int nw) {
  const int tz = 8 * nw, tmax = tz > 8 ? tz : 8;
  return M % tz == 0 && M >= 2 * tmax + P;
}

// FP32 spreading runs on the matrix cores (k_spread_mfma: tiles 16 x 8 x
// 8 nw, 4 nw wavefronts, nw <= 4) where the grid allows, the VALU tiles
// (8 x 8 x 8 nw) elsewhere.
static bool spread_mfma_valid(int M, int P, int nw) {
  const int tz = 8 * nw, tmax = tz > 16 ? tz : 16;
  return nw <= 4 && M % 16 == 0 && M % tz == 0 && M >= 2 * tmax + P;
}

// Built-in tile depth (8 nw): the matrix-core form is fastest with the
// smallest tiles (16 x 8 x 8, measured at 256^3 to 512^3); the VALU tiles
// with 8 x 8 x 32 from 128^3 up (measured best at 256^3 against depths 16
// and 64).
int spread_default_nw(int M, int P, bool fp32) {
  if (fp32 && spread_mfma_valid(M, P, 1)) return 1;
  int nw = M >= 128 ? 4 : (M >= 64 ? 2 : 1);
  while (nw > 1 && !spread_nw_valid(M, P, nw)) nw >>= 1;
  return nw;
}

template <typename T, int P>
static void spread_interp_P(pse_ctx *c, bool spread, const void *vec, void *grid_or_out) {
  using T4 = typename vec4<T>::type;
  const int n = c->n, M = c->p.grid;
  const double h = c->d.h, s2 = c->d.sigma * c->d.sigma;
  const double norm = std::pow(2.0 * 3.14159265358979323846 * s2, -1.5);
  const int blocks = (int)(((long)n * 64 + 255) / 256);
  ProfScope ps(c, spread ? PSE_STAGE_SPREAD : PSE_STAGE_INTERP);
  if (spread) {
    if (spread_tiled(M, P)) {
      auto go = [&](auto nw) {
        constexpr int NW = decltype(nw)::value;
        if constexpr (std::is_same<T, float>::value && NW <= 4) {
          if (spread_mfma_valid(M, P, NW)) {
            k_spread_mfma<P, NW><<<dim3(M / (8 * NW), M / 8, M / 16), 256 * NW, 0, c->stream>>>(
                (const float4 *)c->pos_s, (const float4 *)vec, c->cell_start, c->d.nc, (float)c->d.cs, M, (float)h,
                (float)(1.0 / h), (float)(0.5 / s2), (float)norm, (float *)grid_or_out);
            return;
          }
        }
        const dim3 g(M / (8 * NW), M / 8, M / 8);
        k_spread_tile<T, P, NW><<<g, 64 * NW, 0, c->stream>>>(
            (const T4 *)c->pos_s, (const T4 *)vec, c->cell_start, c->d.nc, (T)c->d.cs, M, (T)h, (T)(1.0 / h),
            (T)(0.5 / s2), (T)norm, (T *)grid_or_out);
      };
      // pse_autotune may pick another valid depth than the built-in one
      const int nw = c->tune_spread_nw ? c->tune_spread_nw : spread_default_nw(M, P, std::is_same<T, float>::value);
      if (nw == 8) go(std::integral_constant<int, 8>{});
      else if (nw == 4) go(std::integral_constant<int, 4>{});
      else if (nw == 2) go(std::integral_constant<int, 2>{});
      else go(std::integral_constant<int, 1>{});
    } else {
      launch_zero_words(c->stream, grid_or_out, sizeof(T) * (size_t)M * M * M * 3 / 4);  // 3 components
      k_spread<T, P><<<blocks, 256, 0, c->stream>>>((const T4 *)c->pos_s, (const T4 *)vec, n, (T *)grid_or_out, M,
                                                    (T)h, (T)(1.0 / h), (T)(0.5 / s2), (T)norm);
    }
  } else {
    // built-in: 8 particles (consecutive in cell order) per workgroup share
    // the L1 (the autotuner's choice at 64^3 to 384^3; 1024 lanes took 2.0
    // against 1.5 ms at 384^3 with 4 10^6 spheres)
    const int nt = c->tune_interp_threads ? c->tune_interp_threads : kInterpLanes;
    k_interp<T, P><<<(int)(((long)n * 64 + nt - 1) / nt), nt, 0, c->stream>>>(
        (const T4 *)c->pos_s, (const T *)vec, n, (T4 *)grid_or_out, M, (T)h, (T)(1.0 / h), (T)(0.5 / s2),
        (T)(norm * h * h * h));
  }
}

template <typename T>
void launch_spread_interp(pse_ctx *c, bool spread, const void *vec, void *grid_or_out) {
  switch (c->p.support) {
    case 2: spread_interp_P<T, 2>(c, spread, vec, grid_or_out); break;
    case 4: spread_interp_P<T, 4>(c, spread, vec, grid_or_out); break;
    case 6: spread_interp_P<T, 6>(c, spread, vec, grid_or_out); break;
    case 8: spread_interp_P<T, 8>(c, spread, vec, grid_or_out); break;
    case 10: spread_interp_P<T, 10>(c, spread, vec, grid_or_out); break;
    case 12: spread_interp_P<T, 12>(c, spread, vec, grid_or_out); break;
    case 14: spread_interp_P<T, 14>(c, spread, vec, grid_or_out); break;
    case 16: spread_interp_P<T, 16>(c, spread, vec, grid_or_out); break;
    default: break;
  }
}

// ------------------------------------------------- batched wave space
// The launches of a system's wave-space part without forces, for every
// system of a group at once: the system index is the last grid dimension
// (x pass, z pass; y pass: component + 3 system) or comes from the block
// map (interpolation).  Same block bodies as the single-system kernels.
template <int M, int TZ, bool FORCES>
__global__ __launch_bounds__(256) void k_xpass_batch(const WaveRep *__restrict__ reps) {
  const WaveRep &r = reps[blockIdx.z];
  xpass_block<float, M, TZ, 256, FORCES, 1>((C<float> *)r.spec, nullptr, r.wc, (const C<float> *)r.tw_M, blockIdx.x,
                                            blockIdx.y, gridDim.x, gridDim.y);
}

// spreading: grid (M / 8 nw, M / 8, M / 8 per system)
template <int P, int NW>
__global__ __launch_bounds__(64 * NW) void k_spread_batch(const WaveRep *__restrict__ reps, int gz) {
  const WaveRep &r = reps[blockIdx.z / gz];
  const int bz = blockIdx.z % gz;
  const int lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * bz), gridDim.x * gridDim.y * gz);
  spread_tile_block<float, P, NW>(r.pos, r.f, r.cell_start, r.nc, r.cs, r.M, r.h, r.invh, r.inv2s2, r.norm, r.rgrid,
                                  lin, gridDim.x, gridDim.y);
}

// the matrix-core form: grid (M / 8 nw, M / 8, M / 16 per system)
template <int P, int NW>
__global__ __launch_bounds__(256 * NW) void k_spread_mfma_batch(const WaveRep *__restrict__ reps, int gz) {
  const WaveRep &r = reps[blockIdx.z / gz];
  const int bz = blockIdx.z % gz;
  const int lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * bz), gridDim.x * gridDim.y * gz);
  spread_mfma_block<P, NW>(r.pos, r.f, r.cell_start, r.nc, r.cs, r.M, r.h, r.invh, r.inv2s2, r.norm, r.rgrid, lin,
                           gridDim.x, gridDim.y);
}

template <int M, int TZ>
__global__ __launch_bounds__(256) void k_fft_y_fwd_batch(const WaveRep *__restrict__ reps) {
  constexpr int H = M / 2;
  const WaveRep &r = reps[blockIdx.z / 3];
  fft_strided_block<float, M, -1, TZ, 256>((C<float> *)r.spec, (size_t)H, (size_t)M * H, (size_t)M * M * H,
                                           (const C<float> *)r.tw_M, blockIdx.x, blockIdx.y, blockIdx.z % 3);
}

template <int M, int NXY>
__global__ __launch_bounds__(256) void k_fft_z_fwd_batch(const WaveRep *__restrict__ reps) {
  const WaveRep &r = reps[blockIdx.y];
  fft_z_aos_block<float, M, -1, NXY, 256>(r.rgrid, r.spec, (const C<float> *)r.tw_H, (const C<float> *)r.tw_M,
                                          blockIdx.x);
}

template <int M, int TZ>
__global__ __launch_bounds__(256) void k_fft_y_inv_batch(const WaveRep *__restrict__ reps) {
  constexpr int H = M / 2;
  const WaveRep &r = reps[blockIdx.z / 3];
  fft_strided_block<float, M, +1, TZ, 256>((C<float> *)r.spec, (size_t)H, (size_t)M * H, (size_t)M * M * H,
                                           (const C<float> *)r.tw_M, blockIdx.x, blockIdx.y, blockIdx.z % 3);
}

template <int M, int NXY>
__global__ __launch_bounds__(256) void k_fft_z_inv_batch(const WaveRep *__restrict__ reps) {
  const WaveRep &r = reps[blockIdx.y];
  fft_z_aos_block<float, M, +1, NXY, 256>(r.spec, r.rgrid, (const C<float> *)r.tw_H, (const C<float> *)r.tw_M,
                                          blockIdx.x);
}

template <int P>
__global__ __launch_bounds__(1024) void k_interp_batch(const WaveRep *__restrict__ reps, const int2 *__restrict__ imap) {
  const int2 rb = imap[xcd_block(blockIdx.x, gridDim.x)];
  const WaveRep &r = reps[rb.x];
  const int s = __builtin_amdgcn_readfirstlane((rb.y * (int)blockDim.x + (int)threadIdx.x) >> 6);
  interp_particle<float, P>(r.pos, r.rgrid, r.n, r.out, r.M, r.h, r.invh, r.inv2s2, r.norm_h3, s);
}

template <int M> static void wave_batch_M(hipStream_t s, const WaveGroup &g) {
  constexpr int H = M / 2;
  constexpr int TZ = GridCfg<float, M>::TZ, TZ1 = GridCfg<float, M>::TZ1;
  constexpr int NX0 = 24576 / (3 * M * (int)sizeof(float));
  constexpr int NXY = NX0 >= 16 ? 16 : (NX0 >= 8 ? 8 : (NX0 >= 4 ? 4 : (NX0 >= 2 ? 2 : 1)));
  if (g.forces) {
    auto spread = [&](auto pp, auto ww) {
      constexpr int PP = decltype(pp)::value, NW = decltype(ww)::value;
      if constexpr (M % (8 * NW) == 0) {
        if constexpr (NW <= 4 && M % 16 == 0) {
          if (spread_mfma_valid(M, PP, NW)) {
            k_spread_mfma_batch<PP, NW><<<dim3(M / (8 * NW), M / 8, (M / 16) * g.nrep), 256 * NW, 0, s>>>(g.reps,
                                                                                                       M / 16);
            return;
          }
        }
        k_spread_batch<PP, NW><<<dim3(M / (8 * NW), M / 8, (M / 8) * g.nrep), 64 * NW, 0, s>>>(g.reps, M / 8);
      }
    };
    auto by_nw = [&](auto pp) {
      if (g.nw == 8) spread(pp, std::integral_constant<int, 8>{});
      else if (g.nw == 4) spread(pp, std::integral_constant<int, 4>{});
      else if (g.nw == 2) spread(pp, std::integral_constant<int, 2>{});
      else spread(pp, std::integral_constant<int, 1>{});
    };
    switch (g.P) {
      case 2: by_nw(std::integral_constant<int, 2>{}); break;
      case 4: by_nw(std::integral_constant<int, 4>{}); break;
      case 6: by_nw(std::integral_constant<int, 6>{}); break;
      case 8: by_nw(std::integral_constant<int, 8>{}); break;
      case 10: by_nw(std::integral_constant<int, 10>{}); break;
      case 12: by_nw(std::integral_constant<int, 12>{}); break;
      case 14: by_nw(std::integral_constant<int, 14>{}); break;
      case 16: by_nw(std::integral_constant<int, 16>{}); break;
      default: break;
    }
    k_fft_z_fwd_batch<M, NXY><<<dim3(M * M / NXY, g.nrep), 256, 0, s>>>(g.reps);
    k_fft_y_fwd_batch<M, TZ1><<<dim3(H / TZ1, M, 3 * g.nrep), 256, 0, s>>>(g.reps);
    k_xpass_batch<M, TZ, true><<<dim3(H / TZ, M, g.nrep), 256, 0, s>>>(g.reps);
  } else {
    k_xpass_batch<M, TZ, false><<<dim3(H / TZ, M, g.nrep), 256, 0, s>>>(g.reps);
  }
  k_fft_y_inv_batch<M, TZ1><<<dim3(H / TZ1, M, 3 * g.nrep), 256, 0, s>>>(g.reps);
  k_fft_z_inv_batch<M, NXY><<<dim3(M * M / NXY, g.nrep), 256, 0, s>>>(g.reps);
  switch (g.P) {
    case 2: k_interp_batch<2><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 4: k_interp_batch<4><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 6: k_interp_batch<6><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 8: k_interp_batch<8><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 10: k_interp_batch<10><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 12: k_interp_batch<12><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 14: k_interp_batch<14><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    case 16: k_interp_batch<16><<<g.nimap, g.nt, 0, s>>>(g.reps, g.imap); break;
    default: break;
  }
}

void launch_wave_batch(hipStream_t s, const WaveGroup *groups, int ngroups) {
  for (int i = 0; i < ngroups; ++i) {
    const WaveGroup &g = groups[i];
    switch (g.M) {
      case 16: wave_batch_M<16>(s, g); break;
      case 24: wave_batch_M<24>(s, g); break;
      case 32: wave_batch_M<32>(s, g); break;
      case 48: wave_batch_M<48>(s, g); break;
      case 64: wave_batch_M<64>(s, g); break;
      case 96: wave_batch_M<96>(s, g); break;
      case 128: wave_batch_M<128>(s, g); break;
      case 192: wave_batch_M<192>(s, g); break;
      case 256: wave_batch_M<256>(s, g); break;
      case 384: wave_batch_M<384>(s, g); break;
      case 512: wave_batch_M<512>(s, g); break;
      default: break;
    }
  }
}

template void launch_grid_op<float>(pse_ctx *, GridOp, const void *, void *, const WaveCoef *, int, int);
template void launch_grid_op<double>(pse_ctx *, GridOp, const void *, void *, const WaveCoef *, int, int);
template void launch_spread_interp<float>(pse_ctx *, bool, const void *, void *);

bool grid_shape_valid(int M, int P, int depth, int interp_lanes) {
  if (depth != 0) {
    const int nw = depth / 8;
    if (depth % 8 || (nw != 1 && nw != 2 && nw != 4 && nw != 8)) return false;
    if (!spread_tiled(M, P) || !spread_nw_valid(M, P, nw)) return false;
  }
  return interp_lanes == 0 || interp_lanes == 256 || interp_lanes == 512 || interp_lanes == 1024;
}

template <typename T> pse_status autotune_grid(pse_ctx *c, int32_t *choice) {
  const int M = c->p.grid, P = c->p.support;
  const uint32_t mask = c->prof_mask;
  c->prof_mask = 0;  // the trial launches are not stage time
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PSE_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PSE_ERR_HIP;
  }
  // any finite per-particle vector serves as the spread source: the sorted
  // positions; the grid and vbuf[5] are scratch that every sample rewrites
  auto time_it = [&](auto launch) -> float {
    launch();  // warm-up
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      float ms = 1e30f;
      if (hipEventRecord(e0, c->stream) != hipSuccess) return 1e30f;
      launch();
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return 1e30f;
      best = ms < best ? ms : best;
    }
    return best;
  };
  const int keep_nw = c->tune_spread_nw, keep_nt = c->tune_interp_threads;
  int best_nw = 0, best_nt = 0;
  if (spread_tiled(M, P)) {
    float tbest = 1e30f;
    for (int nw : {1, 2, 4, 8}) {
      if (!spread_nw_valid(M, P, nw)) continue;
      c->tune_spread_nw = nw;
      const float t = time_it([&] { launch_spread_interp<T>(c, true, c->pos_s, c->rgrid); });
      if (t < tbest) {
        tbest = t;
        best_nw = nw;
      }
    }
  }
  {
    float tbest = 1e30f;
    for (int nt : {256, 512, 1024}) {
      c->tune_interp_threads = nt;
      const float t = time_it([&] { launch_spread_interp<T>(c, false, c->rgrid, c->vbuf[5]); });
      if (t < tbest) {
        tbest = t;
        best_nt = nt;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->prof_mask = mask;
  const pse_status st = hipGetLastError() == hipSuccess ? PSE_OK : PSE_ERR_HIP;
  c->tune_spread_nw = st == PSE_OK && best_nw ? best_nw : keep_nw;
  c->tune_interp_threads = st == PSE_OK && best_nt ? best_nt : keep_nt;
  if (choice) {
    choice[0] = 8 * (c->tune_spread_nw ? c->tune_spread_nw : spread_default_nw(M, P, std::is_same<T, float>::value));
    choice[1] = c->tune_interp_threads ? c->tune_interp_threads : kInterpLanes;
    if (!spread_tiled(M, P)) choice[0] = 0;
  }
  return st;
}
template pse_status autotune_grid<float>(pse_ctx *, int32_t *);
template pse_status autotune_grid<double>(pse_ctx *, int32_t *);
template void launch_spread_interp<double>(pse_ctx *, bool, const void *, void *);

}  // namespace pse
