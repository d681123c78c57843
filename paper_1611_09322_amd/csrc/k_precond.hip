// Learned block preconditioner of the real-space Krylov sample.
//
// The Lanczos iteration of Sec. II B.1 runs on A = P M_r P^T, with P block
// diagonal (one 3x3 block per particle), and the sample is
// y = P^{-1} A^{1/2} z, whose covariance is M_r.  P_i = I + y_i, where y_i
// is the output of a 24 -> 64 -> 64 -> 9 MLP (bf16 weights and activations,
// fp32 sums on the MFMA units) applied to geometry features of the
// particle's near field (computed from the neighbour list).  Blocks
// that are not finite, nearly singular or ill conditioned fall back to I.
// Training kernels (the backward pass on the matrix cores, Adam) run off
// the sampling path.
#include <mutex>

#include "launch.hpp"

namespace pse {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// ------------------------------------------------------------ MLP forward
// One wavefront per 16-particle tile, three layers of 16x16x32 bf16 MFMA.
// Operand layout of v_mfma_f32_16x16x32_bf16: lane l holds row (l % 16) of
// A and column (l % 16) of B over the same 8 consecutive k (group l / 16);
// the 16x16 fp32 result gives lane l rows 4 (l / 16) + i, column l % 16.
// Hidden tiles go through LDS (bf16) to turn result layout into operand
// layout.  Every wavefront runs the same number of tile steps so the
// workgroup barriers are uniform.
constexpr int kTileLd = 64 + 8;  // LDS row stride of an activation tile (elements)

__global__ __launch_bounds__(256) void k_mlp_fwd(const uint16_t *__restrict__ w, const uint16_t *__restrict__ x,
                                                 int n, float *__restrict__ y, uint16_t *__restrict__ cache) {
  __shared__ __attribute__((aligned(16))) uint16_t sw[kWTotal];
  __shared__ __attribute__((aligned(16))) uint16_t sh1[4][16 * kTileLd];
  __shared__ __attribute__((aligned(16))) uint16_t sh2[4][16 * kTileLd];
  for (int i = threadIdx.x; i < kWTotal / 8; i += blockDim.x) ((u32x4 *)sw)[i] = ((const u32x4 *)w)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int ntiles = (n + 15) / 16;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  uint16_t *t1 = sh1[wave], *t2 = sh2[wave];
  for (int base = blockIdx.x * 4; base < ntiles; base += gridDim.x * 4) {
    const int tile = base + wave;
    const int p0 = tile * 16;
    // layer 1: [16 x 32] x [32 x 64], features 24..31 are zero
    u32x4 av = {0u, 0u, 0u, 0u};
    if (tile < ntiles && kg < 3 && p0 + r16 < n) av = *(const u32x4 *)(x + (size_t)(p0 + r16) * kNFeat + 8 * kg);
    const bf16x8 a1 = as_bf16x8(av);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 b = as_bf16x8(*(const u32x4 *)(sw + kW1 + (16 * nb + r16) * 32 + 8 * kg));
      const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, zero, 0, 0, 0);
      const float bias = bf16_to_f32(sw[kB1 + 16 * nb + r16]);
#pragma unroll
      for (int i = 0; i < 4; ++i) t1[(4 * kg + i) * kTileLd + 16 * nb + r16] = f32_to_bf16(fmaxf(d[i] + bias, 0.f));
    }
    __syncthreads();
    // layer 2: [16 x 64] x [64 x 64]
    bf16x8 a2[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) a2[kb] = as_bf16x8(*(const u32x4 *)(t1 + r16 * kTileLd + 32 * kb + 8 * kg));
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      f32x4 d = zero;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 b = as_bf16x8(*(const u32x4 *)(sw + kW2 + (16 * nb + r16) * 64 + 32 * kb + 8 * kg));
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[kb], b, d, 0, 0, 0);
      }
      const float bias = bf16_to_f32(sw[kB2 + 16 * nb + r16]);
#pragma unroll
      for (int i = 0; i < 4; ++i) t2[(4 * kg + i) * kTileLd + 16 * nb + r16] = f32_to_bf16(fmaxf(d[i] + bias, 0.f));
    }
    __syncthreads();
    // layer 3: [16 x 64] x [64 x 16], outputs 9..15 unused
    f32x4 d3 = zero;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const bf16x8 a3 = as_bf16x8(*(const u32x4 *)(t2 + r16 * kTileLd + 32 * kb + 8 * kg));
      const bf16x8 b = as_bf16x8(*(const u32x4 *)(sw + kW3 + r16 * 64 + 32 * kb + 8 * kg));
      d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b, d3, 0, 0, 0);
    }
    if (tile < ntiles && r16 < kNOut) {
      const float bias = bf16_to_f32(sw[kB3 + r16]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = p0 + 4 * kg + i;
        if (p < n) y[(size_t)p * kNOut + r16] = d3[i] + bias;
      }
    }
    if (cache && tile < ntiles) {
      // rows of (h1, h2): 16 rows x 128 bf16 = 256 chunks of 16 bytes
      for (int ch = lane; ch < 256; ch += 64) {
        const int row = ch >> 4, part = ch & 15;  // part < 8: h1, else h2
        const int p = p0 + row;
        if (p < n) {
          const uint16_t *src = (part < 8 ? t1 : t2) + row * kTileLd + 8 * (part & 7);
          *(u32x4 *)(cache + (size_t)p * 2 * kNHid + 8 * part) = *(const u32x4 *)src;
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------- MLP backward
// Gradients of sum_p <dy_p, y_p> for the same network, on the matrix cores.
// A wavefront takes 32 rows at a time; every product of the chain rule is a
// 16x16x32 bf16 MFMA tile product:
//   dh2 = dy W3        (rows x 16 outputs) (16 x 64)
//   gW3 += dy^T h2     (16 x rows) (rows x 64)
//   dz2 = dh2 . [h2 > 0];  gW2 += dz2^T h1;  dh1 = dz2 W2
//   dz1 = dh1 . [h1 > 0];  gW1 += dz1^T x
// h1, h2, x and the weights are bf16 already (exact operands).  The fp32
// factors dy, dz2, dz1 are split into three bf16 parts (hi + mid + lo,
// each the rounded remainder of the previous: 24 significant bits, the
// precision of fp32) and each product is the sum of the three part
// products, accumulated in fp32: the gradient keeps fp32 accuracy.  Bias
// gradients are column sums of dy, dz2, dz1 in fp32.  Each wavefront writes
// its sums to its own slot of `partial`; k_mlp_reduce adds the slots in a
// fixed order (deterministic).
constexpr int kBwdRows = 32;
constexpr int kBwdWaves = 2;  // wavefronts per workgroup

struct BwdLds {
  // per wavefront: the chunk's operands in the layouts the MFMA reads
  uint16_t h1T[64][kBwdRows + 8];        // h1^T (k, p)
  uint16_t h2T[64][kBwdRows + 8];        // h2^T
  uint16_t xT[32][kBwdRows + 8];         // x^T (f, p), f >= 24 zero
  uint16_t dy[3][kBwdRows][32 + 8];      // parts of dy (p, o), o >= 9 zero
  uint16_t dyT[3][16][kBwdRows + 8];     // parts of dy^T (o, p)
  uint16_t dz[3][kBwdRows][64 + 8];      // parts of dz2 (p, j)
  uint16_t dzT[3][64][kBwdRows + 8];     // parts of dz2^T, then dz1^T (j, p)
  float dyf[kBwdRows][16];               // dy in fp32 (bias sums)
};

__device__ __forceinline__ void split3(float v, uint16_t *h, uint16_t *m, uint16_t *l) {
  const uint16_t a = f32_to_bf16(v);
  const float r1 = v - bf16_to_f32(a);
  const uint16_t b = f32_to_bf16(r1);
  const float r2 = r1 - bf16_to_f32(b);
  *h = a;
  *m = b;
  *l = f32_to_bf16(r2);
}

// Each wavefront owns its LDS buffers, so ordering its own writes before
// its own reads needs no workgroup barrier (the wavefronts of a workgroup
// run different numbers of chunks): a fence (the LDS accesses completed)
// and a scheduling barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
  // 8 consecutive bf16 (16 bytes; rows are padded to keep 16-byte alignment)
  return as_bf16x8(*(const u32x4 *)p);
}

__global__ __launch_bounds__(64 * kBwdWaves) void k_mlp_bwd(const uint16_t *__restrict__ w,
                                                            const uint16_t *__restrict__ x,
                                                            const uint16_t *__restrict__ cache,
                                                            const float *__restrict__ dy, int n,
                                                            float *__restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t w3T[64][32 + 8];  // W3^T (k, o), o >= 16 zero
  __shared__ __attribute__((aligned(16))) uint16_t w2s[64][64 + 8];  // W2 (j, k) as stored
  __shared__ __attribute__((aligned(16))) BwdLds L[kBwdWaves];
  for (int e = threadIdx.x; e < 64 * 32; e += blockDim.x) {
    const int k = e >> 5, o = e & 31;
    w3T[k][o] = o < 16 ? w[kW3 + o * 64 + k] : (uint16_t)0;
  }
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) w2s[e >> 6][e & 63] = w[kW2 + e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int gw = blockIdx.x * kBwdWaves + wave, nw = gridDim.x * kBwdWaves;
  BwdLds &S = L[wave];
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gW3[4], gW2[4][4], gW1[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW3[a] = zero;
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[a][b] = zero;
    gW1[a][0] = gW1[a][1] = zero;
  }
  float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f;
  for (int p0 = gw * kBwdRows; p0 < n; p0 += nw * kBwdRows) {
    // ---- stage the chunk (rows past n are zero)
    for (int e = lane; e < kBwdRows * 128; e += 64) {
      const int p = e >> 7, c = e & 127;
      const uint16_t v = p0 + p < n ? cache[(size_t)(p0 + p) * 2 * kNHid + c] : (uint16_t)0;
      if (c < 64) S.h1T[c][p] = v;
      else S.h2T[c - 64][p] = v;
    }
    for (int e = lane; e < kBwdRows * 32; e += 64) {
      const int p = e >> 5, f = e & 31;
      S.xT[f][p] = (f < kNFeat && p0 + p < n) ? x[(size_t)(p0 + p) * kNFeat + f] : (uint16_t)0;
    }
    for (int e = lane; e < kBwdRows * 32; e += 64) {
      const int p = e >> 5, o = e & 31;
      const float v = (o < kNOut && p0 + p < n) ? dy[(size_t)(p0 + p) * kNOut + o] : 0.f;
      uint16_t a, b, c;
      split3(v, &a, &b, &c);
      S.dy[0][p][o] = a;
      S.dy[1][p][o] = b;
      S.dy[2][p][o] = c;
      if (o < 16) {
        S.dyT[0][o][p] = a;
        S.dyT[1][o][p] = b;
        S.dyT[2][o][p] = c;
        S.dyf[p][o] = v;
      }
    }
    wave_sync();
    // ---- bias of the output layer: column sums of dy
    if (lane < 16) {
      float sacc = 0.f;
#pragma unroll 8
      for (int p = 0; p < kBwdRows; ++p) sacc += S.dyf[p][lane];
      gb3 += sacc;
    }
    // ---- gW3 += dy^T h2: M = o (one tile), N = k (4 tiles), K = rows
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x8 b = ld8(&S.h2T[16 * nt + r16][8 * g]);
#pragma unroll
      for (int q = 0; q < 3; ++q)
        gW3[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&S.dyT[q][r16][8 * g]), b, gW3[nt], 0, 0, 0);
    }
    // ---- dh2 = dy W3: M = rows (2 tiles), N = k (4 tiles), K = o (32, zero past 16)
    //      dz2 = dh2 . [h2 > 0], split and stored in both layouts
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const bf16x8 b = ld8(&w3T[16 * nt + r16][8 * g]);
        f32x4 d = zero;
#pragma unroll
        for (int q = 0; q < 3; ++q)
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&S.dy[q][16 * mt + r16][8 * g]), b, d, 0, 0, 0);
        const int k = 16 * nt + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * mt + 4 * g + i;
          const float v = bf16_to_f32(S.h2T[k][p]) > 0.f ? d[i] : 0.f;
          gb2[nt] += v;
          uint16_t a, bb, c;
          split3(v, &a, &bb, &c);
          S.dz[0][p][k] = a;
          S.dz[1][p][k] = bb;
          S.dz[2][p][k] = c;
          S.dzT[0][k][p] = a;
          S.dzT[1][k][p] = bb;
          S.dzT[2][k][p] = c;
        }
      }
    }
    wave_sync();
    // ---- gW2 += dz2^T h1: M = j (4 tiles), N = k (4 tiles), K = rows
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x8 b = ld8(&S.h1T[16 * nt + r16][8 * g]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          gW2[mt][nt] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&S.dzT[q][16 * mt + r16][8 * g]), b, gW2[mt][nt], 0, 0, 0);
    }
    // ---- dh1 = dz2 W2: M = rows (2 tiles), N = k (4 tiles), K = j (2 steps of 32)
    f32x4 dh1[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 d = zero;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          // B[j][k] = W2[j][k]: lane's column k, rows j = 32 ks + 8 g ... + 7
          bf16x8 b;
#pragma unroll
          for (int u = 0; u < 8; ++u) b[u] = __builtin_bit_cast(__bf16, w2s[32 * ks + 8 * g + u][16 * nt + r16]);
#pragma unroll
          for (int q = 0; q < 3; ++q)
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&S.dz[q][16 * mt + r16][32 * ks + 8 * g]), b, d, 0, 0, 0);
        }
        dh1[mt][nt] = d;
      }
    wave_sync();  // dz2^T is read above; dz1^T overwrites it below
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int k = 16 * nt + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * mt + 4 * g + i;
          const float v = bf16_to_f32(S.h1T[k][p]) > 0.f ? dh1[mt][nt][i] : 0.f;
          gb1[nt] += v;
          uint16_t a, bb, c;
          split3(v, &a, &bb, &c);
          S.dzT[0][k][p] = a;
          S.dzT[1][k][p] = bb;
          S.dzT[2][k][p] = c;
        }
      }
    wave_sync();
    // ---- gW1 += dz1^T x: M = j (4 tiles), N = f (2 tiles), K = rows
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const bf16x8 b = ld8(&S.xT[16 * nt + r16][8 * g]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          gW1[mt][nt] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&S.dzT[q][16 * mt + r16][8 * g]), b, gW1[mt][nt], 0, 0, 0);
    }
    wave_sync();  // the chunk's buffers are restaged next
  }
  // hidden-layer bias sums: the four lane groups hold partial sums of the
  // same columns (k = 16 nt + r16)
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    gb1[nt] += __shfl_xor(gb1[nt], 16, 64);
    gb1[nt] += __shfl_xor(gb1[nt], 32, 64);
    gb2[nt] += __shfl_xor(gb2[nt], 16, 64);
    gb2[nt] += __shfl_xor(gb2[nt], 32, 64);
  }
  float *out = partial + (size_t)gw * kWTotal;
  // result layout: lane holds rows 4 g + i, column r16 of each 16x16 tile
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) out[kW3 + (4 * g + i) * 64 + 16 * nt + r16] = gW3[nt][i];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[kW2 + (16 * mt + 4 * g + i) * 64 + 16 * nt + r16] = gW2[mt][nt][i];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[kW1 + (16 * mt + 4 * g + i) * 32 + 16 * nt + r16] = gW1[mt][nt][i];
  if (g == 0) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      out[kB1 + 16 * nt + r16] = gb1[nt];
      out[kB2 + 16 * nt + r16] = gb2[nt];
    }
  }
  if (lane < 16) out[kB3 + lane] = lane < kNOut ? gb3 : 0.f;
}

// Eight interleaved partial sums (slot q goes to sum q mod 8) keep eight
// loads in flight; the order is fixed, so the result is deterministic.
__global__ void k_mlp_reduce(const float *__restrict__ partial, int nparts, float *__restrict__ dw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kWTotal) return;
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int q = 0;
  for (; q + 8 <= nparts; q += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += partial[(size_t)(q + u) * kWTotal + e];
  }
  for (; q < nparts; ++q) v[q & 7] += partial[(size_t)q * kWTotal + e];
  dw[e] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

// Squared-error training loss of the block network: dy = (2/n)(y - t) and
// loss = sum |y - t|^2 / n over the n x 9 outputs; one workgroup, fixed
// summation order (deterministic).
__global__ __launch_bounds__(256) void k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t, int n,
                                                  float *__restrict__ dy, float *__restrict__ loss) {
  __shared__ double sh[16];
  const float sc = 2.0f / (float)n;
  double acc = 0.0;
  for (int e = threadIdx.x; e < n * kNOut; e += blockDim.x) {
    const float r = y[e] - t[e];
    dy[e] = sc * r;
    acc += (double)r * (double)r;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0 && loss) *loss = (float)(acc / n);
}

// Adam (Kingma and Ba) on the fp32 master weights; c1 = 1/(1 - b1^t),
// c2 = 1/(1 - b2^t) are the bias corrections.  Writes the bf16 copy.
__global__ void k_mlp_adam(float *__restrict__ wm, uint16_t *__restrict__ wb, const float *__restrict__ g,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kWTotal) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  const float we = wm[e] - lr * (me * c1) / (sqrtf(ve * c2) + eps);
  wm[e] = we;
  wb[e] = f32_to_bf16(we);
}

// ------------------------------------------------------------- the blocks
// P_i = I + y_i (row-major), rows stored as (x, y, z, 0); P^{-1} likewise.
// Fallback to I: not finite, |det| < 1e-6, or |P|_F |P^-1|_F > 1e3.
// y == nullptr gives I everywhere (no weights: global fallback).  USER: y
// holds the caller's blocks P_i themselves (n x 9, caller order), gathered
// through perm into the sorted order.
template <typename T, bool USER = false>
__global__ void k_pc_blocks(const float *__restrict__ y, int n, T *__restrict__ P, T *__restrict__ Pinv,
                            int *__restrict__ flags, const int *__restrict__ perm = nullptr) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (s < n) {
    T m[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
    T q[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
    if (y) {
      T a[9];
      bool fin = true;
      const size_t row = USER ? (size_t)perm[s] : (size_t)s;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        a[k] = USER ? (T)y[row * kNOut + k] : (T)y[row * kNOut + k] + ((k % 4 == 0) ? T(1) : T(0));
        fin = fin && isfinite(a[k]);
      }
      T det = T(0), nf = T(0), ni = T(0);
      T c[9];
      if (fin) {
        c[0] = a[4] * a[8] - a[5] * a[7];
        c[1] = a[2] * a[7] - a[1] * a[8];
        c[2] = a[1] * a[5] - a[2] * a[4];
        c[3] = a[5] * a[6] - a[3] * a[8];
        c[4] = a[0] * a[8] - a[2] * a[6];
        c[5] = a[2] * a[3] - a[0] * a[5];
        c[6] = a[3] * a[7] - a[4] * a[6];
        c[7] = a[1] * a[6] - a[0] * a[7];
        c[8] = a[0] * a[4] - a[1] * a[3];
        det = a[0] * c[0] + a[1] * c[3] + a[2] * c[6];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          nf += a[k] * a[k];
          ni += c[k] * c[k];
        }
      }
      // |P|_F |P^-1|_F = sqrt(nf) sqrt(ni) / |det|
      if (!fin || !(fabs(det) >= T(1e-6)) || !(sqrt(nf * ni) <= T(1e3) * fabs(det))) {
        bad = 1;
      } else {
        const T id = T(1) / det;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          m[k] = a[k];
          q[k] = c[k] * id;
        }
      }
    } else {
      bad = 1;
    }
    // rows as (x, y, z, 0): one vector store each
    using T4 = typename vec4<T>::type;
    T4 *pp = (T4 *)(P + (size_t)s * 12), *qq = (T4 *)(Pinv + (size_t)s * 12);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      T4 u, v;
      u.x = m[3 * r];
      u.y = m[3 * r + 1];
      u.z = m[3 * r + 2];
      u.w = T(0);
      v.x = q[3 * r];
      v.y = q[3 * r + 1];
      v.z = q[3 * r + 2];
      v.w = T(0);
      pp[r] = u;
      qq[r] = v;
    }
  }
  unsigned long long b = (unsigned long long)bad;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) b += __shfl_xor(b, off, 64);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(&flags[6], (int)b);
}

// ------------------------------------------- preconditioned Lanczos steps
// u = P^T src (sorted order), skipped once the iteration is done.
template <typename T, typename A>
__global__ void k_pc_pre(const typename vec4<T>::type *__restrict__ src, const T *__restrict__ P, int n,
                         typename vec4<T>::type *__restrict__ u, const LzState<A> *st) {
  if (st->done) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const auto v = src[s];
  const auto *pr = (const typename vec4<T>::type *)(P + (size_t)s * 12);  // rows of P_s
  const auto r0 = pr[0], r1 = pr[1], r2 = pr[2];
  typename vec4<T>::type o;
  o.x = r0.x * v.x + r1.x * v.y + r2.x * v.z;
  o.y = r0.y * v.x + r1.y * v.y + r2.y * v.z;
  o.z = r0.z * v.x + r1.z * v.y + r2.z * v.z;
  o.w = T(0);
  u[s] = o;
}

// From t' = M_r P^T src: v_m = src / beta (stored as basis vector m),
// out = P t' / beta, and alpha_m = <v_m, out> reduced in a fixed order with
// the last workgroup finishing (the same contract as the fused product).
template <typename T, typename A>
__global__ __launch_bounds__(256) void k_pc_post(const typename vec4<T>::type *__restrict__ tp,
                                                 const typename vec4<T>::type *__restrict__ src,
                                                 const T *__restrict__ P, int n,
                                                 typename vec4<T>::type *__restrict__ out,
                                                 typename vec4<T>::type *__restrict__ vm_out, LzState<A> *st,
                                                 A *partials, unsigned *counter) {
  __shared__ A sh[16];
  __shared__ int last;
  if (st->done) return;
  const T sc = (T)st->inv_beta;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  A dot = A(0);
  if (s < n) {
    const auto t = tp[s];
    const auto v = src[s];
    const auto *pr = (const typename vec4<T>::type *)(P + (size_t)s * 12);  // rows of P_s
    const auto r0 = pr[0], r1 = pr[1], r2 = pr[2];
    typename vec4<T>::type o, u;
    o.x = (r0.x * t.x + r0.y * t.y + r0.z * t.z) * sc;
    o.y = (r1.x * t.x + r1.y * t.y + r1.z * t.z) * sc;
    o.z = (r2.x * t.x + r2.y * t.y + r2.z * t.z) * sc;
    o.w = T(0);
    u.x = v.x * sc;
    u.y = v.y * sc;
    u.z = v.z * sc;
    u.w = T(0);
    out[s] = o;
    vm_out[s] = u;
    dot = (A)u.x * (A)o.x + (A)u.y * (A)o.y + (A)u.z * (A)o.z;
  }
  const A bs = block_sum(dot, sh);
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

// y = P^{-1} y in place (sorted order).
template <typename T>
__global__ void k_pc_apply(const T *__restrict__ Q, int n, typename vec4<T>::type *__restrict__ y) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const auto v = y[s];
  const auto *qr = (const typename vec4<T>::type *)(Q + (size_t)s * 12);  // rows of P_s^-1
  const auto r0 = qr[0], r1 = qr[1], r2 = qr[2];
  typename vec4<T>::type o;
  o.x = r0.x * v.x + r0.y * v.y + r0.z * v.z;
  o.y = r1.x * v.x + r1.y * v.y + r1.z * v.z;
  o.z = r2.x * v.x + r2.y * v.y + r2.z * v.z;
  o.w = T(0);
  y[s] = o;
}

// Sorted rows -> caller order: out[perm[s]] = in[s] (W elements of E each).
template <typename E, int W>
__global__ void k_unsort_rows(const E *__restrict__ in, const int *__restrict__ perm, int n, E *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int d = perm[s];
#pragma unroll
  for (int k = 0; k < W; ++k) out[(size_t)d * W + k] = in[(size_t)s * W + k];
}

// P blocks (rows of 4, sorted) -> n x 9 fp32 in caller order
template <typename T>
__global__ void k_unsort_blocks(const T *__restrict__ P, const int *__restrict__ perm, int n, float *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int d = perm[s];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[(size_t)d * 9 + 3 * r + k] = (float)P[(size_t)s * 12 + 4 * r + k];
}

// ---------------------------------------------------------------- launchers
static int nblk(long n, int b) { return (int)((n + b - 1) / b); }

void launch_mlp_fwd(const uint16_t *w, const uint16_t *x, int n, float *y, uint16_t *cache, hipStream_t stream) {
  const int ntiles = (n + 15) / 16;
  int blocks = nblk(ntiles, 4);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  k_mlp_fwd<<<blocks, 256, 0, stream>>>(w, x, n, y, cache);
}

// One wavefront per 32-row chunk, up to 256 wavefronts (the chunks are
// shared out round-robin past that); one fp32 slot of kWTotal per wavefront.
int mlp_bwd_parts(int n) {
  int blocks = nblk(nblk(n, kBwdRows), kBwdWaves);
  if (blocks > 256 / kBwdWaves) blocks = 256 / kBwdWaves;
  if (blocks < 1) blocks = 1;
  return blocks * kBwdWaves;
}

void launch_mlp_bwd(const uint16_t *w, const uint16_t *x, const uint16_t *cache, const float *dy, int n, float *dw,
                    float *work, hipStream_t stream) {
  const int parts = mlp_bwd_parts(n);
  k_mlp_bwd<<<parts / kBwdWaves, 64 * kBwdWaves, 0, stream>>>(w, x, cache, dy, n, work);
  k_mlp_reduce<<<nblk(kWTotal, 256), 256, 0, stream>>>(work, parts, dw);
}

// ------------------------------------------ allocation-free backward pass
// The same two kernels with the partial-gradient slots in a fixed device
// array instead of a caller workspace, for callers that cannot allocate.
// Every GPU holds its own copy of the array (7.1 MiB) until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is a host-side stand-in).  The
// backward kernel rewrites every entry of each slot it uses, so nothing has
// to be cleared between calls.  Calls that overlap on one GPU share the
// array and race.
static __device__ __align__(256) float scratch[(size_t)kMlpStaticSlots * kWTotal];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float *scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's scratch array, looked up once per device
// with that device current (nullptr on failure).
static float *static_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    scratch_dev[dev] = (float *)ptr;
  }
  return scratch_dev[dev];
}

pse_status launch_mlp_bwd_static(const uint16_t *w, const uint16_t *x, const uint16_t *cache, const float *dy, int n,
                                 float *dw, hipStream_t stream) {
  if (mlp_bwd_parts(n) > kMlpStaticSlots) return PSE_ERR_INVALID_ARG;
  float *work = static_scratch();
  if (!work) return PSE_ERR_HIP;
  launch_mlp_bwd(w, x, cache, dy, n, dw, work, stream);
  return PSE_OK;
}

void launch_mlp_loss(const float *y, const float *t, int n, float *dy, float *loss, hipStream_t stream) {
  k_mlp_loss<<<1, 256, 0, stream>>>(y, t, n, dy, loss);
}

void launch_mlp_adam(float *wm, uint16_t *wb, const float *g, float *m, float *v, float lr, int t,
                     hipStream_t stream) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, t))), c2 = (float)(1.0 / (1.0 - std::pow(b2, t)));
  k_mlp_adam<<<nblk(kWTotal, 256), 256, 0, stream>>>(wm, wb, g, m, v, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
}

template <typename T> void launch_pc_blocks(pse_ctx *c) {
  ProfScope ps(c, PSE_STAGE_PRECOND);
  const int n = c->n;
  if (c->pc_fixed) {
    // the caller's blocks, in the current sorted order
    k_pc_blocks<T, true><<<nblk(n, 256), 256, 0, c->stream>>>(c->pc_user, n, (T *)c->pc_P, (T *)c->pc_Pinv,
                                                             c->flags, c->perm);
    return;
  }
  if (c->pc_have_w) launch_mlp_fwd(c->pc_w, c->pc_feat, n, c->pc_y, nullptr, c->stream);
  k_pc_blocks<T><<<nblk(n, 256), 256, 0, c->stream>>>(c->pc_have_w ? c->pc_y : nullptr, n, (T *)c->pc_P,
                                                       (T *)c->pc_Pinv, c->flags);
}

template <typename T, typename A> void launch_pc_pre(pse_ctx *c, const void *src, void *u) {
  k_pc_pre<T, A><<<nblk(c->n, 256), 256, 0, c->stream>>>((const typename vec4<T>::type *)src, (const T *)c->pc_P,
                                                         c->n, (typename vec4<T>::type *)u,
                                                         (const LzState<A> *)c->lz);
}

template <typename T, typename A>
void launch_pc_post(pse_ctx *c, const void *tp, const void *src, void *out, void *vm_out) {
  using T4 = typename vec4<T>::type;
  k_pc_post<T, A><<<nblk(c->n, 256), 256, 0, c->stream>>>((const T4 *)tp, (const T4 *)src, (const T *)c->pc_P, c->n,
                                                          (T4 *)out, (T4 *)vm_out, (LzState<A> *)c->lz,
                                                          (A *)c->partials, c->counter);
}

template <typename T> void launch_pc_apply_inv(pse_ctx *c, void *y) {
  ProfScope ps(c, PSE_STAGE_PRECOND);
  k_pc_apply<T><<<nblk(c->n, 256), 256, 0, c->stream>>>((const T *)c->pc_Pinv, c->n, (typename vec4<T>::type *)y);
}

void launch_unsort_features(pse_ctx *c, void *out) {
  k_unsort_rows<uint16_t, kNFeat><<<nblk(c->n, 256), 256, 0, c->stream>>>(c->pc_feat, c->perm, c->n,
                                                                           (uint16_t *)out);
}

template <typename T> void launch_unsort_blocks(pse_ctx *c, float *out) {
  k_unsort_blocks<T><<<nblk(c->n, 256), 256, 0, c->stream>>>((const T *)c->pc_P, c->perm, c->n, out);
}

template void launch_pc_blocks<float>(pse_ctx *);
template void launch_pc_blocks<double>(pse_ctx *);
template void launch_pc_apply_inv<float>(pse_ctx *, void *);
template void launch_pc_apply_inv<double>(pse_ctx *, void *);
template void launch_unsort_blocks<float>(pse_ctx *, float *);
template void launch_unsort_blocks<double>(pse_ctx *, float *);
#define PSE_PC_INST(T, A)                                                          \
  template void launch_pc_pre<T, A>(pse_ctx *, const void *, void *);              \
  template void launch_pc_post<T, A>(pse_ctx *, const void *, const void *, void *, void *);
PSE_PC_INST(float, float)
PSE_PC_INST(float, double)
PSE_PC_INST(double, double)

}  // namespace pse
