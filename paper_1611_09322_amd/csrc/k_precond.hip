// Learned block preconditioner of the real-space Krylov sample.
//
// The Lanczos iteration of Sec. II B.1 runs on A = P M_r P^T, with P block
// diagonal (one 3x3 block per particle), and the sample is
// y = P^{-1} A^{1/2} z, whose covariance is M_r.  P_i = I + y_i, where y_i
// is the output of a 24 -> 64 -> 64 -> 9 MLP (bf16 weights and activations,
// fp32 sums on the MFMA units) applied to geometry features of the
// particle's near field (computed from the neighbour list).  Blocks
// that are not finite, nearly singular or ill conditioned fall back to I.
// Training kernels (backward pass, Adam) run off the sampling path.
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
// Gradients of sum_p <dy_p, y_p> for the same network (fp32, from the bf16
// weights and the cached bf16 activations).  Lane j of a wavefront owns
// hidden unit j: row j of dW2 and of dW1, column j of dW3.  Each wavefront
// writes its sums to its own slot of `partial`; k_mlp_reduce adds the slots
// in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_mlp_bwd(const uint16_t *__restrict__ w, const uint16_t *__restrict__ x,
                                                 const uint16_t *__restrict__ cache, const float *__restrict__ dy,
                                                 int n, float *__restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nw = gridDim.x * (blockDim.x >> 6);
  float w3c[kNOut], w2c[kNHid];
#pragma unroll
  for (int o = 0; o < kNOut; ++o) w3c[o] = bf16_to_f32(w[kW3 + o * 64 + lane]);
#pragma unroll
  for (int j = 0; j < kNHid; ++j) w2c[j] = bf16_to_f32(w[kW2 + j * 64 + lane]);  // W2[j][lane]
  float gW2[kNHid], gW1[kNFeat], gW3[kNOut];
#pragma unroll
  for (int k = 0; k < kNHid; ++k) gW2[k] = 0.f;
#pragma unroll
  for (int f = 0; f < kNFeat; ++f) gW1[f] = 0.f;
#pragma unroll
  for (int o = 0; o < kNOut; ++o) gW3[o] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;
  for (int p = gw; p < n; p += nw) {
    const uint16_t *cp = cache + (size_t)p * 2 * kNHid;
    const float h1 = bf16_to_f32(cp[lane]), h2 = bf16_to_f32(cp[kNHid + lane]);
    float dyo[kNOut];
#pragma unroll
    for (int o = 0; o < kNOut; ++o) dyo[o] = dy[(size_t)p * kNOut + o];
    float dh2 = 0.f;
#pragma unroll
    for (int o = 0; o < kNOut; ++o) {
      dh2 += w3c[o] * dyo[o];
      gW3[o] += dyo[o] * h2;
    }
    if (lane < kNOut) {
      float v = 0.f;
#pragma unroll
      for (int o = 0; o < kNOut; ++o) v = (o == lane) ? dyo[o] : v;
      gb3 += v;
    }
    const float dz2 = h2 > 0.f ? dh2 : 0.f;
    gb2 += dz2;
    float dh1 = 0.f;
#pragma unroll
    for (int k = 0; k < kNHid; ++k) {
      gW2[k] += dz2 * __shfl(h1, k, 64);
      dh1 += w2c[k] * __shfl(dz2, k, 64);
    }
    const float dz1 = h1 > 0.f ? dh1 : 0.f;
    gb1 += dz1;
    const uint16_t *xp = x + (size_t)p * kNFeat;
#pragma unroll
    for (int f = 0; f < kNFeat; ++f) gW1[f] += dz1 * bf16_to_f32(xp[f]);
  }
  float *out = partial + (size_t)gw * kWTotal;
#pragma unroll
  for (int f = 0; f < 32; ++f) out[kW1 + lane * 32 + f] = f < kNFeat ? gW1[f] : 0.f;
  out[kB1 + lane] = gb1;
#pragma unroll
  for (int k = 0; k < kNHid; ++k) out[kW2 + lane * 64 + k] = gW2[k];
  out[kB2 + lane] = gb2;
#pragma unroll
  for (int o = 0; o < 16; ++o) out[kW3 + o * 64 + lane] = o < kNOut ? gW3[o] : 0.f;
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

// About 8 rows per wavefront (each row is a chain of dependent lane
// shuffles), up to 256 wavefronts; one fp32 slot of kWTotal per wavefront.
int mlp_bwd_parts(int n) {
  int blocks = nblk(n, 4 * 8);
  if (blocks > 64) blocks = 64;
  if (blocks < 1) blocks = 1;
  return blocks * 4;
}

void launch_mlp_bwd(const uint16_t *w, const uint16_t *x, const uint16_t *cache, const float *dy, int n, float *dw,
                    float *work, hipStream_t stream) {
  const int parts = mlp_bwd_parts(n);
  k_mlp_bwd<<<parts / 4, 256, 0, stream>>>(w, x, cache, dy, n, work);
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
