// Krylov sample on the full mobility M = M_r + M_w (the comparator of
// Sec. III: Lanczos applied to the whole mobility, each product a complete
// near-field product plus a wave-space M_w v).  Vector kernels of the
// iteration; the host runs the loop and solves the tridiagonal problem.
#include "launch.hpp"

namespace pse {

// Block partial sums of <a, b> over the flat 4n scalars; with add != null
// the kernel first forms t = t + add in place (t = a).
template <typename T, typename A>
__global__ void k_fl_dot(T *__restrict__ t, const T *__restrict__ add, const T *__restrict__ v, int len,
                         A *__restrict__ partials) {
  __shared__ A sh[16];
  A acc = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    T x = t[i];
    if (add) {
      x += add[i];
      t[i] = x;
    }
    acc += (A)x * (A)v[i];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// dst = sum of the partials (fixed order), optionally its square root.
template <typename A> __global__ void k_fl_sum(const A *__restrict__ partials, int nparts, A *dst, int root) {
  __shared__ A sh[16];
  A v = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += partials[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) *dst = root ? sqrt(v) : v;
}

// w = t - alpha_m v_m - beta_m v_{m-1} (alpha, beta from device memory),
// block partials of |w|^2.
template <typename T, typename A>
__global__ void k_fl_update(const T *__restrict__ t, const T *__restrict__ vm, const T *__restrict__ vprev,
                            T *__restrict__ w, int len, const A *alpha, const A *beta, A *__restrict__ partials) {
  __shared__ A sh[16];
  const T al = (T)*alpha, be = vprev ? (T)*beta : T(0);
  A acc = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    T x = t[i] - al * vm[i];
    if (vprev) x -= be * vprev[i];
    w[i] = x;
    acc += (A)x * (A)x;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// dst = src / beta (beta from device memory; 0 stays 0).
template <typename T, typename A>
__global__ void k_fl_scale(const T *__restrict__ src, const A *beta, T *__restrict__ dst, int len) {
  const A b = *beta;
  const T s = b > A(0) ? (T)(A(1) / b) : T(0);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) dst[i] = src[i] * s;
}

// y = sum_{j < m} coef_j V_j.
template <typename T, typename A>
__global__ void k_fl_combine(const T *__restrict__ V, size_t ld, int len, int m, const A *__restrict__ coef,
                             T *__restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    A acc = 0;
    for (int j = 0; j < m; ++j) acc += coef[j] * (A)V[(size_t)j * ld + i];
    y[i] = (T)acc;
  }
}

static int fl_blocks(int len) {
  const int b = (len + 255) / 256;
  return b < kRedBlock ? b : kRedBlock;
}

template <typename T, typename A> void launch_fl_norm(pse_ctx *c, const void *v, void *dst) {
  const int len = 4 * c->n, nb = fl_blocks(len);
  k_fl_dot<T, A><<<nb, 256, 0, c->stream>>>((T *)v, nullptr, (const T *)v, len, (A *)c->partials);
  k_fl_sum<A><<<1, 256, 0, c->stream>>>((const A *)c->partials, nb, (A *)dst, 1);
}

template <typename T, typename A> void launch_fl_alpha(pse_ctx *c, void *t, const void *u, const void *v, void *dst) {
  const int len = 4 * c->n, nb = fl_blocks(len);
  k_fl_dot<T, A><<<nb, 256, 0, c->stream>>>((T *)t, (const T *)u, (const T *)v, len, (A *)c->partials);
  k_fl_sum<A><<<1, 256, 0, c->stream>>>((const A *)c->partials, nb, (A *)dst, 0);
}

template <typename T, typename A>
void launch_fl_update(pse_ctx *c, const void *t, const void *vm, const void *vprev, void *w, const void *alpha,
                      const void *beta, void *beta_next) {
  const int len = 4 * c->n, nb = fl_blocks(len);
  k_fl_update<T, A><<<nb, 256, 0, c->stream>>>((const T *)t, (const T *)vm, (const T *)vprev, (T *)w, len,
                                               (const A *)alpha, (const A *)beta, (A *)c->partials);
  k_fl_sum<A><<<1, 256, 0, c->stream>>>((const A *)c->partials, nb, (A *)beta_next, 1);
}

template <typename T, typename A> void launch_fl_scale(pse_ctx *c, const void *src, const void *beta, void *dst) {
  const int len = 4 * c->n;
  k_fl_scale<T, A><<<fl_blocks(len), 256, 0, c->stream>>>((const T *)src, (const A *)beta, (T *)dst, len);
}

template <typename T, typename A> void launch_fl_combine(pse_ctx *c, int m, void *y) {
  const int len = 4 * c->n;
  k_fl_combine<T, A><<<(len + 255) / 256 < 2048 ? (len + 255) / 256 : 2048, 256, 0, c->stream>>>(
      (const T *)c->fl_V, (size_t)len, len, m, (const A *)c->fl_coef, (T *)y);
}

#define PSE_FL_INST(T, A)                                                                                   \
  template void launch_fl_norm<T, A>(pse_ctx *, const void *, void *);                                     \
  template void launch_fl_alpha<T, A>(pse_ctx *, void *, const void *, const void *, void *);               \
  template void launch_fl_update<T, A>(pse_ctx *, const void *, const void *, const void *, void *,         \
                                       const void *, const void *, void *);                                 \
  template void launch_fl_scale<T, A>(pse_ctx *, const void *, const void *, void *);                       \
  template void launch_fl_combine<T, A>(pse_ctx *, int, void *);
PSE_FL_INST(float, float)
PSE_FL_INST(float, double)
PSE_FL_INST(double, double)

}  // namespace pse
