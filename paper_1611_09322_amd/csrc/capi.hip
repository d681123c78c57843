// C ABI of the sampler: context life cycle and the composition of the hot path
//   dx = dt (M_r + M_w) F + sqrt(2 kT dt) (M_r^{1/2} z1 + M_w^{1/2} z2)
// (eqs. langevin, split).  Real space: cell list -> neighbour list ->
// Lanczos on the near-field product.  Wave space: [spread F -> forward FFT]
// -> B(k) scaling + noise (fused with the x pass) -> inverse FFT ->
// interpolation; the deterministic and stochastic wave terms share one
// inverse FFT (Sec. III).
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <thread>
#include <vector>

#include "launch.hpp"

using namespace pse;

namespace {

struct Alloc {
  pse_status st = PSE_OK;
  void *dev(size_t bytes) {
    if (st != PSE_OK) return nullptr;
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
      st = PSE_ERR_OOM;
      return nullptr;
    }
    return p;
  }
  void *host(size_t bytes) {
    if (st != PSE_OK) return nullptr;
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes ? bytes : 16, hipHostMallocDefault) != hipSuccess) {
      st = PSE_ERR_OOM;
      return nullptr;
    }
    return p;
  }
};

inline size_t tsize(const pse_ctx *c) { return c->dbl ? 8 : 4; }

// The preconditioned iteration runs when blocks exist (weights or the
// caller's blocks) and no global fallback is in progress.
inline bool pc_active(const pse_ctx *c) { return c->pc_on && (c->pc_have_w || c->pc_fixed) && !c->pc_suspend; }
inline size_t asize(const pse_ctx *c) { return c->acc_dbl ? 8 : 4; }

void free_ctx(pse_ctx *c) {
  if (!c) return;
  void *dev[] = {c->pos_w, c->pos_s, c->perm, c->cell_of, c->cell_count, c->cell_start, c->nbr, c->nbr_cnt,
                 c->flags, c->V, c->lz, c->partials, c->counter, c->table, c->series, c->grid, c->rgrid, c->grid2, c->tw_M,
                 c->tw_H, c->pc_w, c->pc_feat, c->pc_y, c->pc_P, c->pc_Pinv, c->pc_user, c->fl_V, c->fl_ab,
                 c->fl_coef};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  for (void *p : c->vbuf)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->flags_h) (void)hipHostFree(c->flags_h);
  if (c->pc_fb_h) (void)hipHostFree(c->pc_fb_h);
  if (c->lz_h) (void)hipHostFree(c->lz_h);
  if (c->fl_ab_h) (void)hipHostFree(c->fl_ab_h);
  delete c;
}

template <typename T> void upload_twiddles(pse_ctx *c, Alloc &al) {
  using CT = typename vec2<T>::type;
  const int M = c->p.grid, H = M / 2;
  std::vector<CT> a(M), b(H);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < M; ++k) {
    a[k].x = (T)std::cos(2 * pi * k / M);
    a[k].y = (T)(-std::sin(2 * pi * k / M));
  }
  for (int k = 0; k < H; ++k) {
    b[k].x = (T)std::cos(2 * pi * k / H);
    b[k].y = (T)(-std::sin(2 * pi * k / H));
  }
  c->tw_M = al.dev(sizeof(CT) * M);
  c->tw_H = al.dev(sizeof(CT) * H);
  if (al.st == PSE_OK) {
    if (hipMemcpy(c->tw_M, a.data(), sizeof(CT) * M, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->tw_H, b.data(), sizeof(CT) * H, hipMemcpyHostToDevice) != hipSuccess)
      al.st = PSE_ERR_HIP;
  }
}

// Neighbour-list capacity: expected count in a sphere of radius rc at the
// mean density, plus margin (grown on overflow in set_positions).
// Always a multiple of 8 (the 16-bit list is stored in chunks of 8).
int nbr_capacity(const pse_ctx *c) {
  const double vol = c->d.L * c->d.L * c->d.L;
  const double expect = c->n / vol * 4.18879020478639 * c->p.rcut * c->p.rcut * c->p.rcut;
  int cap = (int)(1.6 * expect + 48);
  if (cap > c->n) cap = c->n;
  if (cap < 8) cap = 8;
  return (cap + 7) & ~7;
}

WaveCoef wave_coef(const pse_ctx *c, double det_scale, double sto_scale, uint64_t seed, uint64_t counter) {
  const double pi = 3.14159265358979323846;
  const double M = c->p.grid;
  WaveCoef w;
  w.two_pi_over_L = 2 * pi / c->d.L;
  w.a = c->p.a;
  w.inv_4xi2 = 1.0 / (4 * c->p.xi * c->p.xi);
  w.sigma2 = c->d.sigma * c->d.sigma;
  w.det_scale = det_scale;
  w.sto_scale = sto_scale;
  w.w_scale = std::pow(M, -1.5);
  w.seed = seed;
  w.counter = counter;
  w.use_philox = 1;
  w.rng = c->rng_dev;
  (void)M;
  return w;
}

// The wave-space coefficients of a step of length dt: deterministic factor
// dt / (eta M^3), stochastic factor sqrt(2 kT dt) / sqrt(eta V).
WaveCoef step_wave_coef(const pse_ctx *c, double dt, uint64_t seed, uint64_t counter) {
  const double cr = std::sqrt(2.0 * c->p.kT * dt);
  const double V = c->d.L * c->d.L * c->d.L;
  const double M3 = (double)c->p.grid * c->p.grid * c->p.grid;
  return wave_coef(c, dt / (c->p.eta * M3), cr / std::sqrt(c->p.eta * V), seed, counter);
}

pse_status hip_status(hipError_t e) { return e == hipSuccess ? PSE_OK : PSE_ERR_HIP; }

hipEvent_t next_event(pse_ctx *c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// ---------------------------------------------------------- hot path
// The Krylov sample in two halves.  lz_start launches the first chunk of
// iterations (as many as the previous sample needed; the kernels stop
// themselves once converged) and queues the read-back of the state;
// lz_finish, after the stream has been synchronised, continues one
// iteration at a time if needed and combines the iterate.  Split so that a
// batch of contexts needs one synchronisation per stream, not per context.
template <typename T, typename A>
pse_status lz_start(pse_ctx *c, const void *z_sorted) {
  launch_lz_init<T, A>(c, z_sorted);
  if (c->lz_external) {
    // captured batch step: the batch launches the iterations of all its
    // replicas together, and lz_finish reads the state back
    c->lz_launched = c->graph_iters;
    return hip_status(hipGetLastError());
  }
  // without weights every block is I; pc_suspend: the global fallback below
  const bool pc = pc_active(c);
  const int maxit = c->lz_maxit;
  int k = c->last_iters < 2 ? 2 : c->last_iters;
  if (c->graph) k = c->graph_iters;  // no host decision: the kernels stop themselves once converged
  if (k > maxit) k = maxit;
  for (int i = 0; i < k; ++i) {
    if (pc) launch_lz_iter_pc<T, A>(c, i, z_sorted);
    else launch_lz_iter<T, A>(c, i, z_sorted);
  }
  c->lz_launched = k;
  if (c->status_external) return hip_status(hipGetLastError());  // read back with the batch's status
  return hip_status(hipMemcpyAsync(c->lz_h, c->lz, sizeof(LzState<A>), hipMemcpyDeviceToHost, c->stream));
}

// The fallback count of the last set_positions, once its copy has landed
// (the caller has synchronised the stream since, or `synced` is false and
// this waits).
void take_pc_fallbacks(pse_ctx *c, bool synced) {
  if (!c->pc_fb_pending) return;
  if (!synced) (void)hipStreamSynchronize(c->stream);
  c->pc_fallbacks = *c->pc_fb_h;
  c->pc_fb_pending = false;
}

template <typename T, typename A>
pse_status lz_finish(pse_ctx *c, const void *z_sorted, void *y_sorted, pse_stats *stats) {
  if (c->graph) {
    // captured: the iterate of the iterations queued by lz_start (or by the
    // batch); the state copied back tells the host after the replay
    // whether they sufficed
    if (c->lz_external && !c->status_external &&
        hipMemcpyAsync(c->lz_h, c->lz, sizeof(LzState<A>), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return PSE_ERR_HIP;
    launch_lz_combine<T, A>(c, y_sorted);
    if (pc_active(c)) launch_pc_apply_inv<T>(c, y_sorted);
    return hip_status(hipGetLastError());
  }
  take_pc_fallbacks(c, true);
  auto *h = (LzState<A> *)c->lz_h;
  const bool pc = pc_active(c);
  const int maxit = c->lz_maxit;
  while (!h->done && c->lz_launched < maxit) {
    if (pc) launch_lz_iter_pc<T, A>(c, c->lz_launched, z_sorted);
    else launch_lz_iter<T, A>(c, c->lz_launched, z_sorted);
    ++c->lz_launched;
    if (hipMemcpyAsync(h, c->lz, sizeof(LzState<A>), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return PSE_ERR_HIP;
  }
  if (pc && (h->nonfinite || !h->converged)) {
    // global fallback: the preconditioned iteration failed (non-finite, or
    // the tolerance not met within max_iter), so the same z is sampled
    // again with P = I, and every particle counts as fallen back
    c->pc_suspend = true;
    pse_status st = lz_start<T, A>(c, z_sorted);
    if (st == PSE_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = PSE_ERR_HIP;
    if (st == PSE_OK) st = lz_finish<T, A>(c, z_sorted, y_sorted, stats);
    c->pc_suspend = false;
    if (stats) stats->precond_fallbacks = c->n;
    return st == PSE_OK || st == PSE_WARN_PRECOND_FALLBACK ? PSE_WARN_PRECOND_FALLBACK : st;
  }
  launch_lz_combine<T, A>(c, y_sorted);
  if (pc) launch_pc_apply_inv<T>(c, y_sorted);  // y = P^-1 A^1/2 z
  c->last_iters = h->m;
  if (stats) {
    stats->max_neighbors = c->flags_h[5];
    stats->neighbor_pairs = c->pairs;
    stats->nbr_index_bytes = c->lds_B ? 2 : 4;
    stats->lds_block_edge = c->lds_B;
    stats->lanczos_iters = h->m;
    stats->converged = h->converged;
    stats->lanczos_rel_change = (double)h->rel_change;
    stats->precond_fallbacks = c->pc_on ? c->pc_fallbacks : 0;
  }
  if (h->nonfinite) return PSE_ERR_NONFINITE;
  if (!h->converged) return PSE_ERR_NOT_CONVERGED;
  if (c->pc_on && c->pc_fallbacks > 0) return PSE_WARN_PRECOND_FALLBACK;
  return PSE_OK;
}

template <typename T, typename A>
pse_status real_sample_core(pse_ctx *c, const void *z_sorted, void *y_sorted, pse_stats *stats) {
  pse_status st = lz_start<T, A>(c, z_sorted);
  if (st != PSE_OK) return st;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PSE_ERR_HIP;
  return lz_finish<T, A>(c, z_sorted, y_sorted, stats);
}

// Wave-space velocity/displacement in sorted order into `out`:
//   forces (sorted, or null) enter with det_scale, noise with sto_scale.
template <typename T>
pse_status wave_core(pse_ctx *c, const void *f_sorted, int noise, const void *W, const WaveCoef &wc, void *out) {
  const size_t M3 = (size_t)c->p.grid * c->p.grid * c->p.grid;
  if (!f_sorted && noise == 0) {
    ProfScope ps(c, PSE_STAGE_OTHER);
    launch_zero_words(c->stream, out, sizeof(T) * c->n);  // 4 components
    return hip_status(hipGetLastError());
  }
  // caller noise: zeta on the half spectrum as given (NOISE_KSPACE), or
  // the DFT of the grid noise W (scaled by M^{-3/2} in the x pass)
  const bool kspace = (c->p.flags & PSE_FLAG_NOISE_KSPACE) != 0;
  const void *spec = kspace ? W : c->grid2;
  if (noise == 2 && !kspace) {
    launch_grid_op<T>(c, GridOp::FftZ, W, c->grid2, nullptr, -1, 0);
    launch_grid_op<T>(c, GridOp::FftStrided, nullptr, c->grid2, nullptr, 1, -1);
    launch_grid_op<T>(c, GridOp::FftStrided, nullptr, c->grid2, nullptr, 0, -1);
  }
  (void)M3;
  if (f_sorted) {
    launch_spread_interp<T>(c, true, f_sorted, c->rgrid);
    launch_grid_op<T>(c, GridOp::FftZAos, c->rgrid, c->grid, nullptr, -1, 0);
    launch_grid_op<T>(c, GridOp::FftStrided, nullptr, c->grid, nullptr, 1, -1);
  }
  WaveCoef wk = wc;
  if (noise == 2 && kspace) wk.w_scale = 1.0;
  launch_grid_op<T>(c, GridOp::XFused, noise == 2 ? spec : nullptr, c->grid, &wk, f_sorted ? 1 : 0, noise);
  launch_grid_op<T>(c, GridOp::FftStrided, nullptr, c->grid, nullptr, 1, +1);
  launch_grid_op<T>(c, GridOp::FftZAos, c->grid, c->rgrid, nullptr, +1, 0);
  launch_spread_interp<T>(c, false, c->rgrid, out);
  return hip_status(hipGetLastError());
}

// Full displacement.  z1: caller-order real noise (device) or null with
// use_philox; W: grid noise or null.  sample_begin queues everything that
// does not wait for the Krylov stopping decision (noise, the first chunk of
// Lanczos iterations, M_r F, the whole wave-space part); sample_end, after
// the stream is synchronised, finishes the Krylov sample and combines.
struct SampleState {
  bool real = false;   // a real-space sample is part of this call
  bool forces = false; // dt M F is part of this call
  double cr = 0.0;     // sqrt(2 kT dt)
};

template <typename T, typename A>
pse_status sample_begin(pse_ctx *c, bool philox, uint64_t seed, uint64_t counter, const void *z1, const void *W,
                        double dt, const void *forces, SampleState &ss, const void *f_add = nullptr) {
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  if (!(dt >= 0)) return PSE_ERR_INVALID_ARG;
  ss.cr = std::sqrt(2.0 * c->p.kT * dt);
  void *z_s = c->vbuf[0], *wave = c->vbuf[4], *f_s = c->vbuf[6], *ur = c->vbuf[7];
  ss.real = false;
  if (philox) {
    launch_real_noise<T>(c, z_s, seed, counter);  // caller-order noise, written in sorted order
    ss.real = true;
  } else if (z1) {
    launch_gather3<T>(c, z1, z_s);
    ss.real = true;
  }
  ss.real = ss.real && ss.cr > 0;
  if (ss.real) {
    const pse_status st = lz_start<T, A>(c, z_s);
    if (st != PSE_OK) return st;
  }
  ss.forces = (forces || f_add) && dt > 0;
  if (ss.forces) {
    // caller-order forces, plus the sorted overlap repulsion of a Brownian step
    if (f_add) launch_gather3_add<T>(c, forces, f_add, f_s);
    else launch_gather3<T>(c, forces, f_s);
    launch_spmv<T, A>(c, f_s, ur, false, nullptr);
  }
  const WaveCoef wc = step_wave_coef(c, dt, seed, counter);
  const int noise = (ss.cr > 0) ? (philox ? 1 : (W ? 2 : 0)) : 0;
  if (c->wave_external) return hip_status(hipGetLastError());  // the batch launches it
  return wave_core<T>(c, ss.forces ? f_s : nullptr, noise, W, wc, wave);
}

template <typename T, typename A>
pse_status sample_end(pse_ctx *c, const SampleState &ss, double dt, void *disp, pse_stats *stats) {
  void *z_s = c->vbuf[0], *yr = c->vbuf[1], *wave = c->vbuf[4], *ur = c->vbuf[7];
  pse_status st = PSE_OK;
  if (ss.real) {
    st = lz_finish<T, A>(c, z_s, yr, stats);
    if (st < 0 && st != PSE_ERR_NOT_CONVERGED) return st;  // warnings (> 0) continue
  } else if (stats) {
    stats->lanczos_iters = 0;
    stats->converged = 1;
    stats->lanczos_rel_change = 0;
    stats->precond_fallbacks = 0;
  }
  launch_finalize<T>(c, ss.real ? yr : nullptr, ss.cr, ss.forces ? ur : nullptr, dt, wave, disp);
  if (c->graph) {
    // the device flags of this step (list and halo overflow, non-finite
    // positions) for the host's check after the replay
    if (c->status_external) return hip_status(hipGetLastError());
    return hip_status(hipMemcpyAsync(c->flags_h, c->flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream));
  }
  if (stats) {
    stats->max_neighbors = c->flags_h[5];
    stats->neighbor_pairs = c->pairs;
    stats->nbr_index_bytes = c->lds_B ? 2 : 4;
    stats->lds_block_edge = c->lds_B;
  }
  const pse_status se = hip_status(hipGetLastError());
  return se != PSE_OK ? se : st;
}

template <typename T, typename A>
pse_status sample_impl(pse_ctx *c, bool philox, uint64_t seed, uint64_t counter, const void *z1, const void *W,
                       double dt, const void *forces, void *disp, pse_stats *stats) {
  if (!disp) return PSE_ERR_INVALID_ARG;
  SampleState ss;
  const pse_status sb = sample_begin<T, A>(c, philox, seed, counter, z1, W, dt, forces, ss);
  if (sb != PSE_OK) return sb;
  if (ss.real && hipStreamSynchronize(c->stream) != hipSuccess) return PSE_ERR_HIP;
  return sample_end<T, A>(c, ss, dt, disp, stats);
}

#define DISPATCH(ctx, CALL)                                   \
  do {                                                        \
    if ((ctx)->dbl) {                                         \
      using T = double;                                       \
      using A = double;                                       \
      return CALL;                                            \
    } else if ((ctx)->acc_dbl) {                              \
      using T = float;                                        \
      using A = double;                                       \
      return CALL;                                            \
    } else {                                                  \
      using T = float;                                        \
      using A = float;                                        \
      return CALL;                                            \
    }                                                         \
  } while (0)

template <typename T>
pse_status build_neighbors(pse_ctx *c) {
  if (c->lds_B) launch_nbr_lds(c);
  else launch_nbr<T>(c);
  if (hipMemcpyAsync(c->flags_h, c->flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return PSE_ERR_HIP;
  return PSE_OK;
}

template <typename T>
pse_status set_positions_impl(pse_ctx *c, const void *pos) {
  c->have_pos = false;
  launch_bin<T>(c, pos);
  if (c->graph) {
    // captured: block edge, halo capacity and list capacity stay as fixed
    // at capture; the kernels flag what does not fit
    if (c->lds_B) {
      if (!c->nbr_external) launch_nbr_lds(c);  // else the batch's batched launch
    } else {
      launch_nbr<T>(c);
    }
    if (c->pc_on) {
      if (c->lds_B && !c->pc_fixed) launch_feat_lds(c);
      launch_pc_blocks<T>(c);
      if (!c->status_external &&
          hipMemcpyAsync(c->pc_fb_h, c->flags + 6, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return PSE_ERR_HIP;
      c->pc_fb_pending = true;
    }
    c->have_pos = true;
    return hip_status(hipGetLastError());
  }
  // FP32 storage: stage the near-field halo in LDS when it fits.  The block
  // edge B (cells) is the largest whose halo leaves room for two workgroups
  // per CU (one stages while the other computes), searched downwards from
  // the previous choice; blocks of more cells keep enough targets per
  // workgroup when cells hold few particles.  Without such a B, the largest
  // whose halo fits the budget of one workgroup.
  c->lds_B = 0;
  if (sizeof(T) == 4) {
    auto lds_bytes = [](int hmax) {
      // one halo slot more: the zero source read by padding entries
      return (sizeof(float4) + sizeof(float2)) * (size_t)(hmax + 1) + sizeof(float2) * kTableN;
    };
    int hm[5] = {-1, -1, -1, -1, -1};
    auto halo_max = [&](int B) -> pse_status {
      if (hipMemsetAsync(c->flags + 4, 0, sizeof(int), c->stream) != hipSuccess) return PSE_ERR_HIP;
      launch_halo_size(c, B);
      if (hipMemcpyAsync(c->flags_h, c->flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
          hipStreamSynchronize(c->stream) != hipSuccess)
        return PSE_ERR_HIP;
      if (c->flags_h[0]) return PSE_ERR_NONFINITE;
      hm[B] = c->flags_h[4];
      return PSE_OK;
    };
    const int start = c->lds_B_pref ? c->lds_B_pref : 4;
    int pick = 0;
    // B >= 2 with two workgroups per CU, then B >= 2 with one, then B = 1
    for (int pass = 0; pass < 3 && !pick; ++pass) {
      for (int B = pass < 2 ? start : 1; B >= (pass < 2 ? 2 : 1) && !pick; --B) {
        if (c->d.nc < B + 2) continue;
        if (hm[B] < 0) {
          const pse_status hs = halo_max(B);
          if (hs != PSE_OK) return hs;
        }
        const size_t lim = pass == 0 ? kLdsPerCU / 2 - lds_static_extra(B) : kLdsBudget;
        if (hm[B] <= 65535 && lds_bytes(hm[B]) <= lim) pick = B;
      }
    }
    if (pick) {
      c->lds_B = c->lds_B_pref = pick;
      c->hcap = hm[pick] + 1;
      const int nb = (c->d.nc + pick - 1) / pick;
      c->lds_blocks = nb * nb * nb;
    }
  }
  pse_status st = build_neighbors<T>(c);
  if (st != PSE_OK) return st;
  if (c->flags_h[0]) return PSE_ERR_NONFINITE;
  if (c->flags_h[1] > c->nbr_cap) {
    const int cap = (c->flags_h[1] + 32 + 7) & ~7;
    c->graph_stale = true;  // a captured graph holds the old list
    (void)hipFree(c->nbr);
    c->nbr = nullptr;
    if (hipMalloc(&c->nbr, sizeof(int) * (size_t)cap * c->n) != hipSuccess) {
      c->nbr = nullptr;
      c->nbr_cap = 0;
      return PSE_ERR_OOM;
    }
    c->nbr_cap = cap;
    if (hipMemsetAsync(c->flags, 0, sizeof(int) * 8, c->stream) != hipSuccess) return PSE_ERR_HIP;
    st = build_neighbors<T>(c);
    if (st != PSE_OK) return st;
  }
  {
    int64_t pairs;
    std::memcpy(&pairs, c->flags_h + 2, sizeof pairs);
    c->pairs = pairs;
  }
  if (c->pc_on) {
    // features (the LDS path from the list and the staged halo; the global
    // build accumulated them itself), network, blocks, fallbacks; with the
    // caller's blocks only their gather into the new sorted order
    if (c->lds_B && !c->pc_fixed) launch_feat_lds(c);
    launch_pc_blocks<T>(c);
    // the count is taken after the next synchronisation (no wait here)
    if (hipMemcpyAsync(c->pc_fb_h, c->flags + 6, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return PSE_ERR_HIP;
    c->pc_fb_pending = true;
  }
  c->have_pos = true;
  return hip_status(hipGetLastError());
}

// One Euler-Maruyama step of eq. (langevin): rebuild the cell and neighbour
// lists at the current positions (with the overlap repulsion accumulated by
// the same scan), draw the displacement dt M (F_ext + F_rep) + sqrt(2 kT dt)
// M^{1/2} dW with the combined FFT pair, and move the particles.
template <typename T, typename A>
pse_status bd_step_impl(pse_ctx *c, void *pos, const void *fext, double dt, double krep, uint64_t seed,
                        uint64_t step, void *disp, pse_stats *stats) {
  c->rep_k = krep;
  pse_status st = set_positions_impl<T>(c, pos);
  c->rep_k = 0.0;
  if (st != PSE_OK) return st;
  void *out = disp ? disp : c->vbuf[5];  // caller-order 3n scratch when the caller keeps no displacement
  SampleState ss;
  st = sample_begin<T, A>(c, true, seed, step, nullptr, nullptr, dt, fext, ss, krep > 0 ? c->vbuf[kRepBuf] : nullptr);
  if (st != PSE_OK) return st;
  if (ss.real && hipStreamSynchronize(c->stream) != hipSuccess) return PSE_ERR_HIP;
  st = sample_end<T, A>(c, ss, dt, out, stats);
  if (st < 0 && st != PSE_ERR_NOT_CONVERGED) return st;
  launch_advance<T>(c, pos, out);
  const pse_status se = hip_status(hipGetLastError());
  return se != PSE_OK ? se : st;
}

// Krylov sample y = M^{1/2} z on the full mobility M = M_r + M_w (the
// comparator of Sec. III): the Lanczos process of Sec. II B.1 with each
// product a near-field product plus a wave-space product M_w v (spread,
// FFT, B(k), inverse FFT, interpolation), alpha and beta reduced on the
// device, the tridiagonal square root solved on the host in FP64 after
// every iteration, the same successive-iterate stopping rule.
template <typename T, typename A>
pse_status full_sample_impl(pse_ctx *c, const void *z, void *y, pse_stats *stats) {
  using T4 = typename vec4<T>::type;
  constexpr int K = kFullMaxIter;
  const size_t n = (size_t)c->n;
  T4 *V = (T4 *)c->fl_V;
  A *ab = (A *)c->fl_ab, *abh = (A *)c->fl_ab_h;  // alpha_m at [m], beta_m at [K + m]
  void *zs = c->vbuf[0], *t = c->vbuf[2], *w = c->vbuf[3], *u = c->vbuf[4], *ys = c->vbuf[1];
  const int maxit = std::min(c->p.lanczos_max_iter, (int32_t)K);
  auto read_ab = [&]() {
    return hipMemcpyAsync(abh, ab, sizeof(A) * (2 * K + 2), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
           hipStreamSynchronize(c->stream) == hipSuccess;
  };
  launch_gather3<T>(c, z, zs);
  launch_fl_norm<T, A>(c, zs, ab + K);
  launch_fl_scale<T, A>(c, zs, ab + K, V);
  if (!read_ab()) return PSE_ERR_HIP;
  const double beta0 = (double)abh[K];
  if (!std::isfinite(beta0)) return PSE_ERR_NONFINITE;
  const double M3 = (double)c->p.grid * c->p.grid * c->p.grid;
  const WaveCoef wc = wave_coef(c, 1.0 / (c->p.eta * M3), 0.0, 0, 0);
  std::vector<double> d, e, sk, sold;
  int m = 0;
  bool conv = beta0 == 0.0, finite = true;
  double rel = 1.0;
  while (!conv && m < maxit) {
    const T4 *vm = V + (size_t)m * n;
    launch_spmv<T, A>(c, vm, t, false, nullptr);                                   // M_r v_m
    const pse_status ws = wave_core<T>(c, vm, 0, nullptr, wc, u);                   // M_w v_m
    if (ws != PSE_OK) return ws;
    launch_fl_alpha<T, A>(c, t, u, vm, ab + m);                                     // t = M v_m, alpha_m
    launch_fl_update<T, A>(c, t, vm, m ? V + (size_t)(m - 1) * n : nullptr, w, ab + m, ab + K + m,
                           ab + K + m + 1);                                         // w, beta_{m+1}
    if (!read_ab()) return PSE_ERR_HIP;
    ++m;
    d.assign(abh, abh + m);
    e.assign(abh + K + 1, abh + K + m);  // beta_1 .. beta_{m-1}
    const double bnext = (double)abh[K + m];
    sk.assign(m, 0.0);
    finite = std::isfinite(bnext) && tridiag_sqrt_e1_host(m, d.data(), e.data(), sk.data());
    if (!finite) break;
    double num = 0.0, den = 0.0, sc2 = bnext * bnext;
    for (int j = 0; j < m; ++j) {
      const double o = j < (int)sold.size() ? sold[j] : 0.0;
      num += (sk[j] - o) * (sk[j] - o);
      den += sk[j] * sk[j];
      sc2 += d[j] * d[j];
    }
    rel = den > 0.0 ? std::sqrt(num / den) : 0.0;
    conv = (m > 1 && rel <= c->p.lanczos_tol) || bnext <= 1e-11 * std::sqrt(sc2);
    sold = sk;
    if (!conv && m < maxit) launch_fl_scale<T, A>(c, w, ab + K + m, V + (size_t)m * n);  // v_m = w / beta_m
  }
  std::vector<A> coef(std::max(m, 1));
  for (int j = 0; j < m; ++j) coef[j] = (A)(beta0 * sk[j]);
  if (m > 0) {
    if (hipMemcpyAsync(c->fl_coef, coef.data(), sizeof(A) * m, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return PSE_ERR_HIP;
    launch_fl_combine<T, A>(c, m, ys);
  } else if (hipMemsetAsync(ys, 0, sizeof(T) * 4 * n, c->stream) != hipSuccess) {
    return PSE_ERR_HIP;
  }
  launch_finalize<T>(c, ys, 1.0, nullptr, 0.0, nullptr, y);
  // the coefficients are read by the combine before this call returns
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PSE_ERR_HIP;
  if (stats) {
    stats->lanczos_iters = m;
    stats->converged = conv && finite;
    stats->lanczos_rel_change = rel;
    stats->precond_fallbacks = 0;
  }
  if (!finite) return PSE_ERR_NONFINITE;
  if (!conv) return PSE_ERR_NOT_CONVERGED;
  return hip_status(hipGetLastError());
}

template <typename T, typename A>
pse_status real_matvec_impl(pse_ctx *c, const void *v, void *w) {
  launch_gather3<T>(c, v, c->vbuf[0]);
  launch_spmv<T, A>(c, c->vbuf[0], c->vbuf[7], false, nullptr);
  launch_finalize<T>(c, nullptr, 0.0, c->vbuf[7], 1.0, nullptr, w);
  return hip_status(hipGetLastError());
}

template <typename T, typename A>
pse_status real_sample_impl(pse_ctx *c, const void *z, void *y, pse_stats *stats) {
  launch_gather3<T>(c, z, c->vbuf[0]);
  pse_status st = real_sample_core<T, A>(c, c->vbuf[0], c->vbuf[1], stats);
  if (st < 0 && st != PSE_ERR_NOT_CONVERGED) return st;  // warnings (> 0) continue
  launch_finalize<T>(c, c->vbuf[1], 1.0, nullptr, 0.0, nullptr, y);
  const pse_status se = hip_status(hipGetLastError());
  return se != PSE_OK ? se : st;
}

template <typename T>
pse_status wave_sample_impl(pse_ctx *c, const void *W, void *y) {
  const double V = c->d.L * c->d.L * c->d.L;
  WaveCoef wc = wave_coef(c, 0.0, 1.0 / std::sqrt(c->p.eta * V), 0, 0);
  pse_status st = wave_core<T>(c, nullptr, 2, W, wc, c->vbuf[4]);
  if (st != PSE_OK) return st;
  launch_finalize<T>(c, nullptr, 0.0, nullptr, 0.0, c->vbuf[4], y);
  return hip_status(hipGetLastError());
}

template <typename T, typename A>
pse_status wave_apply_impl(pse_ctx *c, const void *F, void *u, bool with_real) {
  const double M3 = (double)c->p.grid * c->p.grid * c->p.grid;
  launch_gather3<T>(c, F, c->vbuf[6]);
  WaveCoef wc = wave_coef(c, 1.0 / (c->p.eta * M3), 0.0, 0, 0);
  pse_status st = wave_core<T>(c, c->vbuf[6], 0, nullptr, wc, c->vbuf[4]);
  if (st != PSE_OK) return st;
  if (with_real) launch_spmv<T, A>(c, c->vbuf[6], c->vbuf[7], false, nullptr);
  launch_finalize<T>(c, nullptr, 0.0, with_real ? c->vbuf[7] : nullptr, 1.0, c->vbuf[4], u);
  return hip_status(hipGetLastError());
}

}  // namespace

namespace pse {
void prof_begin(pse_ctx *c, int stage) {
  if (!(c->prof_mask & (1u << stage)) || c->ev_open >= 0) return;
  hipEvent_t e = next_event(c);
  if (!e) return;
  (void)hipEventRecord(e, c->stream);
  c->ev_open = (int)c->ev_used - 1;
  c->ev_stage.push_back(stage);
}
void prof_end(pse_ctx *c, int stage) {
  if (!(c->prof_mask & (1u << stage)) || c->ev_open < 0 || c->ev_stage.back() != stage) return;
  hipEvent_t e = next_event(c);
  if (!e) return;
  (void)hipEventRecord(e, c->stream);
  c->ev_open = -1;
}
}  // namespace pse

// ---------------------------------------------------------------- batches
// Independent replicas (each its own context) share S streams; one host
// thread per stream queues its replicas' work, so a batch sample needs one
// synchronisation per stream (the Krylov stopping decision) instead of one
// per replica, and the replicas of different streams run concurrently.
struct pse_batch {
  std::vector<pse_ctx *> ctx;
  std::vector<hipStream_t> streams;
  hipStream_t user = nullptr;
  int device = 0;
  hipEvent_t start = nullptr;
  std::vector<hipEvent_t> done;  // per replica: end of its last sample
  std::vector<hipEvent_t> join;  // per stream
  // captured step (pse_batch_graph_*)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t gstream = nullptr;  // capture and replay stream (the caller's may be the null stream)
  hipEvent_t g_in = nullptr, g_out = nullptr;
  uint64_t *rng_h = nullptr, *rng_d = nullptr;  // (seed + r, counter) per replica, pinned host / device
  std::vector<const void *> g_pos, g_forces;
  std::vector<void *> g_disp;
  std::vector<int> g_hcap;  // halo capacity each replica was captured with
  double g_dt = 0.0, g_headroom = 0.0;
  int g_extra = 0;
  // batched Krylov loops of the captured step: the replicas on the LDS
  // product (FP32 storage) without the preconditioner iterate together, one
  // loop per Lanczos scalar type ([0] FP32, [1] FP64)
  struct LzBatch {
    void *reps = nullptr;              // LzRep<A> [nrep], device
    int2 *maps = nullptr;              // product blocks of every group, then the vector blocks
    std::vector<pse::LzGroup> groups;  // pmap pointers into maps
    const int2 *vmap = nullptr;
    int nrep = 0, nv = 0, iters = 0;
    std::vector<int> members;  // replica of each LzRep
  } lzb[2];
  // replicas whose whole captured step is batched ([0] FP32, [1] FP64
  // Lanczos scalars)
  struct FullBatch {
    pse::SampRep *reps = nullptr;
    int2 *maps = nullptr;
    pse::SampMaps m{};
    std::vector<int> members;
  } full[2];
  std::vector<char> is_full;  // per replica
  // batched neighbour build of the captured step (LDS path)
  pse::NbrRep *nb_reps = nullptr;
  int2 *nb_maps = nullptr;
  std::vector<pse::NbrGroup> nb_groups;
  std::vector<int> nb_members;
  // batched wave-space part of the captured step (replicas without forces,
  // FP32 storage, kT > 0)
  pse::WaveRep *wv_reps = nullptr;
  int2 *wv_imap = nullptr;
  std::vector<pse::WaveGroup> wv_groups;
  std::vector<int> wv_members;
  // status of every replica after a replay (one kernel, one copy)
  pse::RepStatusSrc *stat_src = nullptr;
  pse::RepStatus *stat_d = nullptr, *stat_h = nullptr;
};

namespace pse {

static pse_status ctx_begin(pse_ctx *c, uint64_t seed, uint64_t counter, double dt, const void *f, SampleState &ss) {
  if (c->dbl) return sample_begin<double, double>(c, true, seed, counter, nullptr, nullptr, dt, f, ss);
  if (c->acc_dbl) return sample_begin<float, double>(c, true, seed, counter, nullptr, nullptr, dt, f, ss);
  return sample_begin<float, float>(c, true, seed, counter, nullptr, nullptr, dt, f, ss);
}

static pse_status ctx_end(pse_ctx *c, const SampleState &ss, double dt, void *disp, pse_stats *stats) {
  if (c->dbl) return sample_end<double, double>(c, ss, dt, disp, stats);
  if (c->acc_dbl) return sample_end<float, double>(c, ss, dt, disp, stats);
  return sample_end<float, float>(c, ss, dt, disp, stats);
}

// Worse of two statuses: any error beats a warning beats OK.
static pse_status worse(pse_status a, pse_status b) {
  if (a < 0) return a;
  if (b < 0) return b;
  return a > b ? a : b;
}

// Run fn(stream index, replica) for every replica, one host thread per
// stream, replicas of a stream in order; returns the worst status.
template <typename F> static pse_status for_streams(pse_batch *b, F fn) {
  const int S = (int)b->streams.size(), R = (int)b->ctx.size();
  std::vector<pse_status> st(S, PSE_OK);
  std::vector<std::thread> th;
  for (int q = 0; q < S; ++q)
    th.emplace_back([&, q] {
      if (hipSetDevice(b->device) != hipSuccess) {
        st[q] = PSE_ERR_HIP;
        return;
      }
      st[q] = fn(q, R);
    });
  for (auto &t : th) t.join();
  pse_status w = PSE_OK;
  for (pse_status x : st) w = worse(w, x);
  return w;
}

// The replica streams wait for `from` (by default the caller's stream),
// and `from` waits for them.
static pse_status fork(pse_batch *b, hipStream_t from) {
  if (hipEventRecord(b->start, from) != hipSuccess) return PSE_ERR_HIP;
  for (hipStream_t s : b->streams)
    if (hipStreamWaitEvent(s, b->start, 0) != hipSuccess) return PSE_ERR_HIP;
  return PSE_OK;
}
static pse_status fork(pse_batch *b) { return fork(b, b->user); }

static pse_status join(pse_batch *b, hipStream_t to) {
  for (size_t q = 0; q < b->streams.size(); ++q)
    if (hipEventRecord(b->join[q], b->streams[q]) != hipSuccess || hipStreamWaitEvent(to, b->join[q], 0) != hipSuccess)
      return PSE_ERR_HIP;
  return PSE_OK;
}
static pse_status join(pse_batch *b) { return join(b, b->user); }

static void free_graph(pse_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  for (auto &z : b->lzb) {
    if (z.reps) (void)hipFree(z.reps);
    if (z.maps) (void)hipFree(z.maps);
    z = pse_batch::LzBatch{};
  }
  for (auto &f : b->full) {
    if (f.reps) (void)hipFree(f.reps);
    if (f.maps) (void)hipFree(f.maps);
    f = pse_batch::FullBatch{};
  }
  b->is_full.clear();
  if (b->nb_reps) (void)hipFree(b->nb_reps);
  if (b->nb_maps) (void)hipFree(b->nb_maps);
  b->nb_reps = nullptr;
  b->nb_maps = nullptr;
  b->nb_groups.clear();
  b->nb_members.clear();
  if (b->wv_reps) (void)hipFree(b->wv_reps);
  if (b->wv_imap) (void)hipFree(b->wv_imap);
  b->wv_reps = nullptr;
  b->wv_imap = nullptr;
  b->wv_groups.clear();
  b->wv_members.clear();
  if (b->stat_src) (void)hipFree(b->stat_src);
  if (b->stat_d) (void)hipFree(b->stat_d);
  if (b->stat_h) (void)hipHostFree(b->stat_h);
  b->stat_src = nullptr;
  b->stat_d = b->stat_h = nullptr;
}

static void free_batch(pse_batch *b) {
  if (!b) return;
  free_graph(b);
  if (b->rng_h) (void)hipHostFree(b->rng_h);
  if (b->rng_d) (void)hipFree(b->rng_d);
  if (b->g_in) (void)hipEventDestroy(b->g_in);
  if (b->g_out) (void)hipEventDestroy(b->g_out);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  for (pse_ctx *c : b->ctx) free_ctx(c);
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->start) (void)hipEventDestroy(b->start);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

}  // namespace pse

extern "C" {

const char *pse_status_string(pse_status s) {
  switch (s) {
    case PSE_OK: return "ok";
    case PSE_ERR_INVALID_ARG: return "invalid argument";
    case PSE_ERR_OOM: return "device allocation failed";
    case PSE_ERR_HIP: return "HIP runtime error";
    case PSE_ERR_PARAMS: return "parameters rejected by the error model";
    case PSE_ERR_NONFINITE: return "non-finite value";
    case PSE_ERR_NOT_CONVERGED: return "Lanczos did not converge within max_iter";
    case PSE_ERR_NO_POSITIONS: return "positions not set";
    case PSE_WARN_PRECOND_FALLBACK: return "learned preconditioner fell back to identity";
  }
  return "unknown status";
}

pse_status pse_create(const pse_params *p, void *stream, pse_ctx **out) {
  if (!p || !out) return PSE_ERR_INVALID_ARG;
  *out = nullptr;
  Derived d;
  const pse_status ps = derive_params(*p, &d);
  if (ps != PSE_OK) return ps;
  if (p->precond != 0 && p->precond != 1) return PSE_ERR_PARAMS;
  pse_ctx *c = new (std::nothrow) pse_ctx();
  if (!c) return PSE_ERR_OOM;
  c->p = *p;
  c->d = d;
  c->stream = (hipStream_t)stream;
  c->dbl = p->precision == PSE_FP64;
  c->acc_dbl = p->precision != PSE_FP32;
  c->n = p->n;
  c->lz_maxit = std::min(p->lanczos_max_iter, (int32_t)kMaxIter);
  c->ncell = d.nc * d.nc * d.nc;
  Alloc al;
  const size_t n = (size_t)p->n, T = tsize(c), A = asize(c);
  c->pos_w = al.dev(4 * T * n);
  c->pos_s = al.dev(4 * T * n);
  c->perm = (int *)al.dev(sizeof(int) * n);
  c->cell_of = (int *)al.dev(sizeof(int) * 2 * n);  // cells, then slots
  c->cell_count = (int *)al.dev(sizeof(int) * 2 * c->ncell);
  c->cell_start = (int *)al.dev(sizeof(int) * (c->ncell + 1));
  c->nbr_cap = nbr_capacity(c);
  c->nbr = (int *)al.dev(sizeof(int) * (size_t)c->nbr_cap * n);
  c->nbr_cnt = (int *)al.dev(sizeof(int) * n);

  c->flags = (int *)al.dev(sizeof(int) * 8);
  c->flags_h = (int *)al.host(sizeof(int) * 8);
  c->pc_fb_h = (int *)al.host(sizeof(int));
  for (auto &v : c->vbuf) v = al.dev(4 * T * n);  // [8], [9]: preconditioned Lanczos
  c->V = al.dev(4 * T * n * (size_t)(kMaxIter + 1));
  const size_t lzbytes = c->acc_dbl ? sizeof(LzState<double>) : sizeof(LzState<float>);
  c->lz = al.dev(lzbytes);
  c->lz_h = al.host(lzbytes);
  // partial sums: one per block of the widest reduction (256-particle
  // blocks, or one per LDS target block of edge 1 cell)
  const size_t nparts = std::max<size_t>(std::max<size_t>(kRedBlock, (n + 255) / 256), (size_t)c->ncell);
  c->partials = al.dev(A * (nparts + kRedBlock));  // + the alpha partial sums of a Lanczos step
  c->counter = (unsigned *)al.dev(sizeof(unsigned));
  const size_t M3 = (size_t)p->grid * p->grid * p->grid;
  c->grid = al.dev(3 * T * M3);
  c->rgrid = al.dev(4 * T * M3);
  if (p->flags & PSE_FLAG_FULL_LANCZOS) {
    c->fl_V = al.dev(4 * T * n * (size_t)(kFullMaxIter + 1));
    c->fl_ab = al.dev(A * (2 * kFullMaxIter + 2));
    c->fl_ab_h = al.host(A * (2 * kFullMaxIter + 2));
    c->fl_coef = al.dev(A * kFullMaxIter);
  }
  // spectrum of caller grid noise W (not needed when the caller gives zeta)
  if (!(p->flags & PSE_FLAG_NOISE_KSPACE)) c->grid2 = al.dev(3 * T * M3);
  if (p->precond == 1) {
    c->pc_on = true;
    c->pc_w = (uint16_t *)al.dev(sizeof(uint16_t) * kWTotal);
    c->pc_feat = (uint16_t *)al.dev(sizeof(uint16_t) * kNFeat * n);
    c->pc_y = (float *)al.dev(sizeof(float) * kNOut * n);
    c->pc_P = al.dev(12 * T * n);
    c->pc_Pinv = al.dev(12 * T * n);
    c->pc_user = (float *)al.dev(sizeof(float) * 9 * n);
  }
  // real-space tables (FP64 host evaluation of Appendix A)
  double serF[kSeriesTerms], serG[kSeriesTerms];
  fg_series_coeffs(p->xi, p->a, serF, serG);
  for (int i = 0; i < kSeriesTerms; ++i) {
    c->series_h[i] = serF[i];
    c->series_h[kSeriesTerms + i] = serG[i];
  }
  const double thr = fg_small_r_threshold(p->xi, p->a);
  c->small_r2 = thr * thr;
  c->series = (double *)al.dev(sizeof(double) * 2 * kSeriesTerms);
  if (!c->dbl) c->table = (float2 *)al.dev(sizeof(float2) * kTableN);
  if (c->dbl) upload_twiddles<double>(c, al);
  else upload_twiddles<float>(c, al);
  if (al.st != PSE_OK) {
    free_ctx(c);
    return al.st;
  }
  hipError_t e = hipMemcpy(c->series, c->series_h, sizeof(double) * 2 * kSeriesTerms, hipMemcpyHostToDevice);
  if (!c->dbl && e == hipSuccess) {
    std::vector<float2> tab(kTableN);
    fg_build_table(p->xi, p->a, p->rcut, d.mu0, serF, serG, tab.data());
    e = hipMemcpy(c->table, tab.data(), sizeof(float2) * kTableN, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(c->counter, 0, sizeof(unsigned));
  if (e == hipSuccess && c->pc_w) e = hipMemset(c->pc_w, 0, sizeof(uint16_t) * kWTotal);
  if (e != hipSuccess) {
    free_ctx(c);
    return PSE_ERR_HIP;
  }
  *out = c;
  return PSE_OK;
}

pse_status pse_destroy(pse_ctx *ctx) {
  if (ctx) (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
  return PSE_OK;
}

pse_status pse_get_derived(const pse_ctx *c, pse_derived *o) {
  if (!c || !o) return PSE_ERR_INVALID_ARG;
  o->h = c->d.h;
  o->sigma = c->d.sigma;
  o->gauss_m = c->d.gm;
  o->eta_se = c->d.eta_se;
  o->eps_real = c->d.eps_real;
  o->eps_wave = c->d.eps_wave;
  o->eps_quad = c->d.eps_quad;
  o->cells = c->d.nc;
  o->self_real = c->d.self_r;
  o->eps_alias = c->d.eps_alias;
  o->eps_real_tail = c->d.eps_real_tail;
  o->eps_real_coherent = c->d.eps_real_coherent;
  return PSE_OK;
}

pse_status pse_derive(const pse_params *p, pse_derived *o) {
  if (!p || !o) return PSE_ERR_INVALID_ARG;
  Derived d;
  const pse_status st = derive_params(*p, &d);
  if (st != PSE_OK) return st;
  o->h = d.h;
  o->sigma = d.sigma;
  o->gauss_m = d.gm;
  o->eta_se = d.eta_se;
  o->eps_real = d.eps_real;
  o->eps_wave = d.eps_wave;
  o->eps_quad = d.eps_quad;
  o->cells = d.nc;
  o->self_real = d.self_r;
  o->eps_alias = d.eps_alias;
  o->eps_real_tail = d.eps_real_tail;
  o->eps_real_coherent = d.eps_real_coherent;
  return PSE_OK;
}

pse_status pse_choose_params(const pse_params *base, const pse_tuning *t, pse_params *out, pse_tuning_info *info) {
  if (!base || !t || !out) return PSE_ERR_INVALID_ARG;
  return choose_params(*base, *t, out, info);
}

pse_status pse_set_positions(pse_ctx *c, const void *pos) {
  if (!c || !pos) return PSE_ERR_INVALID_ARG;
  if (c->dbl) return set_positions_impl<double>(c, pos);
  return set_positions_impl<float>(c, pos);
}

pse_status pse_sample(pse_ctx *c, uint64_t seed, uint64_t counter, double dt, const void *forces, void *disp,
                      pse_stats *stats) {
  if (!c) return PSE_ERR_INVALID_ARG;
  DISPATCH(c, (sample_impl<T, A>(c, true, seed, counter, nullptr, nullptr, dt, forces, disp, stats)));
}

pse_status pse_sample_with_noise(pse_ctx *c, const void *z1, const void *W, double dt, const void *forces, void *disp,
                                 pse_stats *stats) {
  if (!c) return PSE_ERR_INVALID_ARG;
  DISPATCH(c, (sample_impl<T, A>(c, false, 0, 0, z1, W, dt, forces, disp, stats)));
}

pse_status pse_bd_step(pse_ctx *c, void *pos, const void *forces, double dt, double krep, uint64_t seed,
                       uint64_t step, void *disp, pse_stats *stats) {
  if (!c || !pos || !(dt > 0) || !(krep >= 0)) return PSE_ERR_INVALID_ARG;
  DISPATCH(c, (bd_step_impl<T, A>(c, pos, forces, dt, krep, seed, step, disp, stats)));
}

pse_status pse_full_sample(pse_ctx *c, const void *z, void *y, pse_stats *stats) {
  if (!c || !z || !y) return PSE_ERR_INVALID_ARG;
  if (!c->fl_V) return PSE_ERR_PARAMS;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  DISPATCH(c, (full_sample_impl<T, A>(c, z, y, stats)));
}

pse_status pse_real_matvec(pse_ctx *c, const void *v, void *w) {
  if (!c || !v || !w) return PSE_ERR_INVALID_ARG;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  DISPATCH(c, (real_matvec_impl<T, A>(c, v, w)));
}

pse_status pse_real_sample(pse_ctx *c, const void *z, void *y, pse_stats *stats) {
  if (!c || !z || !y) return PSE_ERR_INVALID_ARG;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  DISPATCH(c, (real_sample_impl<T, A>(c, z, y, stats)));
}

pse_status pse_wave_sample(pse_ctx *c, const void *W, void *y) {
  if (!c || !W || !y) return PSE_ERR_INVALID_ARG;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  if (c->dbl) return wave_sample_impl<double>(c, W, y);
  return wave_sample_impl<float>(c, W, y);
}

pse_status pse_wave_apply(pse_ctx *c, const void *F, void *u) {
  if (!c || !F || !u) return PSE_ERR_INVALID_ARG;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  DISPATCH(c, (wave_apply_impl<T, A>(c, F, u, false)));
}

pse_status pse_autotune(pse_ctx *c, int32_t *choice) {
  if (!c) return PSE_ERR_INVALID_ARG;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  const pse_status st = c->dbl ? autotune_grid<double>(c, choice) : autotune_grid<float>(c, choice);
  if (st != PSE_OK) return st;
  return autotune_spmv(c, choice ? choice + 2 : nullptr);
}

pse_status pse_set_launch_shape(pse_ctx *c, const int32_t *choice) {
  if (!c || !choice) return PSE_ERR_INVALID_ARG;
  const int depth = choice[0], il = choice[1], pl = choice[2];
  if (!grid_shape_valid(c->p.grid, c->p.support, depth, il)) return PSE_ERR_INVALID_ARG;
  if (pl != 0 && pl != 2 && pl != 3 && pl != 4) return PSE_ERR_INVALID_ARG;
  c->tune_spread_nw = depth / 8;
  c->tune_interp_threads = il;
  c->tune_spmv_lanes = pl;
  return PSE_OK;
}

pse_status pse_profile(pse_ctx *c, uint32_t mask) {
  if (!c) return PSE_ERR_INVALID_ARG;
  c->prof_mask = mask & ((1u << PSE_NSTAGES) - 1);
  return PSE_OK;
}

pse_status pse_profile_read(pse_ctx *c, double *ms, int32_t *launches) {
  if (!c || !ms || !launches) return PSE_ERR_INVALID_ARG;
  for (int i = 0; i < PSE_NSTAGES; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PSE_ERR_HIP;
  const size_t npairs = c->ev_stage.size();
  for (size_t i = 0; i < npairs && 2 * i + 1 < c->ev_used; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]) != hipSuccess) return PSE_ERR_HIP;
    ms[c->ev_stage[i]] += t;
    launches[c->ev_stage[i]] += 1;
  }
  c->ev_used = 0;
  c->ev_stage.clear();
  c->ev_open = -1;
  return PSE_OK;
}

pse_status pse_batch_create(const pse_params *p, int32_t n_rep, void *stream, pse_batch **out) {
  if (!p || !out || n_rep < 1) return PSE_ERR_INVALID_ARG;
  *out = nullptr;
  for (int r = 0; r < n_rep; ++r) {
    Derived d;
    const pse_status ps = derive_params(p[r], &d);
    if (ps != PSE_OK) return ps;
  }
  pse_batch *b = new (std::nothrow) pse_batch();
  if (!b) return PSE_ERR_OOM;
  b->user = (hipStream_t)stream;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return PSE_ERR_HIP;
  }
  const int S = std::min(n_rep, 8);
  b->streams.resize(S, nullptr);
  b->join.resize(S, nullptr);
  b->done.resize(n_rep, nullptr);
  bool ok = hipEventCreate(&b->start) == hipSuccess;
  for (int q = 0; ok && q < S; ++q)
    ok = hipStreamCreateWithFlags(&b->streams[q], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[q], hipEventDisableTiming) == hipSuccess;
  for (int r = 0; ok && r < n_rep; ++r) ok = hipEventCreate(&b->done[r]) == hipSuccess;
  if (!ok) {
    free_batch(b);
    return PSE_ERR_HIP;
  }
  for (int r = 0; r < n_rep; ++r) {
    pse_ctx *c = nullptr;
    const pse_status st = pse_create(&p[r], b->streams[r % S], &c);
    if (st != PSE_OK) {
      free_batch(b);
      return st;
    }
    b->ctx.push_back(c);
  }
  *out = b;
  return PSE_OK;
}

pse_status pse_batch_destroy(pse_batch *b) {
  if (!b) return PSE_OK;
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  free_batch(b);
  return PSE_OK;
}

pse_status pse_batch_replica(pse_batch *b, int32_t r, pse_ctx **out) {
  if (!b || !out || r < 0 || r >= (int)b->ctx.size()) return PSE_ERR_INVALID_ARG;
  *out = b->ctx[r];
  return PSE_OK;
}

pse_status pse_batch_set_positions(pse_batch *b, const void *const *pos) {
  if (!b || !pos) return PSE_ERR_INVALID_ARG;
  for (size_t r = 0; r < b->ctx.size(); ++r)
    if (!pos[r]) return PSE_ERR_INVALID_ARG;
  pse_status st = fork(b);
  if (st != PSE_OK) return st;
  const int S = (int)b->streams.size();
  st = for_streams(b, [&](int q, int R) {
    pse_status w = PSE_OK;
    for (int r = q; r < R; r += S) w = worse(w, pse_set_positions(b->ctx[r], pos[r]));
    return w;
  });
  const pse_status sj = join(b);
  return st != PSE_OK ? st : sj;
}

pse_status pse_batch_sample(pse_batch *b, uint64_t seed, uint64_t counter, double dt, const void *const *forces,
                            void *const *disp, pse_stats *stats) {
  if (!b || !disp) return PSE_ERR_INVALID_ARG;
  const int R = (int)b->ctx.size(), S = (int)b->streams.size();
  for (int r = 0; r < R; ++r)
    if (!disp[r]) return PSE_ERR_INVALID_ARG;
  pse_status st = fork(b);
  if (st != PSE_OK) return st;
  st = for_streams(b, [&](int q, int) {
    pse_status w = PSE_OK;
    std::vector<SampleState> ss(R);
    std::vector<pse_status> sb(R, PSE_OK);
    bool any_real = false;
    for (int r = q; r < R; r += S) {
      sb[r] = ctx_begin(b->ctx[r], seed + (uint64_t)r, counter, dt, forces ? forces[r] : nullptr, ss[r]);
      any_real = any_real || ss[r].real;
    }
    if (any_real && hipStreamSynchronize(b->streams[q]) != hipSuccess) return PSE_ERR_HIP;
    for (int r = q; r < R; r += S) {
      pse_status x = sb[r];
      if (x == PSE_OK) x = ctx_end(b->ctx[r], ss[r], dt, disp[r], stats ? &stats[r] : nullptr);
      if (hipEventRecord(b->done[r], b->streams[q]) != hipSuccess) x = worse(x, PSE_ERR_HIP);
      w = worse(w, x);
    }
    return w;
  });
  const pse_status sj = join(b);
  return st != PSE_OK ? st : sj;
}

pse_status pse_batch_autotune(pse_batch *b) {
  if (!b) return PSE_ERR_INVALID_ARG;
  if (hipStreamSynchronize(b->user) != hipSuccess) return PSE_ERR_HIP;
  for (size_t r = 0; r < b->ctx.size(); ++r) {
    pse_ctx *c = b->ctx[r];
    if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
    const pse_ctx *ref = nullptr;  // an earlier replica of the same group
    for (size_t q = 0; q < r && !ref; ++q) {
      const pse_ctx *o = b->ctx[q];
      if (o->p.grid == c->p.grid && o->p.support == c->p.support && o->p.precision == c->p.precision) ref = o;
    }
    if (ref) {
      c->tune_spread_nw = ref->tune_spread_nw;
      c->tune_interp_threads = ref->tune_interp_threads;
    } else {
      const pse_status st = c->dbl ? autotune_grid<double>(c, nullptr) : autotune_grid<float>(c, nullptr);
      if (st != PSE_OK) return st;
    }
    // the product depends on the replica's own density: tuned per replica
    const pse_status st = autotune_spmv(c, nullptr);
    if (st != PSE_OK) return st;
  }
  // then one choice per kernel form (block edge, halo form, Lanczos scalar
  // type): the one most particles of the form chose.  A captured step runs
  // each form's replicas in one launch per iteration, so fewer forms mean
  // fewer, fuller launches; the eager path uses the same choice.
  struct Tally {
    int B, unwrap, dbl;
    long w[5];
  };
  std::vector<Tally> t;
  for (pse_ctx *c : b->ctx) {
    if (c->dbl || !c->lds_B) continue;
    const int uw = c->d.nc >= c->lds_B + 3 ? 1 : 0, ad = c->acc_dbl ? 1 : 0;
    const int G = c->tune_spmv_lanes ? c->tune_spmv_lanes : 3;
    size_t g = 0;
    while (g < t.size() && !(t[g].B == c->lds_B && t[g].unwrap == uw && t[g].dbl == ad)) ++g;
    if (g == t.size()) t.push_back(Tally{c->lds_B, uw, ad, {0, 0, 0, 0, 0}});
    t[g].w[G] += c->n;
  }
  for (pse_ctx *c : b->ctx) {
    if (c->dbl || !c->lds_B) continue;
    const int uw = c->d.nc >= c->lds_B + 3 ? 1 : 0, ad = c->acc_dbl ? 1 : 0;
    for (const Tally &x : t)
      if (x.B == c->lds_B && x.unwrap == uw && x.dbl == ad) {
        int best = 3;
        for (int G = 2; G <= 4; ++G)
          if (x.w[G] > x.w[best]) best = G;
        c->tune_spmv_lanes = best;
      }
  }
  return PSE_OK;
}

}  // extern "C"

namespace pse {

struct LzView {
  int m, done, converged, nonfinite;
  double rel;
};
static LzView lz_view(const pse_ctx *c) {
  if (c->dbl || c->acc_dbl) {
    const auto *h = (const LzState<double> *)c->lz_h;
    return {h->m, h->done, h->converged, h->nonfinite, h->rel_change};
  }
  const auto *h = (const LzState<float> *)c->lz_h;
  return {h->m, h->done, h->converged, h->nonfinite, (double)h->rel_change};
}

static pse_status ctx_set_positions(pse_ctx *c, const void *pos) {
  return c->dbl ? set_positions_impl<double>(c, pos) : set_positions_impl<float>(c, pos);
}

// The forces of replica r in the captured step (null: none).
static const void *batch_forces(const pse_batch *b, int r) {
  return b->g_forces.empty() ? nullptr : b->g_forces[r];
}

// A replica whose whole captured step can run in batched launches: FP32
// storage on the LDS path, no preconditioner, no repulsion, kT > 0, at most
// 65536 particles (the Krylov start's partial sums in the single-system
// layout), and with forces a grid that the tiled spreading covers.
static bool full_candidate(const pse_batch *b, int r) {
  const pse_ctx *c = b->ctx[r];
  if (c->dbl || !c->lds_B || c->pc_on || c->rep_k > 0 || !(c->p.kT > 0) || c->n > kRedBlock * 64) return false;
  if (batch_forces(b, r) && b->g_dt > 0 && !spread_writes_whole_grid(c->p.grid, c->p.support)) return false;
  return true;
}

// A batched Krylov loop of a captured step: every replica with Lanczos
// scalars of type A that runs the LDS product (FP32 storage) without the
// preconditioner, as LzRep records,
// its product blocks grouped by kernel form, and its vector blocks.  Built
// before the capture (device allocation and copies); the loop runs as many
// iterations as the replica that queued the most, the others stop
// themselves once converged.
template <typename A> static pse_status lzb_setup(pse_batch *b) {
  const int R = (int)b->ctx.size();
  pse_batch::LzBatch &z = b->lzb[sizeof(A) == 8 ? 1 : 0];
  std::vector<LzRep<A>> reps;
  std::vector<std::vector<int2>> pm;
  std::vector<LzGroup> gr;
  std::vector<int2> vm;
  int iters = 0;
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    if (c->dbl || c->acc_dbl != (sizeof(A) == 8) || !c->lds_B || pc_active(c) || !(c->p.kT > 0) ||
        c->n > kRedBlock * 256)
      continue;
    const int k = (int)reps.size();
    LzRep<A> q{};
    q.pos = (const float4 *)c->pos_s;
    q.cell_start = c->cell_start;
    q.nbr = (const uint16_t *)c->nbr;
    q.cnt = c->nbr_cnt;
    q.tab = c->table;
    q.ovf = c->flags + 7;
    q.z = (const float4 *)c->vbuf[0];
    q.t = (float4 *)c->vbuf[2];
    q.w = (float4 *)c->vbuf[3];
    q.V = (float4 *)c->V;
    q.st = (LzState<A> *)c->lz;
    q.partials = (A *)c->partials;
    // the fully batched replicas' M_r F runs in the batched plain product
    const bool fr = !b->is_full.empty() && b->is_full[r] && batch_forces(b, r) && b->g_dt > 0;
    q.fs = fr ? (const float4 *)c->vbuf[6] : nullptr;
    q.ur = (float4 *)c->vbuf[7];
    q.cs = (float)c->d.cs;
    q.L = (float)c->d.L;
    q.invL = (float)(1.0 / c->d.L);
    q.inv_dr = (float)(kTableK / c->p.rcut);
    q.self_r = (float)c->d.self_r;
    q.nc = c->d.nc;
    q.n = c->n;
    q.hcap = c->hcap;
    q.maxit = c->lz_maxit;
    q.tol = (A)c->p.lanczos_tol;
    reps.push_back(q);
    z.members.push_back(r);
    const int G = c->tune_spmv_lanes ? c->tune_spmv_lanes : 3, unwrap = c->d.nc >= c->lds_B + 3 ? 1 : 0;
    size_t g = 0;
    while (g < gr.size() && !(gr[g].B == c->lds_B && gr[g].G == G && gr[g].unwrap == unwrap)) ++g;
    if (g == gr.size()) {
      gr.push_back(LzGroup{c->lds_B, G, unwrap, 0, 0, nullptr});
      pm.emplace_back();
    }
    for (int blk = 0; blk < c->lds_blocks; ++blk) pm[g].push_back(make_int2(k, blk));
    const size_t smem = (sizeof(float4) + sizeof(float2)) * (size_t)c->hcap;
    if (smem > gr[g].smem) gr[g].smem = smem;
    for (int v = 0; v < (c->n + 255) / 256; ++v) vm.push_back(make_int2(k, v));
    iters = std::max(iters, c->graph_iters);
  }
  if (reps.empty()) return PSE_OK;
  size_t nmap = vm.size();
  for (auto &x : pm) nmap += x.size();
  if (hipMalloc(&z.reps, sizeof(LzRep<A>) * reps.size()) != hipSuccess ||
      hipMalloc((void **)&z.maps, sizeof(int2) * nmap) != hipSuccess)
    return PSE_ERR_OOM;
  std::vector<int2> all;
  all.reserve(nmap);
  for (size_t g = 0; g < gr.size(); ++g) {
    gr[g].pmap = z.maps + all.size();
    gr[g].nblk = (int)pm[g].size();
    all.insert(all.end(), pm[g].begin(), pm[g].end());
  }
  z.vmap = z.maps + all.size();
  all.insert(all.end(), vm.begin(), vm.end());
  if (hipMemcpy(z.reps, reps.data(), sizeof(LzRep<A>) * reps.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(z.maps, all.data(), sizeof(int2) * nmap, hipMemcpyHostToDevice) != hipSuccess)
    return PSE_ERR_HIP;
  z.groups = gr;
  z.nrep = (int)reps.size();
  z.nv = (int)vm.size();
  z.iters = iters;
  return PSE_OK;
}

template <typename A> static void lzb_launch(pse_batch *b) {
  const pse_batch::LzBatch &z = b->lzb[sizeof(A) == 8 ? 1 : 0];
  for (int m = 0; m < z.iters; ++m)
    launch_lz_batch_iter<A>(b->gstream, (const LzRep<A> *)z.reps, z.nrep, z.groups.data(), (int)z.groups.size(),
                            z.vmap, z.nv, m);
}

// The batched neighbour build of a captured step: every replica on the LDS
// path without the overlap repulsion and without the preconditioner (whose
// features follow the build inside its set_positions), grouped by block
// edge and halo form.
static pse_status nbr_setup(pse_batch *b) {
  const int R = (int)b->ctx.size();
  std::vector<NbrRep> reps;
  std::vector<NbrGroup> gr;
  std::vector<std::vector<int2>> pm;
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    if (c->dbl || !c->lds_B || c->rep_k > 0 || c->pc_on) continue;
    const int k = (int)reps.size();
    NbrRep q{};
    q.pos = (const float4 *)c->pos_s;
    q.cell_start = c->cell_start;
    q.nbr = (uint16_t *)c->nbr;
    q.cnt = c->nbr_cnt;
    q.flags = c->flags;
    q.cs = (float)c->d.cs;
    q.L = (float)c->d.L;
    q.invL = (float)(1.0 / c->d.L);
    q.rc2 = (float)(c->p.rcut * c->p.rcut);
    q.nc = c->d.nc;
    q.n = c->n;
    q.cap = c->nbr_cap;
    q.hcap = c->hcap;
    reps.push_back(q);
    b->nb_members.push_back(r);
    const int unwrap = c->d.nc >= c->lds_B + 3 ? 1 : 0;
    size_t g = 0;
    while (g < gr.size() && !(gr[g].B == c->lds_B && gr[g].unwrap == unwrap)) ++g;
    if (g == gr.size()) {
      gr.push_back(NbrGroup{c->lds_B, unwrap, 0, 0, nullptr});
      pm.emplace_back();
    }
    for (int blk = 0; blk < c->lds_blocks; ++blk) pm[g].push_back(make_int2(k, blk));
    const size_t smem = sizeof(float3) * (size_t)(c->hcap + 3);  // 3 slots read past the last cell
    if (smem > gr[g].smem) gr[g].smem = smem;
  }
  if (reps.empty()) return PSE_OK;
  size_t nmap = 0;
  for (auto &x : pm) nmap += x.size();
  if (hipMalloc((void **)&b->nb_reps, sizeof(NbrRep) * reps.size()) != hipSuccess ||
      hipMalloc((void **)&b->nb_maps, sizeof(int2) * nmap) != hipSuccess)
    return PSE_ERR_OOM;
  std::vector<int2> all;
  all.reserve(nmap);
  for (size_t g = 0; g < gr.size(); ++g) {
    gr[g].pmap = b->nb_maps + all.size();
    gr[g].nblk = (int)pm[g].size();
    all.insert(all.end(), pm[g].begin(), pm[g].end());
  }
  if (hipMemcpy(b->nb_reps, reps.data(), sizeof(NbrRep) * reps.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->nb_maps, all.data(), sizeof(int2) * nmap, hipMemcpyHostToDevice) != hipSuccess)
    return PSE_ERR_HIP;
  b->nb_groups = gr;
  return PSE_OK;
}

// The replicas whose whole captured step runs in batched launches: members
// of the batched Krylov loop, neighbour build and wave-space part alike
// (FP32 storage, LDS path, no preconditioner, no repulsion, no forces,
// kT > 0).  Their binning, noise, Krylov start, combination and final sum
// are batched too, and the capture issues nothing per replica for them.
// After the replicas' rng_dev is set, before the capture.
static pse_status full_setup(pse_batch *b) {
  const int R = (int)b->ctx.size();
  std::vector<char> in_lz(R, 0), in_nb(R, 0), in_wv(R, 0);
  for (const auto &z : b->lzb)
    for (int r : z.members) in_lz[r] = 1;
  for (int r : b->nb_members) in_nb[r] = 1;
  for (int r : b->wv_members) in_wv[r] = 1;
  for (int a = 0; a < 2; ++a) {
    pse_batch::FullBatch &f = b->full[a];
    std::vector<SampRep> reps;
    std::vector<int2> mz, mp, mt, mc, mf;
    for (int r = 0; r < R; ++r) {
      pse_ctx *c = b->ctx[r];
      // 4n vector scalars in at most kRedBlock blocks of 256: the Krylov
      // start's partial sums are laid out as in a single-system launch
      if (!b->is_full[r] || (c->acc_dbl ? 1 : 0) != a) continue;
      if (!(in_lz[r] && in_nb[r] && in_wv[r])) return PSE_ERR_INVALID_ARG;  // the candidate test and the batched sets disagree
      const int k = (int)reps.size(), n = c->n;
      SampRep q{};
      q.pos_in = (const float *)b->g_pos[r];
      q.pos_w = (float4 *)c->pos_w;
      q.pos_s = (float4 *)c->pos_s;
      q.cell_of = c->cell_of;
      q.slot = c->cell_of + n;
      q.cell_count = c->cell_count;
      q.tile_sum = c->cell_count + c->ncell;
      q.cell_start = c->cell_start;
      q.perm = c->perm;
      q.flags = c->flags;
      q.L = (float)c->d.L;
      q.invL = (float)(1.0 / c->d.L);
      q.inv_cs = (float)(1.0 / c->d.cs);
      q.nc = c->d.nc;
      q.ncell = c->ncell;
      q.n = n;
      q.rng = c->rng_dev;
      q.z = (float4 *)c->vbuf[0];
      q.partials = c->partials;
      q.st = c->lz;
      q.V = (const float4 *)c->V;
      q.yr = (float4 *)c->vbuf[1];
      q.wave = (const float4 *)c->vbuf[4];
      q.out = (float *)b->g_disp[r];
      q.cr = (float)std::sqrt(2.0 * c->p.kT * b->g_dt);
      q.f_in = b->g_dt > 0 ? (const float *)batch_forces(b, r) : nullptr;
      q.f_s = (float4 *)c->vbuf[6];
      q.ur = (float4 *)c->vbuf[7];
      q.dt = (float)b->g_dt;
      reps.push_back(q);
      f.members.push_back(r);
      for (int q2 = 0; q2 < (c->ncell + 8 + 255) / 256; ++q2) mz.push_back(make_int2(k, q2));
      for (int q2 = 0; q2 < (n + 255) / 256; ++q2) mp.push_back(make_int2(k, q2));
      for (int q2 = 0; q2 < (c->ncell + kScanTile - 1) / kScanTile; ++q2) mt.push_back(make_int2(k, q2));
      for (int q2 = 0; q2 < (c->ncell + 3) / 4; ++q2) mc.push_back(make_int2(k, q2));
      for (int q2 = 0; q2 < (4 * n + 255) / 256; ++q2) mf.push_back(make_int2(k, q2));
    }
    if (reps.empty()) continue;
    const size_t nmap = mz.size() + mp.size() + mt.size() + mc.size() + mf.size();
    if (hipMalloc((void **)&f.reps, sizeof(SampRep) * reps.size()) != hipSuccess ||
        hipMalloc((void **)&f.maps, sizeof(int2) * nmap) != hipSuccess)
      return PSE_ERR_OOM;
    std::vector<int2> all;
    all.reserve(nmap);
    auto put = [&](const std::vector<int2> &v, const int2 *&ptr, int &cnt) {
      ptr = f.maps + all.size();
      cnt = (int)v.size();
      all.insert(all.end(), v.begin(), v.end());
    };
    put(mz, f.m.zero, f.m.nzero);
    put(mp, f.m.part, f.m.npart);
    put(mt, f.m.tile, f.m.ntile);
    put(mc, f.m.cell, f.m.ncell);
    put(mf, f.m.flat, f.m.nflat);
    f.m.nrep = (int)reps.size();
    if (hipMemcpy(f.reps, reps.data(), sizeof(SampRep) * reps.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(f.maps, all.data(), sizeof(int2) * nmap, hipMemcpyHostToDevice) != hipSuccess)
      return PSE_ERR_HIP;
  }
  return PSE_OK;
}

// The batched wave-space part of a captured step: every replica with FP32
// storage, kT > 0 and no forces, grouped by grid size, support and
// interpolation workgroup size, with the coefficients sample_begin would
// use (key and counter from the replica's device pair).  After the
// replicas' rng_dev is set, before the capture.
static pse_status wave_setup(pse_batch *b) {
  const int R = (int)b->ctx.size();
  struct Key {
    int M, P, nt, nw, forces;
  };
  std::vector<Key> keys;
  std::vector<std::vector<int>> mem;
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    if (c->dbl || !(c->p.kT > 0)) continue;
    const int M = c->p.grid, forces = batch_forces(b, r) && b->g_dt > 0 ? 1 : 0;
    if (forces && !spread_writes_whole_grid(M, c->p.support)) continue;  // the atomic spreading stays per replica
    const int nw = c->tune_spread_nw ? c->tune_spread_nw : spread_default_nw(M, c->p.support, true);
    const Key k{M, c->p.support, c->tune_interp_threads ? c->tune_interp_threads : kInterpLanes, nw, forces};
    size_t g = 0;
    while (g < keys.size() && !(keys[g].M == k.M && keys[g].P == k.P && keys[g].nt == k.nt && keys[g].nw == k.nw &&
                                keys[g].forces == k.forces))
      ++g;
    if (g == keys.size()) {
      keys.push_back(k);
      mem.emplace_back();
    }
    mem[g].push_back(r);
  }
  if (keys.empty()) return PSE_OK;
  const double pi = 3.14159265358979323846;
  std::vector<WaveRep> reps;
  std::vector<int2> imap;
  std::vector<std::pair<size_t, size_t>> span;  // (first rep, first map entry) per group
  for (size_t g = 0; g < keys.size(); ++g) {
    span.emplace_back(reps.size(), imap.size());
    for (int r : mem[g]) {
      pse_ctx *c = b->ctx[r];
      const int k = (int)(reps.size() - span[g].first);
      const double h = c->d.h, s2 = c->d.sigma * c->d.sigma;
      const double norm = std::pow(2.0 * pi * s2, -1.5);
      WaveRep w{};
      w.spec = (float2 *)c->grid;
      w.rgrid = (float *)c->rgrid;
      w.tw_M = (const float2 *)c->tw_M;
      w.tw_H = (const float2 *)c->tw_H;
      w.pos = (const float4 *)c->pos_s;
      w.out = (float4 *)c->vbuf[4];
      w.wc = step_wave_coef(c, b->g_dt, 0, 0);
      w.n = c->n;
      w.M = c->p.grid;
      w.h = (float)h;
      w.invh = (float)(1.0 / h);
      w.inv2s2 = (float)(0.5 / s2);
      w.norm_h3 = (float)(norm * h * h * h);
      w.f = keys[g].forces ? (const float4 *)c->vbuf[6] : nullptr;
      w.cell_start = c->cell_start;
      w.nc = c->d.nc;
      w.cs = (float)c->d.cs;
      w.norm = (float)norm;
      reps.push_back(w);
      b->wv_members.push_back(r);
      const int nt = keys[g].nt;
      const int nb = (int)(((long)c->n * 64 + nt - 1) / nt);
      for (int q = 0; q < nb; ++q) imap.push_back(make_int2(k, q));
    }
  }
  if (hipMalloc((void **)&b->wv_reps, sizeof(WaveRep) * reps.size()) != hipSuccess ||
      hipMalloc((void **)&b->wv_imap, sizeof(int2) * imap.size()) != hipSuccess)
    return PSE_ERR_OOM;
  if (hipMemcpy(b->wv_reps, reps.data(), sizeof(WaveRep) * reps.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->wv_imap, imap.data(), sizeof(int2) * imap.size(), hipMemcpyHostToDevice) != hipSuccess)
    return PSE_ERR_HIP;
  for (size_t g = 0; g < keys.size(); ++g) {
    const size_t r1 = g + 1 < keys.size() ? span[g + 1].first : reps.size();
    const size_t m1 = g + 1 < keys.size() ? span[g + 1].second : imap.size();
    b->wv_groups.push_back(WaveGroup{keys[g].M, keys[g].P, keys[g].nt, keys[g].nw, keys[g].forces,
                                     (int)(r1 - span[g].first), (int)(m1 - span[g].second),
                                     b->wv_reps + span[g].first, b->wv_imap + span[g].second});
  }
  return PSE_OK;
}

// Capture one batch step (every replica's set_positions and sample, on the
// replicas' streams) into b->gexec.  Capacities get the headroom first
// (outside the capture: the list may be reallocated); inside the capture no
// host decision and no synchronisation is taken.
static pse_status batch_capture(pse_batch *b) {
  const int R = (int)b->ctx.size();
  const int hcap_lds = (int)((kLdsBudget - sizeof(float2) * kTableN) / (sizeof(float4) + sizeof(float2)));
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    if (c->lds_B) {
      int want = (int)std::ceil((c->hcap - 1) * (1.0 + b->g_headroom)) + 1;
      if (want > hcap_lds) want = hcap_lds;
      if (want > 65536) want = 65536;  // 16-bit halo-local indices
      if (want > c->hcap) c->hcap = want;
    }
    b->g_hcap[r] = c->hcap;
    const int cap = ((int)std::ceil(c->flags_h[1] * (1.0 + b->g_headroom)) + 32 + 7) & ~7;
    if (cap > c->nbr_cap) {
      if (hipStreamSynchronize(c->stream) != hipSuccess) return PSE_ERR_HIP;
      (void)hipFree(c->nbr);
      c->nbr = nullptr;
      if (hipMalloc(&c->nbr, sizeof(int) * (size_t)cap * c->n) != hipSuccess) {
        c->nbr_cap = 0;
        return PSE_ERR_OOM;
      }
      c->nbr_cap = cap;
    }
    int it = (c->last_iters < 2 ? 2 : c->last_iters) + b->g_extra;
    c->graph_iters = it > c->lz_maxit ? c->lz_maxit : it;
    c->graph_stale = false;
  }
  b->is_full.assign(R, 0);
  for (int r = 0; r < R; ++r) b->is_full[r] = full_candidate(b, r) ? 1 : 0;
  pse_status st0 = lzb_setup<float>(b);
  if (st0 == PSE_OK) st0 = lzb_setup<double>(b);
  if (st0 == PSE_OK) st0 = nbr_setup(b);
  if (st0 != PSE_OK) return st0;
  {
    std::vector<RepStatusSrc> src(R);
    for (int r = 0; r < R; ++r) src[r] = RepStatusSrc{b->ctx[r]->flags, b->ctx[r]->lz, b->ctx[r]->acc_dbl ? 1 : 0};
    if (hipMalloc((void **)&b->stat_src, sizeof(RepStatusSrc) * R) != hipSuccess ||
        hipMalloc((void **)&b->stat_d, sizeof(RepStatus) * R) != hipSuccess ||
        hipHostMalloc((void **)&b->stat_h, sizeof(RepStatus) * R, hipHostMallocDefault) != hipSuccess)
      return PSE_ERR_OOM;
    if (hipMemcpy(b->stat_src, src.data(), sizeof(RepStatusSrc) * R, hipMemcpyHostToDevice) != hipSuccess)
      return PSE_ERR_HIP;
  }
  std::vector<uint32_t> prof(R);
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    prof[r] = c->prof_mask;
    c->prof_mask = 0;
    c->graph = true;
    c->rng_dev = b->rng_d + 2 * r;
  }
  st0 = wave_setup(b);
  if (st0 == PSE_OK) st0 = full_setup(b);
  if (st0 != PSE_OK) {
    for (int r = 0; r < R; ++r) {
      b->ctx[r]->prof_mask = prof[r];
      b->ctx[r]->graph = false;
      b->ctx[r]->rng_dev = nullptr;
    }
    return st0;
  }
  for (const auto &z : b->lzb)
    for (int r : z.members) b->ctx[r]->lz_external = true;
  for (int r : b->wv_members) b->ctx[r]->wave_external = true;
  for (int r : b->nb_members) b->ctx[r]->nbr_external = true;
  for (pse_ctx *c : b->ctx) c->status_external = true;
  pse_status st = hip_status(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeRelaxed));
  if (st == PSE_OK)
    st = hip_status(hipMemcpyAsync(b->rng_d, b->rng_h, sizeof(uint64_t) * 2 * R, hipMemcpyHostToDevice, b->gstream));
  if (st == PSE_OK) st = fork(b, b->gstream);
  // every replica's binning; the batched neighbour build on the capture
  // stream; every replica's first part of the sample; the batched Krylov
  // loops and wave-space part on the capture stream; the rest of each sample
  std::vector<SampleState> ss(R);
  auto full = [&](int r) { return !b->is_full.empty() && b->is_full[r]; };
  for (const auto &f : b->full)
    if (f.m.nrep) launch_samp_batch_bin(b->gstream, f.reps, f.m);
  for (int r = 0; r < R && st == PSE_OK; ++r)
    if (!full(r)) st = ctx_set_positions(b->ctx[r], b->g_pos[r]);
  if (st == PSE_OK && !b->nb_groups.empty()) {
    st = join(b, b->gstream);
    if (st == PSE_OK) {
      launch_nbr_batch(b->gstream, b->nb_reps, b->nb_groups.data(), (int)b->nb_groups.size());
      st = hip_status(hipGetLastError());
    }
    if (st == PSE_OK) st = fork(b, b->gstream);
  }
  if (b->full[0].m.nrep) launch_samp_batch_start<float>(b->gstream, b->full[0].reps, b->full[0].m);
  if (b->full[1].m.nrep) launch_samp_batch_start<double>(b->gstream, b->full[1].reps, b->full[1].m);
  if (!b->g_forces.empty() && b->g_dt > 0) {
    // the fully batched replicas' forces in sorted order, and their M_r F
    for (const auto &f : b->full)
      if (f.m.nrep) launch_samp_batch_forces(b->gstream, f.reps, f.m);
    for (int a = 0; a < 2; ++a) {
      const auto &z = b->lzb[a];
      if (!z.nrep) continue;
      if (a) launch_lz_batch_plain<double>(b->gstream, (const LzRep<double> *)z.reps, z.groups.data(), (int)z.groups.size());
      else launch_lz_batch_plain<float>(b->gstream, (const LzRep<float> *)z.reps, z.groups.data(), (int)z.groups.size());
    }
  }
  for (int r = 0; r < R && st == PSE_OK; ++r)
    if (!full(r)) st = ctx_begin(b->ctx[r], 0, 0, b->g_dt, b->g_forces.empty() ? nullptr : b->g_forces[r], ss[r]);
  if (st == PSE_OK && (b->lzb[0].nrep || b->lzb[1].nrep || !b->wv_groups.empty())) {
    st = join(b, b->gstream);
    if (st == PSE_OK) {
      lzb_launch<float>(b);
      lzb_launch<double>(b);
      launch_wave_batch(b->gstream, b->wv_groups.data(), (int)b->wv_groups.size());
      st = hip_status(hipGetLastError());
    }
    if (st == PSE_OK) st = fork(b, b->gstream);
  }
  if (b->full[0].m.nrep) launch_samp_batch_end<float>(b->gstream, b->full[0].reps, b->full[0].m);
  if (b->full[1].m.nrep) launch_samp_batch_end<double>(b->gstream, b->full[1].reps, b->full[1].m);
  for (int r = 0; r < R && st == PSE_OK; ++r)
    if (!full(r)) st = ctx_end(b->ctx[r], ss[r], b->g_dt, b->g_disp[r], nullptr);
  if (st == PSE_OK) st = join(b, b->gstream);
  if (st == PSE_OK) {
    launch_batch_status(b->gstream, b->stat_src, R, b->stat_d);
    st = hip_status(hipMemcpyAsync(b->stat_h, b->stat_d, sizeof(RepStatus) * R, hipMemcpyDeviceToHost, b->gstream));
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->gstream, &g);
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    c->prof_mask = prof[r];
    c->graph = false;
    c->rng_dev = nullptr;
    c->lz_external = false;
    c->status_external = false;
    c->wave_external = false;
    c->nbr_external = false;
  }
  if (st == PSE_OK && ec != hipSuccess) st = PSE_ERR_HIP;
  if (st != PSE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    b->gexec = nullptr;
    free_graph(b);
    return PSE_ERR_HIP;
  }
  return PSE_OK;
}

}  // namespace pse

extern "C" {

pse_status pse_batch_graph_create(pse_batch *b, const void *const *pos, const void *const *forces,
                                  void *const *disp, double dt, int32_t extra_iters, double headroom) {
  if (!b || !pos || !disp || !(dt > 0) || extra_iters < 0 || !(headroom >= 0)) return PSE_ERR_INVALID_ARG;
  const int R = (int)b->ctx.size();
  for (int r = 0; r < R; ++r)
    if (!pos[r] || !disp[r]) return PSE_ERR_INVALID_ARG;
  free_graph(b);
  b->g_pos.assign(pos, pos + R);
  b->g_forces.clear();
  if (forces) b->g_forces.assign(forces, forces + R);
  b->g_disp.assign(disp, disp + R);
  b->g_hcap.assign(R, 0);
  b->g_dt = dt;
  b->g_extra = extra_iters;
  b->g_headroom = headroom;
  if (!b->gstream) {
    if (hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess) {
      b->gstream = nullptr;
      return PSE_ERR_HIP;
    }
    if (hipEventCreateWithFlags(&b->g_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->g_out, hipEventDisableTiming) != hipSuccess)
      return PSE_ERR_HIP;
  }
  if (!b->rng_h) {
    if (hipHostMalloc((void **)&b->rng_h, sizeof(uint64_t) * 2 * R, hipHostMallocDefault) != hipSuccess) {
      b->rng_h = nullptr;
      return PSE_ERR_OOM;
    }
    if (hipMalloc((void **)&b->rng_d, sizeof(uint64_t) * 2 * R) != hipSuccess) {
      b->rng_d = nullptr;
      return PSE_ERR_OOM;
    }
  }
  // one eager step on these buffers: block edges, halo sizes, list
  // capacities and iteration counts of the positions, and the kernels'
  // launch attributes, before anything is captured
  pse_status st = pse_batch_set_positions(b, pos);
  if (st < 0) return st;
  std::vector<pse_stats> stv(R);
  st = pse_batch_sample(b, 0, 0, dt, forces, disp, stv.data());
  if (st < 0 && st != PSE_ERR_NOT_CONVERGED) return st;
  if (hipStreamSynchronize(b->user) != hipSuccess) return PSE_ERR_HIP;
  return batch_capture(b);
}

pse_status pse_batch_graph_step(pse_batch *b, uint64_t seed, uint64_t counter, pse_stats *stats, int32_t *redone) {
  if (!b) return PSE_ERR_INVALID_ARG;
  if (!b->gexec) return PSE_ERR_NO_POSITIONS;
  const int R = (int)b->ctx.size();
  bool stale = false;
  for (pse_ctx *c : b->ctx) stale = stale || c->graph_stale;
  if (stale) {
    if (hipStreamSynchronize(b->gstream) != hipSuccess) return PSE_ERR_HIP;
    free_graph(b);
    const pse_status sc = batch_capture(b);
    if (sc != PSE_OK) return sc;
  }
  if (hipStreamSynchronize(b->gstream) != hipSuccess) return PSE_ERR_HIP;  // the previous replay has read rng_h
  for (int r = 0; r < R; ++r) {
    b->rng_h[2 * r] = seed + (uint64_t)r;
    b->rng_h[2 * r + 1] = counter;
  }
  // ordered after earlier work on the caller's stream, and later work there after it
  if (hipEventRecord(b->g_in, b->user) != hipSuccess || hipStreamWaitEvent(b->gstream, b->g_in, 0) != hipSuccess ||
      hipGraphLaunch(b->gexec, b->gstream) != hipSuccess || hipEventRecord(b->g_out, b->gstream) != hipSuccess ||
      hipStreamWaitEvent(b->user, b->g_out, 0) != hipSuccess || hipStreamSynchronize(b->gstream) != hipSuccess)
    return PSE_ERR_HIP;
  // the replay's status into each replica's host copies
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    const RepStatus &q = b->stat_h[r];
    std::memcpy(c->flags_h, q.flags, sizeof(int) * 8);
    if (c->pc_on) *c->pc_fb_h = q.flags[6];
    if (c->dbl || c->acc_dbl) {
      auto *h = (LzState<double> *)c->lz_h;
      h->m = q.m;
      h->done = q.done;
      h->converged = q.converged;
      h->nonfinite = q.nonfinite;
      h->rel_change = q.rel_change;
    } else {
      auto *h = (LzState<float> *)c->lz_h;
      h->m = q.m;
      h->done = q.done;
      h->converged = q.converged;
      h->nonfinite = q.nonfinite;
      h->rel_change = (float)q.rel_change;
    }
  }
  pse_status w = PSE_OK;
  int nredo = 0;
  for (int r = 0; r < R; ++r) {
    pse_ctx *c = b->ctx[r];
    const bool real = c->p.kT > 0;
    const LzView v = lz_view(c);
    const bool halo_ovf = c->flags_h[7] != 0, list_ovf = c->flags_h[1] > c->nbr_cap;
    const bool lz_bad = real && !(v.done && v.converged && !v.nonfinite);
    const int fb = c->pc_on ? *c->pc_fb_h : 0;
    if (halo_ovf || list_ovf || lz_bad || c->flags_h[0]) {
      // this replica again, eagerly: capacities from its own positions, the
      // Krylov loop continued as far as needed; the next step captures anew
      ++nredo;
      c->graph_stale = c->graph_stale || halo_ovf || list_ovf || lz_bad;
      pse_status x = ctx_set_positions(c, b->g_pos[r]);
      SampleState ss;
      if (x == PSE_OK)
        x = ctx_begin(c, seed + (uint64_t)r, counter, b->g_dt, b->g_forces.empty() ? nullptr : b->g_forces[r], ss);
      if (x == PSE_OK && hipStreamSynchronize(c->stream) != hipSuccess) x = PSE_ERR_HIP;
      if (x == PSE_OK) x = ctx_end(c, ss, b->g_dt, b->g_disp[r], stats ? &stats[r] : nullptr);
      if (hipStreamSynchronize(c->stream) != hipSuccess) x = worse(x, PSE_ERR_HIP);
      w = worse(w, x);
      continue;
    }
    if (real) c->last_iters = v.m;
    if (stats) {
      pse_stats &o = stats[r];
      o.lanczos_iters = real ? v.m : 0;
      o.converged = 1;
      o.lanczos_rel_change = real ? v.rel : 0.0;
      o.max_neighbors = c->flags_h[5];
      int64_t pairs;
      std::memcpy(&pairs, c->flags_h + 2, sizeof pairs);
      o.neighbor_pairs = pairs;
      o.precond_fallbacks = fb;
      o.nbr_index_bytes = c->lds_B ? 2 : 4;
      o.lds_block_edge = c->lds_B;
    }
  }
  if (redone) *redone = nredo;
  return w;
}

pse_status pse_batch_graph_destroy(pse_batch *b) {
  if (!b) return PSE_ERR_INVALID_ARG;
  if (b->gstream && hipStreamSynchronize(b->gstream) != hipSuccess) return PSE_ERR_HIP;
  free_graph(b);
  return PSE_OK;
}

pse_status pse_batch_latency(pse_batch *b, float *ms) {
  if (!b || !ms) return PSE_ERR_INVALID_ARG;
  for (size_t r = 0; r < b->ctx.size(); ++r) {
    if (hipEventSynchronize(b->done[r]) != hipSuccess ||
        hipEventElapsedTime(&ms[r], b->start, b->done[r]) != hipSuccess)
      return PSE_ERR_HIP;
  }
  return PSE_OK;
}

pse_status pse_precond_set_weights(pse_ctx *c, const void *w_host, size_t bytes) {
  if (!c || !w_host) return PSE_ERR_INVALID_ARG;
  if (!c->pc_on) return PSE_ERR_PARAMS;
  if (bytes != sizeof(uint16_t) * kWTotal) return PSE_ERR_INVALID_ARG;
  if (hipMemcpyAsync(c->pc_w, w_host, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return PSE_ERR_HIP;
  c->pc_have_w = true;
  const bool was_fixed = c->pc_fixed;
  c->pc_fixed = false;
  if (!c->have_pos) return PSE_OK;
  if (was_fixed && c->lds_B) launch_feat_lds(c);  // skipped while the caller's blocks were in use
  // blocks of the current configuration follow the new weights
  if (hipMemsetAsync(c->flags + 6, 0, sizeof(int), c->stream) != hipSuccess) return PSE_ERR_HIP;
  if (c->dbl) launch_pc_blocks<double>(c);
  else launch_pc_blocks<float>(c);
  if (hipMemcpyAsync(c->flags_h, c->flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return PSE_ERR_HIP;
  c->pc_fallbacks = c->flags_h[6];
  c->pc_fb_pending = false;
  return hip_status(hipGetLastError());
}

pse_status pse_precond_set_blocks(pse_ctx *c, const void *P_dev) {
  if (!c) return PSE_ERR_INVALID_ARG;
  if (!c->pc_on) return PSE_ERR_PARAMS;
  if (!P_dev) {
    // back to the network's blocks (or I without weights)
    const bool was_fixed = c->pc_fixed;
    c->pc_fixed = false;
    if (!c->have_pos || !was_fixed) return PSE_OK;
    if (c->lds_B) launch_feat_lds(c);
  } else {
    if (hipMemcpyAsync(c->pc_user, P_dev, sizeof(float) * 9 * (size_t)c->n, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
      return PSE_ERR_HIP;
    c->pc_fixed = true;
    if (!c->have_pos) return PSE_OK;
  }
  if (hipMemsetAsync(c->flags + 6, 0, sizeof(int), c->stream) != hipSuccess) return PSE_ERR_HIP;
  if (c->dbl) launch_pc_blocks<double>(c);
  else launch_pc_blocks<float>(c);
  if (hipMemcpyAsync(c->flags_h, c->flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return PSE_ERR_HIP;
  c->pc_fallbacks = c->flags_h[6];
  c->pc_fb_pending = false;
  return hip_status(hipGetLastError());
}

pse_status pse_precond_features(pse_ctx *c, void *feat_out) {
  if (!c || !feat_out) return PSE_ERR_INVALID_ARG;
  if (!c->pc_on) return PSE_ERR_PARAMS;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  if (c->pc_fixed && c->lds_B) launch_feat_lds(c);  // not kept up to date while the caller's blocks are in use
  launch_unsort_features(c, feat_out);
  return hip_status(hipGetLastError());
}

pse_status pse_precond_blocks(pse_ctx *c, void *P_out, int32_t *fallbacks) {
  if (!c || !P_out) return PSE_ERR_INVALID_ARG;
  if (!c->pc_on) return PSE_ERR_PARAMS;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  if (c->dbl) launch_unsort_blocks<double>(c, (float *)P_out);
  else launch_unsort_blocks<float>(c, (float *)P_out);
  take_pc_fallbacks(c, false);
  if (fallbacks) *fallbacks = c->pc_fallbacks;
  return hip_status(hipGetLastError());
}

pse_status pse_precond_targets(const pse_params *p, const double *pos_host, const int32_t *idx, int32_t m,
                               double radius, double *out) {
  if (!p || !pos_host || (m > 0 && (!idx || !out)) || m < 0) return PSE_ERR_INVALID_ARG;
  Derived d;
  const pse_status ps = derive_params(*p, &d);
  if (ps != PSE_OK) return ps;
  if (!(radius > 0)) radius = p->rcut;
  for (int q = 0; q < m; ++q)
    if (idx[q] < 0 || idx[q] >= p->n) return PSE_ERR_INVALID_ARG;
  std::vector<double> x(3 * (size_t)p->n);
  for (size_t k = 0; k < x.size(); ++k) {
    if (!std::isfinite(pos_host[k])) return PSE_ERR_NONFINITE;
    double v = std::fmod(pos_host[k], d.L);
    x[k] = v < 0 ? v + d.L : v;
  }
  double serF[kSeriesTerms], serG[kSeriesTerms];
  fg_series_coeffs(p->xi, p->a, serF, serG);
  if (!precond_targets(x.data(), p->n, d.L, p->a, p->xi, p->rcut, d.mu0, serF, serG, idx, m, radius, out))
    return PSE_ERR_NOT_CONVERGED;
  return PSE_OK;
}

pse_status pse_mlp_forward(const void *w, const void *x, int32_t n, void *y, void *act_cache, void *stream) {
  if (!w || n < 0 || (n > 0 && (!x || !y))) return PSE_ERR_INVALID_ARG;
  if (((uintptr_t)w | (uintptr_t)x | (uintptr_t)act_cache) & 15) return PSE_ERR_INVALID_ARG;
  if (n == 0) return PSE_OK;
  launch_mlp_fwd((const uint16_t *)w, (const uint16_t *)x, n, (float *)y, (uint16_t *)act_cache,
                 (hipStream_t)stream);
  return hip_status(hipGetLastError());
}

size_t pse_mlp_backward_workspace(int32_t n) {
  return sizeof(float) * kWTotal * (size_t)mlp_bwd_parts(n < 1 ? 1 : n);
}

pse_status pse_mlp_backward(const void *w, const void *x, const void *act_cache, const void *dy, int32_t n, void *dw,
                            void *workspace, size_t workspace_bytes, void *stream) {
  if (!w || !x || !act_cache || !dy || !dw || !workspace || n < 1) return PSE_ERR_INVALID_ARG;
  if (workspace_bytes < pse_mlp_backward_workspace(n)) return PSE_ERR_INVALID_ARG;
  launch_mlp_bwd((const uint16_t *)w, (const uint16_t *)x, (const uint16_t *)act_cache, (const float *)dy, n,
                 (float *)dw, (float *)workspace, (hipStream_t)stream);
  return hip_status(hipGetLastError());
}

pse_status pse_mlp_backward_noalloc(const void *w, const void *x, const void *act_cache, const void *dy, int32_t n,
                                    void *dw, void *stream) {
  if (!w || !x || !act_cache || !dy || !dw || n < 1) return PSE_ERR_INVALID_ARG;
  const pse_status st = launch_mlp_bwd_static((const uint16_t *)w, (const uint16_t *)x, (const uint16_t *)act_cache,
                                              (const float *)dy, n, (float *)dw, (hipStream_t)stream);
  if (st != PSE_OK) return st;
  return hip_status(hipGetLastError());
}

pse_status pse_mlp_loss_grad(const void *y, const void *target, int32_t n, void *dy, void *loss, void *stream) {
  if (!y || !target || !dy || n < 1) return PSE_ERR_INVALID_ARG;
  launch_mlp_loss((const float *)y, (const float *)target, n, (float *)dy, (float *)loss, (hipStream_t)stream);
  return hip_status(hipGetLastError());
}

pse_status pse_mlp_adam(void *w_master, void *w_bf16, const void *dw, void *m, void *v, float lr, int32_t t,
                        void *stream) {
  if (!w_master || !w_bf16 || !dw || !m || !v || t < 1 || !(lr >= 0)) return PSE_ERR_INVALID_ARG;
  launch_mlp_adam((float *)w_master, (uint16_t *)w_bf16, (const float *)dw, (float *)m, (float *)v, lr, t,
                  (hipStream_t)stream);
  return hip_status(hipGetLastError());
}

pse_status pse_mobility_apply(pse_ctx *c, const void *F, void *u) {
  if (!c || !F || !u) return PSE_ERR_INVALID_ARG;
  if (!c->have_pos) return PSE_ERR_NO_POSITIONS;
  DISPATCH(c, (wave_apply_impl<T, A>(c, F, u, true)));
}

}  // extern "C"
