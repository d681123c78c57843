// Kernel launchers shared between the kernel sources and the C ABI.
#pragma once
#include "pse_internal.hpp"

namespace pse {

enum class GridOp { FftZ, FftZAos, FftStrided, XFused };

// Bracket the launches of one stage with events (no-op unless selected).
void prof_begin(pse_ctx *c, int stage);
void prof_end(pse_ctx *c, int stage);
struct ProfScope {
  pse_ctx *c;
  int stage;
  ProfScope(pse_ctx *c_, int s) : c(c_), stage(s) { prof_begin(c, stage); }
  ~ProfScope() { prof_end(c, stage); }
};

// particle side (k_particles.hip)
template <typename T> void launch_bin(pse_ctx *c, const void *pos);
// nwords 32-bit words of p set to 0 by a kernel (capturable in a graph)
void launch_zero_words(hipStream_t s, void *p, size_t nwords);
template <typename T> void launch_nbr(pse_ctx *c);
// LDS-staged near-field path (FP32): halo sizes into flags[4] for block edge B;
// neighbour build with 16-bit LDS indices
void launch_halo_size(pse_ctx *c, int B);
void launch_nbr_lds(pse_ctx *c);
// the LDS neighbour build of every system of the groups in one launch per group
void launch_nbr_batch(hipStream_t s, const NbrRep *reps, const NbrGroup *groups, int ngroups);
void launch_feat_lds(pse_ctx *c);  // preconditioner features from the list and the staged halo
template <typename T, typename A> void launch_spmv(pse_ctx *c, const void *src, void *out, bool lz, void *vm_out);
template <typename T, typename A> void launch_lz_init(pse_ctx *c, const void *z);
template <typename T, typename A> void launch_lz_iter(pse_ctx *c, int m, const void *z);
template <typename T, typename A> void launch_lz_combine(pse_ctx *c, void *y);
template <typename T> void launch_gather3(pse_ctx *c, const void *in, void *out);
// out (sorted) = gather(in, caller order; may be null) + add (sorted; may be null)
template <typename T> void launch_gather3_add(pse_ctx *c, const void *in, const void *add, void *out);
// x += dx over 3n scalars (caller order)
template <typename T> void launch_advance(pse_ctx *c, void *x, const void *dx);
template <typename T>
void launch_finalize(pse_ctx *c, const void *yr, double cr, const void *ur, double dt, const void *wv, void *out);
template <typename T> void launch_real_noise(pse_ctx *c, void *z, uint64_t seed, uint64_t sample);

// full-mobility Krylov sample (k_full.hip); alpha, beta live in device memory
template <typename T, typename A> void launch_fl_norm(pse_ctx *c, const void *v, void *dst);
template <typename T, typename A> void launch_fl_alpha(pse_ctx *c, void *t, const void *u, const void *v, void *dst);
template <typename T, typename A>
void launch_fl_update(pse_ctx *c, const void *t, const void *vm, const void *vprev, void *w, const void *alpha,
                      const void *beta, void *beta_next);
template <typename T, typename A> void launch_fl_scale(pse_ctx *c, const void *src, const void *beta, void *dst);
template <typename T, typename A> void launch_fl_combine(pse_ctx *c, int m, void *y);

// learned block preconditioner (k_precond.hip)
void launch_mlp_fwd(const uint16_t *w, const uint16_t *x, int n, float *y, uint16_t *cache, hipStream_t stream);
int mlp_bwd_parts(int n);  // fp32 slots of kWTotal needed by launch_mlp_bwd's workspace
void launch_mlp_bwd(const uint16_t *w, const uint16_t *x, const uint16_t *cache, const float *dy, int n, float *dw,
                    float *work, hipStream_t stream);
// partial-gradient slots of the allocation-free backward pass (>= mlp_bwd_parts(n) for every n)
constexpr int kMlpStaticSlots = 256;
pse_status launch_mlp_bwd_static(const uint16_t *w, const uint16_t *x, const uint16_t *cache, const float *dy, int n,
                                 float *dw, hipStream_t stream);
void launch_mlp_adam(float *wm, uint16_t *wb, const float *g, float *m, float *v, float lr, int t, hipStream_t stream);
void launch_mlp_loss(const float *y, const float *t, int n, float *dy, float *loss, hipStream_t stream);
template <typename T> void launch_pc_blocks(pse_ctx *c);           // features -> MLP -> P, P^-1 (fallbacks in flags[6])
template <typename T, typename A> void launch_pc_pre(pse_ctx *c, const void *src, void *u);  // u = P^T src
template <typename T, typename A>
void launch_pc_post(pse_ctx *c, const void *tp, const void *src, void *out, void *vm_out);
template <typename T> void launch_pc_apply_inv(pse_ctx *c, void *y);  // y = P^-1 y
void launch_unsort_features(pse_ctx *c, void *out);
template <typename T> void launch_unsort_blocks(pse_ctx *c, float *out);
template <typename T, typename A> void launch_lz_iter_pc(pse_ctx *c, int m, const void *z);
// iteration m of the Lanczos process on nrep systems at once (FP32 storage,
// LDS product, no preconditioner): bit-identical to launch_lz_iter per system
template <typename A>
void launch_lz_batch_iter(hipStream_t s, const LzRep<A> *reps, int nrep, const LzGroup *groups, int ngroups,
                          const int2 *vmap, int nvblk, int m);
// the wave-space part without forces of every system of the groups
// (bit-identical to each system's own launches)
void launch_wave_batch(hipStream_t s, const WaveGroup *groups, int ngroups);
// the fully batched systems of a captured step: binning; noise and Krylov
// start; combination and final sum (A: the Lanczos scalar type)
void launch_samp_batch_bin(hipStream_t s, const SampRep *reps, const SampMaps &m);
// the forces' gather into sorted order (systems with forces)
void launch_samp_batch_forces(hipStream_t s, const SampRep *reps, const SampMaps &m);
// M_r F of every system of the groups whose LzRep carries forces
template <typename A>
void launch_lz_batch_plain(hipStream_t s, const LzRep<A> *reps, const LzGroup *groups, int ngroups);
template <typename A> void launch_samp_batch_start(hipStream_t s, const SampRep *reps, const SampMaps &m);
template <typename A> void launch_samp_batch_end(hipStream_t s, const SampRep *reps, const SampMaps &m);
// out[r] = flags and Krylov outcome of replica r
void launch_batch_status(hipStream_t s, const RepStatusSrc *src, int nrep, RepStatus *out);

// grid side (k_grid.hip)
//   FftZ:       a = src, b = dst, x = direction (-1 forward R2C, +1 inverse C2R)
//   FftZAos:    as FftZ with the real side one packed vector (c0, c1, c2)
//               per node: forward reads the grid that spreading writes,
//               inverse writes the grid that interpolation reads
//   FftStrided: b = data, x = axis (0: x, 1: y), y = direction
//   XFused:     a = transformed grid-noise spectrum (or null), b = data,
//               x = forces present, y = noise (0 none, 1 Philox, 2 grid noise)
template <typename T> void launch_grid_op(pse_ctx *c, GridOp op, const void *a, void *b, const WaveCoef *wc, int x, int y);
template <typename T> void launch_spread_interp(pse_ctx *c, bool spread, const void *vec, void *grid_or_out);
// Spreading writes the packed real grid ((c0, c1, c2) per node) and clears
// it itself (every node written once, or cleared before the atomic
// fallback): no separate clear is needed.  Interpolation reads the packed
// grid that the inverse z pass writes.
bool spread_writes_whole_grid(int M, int P);
// built-in spreading tile depth / 8 for a grid, support and precision
int spread_default_nw(int M, int P, bool fp32);
// times the valid spreading tile depths and interpolation workgroup sizes on
// the current positions and keeps the fastest (c->tune_*)
template <typename T> pse_status autotune_grid(pse_ctx *c, int32_t *choice);
// Times the LDS near-field product at 2, 3 and 4 lanes per target and keeps
// the fastest; *lanes receives the kept value (0 where the product does not
// use the LDS path: FP64, or no LDS block fits).
pse_status autotune_spmv(pse_ctx *c, int32_t *lanes);
// A spreading tile depth (0: built-in) and interpolation workgroup size
// (0: built-in) that the grid's launches accept.
bool grid_shape_valid(int M, int P, int depth, int interp_lanes);

}  // namespace pse
