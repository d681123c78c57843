// Internal declarations of the gfx950 PSE sampler library.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/pse.h"

namespace pse {

constexpr int kMaxIter = 64;     // Lanczos basis capacity
constexpr int kFullMaxIter = 256;  // basis capacity of the full-mobility Krylov sample
constexpr int kTableK = 2048;    // F/G table intervals on [0, rcut]
constexpr int kTableN = kTableK + 2;  // table nodes (float2 (mu0 F, mu0 (G - F)) at r = k rcut / kTableK)
constexpr int kSeriesTerms = 16; // small-r series terms of the wave complement
constexpr uint32_t kKnownFlags = PSE_FLAG_NOISE_KSPACE | PSE_FLAG_FULL_LANCZOS;
constexpr int kRedBlock = 1024;
// cell-count scan: tiles of kScanTile cells, kScanPer per thread of kScanNT
constexpr int kScanPer = 16, kScanNT = 256, kScanTile = kScanPer * kScanNT;
constexpr int kRepBuf = 10;      // work vector holding the overlap repulsion of the Brownian step  // workgroups (partial sums) of the vector reductions
constexpr size_t kLdsPerCU = 160 * 1024;  // LDS of one gfx950 compute unit
constexpr int kInterpLanes = 512;         // built-in interpolation workgroup (one wavefront per particle)
// largest dynamic + table LDS of one workgroup of the staged near-field kernels
constexpr size_t kLdsBudget = 150 * 1024;
// static LDS of the staged near-field product beside its F/G table: the
// halo table of block edge B (cell starts and prefix sums of the (B+2)^3 halo
// cells and the B^3 target cells) plus reduction slots
constexpr size_t lds_static_extra(int B) {
  return 4 * (2 * (size_t)(B + 2) * (B + 2) * (B + 2) + 2 * (size_t)B * B * B + 3) + 256;
}
// Learned preconditioner: 24 features, MLP 24 -> 64 -> 64 -> 9.  Weights are
// one bf16 array: W1 [64][32] (inputs 24..31 zero), b1 [64], W2 [64][64],
// b2 [64], W3 [16][64] (rows 9..15 zero), b3 [16] (entries 9..15 zero).
constexpr int kNFeat = 24, kNHid = 64, kNOut = 9;
constexpr int kW1 = 0, kB1 = kW1 + 64 * 32, kW2 = kB1 + 64, kB2 = kW2 + 64 * 64, kW3 = kB2 + 64,
              kB3 = kW3 + 16 * 64, kWTotal = kB3 + 16;

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> struct vec4;
template <> struct vec4<float> { using type = float4; };
template <> struct vec4<double> { using type = double4; };

// Workgroups go to the 8 XCDs round-robin (workgroup b to XCD b % 8), and
// each XCD has its own L2.  xcd_block renumbers them so that each XCD works
// through one contiguous range of logical workgroups: neighbouring tiles,
// which read overlapping data, then share an L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// ------------------------------------------------------------- reductions
template <typename A> __device__ __forceinline__ A wave_sum(A v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.  sh >= 16 entries.
template <typename A> __device__ __forceinline__ A block_sum(A v, A *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  A r = 0;
  if (wid == 0) {
    r = lane < (int)(blockDim.x >> 6) ? sh[lane] : A(0);
    r = wave_sum(r);
  }
  __syncthreads();
  return r;
}

// bfloat16 <-> float: round to nearest, ties to even; NaN stays NaN.
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float x;
  __builtin_memcpy(&x, &u, 4);
  return x;
}

// Lanczos state kept in device memory (A = accumulation precision).
template <typename A> struct LzState {
  A alpha[kMaxIter];
  A beta[kMaxIter + 1];  // beta[0] = |z|, beta[m+1] couples v_m and v_{m+1}
  A s[kMaxIter];         // T_m^{1/2} e_1 of the latest iterate
  A rel_change;          // |s_m - s_{m-1}| / |s_m|
  A inv_beta;            // scale of the next Lanczos vector
  int m;                 // completed iterations
  int done;              // 1: converged (or broke down / max_iter reached)
  int converged;         // 1: tolerance met or invariant subspace
  int nonfinite;
};

// One system whose whole captured step runs in batched launches (FP32
// storage, LDS path, Philox noise, no forces, no preconditioner): the
// buffers of its binning, noise, Krylov start, combination and final sum.
struct SampRep {
  const float *pos_in;  // caller positions n x 3
  float4 *pos_w, *pos_s;
  int *cell_of, *slot, *cell_count, *tile_sum, *cell_start, *perm, *flags;
  float L, invL, inv_cs;
  int nc, ncell, n;
  const uint64_t *rng;  // (seed, counter) of the Philox noise
  float4 *z;            // real-space noise, sorted
  void *partials;       // A [kRedBlock]
  void *st;             // LzState<A>
  const float4 *V;      // Krylov basis
  float4 *yr;           // Krylov sample, sorted
  const float4 *wave;   // wave-space part, sorted
  float *out;           // displacement, caller order n x 3
  float cr;             // sqrt(2 kT dt)
  const float *f_in;    // caller forces n x 3, or null
  float4 *f_s;          // forces, sorted
  float4 *ur;           // M_r F, sorted
  float dt;
};
// Workgroup maps (system, block) of the batched launches: zero (blocks of
// 256 over ncell + 8), part (256 particles), tile (scan tiles), cell (4
// cells), flat (256 of the 4n vector scalars).
struct SampMaps {
  const int2 *zero, *part, *tile, *cell, *flat;
  int nzero, npart, ntile, ncell, nflat, nrep;
};

// One system of a batched neighbour build (LDS path, no repulsion), and the
// systems sharing one kernel (block edge, halo form): pmap lists (system,
// block) for each of the nblk workgroups, smem the largest halo's LDS.
struct NbrRep {
  const float4 *pos;
  const int *cell_start;
  uint16_t *nbr;
  int *cnt;
  int *flags;
  float cs, L, invL, rc2;
  int nc, n, cap, hcap;
};
struct NbrGroup {
  int B, unwrap, nblk;
  size_t smem;
  const int2 *pmap;
};

// One system of a batched Krylov loop: what the LDS product and the
// Lanczos vector kernels of a single system take as arguments (FP32
// storage, sorted order).
template <typename A> struct LzRep {
  const float4 *pos;        // sorted positions (x, y, z, 0)
  const int *cell_start;    // [ncell + 1]
  const uint16_t *nbr;      // halo-local neighbour list (chunks of 8)
  const int *cnt;           // entries per target
  const float2 *tab;        // (mu0 F, mu0 (G - F)) table
  int *ovf;                 // halo overflow flag
  const float4 *z;          // start vector
  float4 *t, *w, *V;        // product, residual, basis [maxit][n]
  const float4 *fs;         // forces (sorted) of the batched M_r F, or null
  float4 *ur;               // M_r F
  LzState<A> *st;
  A *partials;              // [0, kRedBlock): |w|^2; [kRedBlock, 2 kRedBlock): alpha_m
  float cs, L, invL, inv_dr, self_r;
  int nc, n, hcap, maxit;
  A tol;
};

// The systems of a batched Krylov loop whose LDS products share one kernel:
// block edge B, lanes per target G, halo form; pmap lists (system, block)
// for each of the nblk workgroups, smem the largest halo's LDS.
struct LzGroup {
  int B, G, unwrap, nblk;
  size_t smem;
  const int2 *pmap;
};

// What the host reads back from each replica after a captured batch step:
// the device flags and the Krylov state's outcome, gathered into one array
// by one kernel so that the step needs a single copy.
struct RepStatusSrc {
  const int *flags;  // [8]
  const void *lz;    // LzState<double> (acc_dbl) or LzState<float>
  int acc_dbl;
};
struct RepStatus {
  int flags[8];
  int m, done, converged, nonfinite;
  double rel_change;
};

// Coefficients of the wave-space scaling applied per k (fused x pass).
struct WaveCoef {
  double two_pi_over_L;  // k = 2 pi j / L
  double a;              // sphere radius
  double inv_4xi2;       // 1/(4 xi^2)
  double sigma2;         // Gaussian variance
  double det_scale;      // dt / (eta M^3): deterministic factor before B/ghat^2
  double sto_scale;      // sqrt(2 kT dt) / sqrt(eta V): stochastic factor before sqrt(B)/ghat
  double w_scale;        // M^{-3/2}: grid noise DFT normalisation
  uint64_t seed, counter;
  int use_philox;        // noise from Philox (key (seed,1))
  const uint64_t *rng;   // device (seed, counter) read in place of the two above, or null
};

// One system of a batched wave-space part (FP32 storage): with forces the
// spreading and the forward z and y passes, then the Philox k-space noise
// (and the forces' scaling) through the fused x pass, the inverse y and z
// passes and the interpolation, with the system's own buffers and
// coefficients.
struct WaveRep {
  float2 *spec;              // half spectrum [3][M][M][M/2]
  float *rgrid;              // real grid (packed after the inverse z pass)
  const float2 *tw_M, *tw_H;  // twiddles
  const float4 *pos;         // sorted positions
  float4 *out;               // wave-space displacement, sorted
  WaveCoef wc;
  int n, M;
  float h, invh, inv2s2, norm_h3;
  // with forces: the sorted forces spread onto the packed grid
  const float4 *f;
  const int *cell_start;
  int nc;
  float cs, norm;
};
// The systems of one grid size, support, interpolation workgroup size,
// spreading tile depth (8 nw) and forces flag: nrep consecutive WaveRep
// records; imap lists (system, block) for the interpolation's nimap
// workgroups.
struct WaveGroup {
  int M, P, nt, nw, forces, nrep, nimap;
  const WaveRep *reps;
  const int2 *imap;
};

// ---------------------------------------------------------------- host side
struct Derived {
  double L, h, sigma, gm, eta_se, eps_real, eps_wave, eps_quad, eps_alias;
  double eps_real_tail, eps_real_coherent;  // shell-integral real-space estimates
  double mu0;      // 1 / (6 pi eta a)
  double self_r;   // F_self * mu0
  double cs;       // cell side
  int nc;          // cells per side
};

// Appendix A closed forms and the small-r series, FP64 (fg_host.cpp)
void fg_eval_host(double r, double xi, double a, const double *serF, const double *serG, double *F, double *G);
double fg_self(double xi, double a);
void fg_series_coeffs(double xi, double a, double *serF, double *serG);
double fg_small_r_threshold(double xi, double a);
void fg_build_table(double xi, double a, double rc, double mu0, const double *serF, const double *serG,
                    float2 *tab);
// error model and parameter choice (params_host.cpp)
pse_status derive_params(const pse_params &p, Derived *d);
double eps_wave_bound(double kc, double xi, double a);
void real_tail(double rc, double xi, double a, double rho, double *inc, double *coh);
double eps_quad_bound(int P, double m);
double kcut_for(double tol, double xi, double a);
// (sums on blocks of indices above max_freq frequencies per axis)
double alias_estimate(double L, int M, double xi, double a, double sigma, int max_freq = 96);
// The sigma-free part of alias_estimate (B(k) over the sampled octant),
// reusable across window widths.
struct AliasWeights {
  double L;
  int M, nq;
  std::vector<double> k, w;
  double sum;
  AliasWeights(double L, int M, double xi, double a, int max_freq);
  double estimate(double sigma) const;
};
pse_status choose_params(const pse_params &base, const pse_tuning &t, pse_params *out, pse_tuning_info *info);
// learned-preconditioner training targets (precond_host.cpp); false if a
// patch matrix is not positive definite
bool precond_targets(const double *x, int n, double L, double a, double xi, double rc, double mu0,
                     const double *serF, const double *serG, const int *idx, int m, double radius, double *out);
bool fft_size_supported(int M);
// s = T^{1/2} e_1 of an m x m symmetric tridiagonal (lanczos_host.cpp)
bool tridiag_sqrt_e1_host(int m, const double *d, const double *e, double *s);

}  // namespace pse

struct pse_ctx {
  pse_params p;
  pse::Derived d;
  hipStream_t stream = nullptr;
  bool dbl = false;     // FP64 storage
  bool acc_dbl = true;  // FP64 Lanczos scalars
  int n = 0;
  int ncell = 0;
  bool have_pos = false;
  // graph mode (a batch step captured once, replayed per step): no host
  // decision inside set_positions or the sample; capacities fixed at
  // capture, overflows flagged on the device (flags[7], flags[1]) and the
  // replica redone after the replay
  bool graph = false;
  int graph_iters = 0;              // Lanczos iterations queued per sample in graph mode
  const uint64_t *rng_dev = nullptr;  // device (seed, counter) of the Philox noise, or null
  bool graph_stale = false;         // a buffer the captured graph uses was reallocated
  bool lz_external = false;         // graph mode: the Lanczos iterations run in the batch's batched loop
  bool status_external = false;     // graph mode: the batch reads flags and Krylov state back for all replicas
  bool wave_external = false;       // graph mode: the wave-space part runs in the batch's batched launches
  bool nbr_external = false;        // graph mode: the neighbour build runs in the batch's batched launch
  int last_iters = 4;
  int lz_maxit = 0;         // near-field Lanczos iterations at most: min(lanczos_max_iter, kMaxIter)
  // full-mobility Krylov sample (PSE_FLAG_FULL_LANCZOS)
  void *fl_V = nullptr;     // T4 [(kFullMaxIter + 1) n] basis
  void *fl_ab = nullptr;    // A [2 kFullMaxIter + 2]: alpha_m, then beta_m
  void *fl_ab_h = nullptr;  // pinned copy
  void *fl_coef = nullptr;  // A [kFullMaxIter]: combination coefficients
  int lz_launched = 0;      // Lanczos iterations launched in the current sample
  // device buffers
  void *pos_w = nullptr;    // T4 [n], caller order, wrapped
  void *pos_s = nullptr;    // T4 [n], sorted
  int *perm = nullptr;      // sorted -> caller index
  int *cell_of = nullptr;
  int *cell_count = nullptr;
  int *cell_start = nullptr;
  int *nbr = nullptr;
  int *nbr_cnt = nullptr;
  int nbr_cap = 0;
  int *flags = nullptr;     // [0] nonfinite, [1] list slots needed, [2..3] pairs, [4] max halo,
                            // [5] max neighbours, [6] preconditioner fallbacks
  int *flags_h = nullptr;   // pinned copy
  void *vbuf[11] = {};      // T4 [n] work vectors (sorted order, (x, y, z, 0)); [kRepBuf]: overlap repulsion
  double rep_k = 0.0;       // > 0: the neighbour build also accumulates the overlap repulsion (Brownian step)
  void *V = nullptr;        // T4 [(kMaxIter+1) n] Lanczos basis
  void *lz = nullptr;       // LzState<A>
  void *lz_h = nullptr;     // pinned copy
  void *partials = nullptr; // A [max blocks]
  unsigned *counter = nullptr;
  float2 *table = nullptr;  // F/G table nodes (FP32 modes)
  double *series = nullptr; // [2*kSeriesTerms] series coefficients (device)
  double series_h[2 * pse::kSeriesTerms];
  double small_r2 = 0;      // r^2 below which the series is used
  void *grid = nullptr;     // T [3 M^3]: planar half spectrum [c][jx][jy][jz < M/2] (complex)
  void *rgrid = nullptr;    // T [3 M^3] (allocated 4 M^3): real grid, nodes [x][y][z], packed
                            // (c0, c1, c2) per node
  void *grid2 = nullptr;    // T [3 M^3]: spectrum of caller grid noise W (absent with PSE_FLAG_NOISE_KSPACE)
  void *tw_M = nullptr;     // T2 [M] twiddles exp(-2 pi i k / M)
  void *tw_H = nullptr;     // T2 [M/2]
  // GPU-time accounting (pse_profile)
  uint32_t prof_mask = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_stage;   // stage of each recorded (begin, end) pair
  int ev_open = -1;            // index of the open begin event, -1 if none
  int64_t pairs = 0;
  // LDS-staged near-field path (FP32 storage): block edge B (0 = global path),
  // halo capacity (particles) and number of target blocks
  // launch shapes picked by pse_autotune (0: the built-in choice): depth
  // of the spreading tiles (8 x 8 x 8 nw nodes) and lanes per interpolation
  // workgroup
  int tune_spread_nw = 0;
  int tune_interp_threads = 0;
  // lanes per target of the LDS near-field product (2, 3 or 4; 0: 3)
  int tune_spmv_lanes = 0;
  int lds_B = 0;
  int lds_B_pref = 0;  // block edge of the last configuration (the search starts there)
  int hcap = 0;
  int lds_blocks = 0;
  // learned block preconditioner (params.precond == 1); pc_suspend is set
  // while a failed preconditioned sample is redone with P = I
  bool pc_suspend = false;
  bool pc_on = false;
  bool pc_have_w = false;
  bool pc_fixed = false;       // the caller's blocks (pse_precond_set_blocks) in place of the network's
  float *pc_user = nullptr;    // [n][9] the caller's blocks, caller order
  uint16_t *pc_w = nullptr;    // bf16 [kWTotal]
  uint16_t *pc_feat = nullptr; // bf16 [n][24], sorted order
  float *pc_y = nullptr;       // [n][9] network output, sorted order
  void *pc_P = nullptr;        // T [n][12]: rows of P_i as (x, y, z, 0)
  void *pc_Pinv = nullptr;     // T [n][12]: rows of P_i^-1
  int pc_fallbacks = 0;        // blocks replaced by I at the last set_positions
  int *pc_fb_h = nullptr;      // pinned: the device count, copied back without a wait
  bool pc_fb_pending = false;  // pc_fb_h not yet taken into pc_fallbacks
};
