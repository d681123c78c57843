/* pse.h — C ABI of the MI355X (gfx950) Positively Split Ewald Brownian sampler.
 *
 * Method: Fiore, Balboa Usabiaga, Donev, Swan, "Rapid Sampling of Stochastic
 * Displacements in Brownian Dynamics Simulations" (arXiv:1611.09322).
 *
 * For N equal spheres of radius a in a cubic periodic box of side L, the
 * library returns displacements
 *
 *     dx = dt M F + sqrt(2 kT dt) ( M_r^{1/2} z1 + M_w^{1/2} z2 )      (eqs. langevin, split)
 *
 * with M = M_r + M_w the positively split periodic RPY mobility (eqs. Mwave,
 * Mreal, Appendix A).  M_r^{1/2} z1 is a Lanczos (Krylov) approximation on the
 * near-field real-space sum (Sec. II B.1); M_w^{1/2} z2 is drawn with Gaussian
 * spreading/interpolation on an M^3 grid and FFTs (Spectral Ewald, Sec. II B.2).
 *
 * Conventions shared by every entry point
 *  - Memory: every pointer argument named *_dev is device memory owned by the
 *    caller, read or written on the context's stream; the library never frees
 *    it.  The context owns all scratch (allocated in pse_create).
 *  - Element type: double for PSE_FP64, float for PSE_FP32 and PSE_MIXED.
 *  - Particle vectors (positions, forces, displacements, z1, velocities) are
 *    n x 3, row-major, in the caller's particle order.
 *  - Grid noise W is 3 x M x M x M, component-major, z fastest:
 *    W[((c*M + ix)*M + iy)*M + iz] sits at node (ix, iy, iz) h, h = L/M.
 *  - Calls are asynchronous on the stream given to pse_create, except where
 *    noted: pse_set_positions and the sampling calls synchronise once to read
 *    status (neighbour-list overflow, Lanczos convergence).
 *  - Errors never abort: every call returns a pse_status.  After a non-zero
 *    status the outputs are unspecified unless stated.
 *  - One context per stream; calls on one context must not overlap.
 */
#ifndef PSE_H
#define PSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSE_OK = 0,
  PSE_ERR_INVALID_ARG = -1,   /* null pointer, n < 1, non-positive size ... */
  PSE_ERR_OOM = -2,           /* device allocation failed */
  PSE_ERR_HIP = -3,           /* a HIP runtime call failed */
  PSE_ERR_PARAMS = -4,        /* parameters the error model rejects:
                                 rcut >= L/2, eta_SE >= 1, M < P, odd P,
                                 unsupported grid size, or an error estimate
                                 above params.tol */
  PSE_ERR_NONFINITE = -5,     /* non-finite input or Lanczos scalar */
  PSE_ERR_NOT_CONVERGED = -6, /* Lanczos hit max_iter; best iterate written */
  PSE_ERR_NO_POSITIONS = -7,  /* sampling before pse_set_positions */
  PSE_WARN_PRECOND_FALLBACK = 1
} pse_status;

typedef enum { PSE_FP64 = 0, PSE_FP32 = 1, PSE_MIXED = 2 } pse_precision;

typedef struct {
  int32_t n;                /* number of particles (>= 1) */
  double box;               /* cubic box side L */
  double a;                 /* sphere radius */
  double eta;               /* viscosity */
  double kT;                /* thermal energy */
  double xi;                /* Ewald splitting parameter (eq. green2, eq. Mwave) */
  double rcut;              /* real-space cutoff, < L/2 (minimum image) */
  int32_t grid;             /* M: grid points per side, a power of two,
                               16 <= M <= 512 (PSE_ERR_PARAMS otherwise) */
  int32_t support;          /* P: Gaussian support points per side, even, <= 16 */
  double gauss_m;           /* Gaussian truncation in standard deviations;
                               0 selects sqrt(pi P) (Sec. II C) */
  double lanczos_tol;       /* successive-iterate tolerance of the Krylov sample */
  int32_t lanczos_max_iter; /* <= 64 */
  int32_t precision;        /* pse_precision */
  int32_t precond;          /* 0: none; 1: learned block preconditioner */
  uint32_t flags;           /* PSE_FLAG_* bits below; other bits must be 0 */
  double tol;               /* requested relative error (Sec. II C); when > 0,
                               parameters whose estimates exceed it are
                               rejected: eps_real_tail, eps_wave, and
                               3 eps_quad + eps_alias (pse_derived; the window
                               error of one spreading or interpolation) must
                               each be <= tol.  0: not checked */
} pse_params;

/* pse_params.flags */
#define PSE_FLAG_NOISE_KSPACE 1u /* wave-noise arguments (pse_sample_with_noise,
                                    pse_wave_sample) are zeta itself on the stored
                                    half spectrum: complex [3][M][M][M/2]
                                    (interleaved real, imaginary; element
                                    ((c M + jx) M + jy)(M/2) + jz at the signed
                                    indices of the DFT order), unit variance
                                    E |zeta|^2 = 1.  On the plane jz = 0 only the
                                    canonical member of each (k, -k) pair (signed
                                    jy > 0, or jy = 0 and jx > 0) is read, its
                                    partner is its conjugate; k = 0 and Nyquist
                                    entries are not read.  Without the flag the
                                    argument is real grid noise W and the context
                                    holds one more 3 M^3 buffer for its spectrum */
#define PSE_FLAG_FULL_LANCZOS 2u /* the context also holds the basis of
                                    pse_full_sample (257 vectors of n x 4), and
                                    lanczos_max_iter may be up to 256 there (the
                                    near-field sample still stops at 64) */

typedef struct {
  int32_t lanczos_iters;    /* Krylov iterations used by the last real-space sample */
  int32_t converged;        /* 1 if the tolerance was met */
  double lanczos_rel_change;/* final ||y_m - y_{m-1}|| / ||y_m|| */
  int32_t max_neighbors;    /* largest near-field neighbour count */
  int32_t precond_fallbacks;/* particles whose learned block fell back to I */
  int64_t neighbor_pairs;   /* ordered near-field pairs (sum of neighbour counts) */
  int32_t nbr_index_bytes;  /* bytes per stored neighbour index: 2 on the LDS-staged
                               FP32 path (halo-local), 4 otherwise (global) */
  int32_t lds_block_edge;   /* cells per edge of the target blocks of the LDS-staged
                               near-field kernels (1 ... 4), 0 on the global path */
} pse_stats;

/* Stages of the hot path, for GPU-time accounting (pse_profile). */
typedef enum {
  PSE_STAGE_BIN = 0,      /* wrap, linked-cell counting sort, sorted gather */
  PSE_STAGE_NBR = 1,      /* near-field neighbour list */
  PSE_STAGE_SPMV = 2,     /* one near-field product M_r v (Lanczos or forces) */
  PSE_STAGE_LANCZOS = 3,  /* Lanczos vector update, reductions, tridiagonal solve, combine */
  PSE_STAGE_NOISE = 4,    /* real-space Philox noise */
  PSE_STAGE_SPREAD = 5,   /* Gaussian spreading of forces */
  PSE_STAGE_FFT = 6,      /* z and y FFT passes (forward and inverse) */
  PSE_STAGE_XFUSED = 7,   /* x pass with B(k), projection, noise */
  PSE_STAGE_INTERP = 8,   /* Gaussian interpolation */
  PSE_STAGE_OTHER = 9,    /* gathers, final combine, grid clears */
  PSE_STAGE_PRECOND = 10, /* learned preconditioner: MLP, blocks, P^-1 y */
  PSE_NSTAGES = 11
} pse_stage;

typedef struct {
  double h;                 /* grid spacing L/M */
  double sigma;             /* Gaussian standard deviation P h / (2 m) */
  double gauss_m;           /* m actually used */
  double eta_se;            /* 4 xi^2 sigma^2; must be < 1 */
  double eps_real;          /* exp(-xi^2 rcut^2)                (Sec. II C) */
  double eps_wave;          /* analytic k_cut bound, k_cut = pi/h (Sec. II D) */
  double eps_quad;          /* exp(-pi^2 P^2/2m^2) + erfc(m/sqrt2) (Sec. II C), per
                               axis: the separable window loses about 3 eps_quad */
  int32_t cells;            /* linked cells per side for the near-field sum */
  double self_real;         /* real-space self mobility, eq. (self), / (6 pi eta a) */
  double eps_alias;         /* aliasing estimate of the Gaussian window on the
                               grid: relative error of the wave sample,
                               sqrt(sum_k B(k) sum_{n != 0} rho(k, n)^2 / sum_k B(k)),
                               rho(k, n) = ghat(k + 2 pi n / h) / ghat(k), over
                               the grid k-set and the first alias shell
                               n in {-1, 0, 1}^3 (grids above 96^3: summed on
                               blocks of ceil(M / 96) indices per axis) */
  double eps_real_tail;     /* real-space truncation of a sample or of M F with
                               random forces, relative to the Stokes mobility:
                               sqrt(rho int_rc^inf 4 pi r^2 (2F^2 + G^2)/3 dr),
                               rho = n / L^3 (F, G of eq. Mreal); exp(-xi^2 rc^2)
                               above is its decay alone, without the number of
                               pairs just past rc that multiplies it */
  double eps_real_coherent; /* the same for M F with aligned forces (the pairs
                               add in amplitude): rho int_rc^inf 4 pi r^2
                               |2F + G| / 3 dr */
} pse_derived;

/* Status text for a pse_status value (static string). */
const char *pse_status_string(pse_status s);

typedef struct pse_ctx pse_ctx;
typedef struct pse_batch pse_batch;

/* Create a sampling context for the parameters `p` on HIP stream `stream`
 * (a hipStream_t; NULL = the null stream).  Validates the parameters against
 * the error model (Sec. II C), builds the real-space F/G table (Appendix A,
 * evaluated in FP64), and allocates every scratch buffer: sorted particle
 * arrays, cell list, neighbour list, Lanczos basis (max_iter+1 vectors of 3n)
 * and the 3 M^3 grid.  *out receives the context (NULL on failure).
 * Errors: INVALID_ARG (null pointers), PARAMS (see pse_status), OOM, HIP. */
pse_status pse_create(const pse_params *p, void *stream, pse_ctx **out);

/* Release the context and its scratch.  NULL is accepted. */
pse_status pse_destroy(pse_ctx *ctx);

/* Derived quantities of the error model for this context (host struct). */
pse_status pse_get_derived(const pse_ctx *ctx, pse_derived *out);

/* The same quantities for a parameter set, without a context or a GPU
 * (host only).  Returns the status pse_create would return for `p` on
 * parameter validation (PARAMS, INVALID_ARG); *out is filled on PSE_OK. */
pse_status pse_derive(const pse_params *p, pse_derived *out);

/* Parameter choice (Sec. II C-D): the error sources are controlled
 * separately.  For a sample (and M F with random forces) the real-space,
 * wave-space and Krylov errors are independent and add in variance, so
 * each is held at or below t_s = tol / sqrt 3; for aligned forces
 * (deterministic) the real-space and wave-space errors are systematic and
 * add linearly, t_s = tol / 2:
 *   rc: the smallest with eps_real_tail <= t_s (eps_real_coherent when
 *       deterministic), rho = n / L^3
 *   M:  pi / h at or above the k_cut whose Sec. II D bound is t_s (any
 *       supported size, smallest first)
 *   P, m: even P and a width m in [max(2, P h xi), 1.4 sqrt(pi P)] with
 *       eps_wave + w (3 eps_quad + eps_alias) <= t_s, w = 2 when the step
 *       also spreads forces (with_forces, deterministic: spreading and
 *       interpolation both err), else 1.  3 eps_quad: the separable window
 *       is truncated on three axes.  m = sqrt(pi P) when it passes, else
 *       the width minimising 3 eps_quad + eps_alias (golden section)
 * and xi minimises the work model of eq. (work) for this implementation:
 *   t = c_pair pairs (n_iter + [forces] + 2) + c_node N P^3 (1 + [forces])
 *       + c_fft M^3 log2 M^3 + c_particle N,
 * pairs = N (N / V)(4 pi / 3) rc^3 (hard-sphere structure), scanned over
 * xi a = 0.15 ... 1.5 in steps of 0.01 (or the caller's xi).  The constants
 * are seconds per near-field pair per product, per particle-node of one
 * spreading or interpolation, per M^3 log2 M^3 of the FFT set, per
 * particle; 0 selects values measured on MI355X at 10^6 spheres
 * (1.8e-12, 7.4e-13, 1.5e-12, 3.8e-10).  Host only, no GPU. */
typedef struct {
  double tol;          /* target relative error of every source, (0, 1) */
  double xi;           /* > 0: keep this xi; 0: choose it */
  double n_iter;       /* Lanczos iterations the model assumes (0: 5) */
  double c_pair, c_node, c_fft, c_particle;  /* work-model constants (0: built-in) */
  int32_t max_grid;    /* largest grid to consider (0: 512) */
  int32_t with_forces; /* 1: the step includes dt M F (spreading + one more product) */
  int32_t deterministic; /* 1: tol bounds M F for aligned forces (sedimentation):
                            coherent real-space tail, linear error budget; 0:
                            tol bounds the sample (and M F with random forces) */
} pse_tuning;

typedef struct {
  double model_seconds;       /* work-model time of the chosen parameters */
  double eps_real, eps_wave, eps_quad, eps_alias;
  double pairs_per_particle;  /* model neighbour count (N / V)(4 pi / 3) rc^3 */
  double xi_star;             /* eq. (xistar): the large-N asymptote of the
                                 optimum for the same constants (d_f = 3) */
  double eps_real_tail;       /* the real-space estimate rc was chosen by
                                 (pse_derived.eps_real_tail, or
                                 eps_real_coherent when deterministic) */
} pse_tuning_info;

/* base: n, box, a, eta, kT, lanczos_max_iter, precision, precond, flags are
 * kept; xi, rcut, grid, support, gauss_m (0 when sqrt(pi P)), lanczos_tol
 * (= t_s) and tol (= t->tol) are chosen.  Errors: INVALID_ARG, PARAMS (no feasible choice, e.g. a box
 * too small for rc < L/2 at any xi). */
pse_status pse_choose_params(const pse_params *base, const pse_tuning *t, pse_params *out, pse_tuning_info *info);

/* Set the particle positions (pos_dev: n x 3).  Positions are wrapped into
 * [0, L) (a coordinate equal to L maps to 0); overlapping spheres are allowed
 * (the RPY form stays SPD, eq. pairmobility).  Builds the linked-cell list,
 * the sorted particle order and the near-field neighbour list (Sec. III: the
 * real-space sum uses cell and neighbour lists).  Synchronises once.
 * Errors: NONFINITE (a coordinate is not finite), OOM (neighbour list). */
pse_status pse_set_positions(pse_ctx *ctx, const void *pos_dev);

/* One Brownian displacement with the library's own noise:
 *   disp = dt (M_r + M_w) F + sqrt(2 kT dt)(M_r^{1/2} z1 + M_w^{1/2} z2)
 * z1 and z2 are drawn from Philox-4x64-10 (Salmon et al., SC'11):
 *  - uniforms u = ((w >> 11) + 1/2) 2^-53 (FP64) or ((w >> 40) + 1/2) 2^-24
 *    (FP32/MIXED) from 64-bit words w; Box-Muller on word pairs (wa, wb):
 *    sqrt(-2 ln ua) (cos, sin)(2 pi ub);
 *  - z1[q], q = 3 i + d (caller order): key (seed, 0), counter
 *    (q >> 2, counter, 0, 0), normal number q & 3 of the block;
 *  - z2 on the stored half spectrum, element e = ((c M + jx) M + jy)(M/2) + jz
 *    (jz < M/2): key (seed, 1), counter (e >> 1, counter, 0, 0),
 *    zeta = (n_{2p} + i n_{2p+1})/sqrt 2, p = e & 1; on the plane jz = 0 the
 *    member of each (k, -k) pair with signed jy > 0 (or jy = 0, jx > 0) draws
 *    and its partner is the conjugate; k = 0 and Nyquist indices are zero.
 * The wave
 * part applies B(k)^{1/2} (eq. Mwave) in k-space and one inverse 3D FFT plus
 * Gaussian interpolation; with forces the deterministic wave term shares that
 * inverse FFT (Sec. III, combined FFT pair).  forces_dev may be NULL (then
 * dt M F is omitted).  disp_dev: n x 3 output.  stats may be NULL.
 * Errors: NO_POSITIONS, NOT_CONVERGED (disp still written), NONFINITE. */
pse_status pse_sample(pse_ctx *ctx, uint64_t seed, uint64_t counter, double dt,
                      const void *forces_dev, void *disp_dev, pse_stats *stats);

/* Same displacement with caller-supplied noise: z1_dev (n x 3 standard
 * normals) and W_dev (3 x M^3 real standard normals on the grid nodes; the
 * k-space noise is zeta = DFT(W)/M^{3/2}, fluctuating-hydrodynamics form;
 * under PSE_FLAG_NOISE_KSPACE it is zeta itself, see the flag).
 * Either may be NULL (that part is omitted).  forces_dev may be NULL. */
pse_status pse_sample_with_noise(pse_ctx *ctx, const void *z1_dev, const void *W_dev,
                                 double dt, const void *forces_dev, void *disp_dev,
                                 pse_stats *stats);

/* One Euler-Maruyama step of eq. (langevin) (the divergence term vanishes
 * in a periodic box, Sec. II B):
 *   x <- x + dt M (F_ext + F_rep) + sqrt(2 kT dt) M^{1/2} dW,
 * in place on pos_dev (n x 3, caller order; coordinates are not wrapped, the
 * library wraps them internally).  Each step rebuilds the cell and
 * neighbour lists at the current positions (pse_set_positions) and draws
 * the noise as pse_sample does (key seed, counter step).  F_ext: forces_dev
 * (n x 3) or NULL.  F_rep: the overlap repulsion of near-hard spheres,
 *   F_rep,i = sum_{j: r_ij < 2a} krep (2a - r_ij) (x_i - x_j) / r_ij,
 * accumulated by the neighbour-list scan itself (krep = 0: none).  The
 * deterministic and stochastic wave terms share one FFT pair (Sec. III).
 * disp_dev (n x 3) receives the displacement, or NULL.  Synchronises as
 * pse_set_positions and pse_sample do.
 * Errors: INVALID_ARG (dt <= 0, krep < 0), those of pse_set_positions and
 * pse_sample (on NOT_CONVERGED the positions still move by the best iterate). */
pse_status pse_bd_step(pse_ctx *ctx, void *pos_dev, const void *forces_dev, double dt, double krep, uint64_t seed,
                       uint64_t step, void *disp_dev, pse_stats *stats);

/* w = M_r v (near-field real-space product, eq. Mreal), v_dev/w_dev n x 3. */
pse_status pse_real_matvec(pse_ctx *ctx, const void *v_dev, void *w_dev);

/* y = M_r^{1/2} z1 by Lanczos (Sec. II B.1), z1_dev/y_dev n x 3. */
pse_status pse_real_sample(pse_ctx *ctx, const void *z1_dev, void *y_dev, pse_stats *stats);

/* y = M^{1/2} z1 on the full mobility M = M_r + M_w by the Lanczos process
 * (Chow-Saad, the same stopping rule and tolerance as the near-field
 * sample), each product a near-field product plus a wave-space product
 * M_w v through the FFT pair: the comparator of Sec. III (Lanczos applied to
 * the whole mobility), whose iteration count grows with N as the condition
 * number of M does.  Needs PSE_FLAG_FULL_LANCZOS (PSE_ERR_PARAMS otherwise);
 * at most lanczos_max_iter (<= 256) iterations, NOT_CONVERGED with the best
 * iterate written past that.  Synchronises once per iteration (the
 * tridiagonal square root is solved on the host in FP64).
 * z1_dev, y_dev: n x 3. */
pse_status pse_full_sample(pse_ctx *ctx, const void *z1_dev, void *y_dev, pse_stats *stats);

/* y = M_w^{1/2} z2 with grid noise W_dev (3 x M^3), or with zeta itself
 * under PSE_FLAG_NOISE_KSPACE; y_dev n x 3 (Sec. II B.2). */
pse_status pse_wave_sample(pse_ctx *ctx, const void *W_dev, void *y_dev);

/* u = M_w F (spread, forward FFT, B(k), inverse FFT, interpolate), n x 3. */
pse_status pse_wave_apply(pse_ctx *ctx, const void *forces_dev, void *u_dev);

/* u = (M_r + M_w) F, the deterministic mobility product (n x 3). */
pse_status pse_mobility_apply(pse_ctx *ctx, const void *forces_dev, void *u_dev);

/* ---------------------------------------------------------------------
 * Learned block preconditioner of the real-space Krylov sample.
 *
 * With params.precond = 1 the Lanczos iteration of Sec. II B.1 runs on
 * A = P M_r P^T with P block diagonal (one 3 x 3 block P_i per particle) and
 * the real-space sample is y = P^{-1} A^{1/2} z1; its covariance is still
 * M_r (P^{-1} A P^{-T} = M_r), so the output law is unchanged.  The paper
 * uses no preconditioner: the features, network and training target are
 * this library's (defined below).  P_i = I + reshape(y_i), y_i the output of
 * an MLP 24 -> 64 -> 64 -> 9 (relu; bf16 weights, inputs and hidden values,
 * fp32 sums on the matrix cores) applied to 24 features of the particle's
 * near field, accumulated during pse_set_positions:
 *   0..3   #{r < 2.2a}/4, #{r < 3a}/8, #{r < 4.5a}/16, #{r <= rc}/128
 *   4      sum F / 8
 *   5..10  sum (G - F) dh dh^T        (xx, yy, zz, xy, xz, yz)
 *   11..16 sum_{r < 3a} dh dh^T / 4   (same order)
 *   17..19 sum_{r < 3a} dh / 4
 *   20     sum (G - F);  21  min r / 4.5a (1 without near neighbours)
 *   22     sum_{r < 3a} (3a - r) / a / 4;  23  F_self (eq. self)
 * over near neighbours j (minimum image, r < 4.5a; f3 alone counts all
 * within rc; d = x_i - x_j, dh = d / r or 0 at r = 0), F and G the
 * dimensionless functions of Appendix A.
 * A block falls back to I if it is not finite, |det P_i| < 1e-6 or
 * |P_i|_F |P_i^{-1}|_F > 1e3.  Without weights every block is I.  Global
 * fallback: when the preconditioned Krylov sample fails (a non-finite
 * scalar, or the tolerance not met within lanczos_max_iter), the same z1 is
 * sampled again with P = I, and precond_fallbacks reports n.  Sampling
 * calls return PSE_WARN_PRECOND_FALLBACK when any block fell back (or the
 * status of the plain sample when that fails too); pse_stats.precond_fallbacks
 * counts the blocks.
 *
 * Weights: one bf16 array of PSE_MLP_NPARAM elements, in this order:
 *   W1 [64][32] (input columns 24..31 must be 0), b1 [64], W2 [64][64],
 *   b2 [64], W3 [16][64] (rows 9..15 must be 0), b3 [16] (9..15 must be 0).
 * Device arrays passed to the pse_mlp_* calls must be 16-byte aligned.
 * ------------------------------------------------------------------- */
#define PSE_MLP_NPARAM 7312
#define PSE_MLP_NFEAT 24
#define PSE_MLP_NHIDDEN 64
#define PSE_MLP_NOUT 9

/* Copy the bf16 weights (host, bytes = 2 * PSE_MLP_NPARAM) into the context;
 * the blocks of the current positions are recomputed.  PSE_ERR_PARAMS if
 * the context was created with precond = 0. */
pse_status pse_precond_set_weights(pse_ctx *ctx, const void *weights_host, size_t bytes);

/* Use the caller's blocks P_i (P_dev: n x 9 fp32 row-major, caller order,
 * device; copied) in place of the network's, for the current positions and
 * at every later pse_set_positions, until pse_precond_set_weights is called
 * or P_dev is NULL (back to the network's blocks, or I without weights).
 * Each block passes the same fallback rule.  The sample's covariance is M_r
 * for any invertible blocks, so blocks computed for an earlier
 * configuration remain valid: a Brownian-dynamics caller can refresh the
 * network's blocks (pse_precond_blocks) every k steps and skip the feature
 * pass and the network in between (pse_set_positions then only gathers the
 * blocks into the new sorted order).  Synchronises once.
 * Errors: PARAMS (context without precond = 1), HIP. */
pse_status pse_precond_set_blocks(pse_ctx *ctx, const void *P_dev);

/* Features of the current positions, n x 24 bf16 (device, caller order). */
pse_status pse_precond_features(pse_ctx *ctx, void *feat_dev);

/* The blocks P_i in use, n x 9 fp32 row-major (device, caller order), and
 * the number of fallback blocks (host, may be NULL). */
pse_status pse_precond_blocks(pse_ctx *ctx, void *P_dev, int32_t *fallbacks);

/* Training targets (host, FP64, no GPU): for each caller index idx[q] the
 * symmetric square root of the ii block of M_patch^{-1}, M_patch = M_r
 * restricted to i and the particles within `radius` of it (<= 0: rc),
 * times (mu0 F_self)^{1/2} (an isolated particle gives I); out is m x 9
 * row-major.  pos_host is n x 3 (caller order).  PSE_ERR_NOT_CONVERGED if a
 * patch matrix is not positive definite. */
pse_status pse_precond_targets(const pse_params *params, const double *pos_host, const int32_t *idx, int32_t m,
                               double radius, double *out_host);

/* y = MLP(x): x n x 24 bf16, y n x 9 fp32 (device).  act_cache (device,
 * n x 128 bf16: the hidden activations h1, h2 of each row) may be NULL; the
 * backward pass needs it.  Runs on `stream` (NULL: default stream). */
pse_status pse_mlp_forward(const void *weights_dev, const void *x_dev, int32_t n, void *y_dev, void *act_cache_dev,
                           void *stream);

/* Bytes of device workspace pse_mlp_backward needs for n rows. */
size_t pse_mlp_backward_workspace(int32_t n);

/* dw (device, PSE_MLP_NPARAM fp32) = gradient of sum_rows <dy, y> with
 * respect to every weight, from the forward pass's x and act_cache; padding
 * entries get 0.  The products run on the matrix cores (bf16 MFMA) with
 * the fp32 factors dy and the back-propagated errors split into three bf16
 * parts each, so the gradient has fp32 accuracy.  Deterministic (fixed
 * summation order). */
pse_status pse_mlp_backward(const void *weights_dev, const void *x_dev, const void *act_cache_dev, const void *dy_dev,
                            int32_t n, void *dw_dev, void *workspace_dev, size_t workspace_bytes, void *stream);

/* pse_mlp_backward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation).  The partial gradients go to a fixed
 * device array inside the library instead: 256 slots of PSE_MLP_NPARAM fp32
 * (7.1 MiB), which every GPU the library runs on holds until the process
 * ends.  The pass uses at most 256 slots, so every n >= 1 fits; a count
 * that needed more would be rejected with PSE_ERR_INVALID_ARG.  Allocates
 * nothing.  All calls on one GPU share its array, which keeps the last
 * call's partial sums (each call rewrites every slot entry it reads, so no
 * clearing is needed): calls that overlap on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  dw as in
 * pse_mlp_backward (same kernels, same summation order).
 * Errors: INVALID_ARG (null pointer, n < 1), HIP. */
pse_status pse_mlp_backward_noalloc(const void *weights_dev, const void *x_dev, const void *act_cache_dev,
                                    const void *dy_dev, int32_t n, void *dw_dev, void *stream);

/* Squared-error training loss of the block network and its gradient with
 * respect to the outputs: y_dev, target_dev n x 9 fp32 (device), dy_dev
 * (n x 9, device) = (2/n)(y - target), loss_dev (one fp32 on the device,
 * may be NULL) = sum over rows of |y_p - target_p|^2 / n.  Deterministic
 * (one workgroup, fixed order); no host synchronisation, so a training loop
 * (forward, loss, backward, Adam) stays on the device.
 * Errors: INVALID_ARG (null pointer, n < 1), HIP. */
pse_status pse_mlp_loss_grad(const void *y_dev, const void *target_dev, int32_t n, void *dy_dev, void *loss_dev,
                             void *stream);

/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8, step
 * t >= 1) on the fp32 master weights, with the bf16 copy rewritten. */
pse_status pse_mlp_adam(void *w_master_dev, void *w_bf16_dev, const void *dw_dev, void *m_dev, void *v_dev, float lr,
                        int32_t t, void *stream);

/* ---------------------------------------------------------------------
 * Batches of independent systems (replicas), each with its own parameters
 * and context.  The library spreads the replicas over up to 8 internal
 * streams (default priority) and queues each stream's replicas from its own
 * host thread: the Krylov stopping decision is taken once per stream, not
 * once per replica, and replicas on different streams overlap on the GPU.
 * Calls are ordered after prior work on the caller's stream and later work
 * on that stream waits for them.  Replica r draws its Philox noise with key
 * seed + r (pse_sample's specification otherwise).
 * ------------------------------------------------------------------- */

/* n_rep contexts from params[0 .. n_rep-1]; `stream` is the caller's stream. */
pse_status pse_batch_create(const pse_params *params, int32_t n_rep, void *stream, pse_batch **out);
pse_status pse_batch_destroy(pse_batch *batch);

/* The context of replica r (owned by the batch; for weights, derived
 * parameters or single-replica calls, which run on the replica's stream). */
pse_status pse_batch_replica(pse_batch *batch, int32_t r, pse_ctx **out);

/* pos[r]: device positions of replica r (as pse_set_positions). */
pse_status pse_batch_set_positions(pse_batch *batch, const void *const *pos);

/* One displacement per replica, as pse_sample: forces may be NULL (no
 * forces anywhere) or hold NULL entries; disp[r] device outputs; stats
 * (host, n_rep entries) may be NULL.  Returns the worst status. */
pse_status pse_batch_sample(pse_batch *batch, uint64_t seed, uint64_t counter, double dt, const void *const *forces,
                            void *const *disp, pse_stats *stats);

/* pse_autotune for the batch: the grid shapes are tuned on the first
 * replica of each (grid, support, precision) group (pse_batch_set_positions
 * first) and the others take its choice; the near-field product's lanes per
 * target are tuned on every replica's own positions, and then every replica
 * of one product kernel form (block edge, halo form, Lanczos scalar type)
 * takes the choice of most of the form's particles, so that a captured step
 * runs each form in one launch.  Synchronises every stream. */
pse_status pse_batch_autotune(pse_batch *batch);

/* GPU milliseconds from the start of the last pse_batch_sample to the end
 * of each replica's displacement (host array of n_rep; waits for them). */
pse_status pse_batch_latency(pse_batch *batch, float *ms);

/* A whole batch step captured once into a HIP graph and replayed per step:
 * for every replica, pse_set_positions on pos[r] followed by its sample
 * (Philox noise, key seed + r, counter; dt; forces[r] or none) into
 * disp[r].  The buffers are the caller's device arrays, fixed for the life
 * of the graph (the caller rewrites the positions in place between steps,
 * e.g. by moving the particles by disp).  One replay is one graph launch
 * and one synchronisation for the whole batch, against about 45 launches
 * and two host waits per replica on the eager path.  Inside the graph each
 * stage of the step is one launch for all replicas that share its kernel:
 * binning, neighbour build (block edge, halo form), noise, Krylov start,
 * every Lanczos iteration (product per block edge, halo form and lanes per
 * target; vector kernels and checks for all), wave-space part (grid size,
 * support), combination, final sum and the read-back of every replica's
 * flags and Krylov state, each workgroup finding its replica and block in
 * a table built at capture; with forces, the gather of each replica's
 * forces, its M_r F, its spreading (per grid size and support) and the
 * forward z and y passes join those launches.  Replicas with FP64 storage,
 * the learned preconditioner, more than 65536 particles, or forces on a
 * grid too small for the 8 x 8 x 8 spreading tiles (M < 16 + P, whose
 * spreading adds with atomics and is therefore not bit-reproducible) keep
 * some or all of their own launches inside the same graph.
 *
 * pse_batch_graph_create runs one eager step on the buffers (seed 0,
 * counter 0), then fixes for each replica its block edge, a halo capacity
 * and a neighbour-list capacity `headroom` (e.g. 0.25) above what that step
 * needed, and a Krylov iteration count `extra_iters` above the iterations
 * it needed (the iteration kernels stop themselves once converged), and
 * captures the step.  No host decision and no synchronisation is taken
 * inside a replay: the kernels flag a halo or list that outgrows its
 * capacity (they then skip the work, never write past it), the Krylov
 * state and the flags are copied back, and pse_batch_graph_step, after its
 * one synchronisation, redoes on the eager path every replica whose step
 * overflowed, did not converge within the captured iterations, or met
 * non-finite positions; the next step then captures the batch anew with
 * capacities from the new positions.  The result of every step therefore
 * equals the eager pse_batch_set_positions + pse_batch_sample with the same
 * seed and counter (bit for bit while the block edge stays that of the
 * capture).  stats (n_rep, may be NULL) as pse_batch_sample; *redone (may
 * be NULL) receives the number of replicas redone.  Captured work uses
 * fill kernels, no memset nodes.
 * Errors: INVALID_ARG (null buffers, dt <= 0, extra_iters < 0, headroom
 * < 0), NO_POSITIONS (step without a graph), OOM, HIP, and those of the
 * eager step. */
pse_status pse_batch_graph_create(pse_batch *batch, const void *const *pos_dev, const void *const *forces_dev,
                                  void *const *disp_dev, double dt, int32_t extra_iters, double headroom);
pse_status pse_batch_graph_step(pse_batch *batch, uint64_t seed, uint64_t counter, pse_stats *stats,
                                int32_t *redone);
pse_status pse_batch_graph_destroy(pse_batch *batch);

/* Launch-shape autotuning.  Times, on the context's current positions
 * (pse_set_positions first; PSE_ERR_NO_POSITIONS otherwise), every valid
 * depth D of the owner-computes spreading tiles (D in 8, 16, 32, 64: D
 * divides M and M >= 2 max(8, D) + P; tiles of 8 x 8 x D nodes, or in FP32
 * the matrix-core tiles of 16 x 8 x D where D <= 32, 16 divides M and
 * M >= 2 max(16, D) + P), the interpolation
 * workgroup sizes 256, 512 and 1024 lanes, and 2, 3 and 4 lanes per target
 * particle in the LDS near-field product (FP32 storage), three timed
 * launches each after a warm-up, and keeps the fastest for later calls
 * (the product keeps its built-in 3 lanes unless 2 or 4 is more than 3 %
 * faster).
 * Synchronises the stream; uses the context's scratch only.  choice (host,
 * 3 entries, may be NULL) receives D (0 when the grid is too small for
 * tiles and spreading uses atomics), the interpolation lanes, and the
 * product's lanes per target (0 where the product has no LDS path: FP64,
 * or no LDS block fits).  Results after tuning may differ from those
 * before in the last bits (spreading sums each node's particles in an
 * order that follows the tile's cell scan, and the product splits each
 * row's neighbour chunks over its lanes); they stay deterministic for a
 * given choice. */
pse_status pse_autotune(pse_ctx *ctx, int32_t *choice);

/* Applies a launch-shape choice without timing (one from pse_autotune,
 * kept from an earlier run, or a fixed one): choice (host, 3 entries) holds
 * the spreading tile depth, the interpolation lanes and the product's lanes
 * per target as pse_autotune reports them, with 0 for the built-in choice
 * of an entry.  PSE_ERR_INVALID_ARG (and nothing changed) when the tile
 * depth is not valid for the grid (see pse_autotune), the interpolation
 * lanes are not 256, 512 or 1024, or the product lanes are not 2, 3 or 4.
 * Takes effect for later calls on the context; no synchronisation. */
pse_status pse_set_launch_shape(pse_ctx *ctx, const int32_t *choice);

/* GPU-time accounting: for every stage whose bit (1 << pse_stage) is set in
 * stage_mask, each kernel launch of that stage is bracketed by HIP events on
 * the context stream.  0 switches accounting off.  Events are recorded only
 * for selected stages, so unselected stages run exactly as without it. */
pse_status pse_profile(pse_ctx *ctx, uint32_t stage_mask);

/* Elapsed GPU milliseconds and launch counts per stage since the last read
 * (arrays of PSE_NSTAGES entries, host memory).  Synchronises the stream and
 * resets the accumulators. */
pse_status pse_profile_read(pse_ctx *ctx, double *ms, int32_t *launches);

#ifdef __cplusplus
}
#endif
#endif
