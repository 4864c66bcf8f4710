/*
 * priest.h - C ABI of the MI355X (gfx950) PRIEST planner library, libpriest.so.
 *
 * PRIEST (Rastgar et al., "PRIEST: Projection Guided Sampling-Based
 * Optimization For Autonomous Navigation") plans a trajectory by sampling
 * polynomial coefficient vectors xi from a Gaussian, pushing every sample
 * toward the feasible set with a batched projection optimizer, and refitting
 * the Gaussian to the lowest-cost projected samples (Alg. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers (HIP global memory) unless a comment
 *    says "host".  The caller allocates and owns them; the library owns only
 *    the opaque problem handle and what it allocates inside it.
 *  - Every call that takes a `stream` (a hipStream_t passed as void*, NULL =
 *    the default stream) is asynchronous on that stream: outputs are valid
 *    once the caller synchronises it.  priest_init_problem synchronises once.
 *  - float32 arrays, row-major.  A sample xi has D = dims * n_coeff entries
 *    laid out [dims][n_coeff]: the coefficients of x(t), then y(t), then z(t)
 *    (Sec. II-A, compact form below eq. (3)).
 *  - Scenes:
 *      bc  [dims][6]  per axis (p0, v0, a0, pf, vf, af): boundary values of
 *                     position, velocity, acceleration at t0 and tf
 *                     (eq. (1b)); rows not selected by bc_mask are ignored.
 *      obs [n_obs][8] (cx, cy, cz, vx, vy, vz, a, b): obstacle centre at t=0,
 *                     constant velocity, semi-axes (a, a, b) of eq. (1e);
 *                     in 2D cz, vz and b are ignored (circles of radius a).
 *                     With obs_model PRIEST_OBS_PATH the rows are
 *                     [n_obs][K * dims + 2] instead (positions per step, a, b).
 *  - Return value: PRIEST_OK or a negative status; no exception or abort
 *    crosses the ABI.  priest_last_error() returns a thread-local message
 *    describing the last failure on the calling thread.
 *  - Input validation happens on the host before anything is launched: on
 *    error nothing has been enqueued and outputs are untouched.
 */
#ifndef PRIEST_H_
#define PRIEST_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRIEST_OK 0
#define PRIEST_ERR_INVALID (-1)   /* bad sizes, null required pointer, non-finite scalar */
#define PRIEST_ERR_SINGULAR (-2)  /* boundary rows rank-deficient: KKT matrix singular */
#define PRIEST_ERR_NOMEM (-3)     /* device allocation failed / workspace too small / admission refused */
#define PRIEST_ERR_DEVICE (-4)    /* a HIP runtime call failed */
#define PRIEST_ERR_NONFINITE (-5) /* NaN/Inf met on the device (reported through a status word) */

/* Boundary rows (eq. (3b)): bit i selects row i of
 * [P_0; Pdot_0; Pddot_0; P_-1; Pdot_-1; Pddot_-1] for every axis. */
#define PRIEST_BC_P0 1u
#define PRIEST_BC_V0 2u
#define PRIEST_BC_A0 4u
#define PRIEST_BC_PF 8u
#define PRIEST_BC_VF 16u
#define PRIEST_BC_AF 32u
/* The four rows of the paper's block of A. */
#define PRIEST_BC_DEFAULT (PRIEST_BC_P0 | PRIEST_BC_V0 | PRIEST_BC_A0 | PRIEST_BC_PF)

/* Obstacle models (layout of the obs rows). */
#define PRIEST_OBS_VELOCITY 0 /* obs [n_obs][8]: centre at t = 0, constant velocity, a, b */
#define PRIEST_OBS_PATH 1     /* obs [n_obs][K * dims + 2]: the obstacle's position at every
                                 planning step t_k (x, y[, z] per step), then a, b: the
                                 stacked obstacle positions of eq. (13) given directly.
                                 Projections of such problems use the default tile shape;
                                 the unfused form and the server do not take them. */

#define PRIEST_FP32 0        /* every product in FP32 */
#define PRIEST_BF16_MIXED 1  /* BF16 operands for the right-hand-side assembly F^T(e - F xi),
                                FP32 accumulation, last n_refine_fp32 iterations in FP32 */

#define PRIEST_MAX_COEFF 16
#define PRIEST_MAX_STEPS 256
#define PRIEST_MAX_OBS 1024
#define PRIEST_MAX_SAMPLES 65536

typedef struct priest_problem priest_problem; /* opaque, owned by the library */

/* Shape of a planning problem (Sec. II-A eqs. (1)-(3); Appendix eq. (12)). */
typedef struct priest_problem_desc {
  int32_t dims;          /* 2 or 3 */
  int32_t n_coeff;       /* coefficients per axis, 2..16 (polynomial degree n_coeff-1) */
  int32_t n_steps;       /* planning steps K on t_k = k T/(K-1), 2..256 */
  int32_t n_obs;         /* exact obstacle count (enters I + rho F^T F), 0..1024 */
  double horizon;        /* T > 0, seconds */
  double rho;            /* augmented-Lagrangian weight rho >= 0 (eq. (14)) */
  double v_max;          /* > 0; +inf disables the velocity bound (eq. (1c)) */
  double a_max;          /* > 0; +inf disables the acceleration bound */
  uint32_t bc_mask;      /* PRIEST_BC_* rows; at most n_coeff rows, full rank */
  int32_t precision;     /* PRIEST_FP32 or PRIEST_BF16_MIXED */
  int32_t n_refine_fp32; /* PRIEST_BF16_MIXED: trailing iterations run in FP32 */
  int32_t use_bounds;    /* 0 or 1: workspace bounds s_min <= p(t_k) <= s_max per axis
                            (Appendix, G xi <= tau with G = [-P; P]); their rows enter
                            I + rho F^T F, so they are part of the problem */
  double s_min[3];       /* use_bounds: lower limits per axis (-inf allowed), <= s_max */
  double s_max[3];       /* use_bounds: upper limits per axis (+inf allowed) */
  int32_t obs_model;     /* PRIEST_OBS_VELOCITY or PRIEST_OBS_PATH: layout of obs rows */
  int32_t reserved2;     /* must be 0 */
} priest_problem_desc;

/* Trajectory cost c1 of Alg. 1 (the remark of Sec. II that c1 need not be
 * convex, smooth or analytic; the navigation and steering costs of Sec. V).
 * kind PRIEST_COST_SMOOTH: c1 = sum_k ||a_k||^2 (the point-to-point cost; the
 * weights are ignored).  kind PRIEST_COST_WEIGHTED: c1 = sum_k of
 *   w_acc   ||a_k||^2
 * + w_curv  kappa_k^2,  kappa = |v x a| / (||v||^2 + eps)^(3/2)
 * + w_path  distance of p_k to the segment from p0 to pf of bc (projection
 *           onto the line clamped to the segment; not squared)
 * + w_steer atan(wheelbase * kappa_signed)^2 (2D only: steering angle of a
 *           car-like robot by differential flatness, kappa_signed =
 *           (v_x a_y - v_y a_x) / (||v||^2 + eps)^(3/2)).
 * Weights finite and >= 0; eps > 0; wheelbase > 0 when w_steer > 0. */
#define PRIEST_UPDATE_MPPI 0
#define PRIEST_UPDATE_CMA 1
#define PRIEST_COST_SMOOTH 0
#define PRIEST_COST_WEIGHTED 1
typedef struct priest_cost {
  int32_t kind;
  float w_acc, w_curv, w_path, w_steer;
  float wheelbase;
  float eps;
  int32_t reserved;  /* must be 0 */
} priest_cost;

/* Sampling-loop settings (Alg. 1, eqs. (9a)-(9c)).  A zero-initialised cost
 * is the smoothness cost. */
typedef struct priest_cem_params {
  int32_t n_samples;    /* N_b: samples per CEM iteration, 1..8192 (the selection kernel
                           holds a problem's samples in one block; PRIEST_MAX_SAMPLES
                           bounds the projection calls only) */
  int32_t n_cem;        /* CEM iterations */
  int32_t n_proj_iters; /* projection iterations per CEM iteration */
  int32_t n_proj;       /* N_proj: size of the lowest-residual set, 1..n_samples */
  int32_t n_elite;      /* N_elite: size of the elite set, 1..n_proj */
  int32_t update;       /* PRIEST_UPDATE_MPPI: eqs. (9a)-(9c); PRIEST_UPDATE_CMA: eq. (9a)
                           for the mean and a CMA-ES-style covariance update in place of
                           eq. (9b) (the remark that Alg. 1 is agnostic to the rule):
                           weights w = c_m / sum c_m of eq. (9c), mu_eff = 1 / sum w^2,
                           y_m = xi_bar_m - mu, y_w = sum w y,
                           p_c' = (1 - c_c) p_c + sqrt(c_c (2 - c_c) mu_eff) y_w,
                           Sigma' = (1 - c_1 - c_mu) Sigma + c_1 p_c' p_c'^T
                                    + c_mu sum w y y^T,
                           c_c, c_1, c_mu at the CMA-ES defaults for n = D; the path
                           p_c starts at zero on every plan call (it lives in the
                           workspace); no step-size adaptation */
  float sigma;          /* learning rate of eqs. (9a)/(9b), in [0, 1] */
  float gamma;          /* temperature of eq. (9c), > 0 */
  float cov_jitter;     /* eps = cov_jitter * tr(Sigma)/D added before Cholesky, >= 0 */
  float reserved_f;     /* must be 0 */
  priest_cost cost;     /* c1 (computed in the projection's final pass) */
} priest_cem_params;

/* Outputs of priest_plan; every pointer but best_xi/best_cost may be NULL.
 * Per-sample outputs describe the LAST CEM iteration. */
typedef struct priest_plan_out {
  float* best_xi;      /* [D]: projected sample with the lowest c_aug of the final elite set */
  float* best_cost;    /* [1]: its c_aug = c1 + r */
  int32_t* elite_idx;  /* [n_elite]: elite sample indices, ascending c_aug */
  int32_t* proj_idx;   /* [n_proj]: lowest-residual sample indices, ascending r */
  float* xi;           /* [N][D]: the drawn samples */
  float* xi_bar;       /* [N][D]: projected samples */
  float* resid;        /* [N]: r = ||F xi_bar - e(xi_bar)|| */
  float* c1;           /* [N]: smoothness cost sum_k ||a_k||^2 */
  int32_t* status;     /* [1]: PRIEST_OK, or PRIEST_ERR_NONFINITE if a covariance factorisation failed */
} priest_plan_out;

/* Builds the problem: Bernstein basis P, Pdot, Pddot (eq. (2)), boundary block
 * A (eq. (3b)), and the fixed KKT inverse of eq. (7b), factored once in FP64
 * on the GPU (Sec. III-A, "Scalability": M is computed only once).
 * `out` receives a handle to free with priest_free_problem.  Synchronises
 * `stream`.  Errors: INVALID (bad desc), SINGULAR (rank-deficient boundary
 * rows), NOMEM, DEVICE. */
int32_t priest_init_problem(const priest_problem_desc* desc, void* stream, priest_problem** out);

/* Releases a problem handle (NULL is accepted).  The caller must make sure no
 * work using it is still running. */
int32_t priest_free_problem(priest_problem* p);

/* Number of coefficients per sample, D = dims * n_coeff (host call). */
int32_t priest_problem_dim(const priest_problem* p);

/* Projection optimizer (Sec. III-A eqs. (4)-(7); Appendix eqs. (14)-(15)):
 * pushes each of the N samples xi_in [N][D] toward the feasible set with
 * n_iter alternating-minimisation iterations, starting from xi_bar = xi,
 * lambda = 0.  Writes xi_out [N][D].  resid [N] (r of Alg. 1) and c1 [N]
 * (smoothness cost) of the returned iterate may be NULL.  bc/obs: one scene
 * (layouts above).  xi_in and xi_out may alias.  Errors: INVALID. */
int32_t priest_project(priest_problem* p, const float* bc, const float* obs,
                       const float* xi_in, int32_t N, int32_t n_iter,
                       float* xi_out, float* resid, float* c1, void* stream);

/* priest_project for n_problems problems of the same shape in one launch:
 * bc [P][dims][6], obs [P][n_obs][row] (row 8, or K * dims + 2 for paths),
 * xi_in / xi_out [P][N][D], resid / c1 [P][N] (nullable).  Problem q's
 * samples see only problem q's scene.  Tile shape as priest_project (the
 * first call with a new (N, P) tunes it).  xi_in and xi_out may alias.
 * Errors as priest_project. */
int32_t priest_project_batch(priest_problem* p, int32_t n_problems, const float* bc,
                             const float* obs, const float* xi_in, int32_t N, int32_t n_iter,
                             float* xi_out, float* resid, float* c1, void* stream);

/* priest_project with the residual history of Alg. 1's projection: resid_hist
 * [n_iter][N] receives, for every iteration k and sample i, the norm
 * ||F xi_bar^k - e^{k+1}||_2 of the push-outs that iteration computes from
 * its iterate (Appendix eqs. (15a)-(15f)), i.e. the residual of xi_bar^k;
 * resid (nullable) is that of the returned iterate as in priest_project.
 * Runs the default tile shape (no autotuning); xi_out equals priest_project's
 * output under that shape bit for bit.  Errors as priest_project, and
 * INVALID when resid_hist is NULL. */
int32_t priest_project_hist(priest_problem* p, const float* bc, const float* obs,
                            const float* xi_in, int32_t N, int32_t n_iter, float* xi_out,
                            float* resid, float* c1, float* resid_hist, void* stream);

/* The same projection as priest_project in its plain, unfused form, kept as
 * the baseline the fused kernel is measured against: per iteration three
 * kernels - forward rows p, v, a of every (sample, t) to HBM; closed-form
 * push-outs of every (sample, t) against every obstacle (eqs. (15a)-(15c)) to
 * HBM; g = F^T(e - F xi_bar), the multiplier update and the KKT step per
 * (sample, axis) - then a final forward + push-out pass for r and c1.  No
 * MFMA, no obstacle culling, FP32 only.  Results match priest_project within
 * FP32 rounding (not bit for bit: the sums run in another order).
 * workspace: device buffer of priest_project_unfused_workspace_size bytes
 * (about 2 * N * K * 3 * dims floats).  Errors: INVALID (also for a problem
 * built with PRIEST_BF16_MIXED), NOMEM (workspace too small). */
int32_t priest_project_unfused_workspace_size(const priest_problem* p, int32_t N, size_t* bytes);
int32_t priest_project_unfused(priest_problem* p, const float* bc, const float* obs,
                               const float* xi_in, int32_t N, int32_t n_iter, float* xi_out,
                               float* resid, float* c1, void* workspace, size_t workspace_bytes,
                               void* stream);

/* Bytes of device workspace priest_plan / priest_plan_batch need for
 * n_problems problems with settings `c` (host call): per problem the
 * projected samples, residuals, costs, Cholesky factor, CMA path, status and
 * 48 bytes per obstacle of precomputed obstacle records. */
int32_t priest_plan_workspace_size(const priest_problem* p, const priest_cem_params* c,
                                   int32_t n_problems, size_t* bytes);

/* Alg. 1 for one problem: n_cem iterations of
 *   draw N samples from N(mu, Sigma) -> project -> residual r -> N_proj
 *   lowest r -> c_aug = c1 + r -> N_elite lowest c_aug -> refit (eqs. (9a)-(9c)).
 * mu [D] and cov [D][D] are read and overwritten with the refitted
 * distribution (the warm start of the next call).
 * Draws: if `noise` ([n_cem][N][D] standard normals) is non-NULL it is used;
 * otherwise Philox4x32-10 with key `seed`, counter (sample, d/4, iteration,
 * stream_id), followed by Box-Muller.
 * workspace: device buffer of at least priest_plan_workspace_size bytes.
 * Errors: INVALID, NOMEM (workspace too small). */
int32_t priest_plan(priest_problem* p, const float* bc, const float* obs,
                    const priest_cem_params* c, float* mu, float* cov,
                    uint64_t seed, uint32_t stream_id, const float* noise,
                    const priest_plan_out* out, void* workspace, size_t workspace_bytes,
                    void* stream);

/* priest_plan for callers that cannot allocate device memory - code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc:
 * the same plan, on the same kernels, with its workspace taken from a static
 * device array of the library (PRIEST_STATIC_WORKSPACE_BYTES per GPU, held
 * until the process ends) instead of a caller buffer.  It calls no
 * hipMalloc / hipFree and never synchronises: no autotuning (the tile shape
 * is a forced or already tuned one for this shape, else the default, so the
 * result equals priest_plan's bit for bit), no profiling events or pair
 * counting.  Every call on one GPU shares that GPU's array and leaves the
 * last call's contents in it: calls that overlap on one GPU (on different
 * streams, or from several host threads) race and must be serialised by the
 * caller.  Arguments and outputs as priest_plan.  Errors: INVALID, NOMEM
 * (the plan needs more than PRIEST_STATIC_WORKSPACE_BYTES, which no plan of
 * n_samples <= 8192 and D <= 48 does), DEVICE (the array's address could not
 * be looked up on this device when the problem was built). */
#define PRIEST_STATIC_WORKSPACE_BYTES (2u << 20)
int32_t priest_plan_static(priest_problem* p, const float* bc, const float* obs,
                           const priest_cem_params* c, float* mu, float* cov,
                           uint64_t seed, uint32_t stream_id, const float* noise,
                           const priest_plan_out* out, void* stream);

/* Alg. 1 for n_problems independent problems of the same shape, every CEM
 * step batched over all problems in one launch (the 3D batched workload).
 * Arrays are stacked per problem: bc [P][dims][6], obs [P][n_obs][8],
 * mu [P][D], cov [P][D][D], noise [P][n_cem][N][D] (nullable),
 * out->best_xi [P][D], best_cost [P], elite_idx [P][n_elite], proj_idx [P][n_proj],
 * xi / xi_bar [P][N][D], resid / c1 [P][N], status [P].
 * Problem q draws with stream id stream_base + q.
 * use_graph != 0 captures the whole CEM loop into a hipGraph the first time
 * a given argument set is seen and replays it afterwards.  Errors as priest_plan. */
int32_t priest_plan_batch(priest_problem* p, int32_t n_problems, const float* bc,
                          const float* obs, const priest_cem_params* c, float* mu,
                          float* cov, uint64_t seed, uint32_t stream_base,
                          const float* noise, const priest_plan_out* out, void* workspace,
                          size_t workspace_bytes, int32_t use_graph, void* stream);

/* ------------------------------------------------------------------------
 * Tile shape of the projection kernel
 *
 * The same projection can be laid out on the GPU in several ways: 4 MFMA
 * columns per sample (4 samples per block) or, in 2D, 2 columns per sample
 * (8 samples per block, two items per lane); one or two 16-step time blocks
 * per wave, or every time block of the horizon in one wave (blocks of 16
 * waves, each with its own samples); one block per tile or a persistent grid
 * of resident blocks that loop over tiles (for the whole-horizon shape: one
 * group of samples per wave, or groups that the waves draw from a counter, so
 * that waves whose samples need fewer evaluations take more of them - four
 * per wave from a counter per block, or, in the plan calls, whose workspace
 * then also holds the obstacle records of every problem, from one counter
 * over all (problem, group) pairs of the launch for a grid of resident
 * blocks).  Every shape gives bit-identical results.  By default the
 * library times every candidate the first time a problem handle meets a new
 * (N, n_problems, sampling mode, precision) - one warm-up and two timed
 * launches of a shortened (<= 8 iteration) copy of the real launch, outputs
 * redirected to scratch - and keeps the fastest.  That first call
 * synchronises the stream (and priest_project allocates N*(D+2) floats of
 * scratch for it).  No tuning happens while the stream is being captured
 * into a graph, or with PRIEST_AUTOTUNE=0 in the environment: the default
 * shape (4, 1, 0) is used.
 * ------------------------------------------------------------------------ */
typedef struct priest_tiling {
  int32_t axis_slots; /* MFMA columns per sample: 4; 2 (2D only); or 8 (two samples per
                         block, half the lanes idle in the push-out: more blocks for small N) */
  int32_t row_tiles;  /* 16-step time blocks per wave: 1 or 2 (8 axis slots: 1 only); or 0:
                         each wave carries its samples over the whole horizon (4 axis slots,
                         or 2 in 2D; n_steps <= 128), no block barrier per iteration: for
                         batches large enough to fill the chip */
  int32_t persistent; /* 1: grid of resident blocks looping over tiles; with row_tiles 0:
                         sample groups drawn by the waves from a counter (4 per wave and
                         block; in the plan calls one counter for the whole launch), one
                         group per wave with 0 */
  int32_t reserved;   /* must be 0 */
} priest_tiling;

/* Candidate shapes for p (host call): writes up to max_out of them, n
 * receives the total.  Entry 0 is the default shape. */
int32_t priest_tiling_candidates(const priest_problem* p, priest_tiling* out, int32_t max_out,
                                 int32_t* n);

/* Forces every later projection launch of p to use *t; NULL returns to
 * autotuning.  Errors: INVALID (not a candidate for p). */
int32_t priest_set_tiling(priest_problem* p, const priest_tiling* t);

/* Shape used by p's most recent projection launch; `tuned` (nullable)
 * receives 1 if it came from the autotuner. */
int32_t priest_last_tiling(const priest_problem* p, priest_tiling* out, int32_t* tuned);

/* Profiling hook.  While enabled (process-wide), every projection launch made
 * by priest_project / priest_plan / priest_plan_batch outside graph capture
 * is bracketed by two HIP events on its stream.  priest_profile_read waits
 * for the events recorded since the previous read and returns their count
 * and summed duration in milliseconds (host pointers).  Meant for
 * benchmarks: kernel time measured inside the timed region. */
int32_t priest_profile_enable(int32_t on);
int32_t priest_profile_read(int32_t* n_launches, double* total_ms);

/* Work counter of the same launches.  While on (process-wide, first enabled
 * on the current device, which it stays bound to), every fused projection
 * launch made outside graph capture adds to one device counter the number
 * of (sample, time step, obstacle) pairs whose push-out it evaluated, over
 * all its iterations and the final residual pass; pairs skipped by the
 * obstacle culling (whose push-out is exactly zero) are not counted.
 * Enabling zeroes the counter.  priest_profile_read_pairs synchronises the
 * device, returns the count since the last read or enable (host pointer)
 * and zeroes it.  Errors: INVALID, DEVICE. */
int32_t priest_profile_count_pairs(int32_t on);
int32_t priest_profile_read_pairs(uint64_t* pairs);

/* D-PRIEST (Sec. III-C): n_groups Gaussians (mu [G][D], cov [G][D][D], read
 * and overwritten like priest_plan) each draw c->n_samples samples on ONE
 * scene (bc [dims][6], obs [n_obs][8] shared by all groups).  Every CEM
 * iteration projects the samples of all groups in one launch, then each
 * group selects and refits on its own samples; after n_cem iterations the
 * group whose final best trajectory has the lowest c_aug is picked.
 * out: per-group outputs stacked as for priest_plan_batch (out->best_xi
 * [G][D] and out->best_cost [G] required).  best_xi [D], best_cost [1] and
 * best_group [1] receive the pick (ties: lowest group index; NaN ranks last).
 * Group g draws stream stream_base + g; noise [G][n_cem][N][D] nullable.
 * workspace: priest_plan_workspace_size(p, c, n_groups) bytes.
 * Errors as priest_plan. */
int32_t priest_plan_dpriest(priest_problem* p, int32_t n_groups, const float* bc,
                            const float* obs, const priest_cem_params* c, float* mu, float* cov,
                            uint64_t seed, uint32_t stream_base, const float* noise,
                            const priest_plan_out* out, float* best_xi, float* best_cost,
                            int32_t* best_group, void* workspace, size_t workspace_bytes,
                            void* stream);

/* Debug/parity hook for the closed-form alpha/beta/d step (Appendix eqs.
 * (15a)-(15c), (13)): for samples xi [N][D] writes the per-row push-outs
 * e(xi) - F xi, laid out [N][n_obs + 2][K][dims] (obstacle blocks, then the
 * velocity block, then the acceleration block).  The push-outs rather than
 * alpha, beta, d themselves are returned because the kernels never form the
 * angles: each target of eq. (13) is the obstacle (or origin) plus the
 * scaled direction (cos a sin b, sin a sin b, cos b) d, so alpha, beta and d
 * are the polar coordinates of (push-out + F xi - o) in the obstacle's
 * scaled frame, and comparing push-outs checks all three at once.  Meant for
 * small N (<= 4096). */
int32_t priest_debug_offsets(priest_problem* p, const float* bc, const float* obs,
                             const float* xi, int32_t N, float* offsets, void* stream);

/* Debug/parity hook for the draws: writes z [N][D] standard normals of CEM
 * iteration `iter` for (seed, stream_id), exactly as priest_plan draws them. */
int32_t priest_debug_normals(uint64_t seed, uint32_t stream_id, int32_t iter, int32_t N,
                             int32_t D, float* z, void* stream);

/* Debug/parity hook for the two selections of Alg. 1 (ConstraintEliteSet,
 * then EliteSet), as the refit kernel makes them: from r [N] and c1 [N]
 * (device), writes elite_idx [n_elite] (device), the n_elite lowest
 * c_aug = c1 + r (FP32 sum) among the n_proj lowest r, ascending c_aug with
 * ties in the order of the first selection (ascending r, then index).  With
 * proj_idx non-NULL it also writes that first selection [n_proj] (device),
 * ascending r, and takes the sorting path; with NULL it takes the path the
 * plan takes in its other iterations (radix selects where N <= 2048 and
 * n_elite <= 512).  Requires 1 <= n_elite <= n_proj <= N <= 8192.
 * Allocates and frees scratch; synchronises `stream`. */
int32_t priest_debug_select(int32_t N, int32_t n_proj, int32_t n_elite, const float* r,
                            const float* c1, int32_t* elite_idx, int32_t* proj_idx, void* stream);

/* Copies the problem's FP32 constants to host memory for inspection:
 * which = 0: KKT block M11 [n_coeff][n_coeff]; 1: Pi = M11 Q [n_coeff][n_coeff];
 * 2: M12 [n_coeff][6] (column i multiplies boundary value i of an axis);
 * 3: basis rows [K][3][n_coeff] (P, Pdot, Pddot).  `host_out` must hold
 * `count` floats (host).  Synchronous. */
int32_t priest_debug_constants(const priest_problem* p, int32_t which, float* host_out,
                               int32_t count);

/* ------------------------------------------------------------------------
 * Continuous-batching server (the serving form of Alg. 1)
 *
 * Planning requests of different sizes (n_samples, n_obs, n_steps) from many
 * robots arrive at any time.  Each priest_server_step advances every active
 * request by ONE iteration of Alg. 1 - draw, project (eqs. (4)-(7)), select,
 * refit (eqs. (9a)-(9c)) - with one projection launch per distinct n_steps
 * and one selection/refit launch for all requests, every request on blocks
 * of its own.  A pending request is admitted at a step boundary when a slot
 * is free, its robot has no request in flight, and its device state fits the
 * memory budget (first-fit); it leaves after n_cem iterations.  Each robot's
 * sampling distribution (mu, Sigma) stays on the device between its requests
 * (the warm start of the next plan).  Draws use Philox4x32-10 with key
 * config.seed and counter (sample, d/4, CEM iteration, request.stream_id), so
 * a request's result does not depend on which other requests share its steps.
 *
 * Threading: a server is used from one host thread at a time.  All device
 * work is enqueued on the stream given at creation.
 * ------------------------------------------------------------------------ */
typedef struct priest_server priest_server; /* opaque */

typedef struct priest_server_config {
  int32_t dims;               /* 2 or 3 */
  int32_t n_coeff;            /* coefficients per axis, 2..16 */
  uint32_t bc_mask;           /* PRIEST_BC_* rows of every request */
  int32_t precision;          /* PRIEST_FP32 or PRIEST_BF16_MIXED */
  int32_t n_refine_fp32;      /* see priest_problem_desc */
  int32_t max_active;         /* requests advanced together, 1..8192 */
  int32_t max_robots;         /* robot ids are 0..max_robots-1, 1..65536 */
  int32_t max_inflight_steps; /* steps the device may run behind the host, 1 or 2 */
  int32_t dry_run;            /* 1: admission bookkeeping only, no device call (host tests) */
  int32_t reserved;           /* must be 0 */
  double rho, v_max, a_max;   /* as in priest_problem_desc */
  uint64_t seed;              /* Philox key of every draw */
  uint64_t memory_budget;     /* bytes of device memory for per-request state, >= 4096 */
  float sigma, gamma, cov_jitter; /* as in priest_cem_params */
  float init_std;             /* a reset covariance is init_std^2 I, > 0 */
} priest_server_config;

#define PRIEST_WARM_RESET 0     /* mu = straight line start -> goal, Sigma = init_std^2 I */
#define PRIEST_WARM_KEEP 1      /* keep the robot's mu and Sigma (reset if it has none yet) */
#define PRIEST_WARM_KEEP_MEAN 2 /* keep mu, reset Sigma */

typedef struct priest_request {
  int32_t robot;        /* 0..max_robots-1 */
  int32_t n_steps;      /* 2..256 */
  int32_t n_obs;        /* 0..1024 */
  int32_t n_samples;    /* 1..8192 */
  int32_t n_cem;        /* >= 1 */
  int32_t n_proj_iters; /* >= 0 */
  int32_t n_proj;       /* 1..n_samples */
  int32_t n_elite;      /* 1..n_proj */
  int32_t warm_start;   /* PRIEST_WARM_* */
  uint32_t stream_id;   /* Philox stream of this request's draws */
  double horizon;       /* T > 0 */
  double arrival;       /* caller's timestamp (priest_server_now clock), echoed back */
  const float* bc;      /* HOST [dims][6], copied at submit */
  const float* obs;     /* HOST [n_obs][8], copied at submit */
} priest_request;

typedef struct priest_result {
  int64_t request_id;
  int32_t robot;
  int32_t status;       /* PRIEST_OK or PRIEST_ERR_NONFINITE */
  double arrival;       /* as submitted */
  double t_admit;       /* host clock at admission */
  double t_done;        /* host clock when the completion was observed */
  float best_cost;      /* c_aug of best_xi */
  float best_xi[3 * PRIEST_MAX_COEFF]; /* first D entries valid */
} priest_result;

typedef struct priest_server_stats {
  int64_t submitted, admitted, completed, steps;
  int64_t max_active_seen;
  int64_t arena_used, arena_budget, arena_high_water; /* bytes */
  int64_t sample_iters; /* sum of n_samples * n_proj_iters * n_cem over completed requests */
} priest_server_stats;

/* Host clock in seconds (monotonic) used for the timestamps above. */
double priest_server_now(void);

/* Creates a server: allocates the request arena (memory_budget bytes), the
 * per-robot store (max_robots * (D + D*D) floats) and pinned staging.
 * Errors: INVALID, NOMEM, DEVICE. */
int32_t priest_server_create(const priest_server_config* cfg, void* stream, priest_server** out);

/* Builds (and caches) the problem constants for one (n_steps, n_obs, horizon)
 * ahead of time; otherwise they are built at the first admission of that
 * shape, which synchronises the stream.  No-op in dry-run mode. */
int32_t priest_server_prepare(priest_server* s, int32_t n_steps, int32_t n_obs, double horizon);

/* Queues a request (FIFO).  `id` receives its id (> 0).  Errors: INVALID
 * (bad sizes, non-finite scene values, unknown robot), NOMEM (state larger
 * than the whole budget). */
int32_t priest_server_submit(priest_server* s, const priest_request* r, int64_t* id);

/* Observes finished steps, admits pending requests, and enqueues one CEM
 * iteration of every active request.  Blocks only while max_inflight_steps
 * steps are already running.  n_active (nullable) receives the number of
 * requests in the enqueued step (0: nothing enqueued). */
int32_t priest_server_step(priest_server* s, int32_t* n_active);

/* Moves up to max_results finished requests to `out` (host), oldest first;
 * n receives the count.  Non-blocking. */
int32_t priest_server_poll(priest_server* s, priest_result* out, int32_t max_results, int32_t* n);

/* Waits until every enqueued step has finished on the device. */
int32_t priest_server_flush(priest_server* s);

/* Numbers of queued, active (advanced by the next step) and in-flight steps
 * (any pointer may be NULL). */
int32_t priest_server_counts(const priest_server* s, int32_t* pending, int32_t* active,
                             int32_t* inflight_steps);

int32_t priest_server_stats_get(const priest_server* s, priest_server_stats* out);

/* Copies a robot's current mu [D] and Sigma [D][D] to host memory after
 * waiting for the enqueued work.  Errors: INVALID (robot has no state). */
int32_t priest_server_robot_state(priest_server* s, int32_t robot, float* host_mu,
                                  float* host_cov);

/* Waits for the device, releases everything (NULL accepted).  Requests not
 * yet polled are dropped. */
int32_t priest_server_destroy(priest_server* s);

/* Message of the last failure on this thread ("" if none). */
const char* priest_last_error(void);

/* Library ABI version (increments on incompatible change). */
int32_t priest_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PRIEST_H_ */
