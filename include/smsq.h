/*
 * smsq.h -- C ABI of the MI355X (gfx950) Stein-MAP-Seq hot path.
 *
 * Stein-MAP-Seq (Seo & Kia, arXiv 2312.08684) estimates the MAP state
 * trajectory of a state-space model x_t ~ p(x_t | x_{t-1}),
 * z_t ~ p(z_t | x_t) (Sec. II, eq. SSM) from observations z_{1:T} and a known
 * initial state x_0.  At every step it moves N particles with Stein
 * variational gradient descent toward p(z_t, x_t | x_{t-1}) (Lemma IV.3, eq.
 * SVGD_newupdate), then runs one step of a Viterbi max-plus recursion over the
 * particle lattice (eq. forward_recursion); a final backtrack returns the MAP
 * sequence (Sec. IV-B, Algorithm 2).
 *
 * Conventions for every entry point below:
 *  - Array arguments are DEVICE pointers owned by the caller, row-major and
 *    C-contiguous, in the element type named by the smsq_dtype_t argument
 *    (float for SMSQ_F32, double for SMSQ_F64); index arrays are int32_t,
 *    masks and flags uint8_t.  Host-side arguments are marked (host).
 *  - Calls enqueue work on `stream` and return without waiting.  Argument
 *    errors are returned synchronously and enqueue nothing.  Results of the
 *    enqueued work (including non-finite detection) are read after the
 *    stream is synchronised.
 *  - The library never frees caller memory and never allocates device
 *    memory inside a step call.  Scratch memory is the caller's workspace
 *    `ws` of `ws_bytes` bytes (query its size with smsq_workspace_size and
 *    zero it once after allocation).  The first 256 bytes of a workspace
 *    hold a device status word (see smsq_get_device_status); a workspace may
 *    not be used by two calls that run at the same time.
 *  - Model handles are immutable after creation and may be shared across
 *    streams.
 *  - No exception crosses the ABI.
 */
#ifndef SMSQ_H
#define SMSQ_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMSQ_OK = 0,
    SMSQ_ERR_INVALID = 1,      /* bad argument: null pointer, size <= 0, mismatched d, ... */
    SMSQ_ERR_UNSUPPORTED = 2,  /* shape outside what the kernels handle (e.g. LDS capacity) */
    SMSQ_ERR_HIP = 3,          /* a HIP runtime call failed */
    SMSQ_ERR_NONFINITE = 4,    /* device saw NaN/Inf in particles, scores or path scores */
    SMSQ_ERR_WORKSPACE = 5     /* workspace missing or smaller than smsq_workspace_size */
} smsq_status_t;

typedef enum { SMSQ_F32 = 0, SMSQ_F64 = 1 } smsq_dtype_t;

/* Model families (the paper's scenario shapes, Sec. V, plus a
 * linear-Gaussian model).  Every family has a Gaussian transition
 * x_t ~ N(f_t(x_{t-1}), diag(q_var)); `params` layout per family:
 *   GROWTH1D  d=1, obs_dim=n_obs=1.  f_t(x)=p0 x + p1 x/(1+x^2) + p2 cos(p3 t + p4);
 *             z = p5 x^2 + N(0, p6).
 *   RANGE2D   d=2, obs_dim=n_obs=nb<=16.  f(x)=x; z_b = |x - beacon_b| + N(0, p0);
 *             p1 = nb, beacon b at (p[2+2b], p[3+2b]); mask[b]=0 hides beacon b.
 *   CV4D      d=4 (px,py,vx,vy), n_obs=M<=16 detections, obs_dim=2M.
 *             f(x)=(px+p0 vx, py+p0 vy, vx, vy); p(Z|x) = V^-(M-1) [(1-P_D)/V
 *             + (P_D/M) sum_m N(z_m; (px,py), p1 I)], P_D=p2, V=p3; mask[m]=0
 *             drops detection m.
 *   ARM7      d=7 joint angles, obs_dim=3, n_obs=1.  f(x)=x; z = end-effector
 *             position of the standard-DH chain A_i = Rz(q_i) Tz(d_i) Tx(a_i)
 *             Rx(alpha_i) + N(0, p0 I); a_i = p[1+i], alpha_i = p[8+i], d_i = p[15+i].
 *   LINGAUSS  d<=4, obs_dim<=4, n_obs=1.  f(x) = A x with A = p[0..d*d) row-major;
 *             z = C x + N(0, diag r), C = p[16..16+obs_dim*d), r = p[32..32+obs_dim).
 *   SE2       d=3 (px, py, heading), obs_dim=2, n_obs=1 (Sec. V-B).  With
 *             dt=p0, v=p1, omega=p2: th' = th + omega dt, f(x) = (px + v dt
 *             cos th', py + v dt sin th', th').  z = (range, bearing) from one
 *             of n_l = p5 <= 8 landmarks (p[6+2l], p[7+2l]) of unknown
 *             identity: p(z|x) = (1/n_l) sum_l N(z_r; |P - G_l|, p3)
 *             N(wrap(z_b - atan2(py - G_l,y, px - G_l,x)); 0, p4), the bearing
 *             residual mapped into [-pi, pi).  Batched plans reject it.
 *   ARM14     d=14 (7 joint angles q, 7 joint velocities qdot), obs_dim=3,
 *             n_obs=1 (Sec. V-D).  The DH chain and r_var use ARM7's slots
 *             p[0..22); dt=p22, amp=p23, freq=p24, phase_step=p25:
 *             f_t(x) = (q + qdot dt, qdot + u_{t-1} dt), u_{t-1,i} = amp
 *             sin(freq (t-1) + phase_step i), i = 0..6; z = end-effector
 *             position of q + N(0, p0 I).  Runs on the vector-ALU step
 *             kernel; batched plans reject it.
 */
typedef enum {
    SMSQ_MODEL_GROWTH1D = 0,
    SMSQ_MODEL_RANGE2D = 1,
    SMSQ_MODEL_CV4D = 2,
    SMSQ_MODEL_ARM7 = 3,
    SMSQ_MODEL_LINGAUSS = 4,
    SMSQ_MODEL_SE2 = 5,
    SMSQ_MODEL_ARM14 = 6
} smsq_model_kind_t;

typedef struct {
    int kind;           /* smsq_model_kind_t */
    int d;              /* state dimension */
    int obs_dim;        /* length of one observation vector z_t */
    int n_obs;          /* length of one mask row (beacons / detections / 1) */
    double q_var[16];   /* diagonal transition variances, first d used, > 0 */
    double params[64];  /* family constants, layout above */
} smsq_model_desc_t;

typedef struct smsq_model_s *smsq_model_t;

/* Kernel of the Stein direction (Sec. V-E ablation), functions of the squared
 * distance D = |x_i - x_k|^2 and the bandwidth h:
 *   SMSQ_KERNEL_RBF       exp(-D / h)                  (Sec. III; default)
 *   SMSQ_KERNEL_IMQ       (1 + D / h)^(-1/2)           inverse multiquadric
 *   SMSQ_KERNEL_MATERN32  (1 + a) exp(-a), a = sqrt(3 D / h)   Matern, nu = 3/2
 * The paper names the three and cites their sources without formulas; these
 * are the common forms (its printed nu = 2/3 read as 3/2).  IMQ and Matern
 * run on the vector-ALU step kernel; batched plans take RBF only. */
typedef enum { SMSQ_KERNEL_RBF = 0, SMSQ_KERNEL_IMQ = 1, SMSQ_KERNEL_MATERN32 = 2 } smsq_kernel_t;

/* SVGD options (Sec. V set-up: fixed iteration count and step size).
 *  n_iter      iterations per time step (>= 0)
 *  step        step size epsilon of x <- x + epsilon phi (finite)
 *  bw_scale    multiplier s of the median-heuristic bandwidth h = s med / ln N
 *              (> 0; the paper's ablation uses 0.5, 1 and 3)
 *  bw_mode     0: h recomputed from the particles of every iteration;
 *              1: h computed once from the initial particles of the step
 *  trans_mode  0: transition term of the score is grad_x log sum_j w_j
 *              p(x | x_{t-1}^j) (log-sum-exp over the previous particles);
 *              1: the equation's literal average of the per-j gradients.
 *  kernel      smsq_kernel_t (0 = RBF; zero-initialised options keep RBF).
 *  weights     mixture weights w_j of the previous particles in the
 *              transition term (trans_mode 0): 0 uniform (or log_w_prev where
 *              a call takes it); 1 w_j proportional to exp(phi_{t-1}(j)), the
 *              previous step's forward-recursion scores, in the drivers that
 *              hold them (smsq_batch_step, smsq_run_batch, smsq_run_sequence,
 *              batched plans): the step's target is conditioned on the MAP
 *              recursion so far.  smsq_svgd_step takes log_w_prev as given.
 *  step_kernel smsq_step_kernel_t: which step kernel runs the step (0 =
 *              automatic choice by size, precision and kernel; the others
 *              force one kernel wherever the shape fits it, else the
 *              automatic choice applies).  Results agree to rounding.
 *              Batched plans run their own persistent kernel and require 0. */
typedef struct {
    int n_iter;
    double step;
    double bw_scale;
    int bw_mode;
    int trans_mode;
    int kernel;
    int weights;
    int step_kernel;
} smsq_svgd_opts_t;

/* Step kernels (see smsq_svgd_step for the automatic choice). */
typedef enum {
    SMSQ_STEP_AUTO = 0,
    SMSQ_STEP_WAVE = 1,   /* one wave per sequence, particles in registers (n, n_prev <= 64) */
    SMSQ_STEP_VALU = 2,   /* one workgroup per sequence on the vector ALU (any kernel, FP64) */
    SMSQ_STEP_MFMA = 3,   /* one workgroup per sequence on the matrix cores (FP32, RBF, d <= 7) */
    SMSQ_STEP_COOP = 4    /* matrix cores, several workgroups per sequence: the Algorithm 2
                             drivers at any size that splits evenly (see smsq_run_batch);
                             elsewhere the automatic choice */
} smsq_step_kernel_t;

/* Validates a model description and copies it into an immutable handle.
 * Returns SMSQ_ERR_INVALID for an unknown kind, a d or observation size that
 * does not match the family, or a non-positive variance. (host only) */
smsq_status_t smsq_model_create(const smsq_model_desc_t *desc, smsq_model_t *out);
smsq_status_t smsq_model_destroy(smsq_model_t model);

/* Bytes of workspace needed by smsq_run_batch for `batch` sequences of T
 * steps with n particles (also enough for smsq_run_sequence with batch = 1
 * and for the single-step calls, which need only the 256-byte header).
 * Includes the exchange areas of the multi-workgroup steps where the shape
 * can take them (see smsq_run_batch). */
smsq_status_t smsq_workspace_size(smsq_model_t model, smsq_dtype_t dtype, int batch, int T,
                                  int n, size_t *bytes);

/* One time step of SVGD (Algorithm 2, steps 1 and 2; eq. SVGD_newupdate, and
 * eq. SVGD_initial_newupdate when n_prev = 1 and x_prev = x_0).
 *  t           step index (>= 1), the time argument of f_t
 *  x_prev      [n_prev, d] particles of step t-1 (x_0 for t = 1)
 *  log_w_prev  [n_prev] log-weights of those particles, or NULL for uniform
 *  z_t         [obs_dim] observation; z_mask [n_obs] or NULL (all present)
 *  x           [n, d] in: initial particles, out: particles after n_iter
 *              iterations; all particles move together from the state of
 *              the previous iteration
 *  h_out       [n_iter] bandwidth used by each iteration, or NULL
 * Requires n >= 1, n_prev >= 1; SMSQ_ERR_UNSUPPORTED when the particle sets
 * do not fit one compute unit's LDS.
 * Kernel choice (also for smsq_batch_step, smsq_run_batch and
 * smsq_run_sequence): up to 32 particles (FP32 states of one or two
 * dimensions: 40) and at most 64 previous ones, a one-wave kernel with the
 * particles in registers;
 * otherwise FP32 with the RBF kernel, d <= 7 and up to 1024 particles runs
 * on the matrix cores, and FP64, the IMQ and Matern kernels, d > 7 or more
 * than 1024 particles on the workgroup vector-ALU kernel.  opts->step_kernel
 * forces one of them wherever it fits; results agree to rounding. */
smsq_status_t smsq_svgd_step(smsq_model_t model, smsq_dtype_t dtype, int t,
                             int n_prev, const void *x_prev, const void *log_w_prev,
                             const void *z_t, const uint8_t *z_mask,
                             int n, void *x, const smsq_svgd_opts_t *opts /* host */,
                             void *h_out, void *ws, size_t ws_bytes, hipStream_t stream);

/* One forward-recursion step (eq. forward_recursion):
 *   c_ij = A_ij + phi_prev(j),  psi(i) = lowest j attaining max_j c_ij,
 *   phi(i) = c_{i psi(i)} + loglik_i,
 * with A_ij = log p(x_t^i | x_{t-1}^j) and loglik_i = log p(z_t | x_t^i),
 * both with their normalising constants.
 * Lattice mode (lattice != NULL): A is the given [n, n_prev] matrix and
 * loglik the given [n] vector; model, t, x_prev, z_t, z_mask and x are
 * ignored (may be NULL).  Particle mode (lattice == NULL): A and loglik are
 * computed from x_prev [n_prev, d], x [n, d] and z_t over the whole chip
 * (rows i spread over workgroups, each holding the n_prev transition means
 * in LDS).  FP32 states of d <= 8 and FP64 of d <= 4 take 4..16 rows per
 * workgroup pass (with or without tie flags) and rank c_ij in log2 units
 * (c_ij log2 e, one fused multiply-subtract per coordinate; equal scores
 * are equal in that form), in (d + 1) * n_prev element slots with n_prev
 * rounded up to a multiple of 512, 1024 or 2048; the other cases, and these
 * when that does not fit, take two waves per row in n_prev * (dpad(d) + 1)
 * slots with dpad(d) = 1, 2, 4, 8 or 16.  Any n, and n_prev up to what fits one compute unit's
 * LDS (e.g. 13,000 previous particles in FP32 at d = 2), else
 * SMSQ_ERR_UNSUPPORTED.
 *  phi_prev    [n_prev] accumulated scores of step t-1 (zeros for t = 1)
 *  phi, psi    [n] outputs; tie_flags [n] output or NULL: 1 where the best
 *              c_ij over j != psi(i) is >= best - tie_tol * max(1, |best|)
 * NaN in any c_ij or loglik_i sets SMSQ_ERR_NONFINITE in the workspace
 * status; -inf is a valid score (a row of -inf gives psi = 0). */
smsq_status_t smsq_viterbi_step(smsq_model_t model, smsq_dtype_t dtype, int t,
                                int n_prev, const void *x_prev, const void *phi_prev,
                                const void *z_t, const uint8_t *z_mask, int n, const void *x,
                                const void *lattice, const void *loglik,
                                void *phi, int32_t *psi, uint8_t *tie_flags, double tie_tol,
                                void *ws, size_t ws_bytes, hipStream_t stream);

/* Lattice-mode forward recursion (eq. forward_recursion, as
 * smsq_viterbi_step with a lattice) of `batch` independent lattices in one
 * launch: lattice [batch][n][n_prev], loglik [batch][n], phi_prev
 * [batch][n_prev], outputs phi [batch][n], psi [batch][n] and tie_flags
 * [batch][n] (or NULL), all C-contiguous.  batch <= 65535.  NaN sets
 * SMSQ_ERR_NONFINITE in the workspace status. */
smsq_status_t smsq_viterbi_lattice_batch(smsq_dtype_t dtype, int batch, int n, int n_prev, const void *lattice,
                                         const void *loglik, const void *phi_prev, void *phi, int32_t *psi,
                                         uint8_t *tie_flags, double tie_tol, void *ws, size_t ws_bytes,
                                         hipStream_t stream);

/* Backtracking (Sec. IV-B; Algorithm 2, step 4) over `batch` independent
 * sequences.  psi [batch, T, n]: row t-1 holds psi_t (entries of row 0 are
 * ignored).  phi_T [batch, n].  Outputs idx_out [batch, T] (entry t-1 is
 * i_t; i_T = lowest argmax of phi_T) and logpost_out [batch] = phi_T(i_T).
 * If particles [batch, T, n, d], x0 [batch, d] and xmap_out [batch, T+1, d]
 * are all non-NULL, the MAP states are gathered: xmap[0] = x0,
 * xmap[t] = particles[t-1][i_t]. */
smsq_status_t smsq_backtrack(smsq_dtype_t dtype, int batch, int T, int n, int d,
                             const int32_t *psi, const void *phi_T, int32_t *idx_out,
                             void *logpost_out, const void *particles, const void *x0,
                             void *xmap_out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Backtracking (Sec. IV-B; Algorithm 2, step 4) of one sequence whose
 * particle count changes from step to step.  n_t (host) [T+1]: n_t[0] = 1
 * (the known x_0), 1 <= n_t[t] <= n_max for t = 1..T.  psi [T, n_max]
 * (device, int32): entries 0..n_t[t]-1 of row t-1 hold psi_t, indices into
 * step t-1's n_t[t-1] particles (row 0 is never read).  phi_T [n_t[T]]
 * (device).  Outputs idx_out [T] (device; entry t-1 is i_t, i_T = the lowest
 * argmax of phi_T) and logpost_out [1] = phi_T(i_T).  A back-pointer outside
 * [0, n_t[t-1]) or a non-finite J sets SMSQ_ERR_NONFINITE in the workspace
 * status (the walk goes on from index 0).  The counts are copied into the
 * workspace, which needs 256 + 4 (T + 1) bytes; n_t may be freed when the
 * call returns (not for stream capture: the copy is from pageable memory).
 * Errors: SMSQ_ERR_INVALID (sizes, counts or pointers), SMSQ_ERR_WORKSPACE. */
smsq_status_t smsq_backtrack_steps(smsq_dtype_t dtype, int T, const int *n_t, int n_max, const int32_t *psi,
                                   const void *phi_T, int32_t *idx_out, void *logpost_out, void *ws,
                                   size_t ws_bytes, hipStream_t stream);

/* One step of Algorithm 2 for `batch` independent sequences that share a
 * model and sizes, in one launch: initial particles, n_iter SVGD iterations
 * and the forward recursion.
 *  t              step (>= 1).  For t = 1, n_prev must be 1, x_prev is x_0
 *                 [batch, d] and phi_prev may be NULL (zeros).
 *  x_prev         [batch, n_prev, d] (element stride between sequences is
 *                 x_prev_stride)
 *  phi_prev       n_prev accumulated scores of step t-1 per sequence, element
 *                 stride out_stride between sequences (NULL: zeros)
 *  z, z_mask      observation of step t of each sequence: element
 *                 b * z_stride (mask: b * mask_stride) starts sequence b's row
 *  x              [batch, n, d] (stride x_stride): the step's particles; if
 *                 init_given != 0 it holds the initial particles on entry,
 *                 else they are drawn as f_t(x_prev[i mod n_prev]) +
 *                 sqrt(q) * xi with xi standard normals from Philox4x32-10
 *                 keyed by `seed`, counter (i, t, seq_offset + b, block)
 *  phi, psi       outputs of the forward recursion, n per sequence with
 *                 element stride out_stride between sequences; tie_flags
 *                 likewise, or NULL.  Keeping phi and psi of every step in
 *                 [batch, T, n] buffers gives out_stride = T n. */
smsq_status_t smsq_batch_step(smsq_model_t model, smsq_dtype_t dtype, int batch, int t,
                              int n_prev, const void *x_prev, long x_prev_stride,
                              const void *phi_prev, const void *z, long z_stride,
                              const uint8_t *z_mask, long mask_stride,
                              int n, void *x, long x_stride, int init_given,
                              uint64_t seed, uint32_t seq_offset,
                              const smsq_svgd_opts_t *opts /* host */,
                              void *phi, int32_t *psi, uint8_t *tie_flags, long out_stride,
                              double tie_tol, void *ws, size_t ws_bytes, hipStream_t stream);

/* Algorithm 2 end to end for `batch` independent sequences (Monte-Carlo
 * runs) sharing a model and sizes.
 * Multi-workgroup steps: in FP32 with the RBF kernel (families GROWTH1D,
 * RANGE2D, CV4D, ARM7, d <= 7), when a sequence has at least 512 particles
 * and the batch keeps at most a quarter of the compute units busy with one
 * workgroup per sequence, each step of a sequence runs on G workgroups (the
 * largest power of two dividing its 64-particle tasks with batch * G within
 * the compute units) that own its target particles and exchange particles,
 * score rows and the median's data through the workspace every SVGD
 * iteration (a cooperative launch; on a stream under graph capture the
 * one-workgroup kernels run instead).  opts->step_kernel = SMSQ_STEP_COOP
 * takes this path at any size that splits evenly, SMSQ_STEP_MFMA never.
 * Results agree with the one-workgroup kernels to rounding.  A step whose
 * workgroups fail to meet at a barrier within a bounded wait (they did not
 * all run at once) sets the device status to SMSQ_ERR_HIP.
 *  x0 [batch, d], z [batch, T, obs_dim], z_mask [batch, T, n_obs] or NULL
 *  seed           Philox key of the predictive initial particles (sequence b
 *                 uses counter word 2 = b)
 *  xmap_out       [batch, T+1, d] MAP trajectories (x_0 first)
 *  logpost_out    [batch] J = sum_t log p(z_t, x_t | x_{t-1}) along the MAP
 *                 path (Theorem IV.1's score without the constant log p(x_0))
 *  particles_out  [batch, T, n, d] every step's particles, or NULL (then
 *                 they are kept in the workspace)
 * The workspace must hold smsq_workspace_size(model, dtype, batch, T, n). */
smsq_status_t smsq_run_batch(smsq_model_t model, smsq_dtype_t dtype, int batch, int T, int n,
                             const void *x0, const void *z, const uint8_t *z_mask, uint64_t seed,
                             const smsq_svgd_opts_t *opts /* host */, void *xmap_out,
                             void *logpost_out, void *particles_out, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/* smsq_run_batch with batch = 1. */
smsq_status_t smsq_run_sequence(smsq_model_t model, smsq_dtype_t dtype, int T, int n,
                                const void *x0, const void *z, const uint8_t *z_mask,
                                uint64_t seed, const smsq_svgd_opts_t *opts /* host */,
                                void *xmap_out, void *logpost_out, void *particles_out,
                                void *ws, size_t ws_bytes, hipStream_t stream);

/* smsq_run_sequence for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, but the run's scratch memory
 * (status word, the particles of every step when particles_out is NULL, the
 * back-pointers and the ping-pong scores) lives in one 16 MiB array of the
 * library's own device memory on each GPU, held until the process ends.  The
 * call allocates and frees nothing; no workspace argument.
 *  status_out  [1] int32 (device) or NULL: receives SMSQ_OK or
 *              SMSQ_ERR_NONFINITE for this run once the stream reaches it
 *              (the status word is cleared at the start of every run)
 * Sizes: 256 + a(T n d e) + a(4 T n) + a(2 n e) + a(4 T) bytes must not
 * exceed 16 MiB, with e the element size and a() rounding up to 256 bytes
 * (e.g. T n = 500,000 particle-steps of a 7-D FP32 state), else
 * SMSQ_ERR_WORKSPACE is returned and nothing is enqueued.  Every call on one
 * GPU shares that GPU's array: calls that overlap in time on one GPU (two
 * streams, two threads) race and give undefined results; calls ordered on
 * one stream are safe. */
smsq_status_t smsq_run_sequence_noalloc(smsq_model_t model, smsq_dtype_t dtype, int T, int n,
                                        const void *x0, const void *z, const uint8_t *z_mask,
                                        uint64_t seed, const smsq_svgd_opts_t *opts /* host */,
                                        void *xmap_out, void *logpost_out, void *particles_out,
                                        int32_t *status_out, hipStream_t stream);

/* ---- Batched ragged form ------------------------------------------------
 * Thousands of independent sequences of different model family, particle
 * count n and length T run Algorithm 2 together: every time step t is one
 * persistent launch over all sequences with T >= t (one workgroup per
 * sequence step, taken longest first from an atomic queue), followed at the
 * end by one backtrack launch over all sequences.  FP32, matrix-core step
 * kernel, RBF kernel; families GROWTH1D, RANGE2D, CV4D, ARM7, SE2 and
 * LINGAUSS at d = 2 (ARM14 and the other linear-Gaussian sizes run through
 * smsq_run_batch / smsq_run_sequence).
 *
 * The plan owns its device storage (every step's particles, forward-
 * recursion scores and backpointers of every sequence), allocated at
 * creation; runs allocate nothing.  Caller arrays named in
 * smsq_batch_seq_t are device pointers that must stay valid while the plan
 * runs.  A sequence's results equal those of smsq_run_sequence with the same
 * model, n, T, seed and options. */
typedef struct smsq_batch_plan_s *smsq_batch_plan_t;

typedef struct {
    int model;              /* index into the plan's model/options arrays */
    int n;                  /* particles per step, 1..1024 */
    int T;                  /* steps, >= 1 */
    int use_proposal;       /* 1: when the plan has a proposal network
                               (smsq_batch_plan_set_init), the initial particles
                               of steps t >= 2 are drawn from it; 0: always the
                               predictive initialisation (Philox, as in
                               smsq_batch_step with seq_offset 0) */
    uint64_t seed;
    const void *x0;         /* [d] FP32 known initial state */
    const void *z;          /* [T][obs_dim] FP32 observations */
    const uint8_t *z_mask;  /* [T][n_obs] or NULL */
    void *xmap_out;         /* [T+1][d] FP32 MAP trajectory out (x_0 first) */
    void *logpost_out;      /* [1] FP32 J out */
} smsq_batch_seq_t;

typedef struct {
    int count;              /* sequences */
    int T_max;              /* launches per run: T_max steps + 1 backtrack */
    int waves;              /* waves per workgroup of the step launches (8 or 16) */
    int grid;               /* persistent workgroups per step launch */
    size_t lds_bytes;       /* dynamic LDS per workgroup */
    size_t device_bytes;    /* device memory held by the plan */
    double tuned_ms[2];     /* autotuner timings per step: 16 waves, 8 waves (0 if not run) */
} smsq_batch_info_t;

/* Validates the sequences, orders every step's active sequences by
 * descending n^2 L and allocates the plan's storage.  models[k] and
 * opts[k] (host) describe model index k; n_models >= 1.  Starts with 16
 * waves per workgroup.  Errors: SMSQ_ERR_INVALID (bad index, size, pointer
 * or options), SMSQ_ERR_UNSUPPORTED (family not carried, n too large for
 * LDS), SMSQ_ERR_HIP (allocation). (host) */
smsq_status_t smsq_batch_plan_create(const smsq_model_t *models, const smsq_svgd_opts_t *opts,
                                     int n_models, const smsq_batch_seq_t *seqs, int count,
                                     smsq_batch_plan_t *out);

/* Autotuner: runs the first `steps` (>= 2) steps eagerly on `stream` with
 * each workgroup shape (16 waves, one 64-particle task per wave; 8 waves,
 * two tasks per wave) and grid size from the occupancy of that shape, times
 * the steps after the first with HIP events, and keeps the faster shape.
 * Synchronises the stream.  The choice and its timings are remembered for
 * the rest of the process per device architecture (name and compute units)
 * and plan shape (every sequence's family, d, n, T, L and proposal switch
 * in order, the learned-initialisation setting, the number of steps): a
 * later plan of the same shape on the same kind of device takes them
 * without running anything. (host) */
smsq_status_t smsq_batch_plan_tune(smsq_batch_plan_t plan, int steps, hipStream_t stream);

/* Runs every sequence end to end on `stream` (asynchronous).  use_graph:
 * the T_max + 1 launches (and the reset of the queue counters and status)
 * are captured once into a hipGraph on first use and replayed afterwards;
 * `stream` must then be a non-default stream. */
smsq_status_t smsq_batch_run(smsq_batch_plan_t plan, int use_graph, hipStream_t stream);

/* Device pointers of sequence `seq`'s storage in the plan: particles
 * [T][n][d], forward-recursion scores [T][n], backpointers [T][n].  Any
 * output pointer may be NULL. (host) */
smsq_status_t smsq_batch_storage(smsq_batch_plan_t plan, int seq, void **particles, void **phi,
                                 int32_t **psi);

smsq_status_t smsq_batch_plan_info(smsq_batch_plan_t plan, smsq_batch_info_t *out);
/* Device status of the last run (after stream sync): SMSQ_OK or SMSQ_ERR_NONFINITE. */
smsq_status_t smsq_batch_status(smsq_batch_plan_t plan, smsq_status_t *out);
smsq_status_t smsq_batch_plan_destroy(smsq_batch_plan_t plan);

/* ---- Learned initial particles (proposal network) ------------------------
 * A small MLP (64 -> 256 -> 256 -> 120, ReLU) maps features of a sequence
 * step (summary of the previous particle set around its best particle, the
 * likelihood gradient of the new observation there) to an 8-component
 * diagonal Gaussian mixture over the step's state, from which the initial
 * particles are drawn.  It is trained on particle sets the method itself
 * converged to, by the mixture negative log-likelihood.  GEMMs use BF16
 * operands with FP32 accumulation; parameters and Adam state are FP32.
 * Families GROWTH1D, RANGE2D, CV4D, ARM7; d <= 7.
 *
 * Parameters: one FP32 array of 113,272 values, W1 [256][64], b1 [256],
 * W2 [256][256], b2 [256], W3 [120][256], b3 [120].  Outputs per example:
 * component c (0..7) has the logit out[15c], mean offsets out[15c+1+k] and
 * log-scales out[15c+8+k] (clamped to [-7, 3]) for dimensions k < d: mean
 * a_k + s_k mu, standard deviation s_k exp(rho), with a the transition mean
 * of the best previous particle and s = sqrt(q). */
typedef struct smsq_init_mlp_s *smsq_init_mlp_t;
typedef struct smsq_init_set_s *smsq_init_set_t;

typedef struct {
    int model;              /* index into the models array */
    int t;                  /* step of the proposed particles (>= 2) */
    int n;                  /* particles of the step */
    int n_prev;             /* particles of step t - 1 */
    const void *x_prev;     /* [n_prev][d] FP32 particles of step t - 1 */
    const void *phi_prev;   /* [n_prev] FP32 forward-recursion scores of step t - 1 */
    const void *z;          /* [obs_dim] FP32 observation of step t */
    const uint8_t *z_mask;  /* [n_obs] or NULL */
    void *particles;        /* [n][d] FP32: converged particles (training) or the
                               proposal's samples (sampling, written) */
    uint64_t seed;          /* Philox key of the sampler */
    int seq;                /* Philox counter word 2 of the sampler */
} smsq_init_example_t;

/* Network with He-initialised weights (Philox normals keyed by seed) and
 * zero biases; buffers for batches of up to max_batch examples.  (host) */
smsq_status_t smsq_init_mlp_create(uint64_t seed, int max_batch, smsq_init_mlp_t *out);
smsq_status_t smsq_init_mlp_destroy(smsq_init_mlp_t mlp);
/* Device pointers of the FP32 parameters and of their gradient buffer
 * (written by smsq_init_mlp_backward / _train_step); count = 113,272. */
smsq_status_t smsq_init_mlp_params(smsq_init_mlp_t mlp, float **params, float **grads, size_t *count);
/* After the caller wrote the parameters (e.g. loaded them): refresh the BF16
 * weight copies and reset the Adam state. */
smsq_status_t smsq_init_mlp_sync(smsq_init_mlp_t mlp, hipStream_t stream);

/* A set of examples (host array of device pointers, copied). (host) */
smsq_status_t smsq_init_set_create(const smsq_model_t *models, int n_models, const smsq_init_example_t *ex,
                                   int count, smsq_init_set_t *out);
smsq_status_t smsq_init_set_destroy(smsq_init_set_t set);

/* Features of examples [first, first + count) into features [count][64]
 * (FP32) and anchors / scales [count][8] (a, s; NULL allowed). */
smsq_status_t smsq_init_features(smsq_init_mlp_t mlp, smsq_init_set_t set, int first, int count,
                                 void *features, void *anchors, void *scales, hipStream_t stream);
/* out [batch][120] = MLP(features [batch][64]), BF16 operands. */
smsq_status_t smsq_init_mlp_forward(smsq_init_mlp_t mlp, int batch, const void *features, void *out,
                                    hipStream_t stream);
/* Gradient buffer = d(sum_e <dout_e, out_e>)/d(parameters) at the last
 * forward of the same batch (call smsq_init_mlp_forward first). */
smsq_status_t smsq_init_mlp_backward(smsq_init_mlp_t mlp, int batch, const void *dout, hipStream_t stream);
/* Mixture NLL (mean over each example's particles) of examples [first,
 * first + count) under outputs out [count][120]: loss [count], and
 * dout [count][120] = gscale * d loss_e / d out_e. */
smsq_status_t smsq_init_mixture_nll(smsq_init_set_t set, int first, int count, const void *out,
                                    const void *anchors, const void *scales, double gscale, void *loss,
                                    void *dout, hipStream_t stream);
/* One Adam step (lr; beta 0.9, 0.999; eps 1e-8) on the mean NLL over
 * examples [first, first + count): features, forward, loss, backward,
 * update.  loss_out [1] (device, FP32) receives the mean loss, or NULL. */
smsq_status_t smsq_init_mlp_train_step(smsq_init_mlp_t mlp, smsq_init_set_t set, int first, int count,
                                       double lr, void *loss_out, hipStream_t stream);
/* Draws each example's n particles from its proposal into `particles`
 * (Philox4x32-10 keyed by seed, counter (i, t, seq, 2..4)); used [count]
 * (device, int32, or NULL) is 1 where the outputs were finite and the
 * samples written, 0 where nothing was written. */
smsq_status_t smsq_init_mlp_sample(smsq_init_mlp_t mlp, smsq_init_set_t set, int first, int count,
                                   int32_t *used, hipStream_t stream);

/* Batched plans: initial particles of steps t >= 2 of the sequences with
 * use_proposal = 1 from the proposal (NULL: the predictive initialisation
 * everywhere).  Per step the plan then also runs the features, the forward
 * pass and the sampler; a sequence whose proposal is not finite falls back
 * to the predictive initialisation for that step.
 * max_batch of the network must cover the plan's sequences.  The proposal's
 * features cover GROWTH1D, RANGE2D, CV4D and ARM7: a plan holding another
 * family gets SMSQ_ERR_UNSUPPORTED for a non-NULL mlp. (host) */
smsq_status_t smsq_batch_plan_set_init(smsq_batch_plan_t plan, smsq_init_mlp_t mlp);

/* Reads the workspace status word (synchronous device-to-host copy; call
 * after the work has been synchronised).  *out is SMSQ_OK,
 * SMSQ_ERR_NONFINITE, or SMSQ_ERR_HIP for a multi-workgroup step whose
 * workgroups did not all run at once (see smsq_run_batch). */
smsq_status_t smsq_get_device_status(const void *ws, smsq_status_t *out);
/* Enqueues a reset of the workspace status word to SMSQ_OK. */
smsq_status_t smsq_clear_device_status(void *ws, hipStream_t stream);

/* Static text for a status code. (host) */
const char *smsq_status_string(smsq_status_t status);

/* Maximum particles per step the single-compute-unit kernels accept for a
 * model and dtype (limited by LDS capacity), for n_prev = n. (host) */
int smsq_max_particles(smsq_model_t model, smsq_dtype_t dtype);

#ifdef __cplusplus
}
#endif
#endif /* SMSQ_H */
