/*
 * dino.h - C ABI of the MI355X (gfx950) hot path of DINO-accelerated geometric MCMC
 * (Cao, O'Leary-Roseberry & Ghattas, arXiv 2403.08220).
 *
 * The library runs the first stage of Alg. 1 (surrogate-driven mMALA with the
 * surrogate misfit deciding acceptance, eq. da_dino_trr_1) for many independent
 * chains at once, together with the pCN move of the complement subspace
 * (splitting proposition of Sec. 5.3, item 1). Every step of the path runs in HIP kernels on the device:
 * reduced proposal (eq. reduced_space_sampling), surrogate forward and reduced
 * Jacobian (eq. rb_dino and the reduced Jacobian that follows it), surrogate
 * misfit, reduced ppg and reduced ppGNH (Sec. 5.1), Cholesky factor of I + H,
 * reduced RN derivative and first-stage ratio (Sec. 5.4), MH decision, complement
 * update, trace and statistics.
 *
 * Conventions
 *  - Every call returns a dino_status; nothing throws or aborts across the ABI.
 *    On failure dino_last_error() returns a message for the calling thread.
 *  - Host pointers are borrowed for the duration of the call and copied.
 *    Pointers documented as "device" must address device memory of the
 *    context's GPU that stays valid until the call's stream work completes.
 *  - Matrices are row-major. Reduced coordinates are whitened KLE coordinates
 *    (prior N(0, I)), so x in R^r and the complement z in R^(d_m - r).
 *  - "stream" is a hipStream_t passed as void*; NULL means the null stream.
 *    Work is enqueued asynchronously; dino_read_* calls synchronise the stream
 *    they last ran on.
 *  - No call allocates device memory in dino_step; setup calls (dino_load_*,
 *    dino_problem_create without a caller workspace) allocate with hipMalloc.
 */
#ifndef DINO_H
#define DINO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dino_status;
#define DINO_OK 0
#define DINO_EINVAL (-1)   /* bad argument (size, pointer, range) */
#define DINO_ENOMEM (-2)   /* device allocation failed or workspace too small */
#define DINO_EDEVICE (-3)  /* a HIP runtime call failed */
#define DINO_ESTATE (-4)   /* call made in the wrong order (e.g. step before init) */
#define DINO_ENUMERIC (-5) /* non-finite input data */

typedef struct dino_ctx dino_ctx;
typedef struct dino_problem dino_problem;

/* Message describing the last failure on the calling thread ("" if none). */
const char* dino_last_error(void);
/* Library version string. */
const char* dino_version(void);

/* Context on one GPU. device: HIP device ordinal. Holds the prior/basis and the
 * network. Destroying a context with live problems is an error (DINO_ESTATE). */
dino_status dino_ctx_create(int device, dino_ctx** out);
dino_status dino_ctx_destroy(dino_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Prior and KLE basis (Sec. 2.1 Assumption 2; Sec. 4.2 KLE reduced basis).
 * Grid Matern prior C_pr = (gamma(-Lap_h) + delta I)^-2 on an n x n unit-square
 * grid (h = 1/(n-1), node p = j*n + i with i the x-index) with the zero-flux
 * 5-point Laplacian. The basis is the closed-form DCT-II eigenbasis ordered by
 * decreasing eigenvalue with exact ties broken by (k1, k2) ascending (k1 the
 * x-frequency); the first r modes are kept. n >= 2, 1 <= r <= n*n,
 * gamma > 0, delta > 0. Replaces a previously loaded prior.
 */
dino_status dino_load_prior(dino_ctx* ctx, int n, double gamma, double delta, int r);

/* A dense reduced basis (Sec. 4.2), e.g. a derivative-informed (DIS) basis (eq.
 * jtj_eigenvalue, eq. dis_gnh), replacing the KLE reduced basis of the loaded prior:
 * U (host, d_m x r, row-major) holds orthonormal columns u_j in whitened KLE coordinates
 * (KLE order of dino_read_basis's modes), so psi_j = Q Lambda^1/2 u_j is H_mu-orthonormal;
 * lam_dis (host, r, >= 0, or NULL) its eigenvalues, the fixed metric diag(lam_dis) of
 * DIS-mMALA. The reduced coordinates of a field with whitened coordinates z are x = U^T z.
 * A problem on a dense basis keeps the unprojected complement draw w (n_chains x d_m,
 * moved by the same pCN rule); the complement of the state is (I - U U^T) w, and the full
 * parameter U x + (I - U U^T) w (Alg. 1's assembly of m+) is formed where it is needed:
 * the second stage of delayed acceptance (per step), decode and statistics. dino_encode
 * then returns z_perp = z - U x (n_fields x d_m) and dino_decode takes one. EINVAL unless
 * U^T U = I within 1e-10, 1 <= r <= 512; ESTATE without a prior or under live problems.
 * dino_load_prior restores a KLE basis. */
dino_status dino_load_basis(dino_ctx* ctx, int r, const double* U, const double* lam_dis);

/* Copies of the basis to host buffers (any may be NULL):
 *   dec      d_m x r   decoder Psi_r (columns psi_j = sqrt(lambda_j) eta_j)
 *   lam      r         eigenvalues lambda_j
 *   var_perp d_m       pointwise prior variance of the complement,
 *                      sum_{k >= r} lambda_k eta_k(p)^2
 *   modes    r x 2     (k1, k2) of every kept mode
 * For a dense basis: dec = Q Lambda^1/2 U, lam = its DIS eigenvalues (0 if none were
 * given), var_perp = diag(C_pr) - sum_j psi_j(p)^2, modes -1. */
dino_status dino_read_basis(dino_ctx* ctx, double* dec, double* lam, double* var_perp, int32_t* modes);

/* ---------------------------------------------------------------------------
 * Surrogate network f_NN (eq. rb_dino): a chain of layers, W_k of shape
 * fan_out x fan_in (row-major, host FP64), b_k of length fan_out (NULL = 0).
 *   DINO_LAYER_LINEAR: h <- W h + b
 *   DINO_LAYER_ACT:    h <- gelu(W h + b)
 *   DINO_LAYER_RESID:  h <- h + gelu(W h + b)        (fan_in == fan_out)
 * gelu is the exact GELU z Phi(z). The first layer's fan_in is the reduced
 * dimension r (must equal the prior's r); the last layer must be LINEAR and its
 * fan_out is the number of network outputs d_out. At most 16 layers, widths <= 1024.
 * The library keeps FP64, FP32 and BF16 copies of the weights.
 */
#define DINO_LAYER_LINEAR 0
#define DINO_LAYER_ACT 1
#define DINO_LAYER_RESID 2
dino_status dino_load_network(dino_ctx* ctx, int n_layers, const int32_t* kinds, const int32_t* fan_out,
                              const int32_t* fan_in, const double* const* W, const double* const* b);

/* ---------------------------------------------------------------------------
 * True model of delayed acceptance (Alg. 1 second stage; Sec. 2.5): the paper's true
 * parameter-to-observable map is a PDE solve, out of scope here; its stand-in is a second
 * network with the layer format of dino_load_network whose input is the first r_T
 * whitened KLE coordinates of the full parameter, (x, z_perp[0 : r_T - r]) with
 * r <= r_T <= d_m (checked when a DA_MMALA problem is created). A problem observes its
 * first d_y outputs with the problem's noise variances. It runs in FP64 on DINO_PREC_F64
 * problems and in FP32 on DINO_PREC_BF16 problems. Replaces a previously loaded one.
 */
dino_status dino_load_true_model(dino_ctx* ctx, int n_layers, const int32_t* kinds, const int32_t* fan_out,
                                 const int32_t* fan_in, const double* const* W, const double* const* b);

/* ---------------------------------------------------------------------------
 * Problem: one inverse problem (data y, noise, step size) with n_chains chains.
 *
 * precision:
 *   DINO_PREC_F64   every stage in FP64 (the plain FP64 GPU path).
 *   DINO_PREC_BF16  surrogate forward in FP32; reduced Jacobian and GN Hessian
 *                   from BF16 MFMA products with FP32 accumulation; proposal,
 *                   Cholesky, log-densities and MH ratio in FP64.
 *   DINO_PREC_FP8   as DINO_PREC_BF16, but the reverse sweep of the reduced Jacobian
 *                   multiplies in OCP FP8 e4m3 (FP32 accumulation): the weights W_l^T
 *                   with one power-of-two scale per output channel (column of W_l),
 *                   quantised when the network is loaded; the sweep's left operand
 *                   Lambda diag(gelu') in MX blocks (one power-of-two scale per 32
 *                   values of a row) as a two-term e4m3 expansion hi + lo (~2^-8
 *                   relative error; two products per weight operand). Lambda is kept
 *                   in BF16 between layers, the output layer's rows in FP32. Layers of
 *                   at most 800 units (at that width, d_y >= 5).
 *   DINO_PREC_FP8_SINGLE  as DINO_PREC_FP8 with the left operand as a single e4m3 term
 *                   (one product per weight operand, ~2^-4 relative error). Its error
 *                   varies from state to state, and at the largest shapes the metric's
 *                   roughness lowers mMALA's acceptance far below the FP64 path's.
 * d_y: observed outputs (the first d_y of the network's d_out outputs).
 * noise_var: diagonal of Gamma (d_y values > 0; +inf means the output carries no
 *   information). Gamma is diagonal here: a caller with a full noise covariance
 *   Gamma = L L^T whitens its data and the network's output layer by L^-1 and passes
 *   unit variances. dt > 0 is the step size (s = (4-dt)/(4+dt), eq. mmala).
 * seed, request_id: the Philox4x64-10 key. Draw k of stream S for chain c at
 *   step t uses counter (k/4, S, t, c): S = 0 proposal normals, 1 complement
 *   normals, 2 MH uniform, 3 initial x, 4 initial z.
 * track_complement: keep the complement state z (n_chains x (d_m - r) FP32).
 * trace_capacity: number of steps whose reduced states (FP32) and misfits are
 *   recorded for diagnostics (0 = none).
 * factorization: DINO_FACTOR_PRIMAL factorises I + H (r x r) and draws the proposal
 *   noise L^-T xi; DINO_FACTOR_DUAL factorises I + B B^T (d_y x d_y, B = Gamma^-1/2 J),
 *   applies (I + H)^-1 by Woodbury and draws the noise (I + H)^-1 (xi_1 + B^T xi_2)
 *   (the same law, N(0, (I + H)^-1); xi_2 = the d_y normals of stream 0 after the
 *   first r); DINO_FACTOR_AUTO takes the dual form when d_y < r. The order of the
 *   factorised matrix must not exceed 512. On the BF16 and FP8 paths the dual form
 *   stages each chain's B (d_y x r) and its work vectors in one block's LDS: a shape
 *   that does not fit is refused with DINO_EINVAL by dino_problem_workspace_bytes and
 *   dino_problem_create (the primal form's Gauss-Newton kernel stages B^T when it fits
 *   and otherwise streams B through LDS in 64 x 64 output tiles). The BF16 reverse
 *   sweep holds at most 512 rows: networks with a hidden layer wider than 512 units
 *   need DINO_PREC_FP8 or DINO_PREC_F64 (refused with DINO_EINVAL otherwise).
 */
#define DINO_PREC_F64 0
#define DINO_PREC_BF16 1
#define DINO_PREC_FP8 2
#define DINO_PREC_FP8_SINGLE 3
#define DINO_FACTOR_PRIMAL 0
#define DINO_FACTOR_DUAL 1
#define DINO_FACTOR_AUTO 2
/* Transition kernel of a problem's chains.
 * MMALA: the surrogate mMALA first stage (Alg. 1, the splitting proposition of Sec. 5.3).
 * PCN: the pCN baseline (Sec. 2.6, eq. pCN_proposal; the pCN row of the baselines of
 *   Sec. 6.1): x+ = s x + beta xi with xi the first r normals of the proposal stream and
 *   s = (4 - dt)/(4 + dt), accepted with exp(Phi(x) - Phi(x+)); the complement moves as
 *   for MMALA. A step evaluates the network forward only (no Jacobian, metric or factor);
 *   the cache's g and factor then stay those of dino_chains_init.
 * MALA: the MALA baseline (the MALA row of the baselines of Sec. 6.1): the MMALA
 *   transition with the metric removed (H = 0) and the ppg kept, x+ = s x - (1 - s) g +
 *   beta xi, log rho_0(m1, m2) = -(dt/8)||g(m1)||^2 - (sqrt(dt)/2) mhat . g(m1). A step
 *   forms the misfit and ppg at x+ (forward and Jacobian); the cache's factor stays that
 *   of dino_chains_init.
 * LAPCN: the LA-pCN baseline (eq. MAP and the LA-pCN proposal after it; the LA-pCN row
 *   of the baselines of Sec. 6.1), the pCN move about the MAP with the Laplace
 *   covariance: x+ = x_map + s (x - x_map) + beta L^-T xi, with L L^T = I + H(x_map)
 *   fixed by dino_set_fixed_metric, and log rho = Phi(x) - Phi(x+) + (|x|^2 - |x+|^2)/2
 *   + (|L^T (x+ - x_map)|^2 - |L^T (x - x_map)|^2)/2. The printed proposal mean
 *   m_MAP - s m is read as m_MAP + s (m - m_MAP): only that form is reversible with
 *   respect to the Laplace approximation. A step evaluates the network forward only.
 * DA_MMALA: delayed acceptance (Alg. 1 with its second stage; Sec. 2.5, eq. da_dino_trr_2):
 *   the MMALA first stage, then, for the proposals it passes, the full proposal (x+ and the
 *   pCN move of the complement, drawn only then) judged by the true misfit Phi of the true
 *   model loaded with dino_load_true_model: log rho^(2) = (Phi~(x+) - Phi~(x)) +
 *   (Phi(m) - Phi(m+)), accepted iff log u2 <= log rho^(2) with u2 word 0 of block 0 of
 *   Philox stream 5 at (step, chain). The state keeps its true misfit. The true model runs
 *   on the first-stage passes only (compacted). Needs track_complement when the true model
 *   reads complement coordinates.
 * DIS_MMALA: the DIS-mMALA baseline (the DIS-mMALA row of the baselines of Sec. 6.1): the
 *   MMALA transition with the metric fixed at the DIS approximation of the expected ppGNH
 *   (eq. dis_gnh), diag(lam_dis) in the coordinates of a dense basis loaded with its DIS
 *   eigenvalues, and the ppg kept: x+_j = ((lam_j + s) x_j - (1 - s) g_j)/(1 + lam_j) +
 *   beta xi_j / sqrt(1 + lam_j). A step forms the misfit and ppg at x+ (no metric or
 *   factor). lam = 0 is MALA.
 * PCN, MALA, LAPCN, DA_MMALA and DIS_MMALA are not available to the serving pools. */
#define DINO_METHOD_MMALA 0
#define DINO_METHOD_PCN 1
#define DINO_METHOD_MALA 2
#define DINO_METHOD_LAPCN 3
#define DINO_METHOD_DA_MMALA 4
#define DINO_METHOD_DIS_MMALA 5
typedef struct {
    int32_t n_chains;
    int32_t d_y;
    int32_t precision;
    int32_t track_complement;
    int32_t trace_capacity;
    int32_t factorization;
    double dt;
    uint64_t seed;
    uint64_t request_id;
    int32_t method;           /* DINO_METHOD_MMALA (0), _PCN, _MALA or _LAPCN */
} dino_problem_desc;

/* Device bytes a problem needs (state, caches, scratch, trace). */
dino_status dino_problem_workspace_bytes(const dino_ctx* ctx, const dino_problem_desc* desc, size_t* bytes);

/* Create a problem. y and noise_var are host arrays of d_y values.
 * dev_ws/ws_bytes: caller-owned device workspace of at least
 * dino_problem_workspace_bytes() bytes, 256-byte aligned; NULL lets the library
 * allocate (and free it at destroy). EINVAL for dt <= 0, d_y outside
 * [1, d_out], non-positive noise variances; ENUMERIC for non-finite y. */
dino_status dino_problem_create(dino_ctx* ctx, const dino_problem_desc* desc, const double* y,
                                const double* noise_var, void* dev_ws, size_t ws_bytes, dino_problem** out);
dino_status dino_problem_destroy(dino_problem* p);

/* Initial states: x0 (n_chains x r, host FP64) and z0 (n_chains x (d_m - r),
 * host FP32); NULL draws them from the prior (streams 3 and 4). Evaluates the
 * geometry cache at x0 (Alg. 1 "known at m_j") and resets the step counter,
 * acceptance counts and trace. */
dino_status dino_chains_init(dino_problem* p, const double* x0, const float* z0, void* stream);

/* The fixed metric of an LAPCN problem: x_map (host, r FP64, the reduced MAP) and L_map
 * (host, r x r FP64 row-major, the lower Cholesky factor of I + H(x_map); the upper
 * triangle is not read). Copied to the problem's workspace. EINVAL unless the problem's
 * method is DINO_METHOD_LAPCN, for null pointers, or a non-positive diagonal; ENUMERIC
 * for non-finite entries. An LAPCN problem refuses dino_step (ESTATE) until this call. */
dino_status dino_set_fixed_metric(dino_problem* p, const double* x_map, const double* L_map);

/* How dino_step launches its kernels. DINO_LAUNCH_GRAPH (the default, 8 steps per graph):
 * the step loop of steps_per_graph transitions (1..256) is captured once as a HIP graph
 * and replayed (one graph of the remainder too); DINO_LAUNCH_EAGER: one launch per kernel.
 * Both run the same kernels with the same arguments, so their results are identical.
 * Stage profiling always runs eagerly. Waits for the problem's last stream. */
#define DINO_LAUNCH_EAGER 0
#define DINO_LAUNCH_GRAPH 1
dino_status dino_set_launch_mode(dino_problem* p, int mode, int steps_per_graph);

/* Autotuner. Times the implementations that can run a stage of this problem at its
 * shapes, on the problem's own buffers between steps (stage outputs that every step
 * overwrites; the chains' states are not touched), and keeps the fastest in a
 * process-wide table keyed by stage and shape, which every later launch of that shape
 * uses (other problems and serving pools included):
 *   kind DINO_TUNE_CHOL  (a, b, c) = (chains, factor order, 0): the factor kernel,
 *        0-2 one wavefront per chain (orders up to 32 / 56 / 104), 3-4 one block per
 *        chain with the triangle in registers (up to 128 / 208), 5 the LDS panel kernel,
 *        6 the transposed-panel kernel (one-wave diagonal block, row-parallel panel solve;
 *        up to 512);
 *   kind DINO_TUNE_FWD64 (rows, fan_in, fan_out): FP64 forward tile of 16, 32 or 64 outputs;
 *   kind DINO_TUNE_FWD32 (rows, fan_in, fan_out): FP32 MFMA forward block order, 0 row-major,
 *        1 the tiles of a 32-row block on one XCD;
 *   kind DINO_TUNE_HESS  (r, d_y, 0): the BF16/FP8 paths' Gauss-Newton kernel of the primal
 *        form, 0 one block per chain with B^T staged in LDS (where it fits), 1 one block per
 *        64 x 64 output tile streaming B (the only choice where B^T does not fit);
 *   kind DINO_TUNE_FWDCHAIN (chains, layers, widest hidden layer): the mixed paths' FP32
 *        forward, 0 one launch per layer (the default), 1 one launch for all layers (row
 *        blocks hand layers on through device counters; taken only where all its blocks
 *        are resident at once);
 *   kind DINO_TUNE_DUALSOLVE (d_y, 0, 0): the triangular solves of the dual proposal and
 *        acceptance on the mixed path, 1 (the default where the fused Gram + factor kernel
 *        makes the factors) blocks of 32 rows through their inverted diagonal blocks,
 *        which that kernel stores in the factor's unused upper triangle, 0 serial
 *        substitution in every block. Not timed by dino_autotune (timing it would move the
 *        chains); set by dino_tune_set.
 * Every choice computes the same quantities (rounding order may differ between factor
 * kernels and between the two solves). n_entries (optional): table entries written. Releases the problem's launch
 * graphs (they hold the earlier choices). dino_tune_set sets or (choice < 0) erases an
 * entry; dino_tuning_table writes the table as text lines "kind a b c choice ms...". */
#define DINO_TUNE_CHOL 0
#define DINO_TUNE_FWD64 1
#define DINO_TUNE_FWD32 2
#define DINO_TUNE_HESS 3
#define DINO_TUNE_FWDCHAIN 4
#define DINO_TUNE_DUALSOLVE 5
dino_status dino_autotune(dino_problem* p, void* stream, int32_t* n_entries);
dino_status dino_tune_set(int32_t kind, int32_t a, int32_t b, int32_t c, int32_t choice);
dino_status dino_tuning_table(char* buf, size_t cap, size_t* length);

/* Advance every chain n_steps transitions (Alg. 1 first stage + the splitting proposition of Sec. 5.3).
 * Asynchronous on stream. Per-chain numerical failures (non-finite misfit,
 * I + H not positive definite) reject the proposal and are counted; they do
 * not fail the call. */
dino_status dino_step(dino_problem* p, int n_steps, void* stream);

/* Host copies of the state (any pointer may be NULL). x: n_chains x r FP64;
 * z: n_chains x (d_m - r) FP32 (ESTATE if not tracked). */
dino_status dino_read_states(dino_problem* p, double* x, float* z);

/* Host copies of the cache at the current states: misfit (n_chains), reduced
 * ppg (n_chains x r) and the lower Cholesky factor of I + H (n_chains x r x r,
 * upper triangle unspecified; in the dual form the factor of I + B B^T, d_y x d_y
 * with row stride d_y, in the first d_y^2 entries of each chain's r x r block). Any
 * pointer may be NULL. */
dino_status dino_read_cache(dino_problem* p, double* phi, double* g, double* L);

/* Per-chain accepted moves and numerical failures since init, and the number of
 * steps taken. Any pointer may be NULL. */
dino_status dino_read_diagnostics(dino_problem* p, int64_t* accepts, int64_t* failures, int64_t* steps);

/* Delayed acceptance: host copies of the true misfit of the current states (n_chains) and
 * of the first-stage passes per chain since init (the true-model evaluations). EINVAL
 * unless the problem's method is DINO_METHOD_DA_MMALA. */
dino_status dino_read_delayed(dino_problem* p, double* phi_true, int64_t* passes);

/* Delayed acceptance: the true misfit (n) of n full parameters given as the r_T
 * coordinates the true model reads (device, n x r_T FP64), evaluated as the second stage
 * evaluates it. EINVAL unless the method is DINO_METHOD_DA_MMALA. */
dino_status dino_eval_true_misfit(dino_problem* p, int n, const double* z_in, double* phi_true, void* stream);

/* Recorded trace: x_trace (steps x n_chains x r FP32) and phi_trace
 * (steps x n_chains FP64) for the min(steps, trace_capacity) first steps. */
dino_status dino_read_trace(dino_problem* p, float* x_trace, double* phi_trace, int64_t* n_recorded);

/* Posterior field mean and pointwise variance (d_m each, host FP64) from the
 * recorded trace after discarding the first burn_in recorded steps: mean =
 * Psi_r xbar and var = diag(Psi_r S Psi_r^T) + var_perp (the complement is
 * prior distributed and independent of the reduced part, the Gaussian lemma of Sec. 5.3). Also the
 * reduced mean xbar (r) and covariance S (r x r) if the pointers are non-NULL.
 * Computed on the device. */
dino_status dino_posterior(dino_problem* p, int burn_in, double* mean, double* var, double* xbar, double* S);

/* Multichain ESS fraction (Sec. 6.2.2, eq. ess; rho_t with lag-t
 * autocovariances, Geyer truncation on positive pair sums) of every reduced
 * coordinate from the recorded trace after burn_in steps; ess: r values. */
dino_status dino_ess(dino_problem* p, int burn_in, double* ess);

/* ---------------------------------------------------------------------------
 * Stage timing. With profiling enabled, dino_step records HIP events on its
 * stream around every stage of every step into a ring of steps that is read
 * back (one host wait) when it fills or when the profile is read (slower;
 * meant for measurement passes). Stages: 0 proposal, 1 surrogate forward,
 * 2 reduced Jacobian, 3 misfit and ppg, 4 GN Hessian, 5 Cholesky,
 * 6 acceptance, 7 second stage (delayed acceptance), 8 complement, 9 trace. stage_ms: total milliseconds per stage;
 * launches: kernel launches per stage per step (0 where the stage's work runs
 * inside another stage's kernel: the misfit on the BF16 path, in the GN
 * kernel; the trace and step counters, in the acceptance kernel); steps:
 * profiled steps.
 */
#define DINO_N_STAGES 10
dino_status dino_set_profiling(dino_problem* p, int enable);
dino_status dino_read_profile(dino_problem* p, double* stage_ms, int32_t* launches, int64_t* steps);
const char* dino_stage_name(int stage);

/* ---------------------------------------------------------------------------
 * Stage entry points on explicit device buffers (used to check each stage).
 * All pointers are device pointers; n <= n_chains of the problem; chain
 * index k of the batch uses counters of chain k.
 */

/* Geometry at reduced points x (n x r): network output f (n x d_y), surrogate
 * misfit phi (n), reduced ppg g (n x r), reduced ppGNH H (n x r x r, full),
 * lower Cholesky factor L of I + H (n x r x r), logdet = sum log L_ii (n) and
 * ok (n int32: 1 if finite and positive definite). H may be NULL. In the dual form
 * L receives the factor of I + B B^T (d_y x d_y, row stride d_y, in the first d_y^2
 * entries of each chain's block; log det is the same) and H is B^T B formed from the
 * stored B. dino_eval_propose and dino_eval_log_rho serve the primal form,
 * dino_eval_propose_dual and dino_eval_log_rho_dual the dual form. */
dino_status dino_eval_geometry(dino_problem* p, int n, const double* x, double* f, double* phi, double* g,
                               double* H, double* L, double* logdet, int32_t* ok, void* stream);

/* Reduced proposal (eq. reduced_space_sampling, noise mapped through L^-T) from
 * states x with cache (g, L) and given normals xi (all n x r / n x r x r):
 * xp = L^-T (L^-1 [L L^T x - (1-s) x - (1-s) g] + sqrt(1-s^2) xi). */
dino_status dino_eval_propose(dino_problem* p, int n, const double* x, const double* g, const double* L,
                              const double* xi, double* xp, void* stream);

/* log of the first-stage ratio rho^(1)_r(x, xp) (eq. da_dino_trr_1) from the
 * two states and their caches (phi, g, L, logdet). */
dino_status dino_eval_log_rho(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                              const double* L_x, const double* logdet_x, const double* xp,
                              const double* phi_p, const double* g_p, const double* L_p,
                              const double* logdet_p, double* log_rho, void* stream);

/* Whitened reduced Jacobian B = Gamma^-1/2 J (the surrogate Jacobian of eq. rb_dino at
 * x, whitened as in Sec. 5.1) of n points x (n x r), as the problem's Jacobian stage
 * computes and stores it (BF16 problems: BF16 values), returned as FP64 in B
 * (n x d_y x r, row-major). Runs the forward and Jacobian stages. */
dino_status dino_eval_jacobian(dino_problem* p, int n, const double* x, double* B, void* stream);

/* Row stride ldb of the Jacobian the dual stage entry points take: r for DINO_PREC_F64
 * problems (B in doubles), ceil(r / 32) * 32 for DINO_PREC_BF16 problems (B as
 * bfloat16 bit patterns; the entries of a row past r are not read). */
dino_status dino_jacobian_ld(const dino_problem* p, int32_t* ldb);

/* Observation-space (dual) form of the reduced proposal (eq. reduced_space_sampling,
 * noise drawn as beta (I + H)^-1 (xi_1 + B^T xi_2), H = B^T B) and of the forward term
 * lfwd = log rho_0(x -> xp) of the reduced RN derivative (Sec. 5.4), with the kernels
 * dino_step runs for a dual problem. Device buffers: x, g (n x r), B (n x d_y x ldb, see
 * dino_jacobian_ld, in the problem's Jacobian type), K (n x d_y x d_y, the lower Cholesky
 * factor of I + B B^T, row-major, upper triangle not read), logdet (n, sum log K_ii), xi
 * (n x (r + d_y): xi_1 then xi_2); outputs xp (n x r) and lfwd (n). EINVAL for a primal
 * problem or a method other than MMALA. */
dino_status dino_eval_propose_dual(dino_problem* p, int n, const double* x, const double* g, const void* B,
                                   const double* K, const double* logdet, const double* xi, double* xp, double* lfwd,
                                   void* stream);

/* log of the first-stage ratio rho^(1)_r(x, xp) (eq. da_dino_trr_1) of the dual form from
 * the two states and their caches (phi, g, B, K, logdet, laid out as for
 * dino_eval_propose_dual); both transition terms are evaluated with the code of the
 * acceptance kernel's reverse term. */
dino_status dino_eval_log_rho_dual(dino_problem* p, int n, const double* x, const double* phi_x, const double* g_x,
                                   const void* B_x, const double* K_x, const double* logdet_x, const double* xp,
                                   const double* phi_p, const double* g_p, const void* B_p, const double* K_p,
                                   const double* logdet_p, double* log_rho, void* stream);

/* Philox4x64-10 normals of one stream for n chains at one step: out n x count. */
dino_status dino_eval_normals(dino_problem* p, int n, int stream_id, int64_t step, int count, double* out,
                              void* stream);

/* Whitened KLE coordinates of nodal fields (the encoder of eq. projector extended to
 * all d_m modes, Sec. 4.2 with the prior of this library): z = Lambda^-1/2 Q^T m in KLE
 * order, computed through the separable DCT-II basis; x = z[0:r] is the reduced part
 * and z_perp = z[r:] the complement. fields: device, n_fields x d_m (node p = j n + i);
 * x: device, n_fields x r; z_perp: device, n_fields x (d_m - r); one of x and z_perp
 * may be NULL. The call allocates 2 n_fields d_m doubles of device scratch and
 * synchronises the stream. */
dino_status dino_encode(dino_ctx* ctx, int n_fields, const double* fields, double* x, double* z_perp,
                        void* stream);
/* Nodal fields m = Q Lambda^1/2 z from whitened coordinates (the decoder Psi_r x plus
 * the complement); z_perp == NULL decodes the reduced part alone. Same layouts and
 * scratch as dino_encode. */
dino_status dino_decode(dino_ctx* ctx, int n_fields, const double* x, const double* z_perp, double* fields,
                        void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dino_encode without any allocation.
 * Same arguments, layouts and results as dino_encode; its two transform buffers live in
 * a library-owned static device buffer of DINO_NOALLOC_SCRATCH_BYTES per GPU (held until
 * the process ends), so 2 * n_fields * d_m * sizeof(double) must not exceed it (else
 * DINO_EINVAL, e.g. at most 63 fields on a 129 x 129 grid). The call is asynchronous on
 * stream and does not synchronise it. Every call on one GPU shares that GPU's buffer:
 * calls that overlap on one GPU (other streams, other threads, other contexts) race and
 * must be ordered by the caller. */
#define DINO_NOALLOC_SCRATCH_BYTES (16u << 20)
dino_status dino_encode_noalloc(dino_ctx* ctx, int n_fields, const double* fields, double* x, double* z_perp,
                                void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of many inverse problems (one problem = one request:
 * its own data y, noise variances, observation count, chain count and step budget)
 * on the context's GPU. Each request runs the same chains as dino_step would
 * (Alg. 1 first stage + the splitting proposition of Sec. 5.3) with Philox key
 * (seed, request_id), prior initial states drawn from streams 3 and 4, and chain
 * index 0..n_chains-1, so its draws do not depend on what else is served.
 *
 * Every bucket b serves requests with d_y <= bucket_dy[b] that no smaller bucket
 * serves, in a pool of bucket_slots[b] preallocated chain slots and max_requests
 * request rows; outputs beyond a request's d_y are unobserved (Gamma^-1/2 = 0), the
 * request observing the first d_y network outputs. A request is admitted, in arrival
 * order, when its chains fit a contiguous free slot range and a row is free; all
 * occupied slots of a pool advance together in quanta of steps_per_quantum steps on
 * the pool's own stream, and the pools of different buckets overlap on the device.
 * A request's result is its posterior mean field Psi_r xbar (xbar: the mean of the
 * reduced states after the first 20% of its steps, over its chains and steps; the
 * complement has mean zero, the Gaussian lemma of Sec. 5.3) with its acceptance
 * counts and server-clock timestamps. The library allocates the pools in
 * dino_server_create (hipMalloc, pinned host buffers) and nothing afterwards. */
#define DINO_MAX_BUCKETS 8

typedef struct dino_server dino_server;

typedef struct {
    int32_t n_buckets;                        /* 1..DINO_MAX_BUCKETS */
    int32_t bucket_dy[DINO_MAX_BUCKETS];      /* ascending observation counts, <= network outputs */
    int32_t bucket_slots[DINO_MAX_BUCKETS];   /* chain slots of each bucket's pool */
    int32_t max_requests;                     /* request rows per pool (concurrent requests) */
    int32_t steps_per_quantum;                /* steps enqueued per pool between scheduling passes */
    int32_t precision;                        /* DINO_PREC_F64 or DINO_PREC_BF16 */
    int32_t track_complement;                 /* keep and move the complement state */
    int32_t factorization;                    /* DINO_FACTOR_* of every pool (AUTO: per bucket) */
    double dt;                                /* step size of every request */
    double hbm_budget_bytes;                  /* > 0: DINO_ENOMEM if the pools need more */
} dino_server_cfg;

typedef struct {
    uint64_t seed;                            /* Philox key word 0 */
    uint64_t request_id;                      /* Philox key word 1, and the result's id */
    int32_t d_y;                              /* observed outputs: the first d_y of the network */
    int32_t n_chains;                         /* 1..slots of its bucket */
    int64_t n_steps;                          /* Markov steps per chain (burn-in: the first 20%) */
    const double* y;                          /* host, d_y; copied by dino_server_submit */
    const double* noise_var;                  /* host, d_y; > 0 (inf: unobserved) */
    double arrival;                           /* server-clock seconds from which it may be admitted */
} dino_request;

typedef struct {
    uint64_t request_id;
    int32_t d_y, n_chains;
    int64_t n_steps;
    double arrival, admitted, finished;       /* server-clock seconds; finished = mean in host memory */
    int64_t accepts, failures;                /* summed over the request's chains */
} dino_result;

/* Pools for cfg on ctx's device (prior and network loaded). Errors: DINO_EINVAL (bad
 * cfg), DINO_ESTATE (ctx not ready), DINO_ENOMEM (pools exceed hbm_budget_bytes or the
 * device). The context must outlive the server. */
dino_status dino_server_create(dino_ctx* ctx, const dino_server_cfg* cfg, dino_server** out);
dino_status dino_server_destroy(dino_server* srv);
/* Seconds since dino_server_create (monotonic clock of the server). */
dino_status dino_server_clock(const dino_server* srv, double* seconds);
/* Queues a request (its data is copied). DINO_EINVAL if no bucket serves d_y or
 * n_chains exceeds the bucket's slots; DINO_ENUMERIC on non-finite data. */
dino_status dino_server_submit(dino_server* srv, const dino_request* req);
/* Runs the scheduler in the calling thread until every submitted request has
 * finished, or until the server clock reaches `until` (until >= 0). n_finished
 * (optional) receives the number of requests finished during the call. */
dino_status dino_server_run(dino_server* srv, double until, int* n_finished);
/* Moves up to max finished results, oldest first, into out[0..n) and, if means is not
 * NULL, their mean fields into means (max x d_m doubles, caller-owned). */
dino_status dino_server_poll(dino_server* srv, int max, dino_result* out, double* means, int* n);
/* Chain-steps of the finished requests, and counts of waiting and admitted requests. */
dino_status dino_server_stats(const dino_server* srv, int64_t* chain_steps, int64_t* pending, int64_t* live);

#ifdef __cplusplus
}
#endif
#endif /* DINO_H */
