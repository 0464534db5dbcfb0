/*
 * bdrpy.h -- C ABI of libbdrpy, the MI355X (gfx950) hot path of bead-rod
 * Brownian dynamics with Rotne-Prager-Yamakawa hydrodynamic interactions
 * (arXiv 2208.06559).
 *
 * One timestep of one chain (Section 3, Eq. 6 with Eqs. 7-10; the per-step
 * order of Section 4's flowchart):
 *   1. bd_rpy_assemble  D = D(x), the 3N x 3N RPY diffusion tensor
 *   2. bd_cholesky      D = B B^T, B lower (in place)
 *   3. bd_brownian      y = c_B B xi, xi from a counter-based Philox stream
 *   4. predictor        x* = x + dt kappa.x + y       (inside bd_step)
 *   5. bd_constrain     rod tensions T with |Q_k| = b, then x^{t+dt}
 *   bd_step runs 1-5 on the handle's stream.
 *
 * Conventions shared by every entry point
 *   - N beads (the paper's beads 0..N are N+1 beads; here N counts beads),
 *     N-1 rods Q_k = r_{k+1} - r_k, matrix order n = 3N.
 *   - Scalar index e = 3i + alpha (bead-major, component-minor), the block
 *     layout of the paper's two-bead example (Section 4, Eqs. 18-20).
 *   - Positions x: row-major N x 3 doubles.  Matrices: column-major with
 *     leading dimension ld >= n, FP64.
 *   - Units zeta = kT = 1 (so D_ii = I, Eq. 7); lengths in Kuhn steps b.
 *   - Pointers named d_* are device pointers, caller-owned; the library never
 *     allocates or frees caller buffers.  Scratch memory is the caller's
 *     workspace, sized by bd_workspace_size.  The handle owns only a few
 *     bytes of device state (status word, Newton state).
 *   - Calls are asynchronous on the handle's stream.  Argument errors are
 *     returned synchronously; numerical errors (non-positive pivot, Newton
 *     non-convergence) are recorded in device memory and reported by
 *     bd_get_info, which synchronises the stream.  On an error return the
 *     outputs are unspecified, but no write goes outside the caller's
 *     buffers.  No C++ exception crosses this interface.
 *   - Results are bitwise reproducible run to run on one GPU (no floating
 *     point atomics).  A handle must not be used from two host threads at
 *     once.
 */
#ifndef BDRPY_H
#define BDRPY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BD_OK = 0,
  BD_ERR_PARAM = 1,       /* invalid argument (null pointer, size, range)      */
  BD_ERR_NOT_SPD = 2,     /* non-positive pivot in the Cholesky factorisation  */
  BD_ERR_NO_CONVERGE = 3, /* tension Newton did not reach newton_tol           */
  BD_ERR_HIP = 4,         /* a HIP runtime call failed                         */
  BD_ERR_ALLOC = 5,       /* the handle's own small allocation failed          */
  BD_ERR_UNSUPPORTED = 6  /* device is not gfx950                              */
} bd_status_t;

typedef enum {
  BD_PREC_FP64 = 0, /* every step in FP64                                       */
  BD_PREC_MIXED = 1 /* Cholesky trailing updates on FP32 MFMA with FP32
                       accumulation into FP64 storage; diagonal blocks, panel
                       solves, noise and the tension solve stay FP64          */
} bd_precision_t;

typedef enum {
  BD_NOISE_GAUSSIAN = 0,     /* xi ~ N(0,1), y = sqrt(2 dt) B xi               */
  BD_NOISE_UNIFORM_PAPER = 1 /* n uniform on [-1,1] (Eq. 2), y = sqrt(6 dt) B n */
} bd_noise_t;

typedef enum { BD_FILL_LOWER = 0, BD_FILL_FULL = 1 } bd_fill_t;

typedef enum {
  BD_OP_CHOLESKY = 0,
  BD_OP_BROWNIAN = 1,
  BD_OP_CONSTRAIN = 2,
  BD_OP_STEP = 3,
  BD_OP_CHOLESKY_ADJOINT = 4,
  BD_OP_STEP_ADJOINT = 5
} bd_op_t;

/* Model and step parameters (Sections 3 and 5). */
typedef struct {
  int32_t n_beads;      /* N >= 2                                             */
  int32_t noise;        /* bd_noise_t                                          */
  double b;             /* rod length, > 0                                     */
  double hstar;         /* HI strength h* of Eqs. 8-9, 0 <= h* <= a (0: HI off) */
  double a;             /* bead radius of Eqs. 8-9, > 0                        */
  double dt;            /* timestep, > 0                                       */
  double kappa[9];      /* row-major (grad v)^T, flow velocity v = kappa . r (Eq. 5) */
  uint64_t seed;        /* Philox4x64-10 key word 0                            */
  uint64_t chain_id;    /* Philox4x64-10 key word 1                            */
  double newton_tol;    /* stop when max_k | |Q_k|/b - 1 | <= newton_tol        */
  int32_t newton_maxit; /* >= 1, Newton steps before BD_ERR_NO_CONVERGE        */
  int32_t reserved;     /* must be 0                                           */
} bd_params_t;

/* Result of the most recent call on a handle. */
typedef struct {
  int32_t status;         /* bd_status_t                                      */
  int32_t newton_iters;   /* Newton steps performed by the last constraint    */
  int64_t potrf_info;     /* 0, or 1-based column of the first non-positive pivot */
  double max_rod_err;     /* max_k | |Q_k|/b - 1 | after the last constraint  */
  double last_newton_res; /* max_k | |Q_k|^2 - b^2 | at the last Newton check */
  int32_t krylov_iters;   /* GMRES iterations summed over those Newton steps  */
  int32_t reserved;
} bd_info_t;

typedef struct bd_handle_s* bd_handle_t;

/* Create a handle on HIP device `device` that launches on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Fails with BD_ERR_UNSUPPORTED
 * unless the device is gfx950. */
bd_status_t bd_create(bd_handle_t* h, int device, void* hip_stream);
bd_status_t bd_destroy(bd_handle_t h);
bd_status_t bd_set_stream(bd_handle_t h, void* hip_stream);

/* Factorisation schedule for calls of matrix order n <= n_max in precision
 * prec (the first matching row of the handle's table applies): the trailing
 * matrix is updated by up to step_panels (1, 2 or 4) panels of 128 columns
 * per pass while more than wide_rows rows remain, by two after.  Results of
 * different schedules differ only in rounding order. */
typedef struct {
  int64_t n_max;
  int32_t prec;         /* bd_precision_t */
  int32_t step_panels;  /* 1, 2 or 4 */
  int64_t wide_rows;    /* >= 0 */
} bd_schedule_t;

/* Copy a table of schedules into the handle (count = 0: back to the
 * defaults, four panels while more than 4096 rows remain, or the
 * BDRPY_STEP_PANELS / BDRPY_WIDE_ROWS environment variables read at
 * bd_create).  The table is meant to come from measured timings: the
 * package's autotuner (tune.py) writes one for this GPU. */
bd_status_t bd_set_schedules(bd_handle_t h, const bd_schedule_t* rows, int32_t count);

/* Panels per factorisation step (2 or 4; 0: the default, four, or
 * BDRPY_ENS_PANELS) of the ensembles created on this handle afterwards, in
 * precision prec. */
bd_status_t bd_set_ensemble_panels(bd_handle_t h, bd_precision_t prec, int32_t panels);

/* Bytes of device workspace the operation needs for matrix order n = 3N
 * (for BD_OP_CHOLESKY, n is the matrix order of the call). */
bd_status_t bd_workspace_size(bd_op_t op, int64_t n, bd_precision_t prec, size_t* bytes);

/* D(x) per Eqs. 7-9: D_ii = I; for i != j with R = r_i - r_j, |R| >= 2a the
 * far-field block (Eq. 8), else the near-field block (Eq. 9).
 * d_x: N x 3; d_D: n x n column-major, ld >= n.  BD_FILL_LOWER writes the
 * lower triangle including the diagonal and leaves the rest untouched;
 * BD_FILL_FULL writes every element. */
bd_status_t bd_rpy_assemble(bd_handle_t h, const bd_params_t* p, const double* d_x, double* d_D,
                            int64_t ld, bd_fill_t fill);

/* Adjoint of the assembly (Eqs. 7-9), the first step of differentiating
 * the path: for phi = sum_ij <Dbar_ij, D_ij(x)> with Dbar a full n x n
 * matrix (d_Dbar, column-major, ld >= n, both triangles read), writes
 * d phi/d x to d_xbar (N x 3) and d phi/d h* to d_hbar (one double).
 * d_ws: at least 8 N bytes.  Coincident beads (where the near-field block
 * is not differentiable) set status BD_ERR_PARAM in bd_get_info; the
 * outputs are then unspecified. */
bd_status_t bd_rpy_assemble_adjoint(bd_handle_t h, const bd_params_t* p, const double* d_x,
                                    const double* d_Dbar, int64_t ld, double* d_xbar,
                                    double* d_hbar, void* d_ws, size_t ws_bytes);

/* Adjoint of the noise product y = c_B B xi (bd_brownian): for the
 * gradient ybar of a scalar in y, writes Lbar = c_B ybar xi^T on the lower
 * triangle of d_Lbar (n x n column-major, ldb >= n; the strict upper part
 * is not touched) and xibar = c_B B^T ybar to d_xibar (n).  d_L: the lower
 * triangle of B (ld >= n); d_xi: the noise of the forward call (its
 * d_xi_out).  n <= 65535 (BD_ERR_UNSUPPORTED above). */
bd_status_t bd_brownian_adjoint(bd_handle_t h, const bd_params_t* p, const double* d_L,
                                int64_t ld, const double* d_xi, const double* d_ybar,
                                double* d_Lbar, int64_t ldb, double* d_xibar);

/* In-place Cholesky D = B B^T (Eq. 10) of the lower triangle of d_A
 * (n x n column-major, ld >= n); B overwrites the lower triangle, the strict
 * upper triangle is not touched.  Blocked right-looking: FP64 diagonal
 * blocks and panel solves; trailing updates on MFMA in FP64 or (MIXED) FP32.
 * d_ws: workspace of bd_workspace_size(BD_OP_CHOLESKY, n, prec) bytes.
 * A non-positive pivot sets potrf_info (see bd_get_info). */
bd_status_t bd_cholesky(bd_handle_t h, int64_t n, double* d_A, int64_t ld, bd_precision_t prec,
                        void* d_ws, size_t ws_bytes);

/* Adjoint of the factorisation (Eq. 10), in the matrix form of Murray
 * (2016): for the gradient Lbar of a scalar phi in the lower-triangular
 * entries of B (d_Lbar, n x n column-major, ldb >= n; its strict upper part
 * is not read), writes to d_Abar (n x n, lda >= n, every element) the
 * symmetric gradient of phi in A = B B^T,
 *   Abar = (P + P^T)/2,  P = B^-T Phi(B^T Lbar) B^-1,
 * Phi keeping the lower triangle with the diagonal halved, so that
 * d phi = <Abar, dA> for every symmetric dA.  d_L: the lower triangle of B
 * (bd_cholesky's output; the strict upper part is not read).  FP64 on
 * matrix cores; d_ws: bd_workspace_size(BD_OP_CHOLESKY_ADJOINT, n, FP64)
 * bytes.  n <= 65535. */
bd_status_t bd_cholesky_adjoint(bd_handle_t h, int64_t n, const double* d_L, int64_t ld,
                                const double* d_Lbar, int64_t ldb, double* d_Abar, int64_t lda,
                                void* d_ws, size_t ws_bytes);

/* y = c_B B xi: the Brownian term of Eq. 6 times dt.  xi_e for e = 3i+alpha
 * comes from Philox4x64-10 with key (seed, chain_id) and counter
 * (e/4, step, 0, 0), lane e%4; Gaussian by Box-Muller on lane pairs
 * (0,1), (2,3), or 2u-1 in the paper's uniform mode.  d_L: the lower
 * triangle of B (n x n, ld >= n); d_y: n; d_xi_out: n or NULL. */
bd_status_t bd_brownian(bd_handle_t h, const bd_params_t* p, int64_t step, const double* d_L,
                        int64_t ld, double* d_y, double* d_xi_out, void* d_ws, size_t ws_bytes);

/* bd_brownian without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  The same kernels and results as bd_brownian; their
 * scratch (xi and the per-tile partial sums, 4.8 MB) is a fixed device array
 * of the library, one per GPU, held until the process ends, sized for
 * n = 3N <= 12288 (BD_ERR_UNSUPPORTED above).  The call allocates nothing.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two streams, two handles or two host threads at once) race and give
 * wrong results; calls ordered on one stream are safe.  Arguments as for
 * bd_brownian. */
bd_status_t bd_brownian_noalloc(bd_handle_t h, const bd_params_t* p, int64_t step,
                                const double* d_L, int64_t ld, double* d_y, double* d_xi_out);

/* Rigid-rod constraint: tensions T_k along the rod directions u_k of d_x_old
 * such that x^{t+dt} = x* - dt D(x_old) Delta^T U T has |Q_k| = b for every
 * rod (the infinite-stiffness limit of the semi-implicit spring update of
 * Eqs. 13-17, every tension coupled through the full D of Eqs. 7-9).
 * Inexact Newton from T = 0; each correction by GMRES right-preconditioned
 * with the tridiagonal part of the Jacobian; products with D are
 * matrix-free.  d_x_pred_inout: x* in, x^{t+dt} out (N x 3); d_T_out: N-1
 * or NULL.  N <= 8193 (BD_ERR_UNSUPPORTED above).  The call synchronises
 * the stream a few times to stop the iteration once it has converged. */
bd_status_t bd_constrain(bd_handle_t h, const bd_params_t* p, const double* d_x_old,
                         double* d_x_pred_inout, double* d_T_out, void* d_ws, size_t ws_bytes);

/* Adjoint of the tension solve (bd_constrain), by the implicit-function
 * theorem.  The constraint maps x* to x^{t+dt} = x* - dt D Delta^T U T with
 * T fixed by g_k = |Q_k|^2 - b^2 = 0, Q = Delta x^{t+dt} (U: the rod
 * directions of d_x_old, D = D(x_old)).  For the gradient d_xbar (N x 3) of
 * a scalar in x^{t+dt} (d_x_new, bd_constrain's output), writes
 *   z = xbar - 2 Delta^T (Q mu),  J^T mu = -dt U^T Delta D xbar,
 * with J = dg/dT = -2 dt diag(Q)^T Delta D Delta^T U, to d_z (N x 3): the
 * gradient of that scalar in x* (and in anything x^{t+dt} depends on at
 * fixed T).  J^T mu = rhs is solved by GMRES right-preconditioned with the
 * tridiagonal part of J^T (J with u and Q exchanged), products with D
 * matrix-free, to a residual of newton_tol |rhs| (BD_ERR_NO_CONVERGE in
 * bd_get_info otherwise).  d_ws: bd_workspace_size(BD_OP_CONSTRAIN, 3N)
 * bytes; N <= 8193.  Synchronises the stream a few times, as bd_constrain. */
bd_status_t bd_constrain_adjoint(bd_handle_t h, const bd_params_t* p, const double* d_x_old,
                                 const double* d_x_new, const double* d_xbar, double* d_z,
                                 void* d_ws, size_t ws_bytes);

/* Adjoint of one FP64 step (bd_step at BD_PREC_FP64 with the same
 * arguments), at fixed noise: for the gradient d_xbar of a scalar in
 * x^{t+dt}, overwrites d_xbar with its gradient in x^t (d_x, N x 3, not
 * modified) and adds its gradients in h* to d_hbar[0] and in kappa
 * (row-major) to d_kbar[0..8].  The forward step is recomputed from d_x
 * (D, B, xi, y, x*, T, x^{t+dt}); then the tension solve's adjoint gives z,
 * the gradient in x^{t+dt} at fixed T, and z is carried back through
 * x^{t+dt} = x* + dt D(x) f(T, u(x)) (Dbar = dt z f^T and the rod
 * directions), through x* = x + dt kappa x + c_B B xi (Lbar = c_B z xi^T),
 * the factorisation (bd_cholesky_adjoint's Abar added into Dbar) and the
 * assembly (bd_rpy_assemble_adjoint of Dbar, Eqs. 7-9).  d_ws:
 * bd_workspace_size(BD_OP_STEP_ADJOINT, 3N, FP64) bytes (about four n x n
 * matrices plus bd_step's workspace); N <= 8193.  Status (pivot, tension or
 * adjoint non-convergence, coincident beads) via bd_get_info. */
bd_status_t bd_step_adjoint(bd_handle_t h, const bd_params_t* p, int64_t step, const double* d_x,
                            double* d_xbar, double* d_hbar, double* d_kbar, void* d_ws,
                            size_t ws_bytes);

/* One timestep of one chain: steps 1-5 above with noise counter `step`.
 * d_x_inout: N x 3 (N <= 8193, BD_ERR_UNSUPPORTED above; the paper's
 * longest chain, 6400 rods, is N = 6401), advanced in place, or left
 * unchanged when the step fails (non-positive pivot, tensions not
 * converged; see bd_get_info).  The tension solve synchronises the stream
 * a few times, unless the handle was created with the environment variable
 * BDRPY_CONSTRAIN=onelaunch: then the whole step is asynchronous on the
 * stream (the solve runs as one launch with grid barriers, at most one
 * workgroup per compute unit, which must all be resident at once) and can
 * be captured in a HIP graph; a replay repeats the captured noise counter. */
bd_status_t bd_step(bd_handle_t h, const bd_params_t* p, int64_t step, double* d_x_inout,
                    bd_precision_t prec, void* d_ws, size_t ws_bytes);

/* One timestep with the paper's own stiff Fraenkel springs (Eq. 3) in
 * place of rigid rods: D, B and y = c_B B xi as in bd_step, then the
 * semi-implicit link update of Eqs. 13-17.  Spring k pulls bead k with
 * F_k = K (|Q_k| - b) Q_k/|Q_k| (K = k_spring > 0) and bead k+1 with -F_k;
 * with v = D f (f the net bead forces at t, matrix-free product)
 *   Y_k = Q_k + dt [kappa.Q_k + v_{k+1} - v_k + 2 F_k] + y_{k+1} - y_k,
 *   |Q_k'| = (|Y_k| + 2 dt K b) / (1 + 2 dt K) along Y_k (Eq. 17);
 * bead 0 moves by its explicit equation of motion,
 * x_0' = x_0 + dt (kappa.x_0 + v_0) + y_0, and x_{k+1}' = x_k' + Q_k'.
 * d_x_inout: N x 3 (N <= 8193, BD_ERR_UNSUPPORTED above), advanced in
 * place; d_ws: bd_workspace_size(BD_OP_STEP, 3N, prec) bytes.  max_rod_err
 * of bd_get_info receives max_k | |Q_k'|/b - 1 |; the Newton fields are 0.
 * A non-positive pivot leaves the positions unchanged. */
bd_status_t bd_step_fraenkel(bd_handle_t h, const bd_params_t* p, double k_spring, int64_t step,
                             double* d_x_inout, bd_precision_t prec, void* d_ws, size_t ws_bytes);

/* Observables of the paper's flow studies (Section 5) for n_chains chains
 * packed in d_x: chain c is beads d_offsets[c] .. d_offsets[c+1]-1 (rows of
 * d_x, N x 3 each; d_offsets: device, n_chains + 1 increasing values, every
 * chain at least one bead; the call does not check them).  d_out (device,
 * 4 n_chains doubles) receives per chain the end-to-end vector
 * R_ee = r_{N-1} - r_0 (three components: stretch |R_ee| / ((N-1) b),
 * R_ee,y, ...) and R_g^2 = (1/N) sum_i |r_i - r_cm|^2.  Asynchronous on
 * the handle's stream. */
bd_status_t bd_observables(bd_handle_t h, int32_t n_chains, const double* d_x,
                           const int64_t* d_offsets, double* d_out);

/* Kramers stress (Section 5, Eq. 28) and first normal stress difference
 * (Eq. 29) of n_chains chains packed in d_x as for bd_observables (d_x,
 * d_offsets: the same layout; every chain at least two beads, not checked).
 * Per chain, over its M = N - 1 connectors Q_k = r_{k+1} - r_k,
 *   tau = sum_k F_k Q_k^T - M I,   N1 = tau_xx - tau_yy   (units of kT),
 * with F_k the connector's force along Q_k: for rigid rods (d_T given)
 * the tension T_k times Q_k/|Q_k|, d_T packing chain c's M tensions (as
 * bd_constrain returns them, at the start-of-step positions) from index
 * d_offsets[c] - c; for the paper's Fraenkel springs (d_T = NULL) the
 * force of Eq. 3, K (|Q_k| - b) Q_k/|Q_k| with K = k_spring > 0.  The sign
 * of the isotropic part is the one that makes tau vanish at equilibrium
 * (<Q F^T> = kT I per connector); N1 does not depend on it.  d_out (device,
 * 7 n_chains doubles) receives per chain tau_xx, tau_yy, tau_zz, tau_xy,
 * tau_xz, tau_yz, N1; the ensemble average is the mean over chains.
 * Asynchronous on the handle's stream. */
bd_status_t bd_stress(bd_handle_t h, int32_t n_chains, const double* d_x,
                      const int64_t* d_offsets, const double* d_T, double k_spring, double b,
                      double* d_out);

/* Synchronise the handle's stream and return the info of the last call. */
bd_status_t bd_get_info(bd_handle_t h, bd_info_t* out);

/* ---- Ensembles: many independent chains advanced together.  The paper's
 * production runs average over many independent chains with no exchange
 * between them (Section 4, one chain per MPI process; Section 5, 128 and
 * 1000 chains); here every chain of an ensemble shares each launch of each
 * kernel (the chain is the third grid dimension), so a step of the whole
 * ensemble costs one launch sequence.
 *
 * p[0..n_chains-1]: per-chain parameters (sizes, flows, seeds may all
 * differ; 1 <= n_chains <= 65535, every N <= 4097).  Positions are packed:
 * chain c is the N_c x 3 block starting at row sum_{c' < c} N_c' of d_x.
 * A step of the ensemble advances every chain as bd_step with the same
 * parameters and `step` would (the same kernels, arithmetic and reduction
 * orders) except that every chain's Cholesky takes steps of four panels
 * (environment BDRPY_ENS_PANELS=2 at creation: two).  bd_step takes
 * four-panel steps while more than BDRPY_WIDE_ROWS rows remain (read at
 * bd_create, default 4096) and two after, so with BDRPY_WIDE_ROWS=0 (or
 * BDRPY_ENS_PANELS=2 and n <= 4096) each chain's result is bitwise that of
 * bd_step; otherwise the two differ only in rounding order. */
typedef struct bd_ensemble_s* bd_ensemble_t;

/* Bytes of device workspace for the ensemble p[0..n_chains-1] in `prec`. */
bd_status_t bd_ensemble_workspace_size(int32_t n_chains, const bd_params_t* p,
                                       bd_precision_t prec, size_t* bytes);

/* Build an ensemble on handle h (its stream, lookahead stream and events).
 * p is copied.  d_x (3 sum_c N_c doubles) and d_ws (>= the size above) stay
 * caller-owned and bound to the ensemble until bd_ensemble_destroy.  The
 * ensemble allocates a device table of its chains and one status block per
 * chain (BD_ERR_ALLOC if that fails). */
bd_status_t bd_ensemble_create(bd_handle_t h, int32_t n_chains, const bd_params_t* p,
                               bd_precision_t prec, double* d_x, void* d_ws, size_t ws_bytes,
                               bd_ensemble_t* out);

/* One timestep of every chain with noise counter `step`; d_x is advanced in
 * place.  A chain whose step fails (non-positive pivot, tensions not
 * converged) keeps its positions; its status
 * and those of the others are reported by bd_ensemble_get_info.  The call
 * synchronises the stream a few times during the tension solves. */
bd_status_t bd_ensemble_step(bd_ensemble_t e, int64_t step);

/* Capture one step of the ensemble in a HIP graph; from then on
 * bd_ensemble_step replays it (one graph launch per step, no host round
 * trip: asynchronous on the handle's stream).  The captured step differs
 * from the plain one in two ways: its noise counter is kept on the device
 * (set from `step` when a call does not follow the previous one, advanced
 * by each replay), and its tension solves take exactly max_products
 * (product with D, controller) pairs (0: 5/4 of the products the previous
 * plain step needed plus 4), launches for a converged chain returning at
 * once; a chain that needs more reports BD_ERR_NO_CONVERGE in
 * bd_ensemble_get_info and keeps its positions.  Results are otherwise
 * bitwise those of plain steps.  Not with profiling on (BD_ERR_PARAM);
 * BD_ERR_HIP if the capture fails. */
bd_status_t bd_ensemble_capture(bd_ensemble_t e, int32_t max_products);

/* Synchronise and write the info of the last step of every chain to
 * out[0..n_chains-1], in the order of p. */
bd_status_t bd_ensemble_get_info(bd_ensemble_t e, bd_info_t* out);
bd_status_t bd_ensemble_destroy(bd_ensemble_t e);

/* Per-kernel timing (instrumentation, not part of the method).  Between
 * bd_profile_begin and bd_profile_end every kernel the handle launches is
 * bracketed by HIP events on the handle's stream.  bd_profile_end
 * synchronises, writes up to max_out entries (one per kernel name: launch
 * count and summed duration), sets *n_out to the number of distinct kernels
 * and switches timing off. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} bd_kernel_stat_t;

bd_status_t bd_profile_begin(bd_handle_t h);
bd_status_t bd_profile_end(bd_handle_t h, bd_kernel_stat_t* out, int32_t max_out, int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif /* BDRPY_H */
