/*
 * bdo.h -- plain CPU FP64 oracle for one timestep of bead-rod Brownian
 * dynamics with Rotne-Prager-Yamakawa hydrodynamic interactions
 * (arXiv 2208.06559, Sections 3-4).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.  It shares no header, table or
 * helper with the HIP implementation.
 *
 * Conventions (all arrays are caller-owned host memory, FP64 unless noted):
 *   N beads r_0..r_{N-1} (the paper numbers its beads 0..N, so its "N+1" is
 *   our N); N-1 rods Q_k = r_{k+1} - r_k; matrix order n = 3N with scalar
 *   index e = 3i + alpha (bead-major, component-minor: the block layout of
 *   the paper's two-bead example, Section 4 "Diffusion Tensor and
 *   Multiplication").
 *   Positions x: row-major N x 3.  Matrices: column-major, leading dim ld.
 *   Units: zeta = kT = 1 (so D_ii = I, Eq. 7), lengths in Kuhn steps.
 */
#ifndef BDO_H
#define BDO_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { BDO_OK = 0, BDO_ERR_PARAM = 1, BDO_ERR_NOT_SPD = 2, BDO_ERR_NO_CONVERGE = 3 };
enum { BDO_NOISE_GAUSSIAN = 0, BDO_NOISE_UNIFORM_PAPER = 1 };
enum { BDO_FILL_LOWER = 0, BDO_FILL_FULL = 1 };
enum { BDO_PURPOSE_NOISE = 0 };

typedef struct {
  int32_t n_beads;      /* N >= 2                                          */
  int32_t noise;        /* BDO_NOISE_*                                     */
  double b;             /* rod length > 0                                  */
  double hstar;         /* HI strength, 0 <= h* <= a (0: HI off)           */
  double a;             /* bead radius > 0                                 */
  double dt;            /* timestep > 0                                    */
  double kappa[9];      /* row-major velocity gradient transpose, v = kappa.r */
  uint64_t seed;        /* Philox key word 0                               */
  uint64_t chain_id;    /* Philox key word 1                               */
  double newton_tol;    /* stop when max_k | |Q_k|/b - 1 | <= tol          */
  int32_t newton_maxit; /* >= 1, Newton steps before NO_CONVERGE          */
  int32_t pad_;
} bdo_params;

typedef struct {
  int32_t status;         /* BDO_*                                         */
  int32_t newton_iters;   /* Newton steps performed                        */
  int64_t potrf_info;     /* 0 or 1-based column of the failing pivot      */
  double max_rod_err;     /* max_k | |Q_k|/b - 1 | after the step          */
  double last_newton_res; /* max_k | |Q_k|^2 - b^2 | at the last check     */
  int32_t krylov_iters;   /* GMRES iterations summed over Newton steps     */
  int32_t pad_;
} bdo_info;

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) applied once to the
 * 256-bit counter ctr with the 128-bit key; writes 4 x u64. */
void bdo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Noise vector of length n for (seed, chain_id, step): Gaussian N(0,1)
 * (Box-Muller) or the paper's uniform on [-1,1] (Eq. 2).  Element e uses
 * Philox block e/4 with counter (e/4, step, purpose, 0), lane e%4. */
void bdo_noise(const bdo_params* p, int64_t step, int64_t n, double* xi);

/* One 3x3 RPY block D_ij for Rvec = r_i - r_j, i != j (Eqs. 8-9),
 * row-major out[9]. */
void bdo_rpy_block(double hstar, double a, const double Rvec[3], double out[9]);

/* Assemble D (n x n, column-major, ld >= n) from x (N x 3): Eqs. 7-9.
 * fill = LOWER writes the lower triangle incl. diagonal only. */
int bdo_rpy_assemble(const bdo_params* p, const double* x, double* D, int64_t ld, int32_t fill);

/* Unblocked Cholesky (Crout order), lower, in place: Eq. 10.  Reads the
 * lower triangle of A; the strict upper triangle is left untouched.
 * Returns 0, or the 1-based column of the first non-positive pivot. */
int64_t bdo_cholesky(int64_t n, double* A, int64_t ld);

/* y = c_B * L * xi with c_B = sqrt(2 dt) (Gaussian) or sqrt(6 dt)
 * (uniform, Eq. 2 times dt), xi = bdo_noise(step).  xi_out may be NULL. */
int bdo_brownian(const bdo_params* p, int64_t step, const double* L, int64_t ld,
                 double* y, double* xi_out);

/* Rigid-rod tension solve and corrector: inexact Newton from T = 0, each
 * step solved by GMRES right-preconditioned with the tridiagonal part of the
 * Jacobian; the residual always uses the full D (matrix-free).
 * x_old: positions at t (N x 3); x_pred_inout: predictor x* in, x^{t+dt}
 * out; T_out (N-1, may be NULL). */
int bdo_constrain(const bdo_params* p, const double* x_old, double* x_pred_inout,
                  double* T_out, bdo_info* info);

/* Same root by Newton with the dense Jacobian and LU with partial
 * pivoting (used to check the band iteration). */
int bdo_constrain_dense(const bdo_params* p, const double* x_old, double* x_pred_inout,
                        double* T_out, bdo_info* info);

/* One full timestep: assemble, factor, noise, predictor, constraint. */
int bdo_step(const bdo_params* p, int64_t step, double* x_inout, bdo_info* info);

/* One timestep with the paper's own stiff Fraenkel springs (Eq. 3) in
 * place of rigid rods: the semi-implicit link update of Eqs. 13-17.
 * Spring k (k = 0..N-2) acts on bead k with F_k = K (|Q_k| - b) Q_k/|Q_k|
 * and on bead k+1 with -F_k; f = the net bead forces at t.  With v = D f,
 *   Y_k = Q_k + dt [kappa.Q_k + v_{k+1} - v_k + 2 F_k] + y_{k+1} - y_k  (Eq. 14)
 *   |Q_k'| = (|Y_k| + 2 dt K b) / (1 + 2 dt K),  Q_k' = Y_k |Q_k'|/|Y_k|  (Eqs. 15-17)
 * and the positions: bead 0 by its explicit equation of motion,
 * x_0' = x_0 + dt (kappa.x_0 + v_0) + y_0, then x_{k+1}' = x_k' + Q_k'.
 * info->max_rod_err receives max_k | |Q_k'|/b - 1 |.  k_spring > 0. */
int bdo_step_fraenkel(const bdo_params* p, double k_spring, int64_t step, double* x_inout,
                      bdo_info* info);

/* nsteps consecutive steps (step0, step0+1, ...) of one chain. */
int bdo_run(const bdo_params* p, int64_t step0, int64_t nsteps, double* x_inout, bdo_info* info);

/* Independent chains c = 0..nchains-1 with chain_id = chain_ids[c] and
 * positions x + c*3N, each advanced nsteps from step0; chains run in
 * parallel.  status_out[c] receives each chain's final status. */
int bdo_run_many(const bdo_params* p, int32_t nchains, const uint64_t* chain_ids,
                 int64_t step0, int64_t nsteps, double* x, int32_t* status_out);

/* OpenMP threads the oracle's parallel loops use. */
int bdo_num_threads(void);
void bdo_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
