// Internal declarations shared by the HIP translation units of libbdrpy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/bdrpy.h"

namespace bd {

// Device-resident status and Newton state of one handle.  The first block
// mirrors bd_info_t so it can be copied out verbatim.
struct DevState {
  int32_t status;
  int32_t newton_iters;
  int64_t potrf_info;
  double max_rod_err;
  double last_newton_res;
  int32_t krylov_iters;
  int32_t reserved;
  // end of the bd_info_t mirror
  int32_t done;  // 1 once the tension iteration has finished (either way)
  int32_t pad[3];
};
static_assert(sizeof(bd_info_t) == 40, "bd_info_t layout");

// Launch-bound / common constants
constexpr int kWave = 64;

// Cholesky blocking: trailing-update block (panel width) and MFMA tile.
constexpr int kNB = 128;       // panel width
constexpr int kTile = 128;     // trailing-update workgroup tile (square)
constexpr int kMaxStep = 4 * kNB;  // widest factorisation step (four panels)

// ---------------------------------------------------------------- launchers
// rpy.hip
hipError_t launch_rpy_assemble(hipStream_t s, const bd_params_t& p, const double* x, double* D,
                               int64_t ld, int fill);

hipError_t launch_rpy_adjoint(hipStream_t s, const bd_params_t& p, const double* x,
                              const double* Dbar, int64_t ld, double* xbar, double* hbar,
                              double* hpart, DevState* st);

// cholesky.hip
size_t cholesky_workspace_bytes(int64_t n, bd_precision_t prec);
// With xi and ypart non-null the noise product y = cB L xi follows the
// factorisation: one pass stores each panel's share of every row below it
// in ypart (one row of n per panel, noise_part_bytes(n)), a second adds
// them in panel order with the diagonal blocks' share (the sums, in their
// order, of the ensemble's fused noise product).
hipError_t launch_cholesky(hipStream_t s, hipStream_t aux, hipEvent_t ev[4], int64_t n, double* A,
                           int64_t ld, bd_precision_t prec, void* ws, DevState* st,
                           int max_panels, int64_t wide_rows, bool tile_potrf,
                           const double* xi = nullptr, double* y = nullptr, double cB = 0.0,
                           double* ypart = nullptr);

// adjoint.hip
size_t cholesky_adjoint_workspace_bytes(int64_t n);
hipError_t launch_cholesky_adjoint(hipStream_t s, int64_t n, const double* L, int64_t ld,
                                   int64_t sL, const double* Lbar, int64_t ldb, int64_t sLb,
                                   double* Abar, int64_t lda, int64_t sAb, double alpha,
                                   double beta, int batch, void* ws);

// The step adjoint's local parts (adjoint.hip): rod forces f(T, u(x)),
// Dbar = dt z f^T (every element), the gradient through u, the predictor
// and kappa (xbar overwritten, kbar accumulated), and the final sums.
hipError_t launch_rod_forces(hipStream_t s, const double* x, const double* T, int N, double* f);
hipError_t launch_rank1(hipStream_t s, const double* z, const double* f, double c, int64_t n,
                        double* Dbar, int64_t ld);
hipError_t launch_step_adjoint_local(hipStream_t s, const bd_params_t& p, const double* x,
                                     const double* T, const double* z, const double* Dz,
                                     double* xbar, double* kbar);
hipError_t launch_step_adjoint_finish(hipStream_t s, int64_t n, const double* xbD,
                                      const double* hstep, double* xbar, double* hbar);

// brownian.hip
size_t brownian_workspace_bytes(int64_t n);
hipError_t launch_brownian(hipStream_t s, const bd_params_t& p, int64_t step, const double* L,
                           int64_t ld, double* y, double* xi_out, void* ws);
hipError_t launch_predictor(hipStream_t s, const bd_params_t& p, const double* x, const double* y,
                            double* xs);
// The device address of this device's fixed scratch array of the
// allocation-free noise product (looked up once per device; the caller has
// made `device` current), and the largest matrix order it holds.
hipError_t brownian_scratch_init(int device, void** out);
int64_t brownian_scratch_max_n();
// The noise coefficient c_B (sqrt(2 dt), or sqrt(6 dt) for the paper's
// uniform noise); the noise xi of one step.
double noise_coeff(const bd_params_t& p);
hipError_t launch_noise(hipStream_t s, const bd_params_t& p, int64_t step, double* xi);
hipError_t launch_brownian_adjoint(hipStream_t s, const bd_params_t& p, const double* L,
                                   int64_t ld, const double* xi, const double* ybar,
                                   double* Lbar, int64_t ldb, double* xibar);
// Only the L part of it: Lbar = c_B tril(ybar xi^T).
hipError_t launch_brownian_adjoint_lbar(hipStream_t s, const bd_params_t& p, const double* xi,
                                        const double* ybar, double* Lbar, int64_t ldb);

// constrain.hip
size_t constrain_workspace_bytes(int64_t n_beads);
// n_cu > 0: the whole solve in one launch of at most n_cu workgroups (no
// host round trip, capturable); n_cu = 0: alternating launches polled by
// the host.
hipError_t launch_constrain(hipStream_t s, const bd_params_t& p, const double* x_old, double* xs,
                            double* T_out, void* ws, DevState* st, DevState* host_state_pinned,
                            int* pairs_hint, int n_cu);

// Adjoint of the tension solve (bd_constrain_adjoint): z = xbar - 2 Delta^T
// (Q mu) with J^T mu = -dt U^T Delta D(x_old) xbar; polls like
// launch_constrain.  ws: constrain_workspace_bytes(N).
hipError_t launch_constrain_adjoint(hipStream_t s, const bd_params_t& p, const double* x_old,
                                    const double* x_new, const double* xbar, double* z, void* ws,
                                    DevState* st, DevState* host_state);

// r = D(x) f, matrix-free (the tension solve's product); returns at once
// when st is given and st->done is set.
hipError_t launch_dmatvec(hipStream_t s, const bd_params_t& p, const double* x, const double* f,
                          double* r, const DevState* st);

// observables.hip
hipError_t launch_observables(hipStream_t s, int32_t n_chains, const double* x,
                              const int64_t* off, double* out);
// Kramers stress and N1 of packed chains: rigid rods when T (packed
// tensions, chain c's at offset off[c] - c) is given, else springs of
// stiffness K and rest length b.
hipError_t launch_stress(hipStream_t s, int32_t n_chains, const double* x, const int64_t* off,
                         const double* T, double K, double b, double* out);

// fraenkel.hip
int fraenkel_max_beads();
hipError_t launch_spring_forces(hipStream_t s, const double* x, int N, double K, double b,
                                double* f);
hipError_t launch_fraenkel_update(hipStream_t s, const bd_params_t& p, double K, double* x,
                                  const double* v, const double* y, DevState* st);

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
// One FP32 panel copy of the mixed-precision factorisation: n x kMaxStep
// floats plus kP32Tail of slack, since the trailing update's 16-byte
// operand loads may run up to three floats past a column's last row.
constexpr int kP32Tail = 64;
// Its column stride: n rounded up to 16 bytes, so that columns stay aligned.
__host__ __device__ inline int64_t p32_ld(int64_t n) { return (n + 3) / 4 * 4; }
// The noise product's partial sums: one row of n per panel.
inline size_t noise_part_bytes(int64_t n) {
  return align_up(sizeof(double) * (size_t)((n + kNB - 1) / kNB) * (size_t)n, 256);
}
__host__ __device__ inline size_t p32_copy_bytes(int64_t n) {
  return align_up(sizeof(float) * ((size_t)p32_ld(n) * kMaxStep + kP32Tail), 256);
}

// ---------------------------------------------------------------- ensembles
// One chain of an ensemble as the batched kernels see it: the chain's
// parameters and the absolute device addresses of its data.  A batched
// launch takes a table of these and works on chain blockIdx.z of it; each
// workgroup derives its chain's sizes from the entry and returns at once if
// the chain has no work at its grid position.
struct ChainDesc {
  int32_t N;          // beads
  int32_t uniform;    // 1: the paper's uniform noise (Eq. 2), 0: Gaussian
  int64_t n;          // 3N
  int64_t ld;         // leading dimension of D
  double hstar, a, b, dt, tol, cB;  // cB: noise coefficient sqrt(2 dt) or sqrt(6 dt)
  int32_t maxit;
  int32_t index;      // position of the chain in the caller's order
  double kappa[9];
  uint64_t seed, chain_id;
  double* x;          // N x 3 positions (in the packed array of the ensemble)
  double* D;          // n x ld diffusion tensor, then its factor
  double* W;          // Cholesky: inverses of the diagonal sub-blocks
  float* P32[2];      // Cholesky MIXED: FP32 panel copies of alternate steps (p32_ld(n) x kMaxStep)
  double* xi;         // noise (n)
  double* y;          // Brownian displacement (n), formed by the factorisation
  double* ypart;      // its panels' partial sums (noise_part_bytes(n))
  double* xs;         // predictor / new positions (N x 3)
  void* cons;         // tension-solve workspace
  DevState* st;       // status of this chain
};

// Flattened grids: chain c owns workgroups prefix[c] .. prefix[c+1]-1 of a
// launch (prefix has count + 1 entries, prefix[0] = 0); returns c for
// workgroup t by bisection (wave-uniform scalar loads).
__device__ __forceinline__ int find_chain(const int32_t* __restrict__ prefix, int count, int t) {
  int lo = 0, hi = count;  // prefix[lo] <= t < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Bytes each chain of an ensemble needs in the Cholesky workspace.
size_t cholesky_batched_workspace_bytes(int64_t n, bd_precision_t prec);
// Flattened grids of the batched factorisation: one prefix array (chain ->
// first workgroup) per launch, in launch order.  A recording pass at plan
// creation builds them on the host (no launches); they are uploaded once
// and every step reads them back in the same order.
struct BatchTables {
  std::vector<int32_t> host;
  const int32_t* dev = nullptr;
  size_t cur = 0;
  bool record = false;
};
// The chains of `cd` (device table, `cd_host` its host copy) ordered by
// decreasing n, `count` of them; every chain is factored in place with the
// schedule of launch_cholesky at `panels` (2 or 4) panels per step; with
// `noise`, each chain's y += cB L xi on the way (as launch_cholesky).
hipError_t launch_cholesky_batched(hipStream_t s, hipStream_t aux, hipEvent_t ev[4],
                                   const ChainDesc* cd, const ChainDesc* cd_host, int count,
                                   bd_precision_t prec, int panels, BatchTables* tb,
                                   bool noise = false);
// Flattened grid of the assembly: workgroups per chain, and the launcher
// taking the prefix array over the table.
int rpy_batched_blocks(int n_beads);
hipError_t launch_rpy_assemble_batched(hipStream_t s, const ChainDesc* cd, int count,
                                       const int32_t* prefix, int blocks);
// Each chain's noise xi (d_step non-null: the step counter from device
// memory).
hipError_t launch_noise_batched(hipStream_t s, const ChainDesc* cd, int count, int64_t max_n,
                                int64_t step, const int64_t* d_step = nullptr);
hipError_t launch_predictor_batched(hipStream_t s, const ChainDesc* cd, int count, int max_beads);
// Runs the tension solve of every chain; returns once every chain's
// iteration has finished (polls the `count` states at `st`, which are
// contiguous, through the pinned `host_states`).
// mv_prefix: workgroups of the matrix-free product per chain, flattened
// (constrain_mv_blocks(N) for chain c of the table), mv_blocks in all.
int constrain_mv_blocks(int n_beads);
// budget > 0: exactly `budget` (product, controller) pairs, no host round
// trip (a chain not finished by then reports BD_ERR_NO_CONVERGE); 0: polled.
hipError_t launch_constrain_batched(hipStream_t s, const ChainDesc* cd, int count, int max_beads,
                                    const int32_t* mv_prefix, int mv_blocks, int newton_maxit,
                                    DevState* st, DevState* host_states, int* pairs_hint,
                                    int budget = 0);

}  // namespace bd
