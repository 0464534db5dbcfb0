// Internal declarations shared by the HIP translation units of libbdrpy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// cholesky.hip
size_t cholesky_workspace_bytes(int64_t n, bd_precision_t prec);
hipError_t launch_cholesky(hipStream_t s, hipStream_t aux, hipEvent_t ev[4], int64_t n, double* A,
                           int64_t ld, bd_precision_t prec, void* ws, DevState* st,
                           int max_panels, int64_t wide_rows, bool tile_potrf);

// brownian.hip
size_t brownian_workspace_bytes(int64_t n);
hipError_t launch_brownian(hipStream_t s, const bd_params_t& p, int64_t step, const double* L,
                           int64_t ld, double* y, double* xi_out, void* ws);
hipError_t launch_predictor(hipStream_t s, const bd_params_t& p, const double* x, const double* y,
                            double* xs);

// constrain.hip
size_t constrain_workspace_bytes(int64_t n_beads);
hipError_t launch_constrain(hipStream_t s, const bd_params_t& p, const double* x_old, double* xs,
                            double* T_out, void* ws, DevState* st, DevState* host_state_pinned,
                            int* pairs_hint);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace bd
