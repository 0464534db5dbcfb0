// RPY diffusion-tensor assembly (Eqs. 7-9), column-major D with ld.
//
// One work-item evaluates one 3x3 block D_ij (one sqrt, one divide chain)
// and stores its three columns; consecutive work-items take consecutive
// beads i, so each of the three column stores of a wavefront covers a
// contiguous 64*24-byte run of one matrix column.  With BD_FILL_LOWER only
// blocks with i >= j are touched and the diagonal block keeps its lower
// part only.
#include "common.hpp"
#include "profile.hpp"
#include "rpy_device.hpp"

namespace bd {

namespace {

constexpr int kRpyThreads = 256;

__global__ __launch_bounds__(kRpyThreads) void rpy_assemble_kernel(
    const double* __restrict__ x, double* __restrict__ D, int64_t ld, int N, double hstar,
    double a, int fill_full) {
  const int j = blockIdx.y;                         // column bead
  const int i = blockIdx.x * kRpyThreads + threadIdx.x;  // row bead
  if (!fill_full && (blockIdx.x + 1) * kRpyThreads <= j) return;  // block entirely above
  if (i >= N) return;
  if (!fill_full && i < j) return;
  double blk[3][3];
  if (i == j) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) blk[r][c] = (r == c) ? 1.0 : 0.0;
  } else {
    const double R0 = x[3 * i] - x[3 * j];
    const double R1 = x[3 * i + 1] - x[3 * j + 1];
    const double R2c = x[3 * i + 2] - x[3 * j + 2];
    const double R2 = R0 * R0 + R1 * R1 + R2c * R2c;
    double cI, cRR;
    rpy_coeffs(R2, hstar, a, cI, cRR);
    const double Rv[3] = {R0, R1, R2c};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) blk[r][c] = (r == c ? cI : 0.0) + cRR * Rv[r] * Rv[c];
  }
  const int64_t row0 = 3 * (int64_t)i;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double* col = D + (3 * (int64_t)j + c) * ld + row0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (!fill_full && i == j && r < c) continue;  // strict upper part of the diagonal block
      col[r] = blk[r][c];
    }
  }
}

}  // namespace

hipError_t launch_rpy_assemble(hipStream_t s, const bd_params_t& p, const double* x, double* D,
                               int64_t ld, int fill) {
  const int N = p.n_beads;
  dim3 grid((N + kRpyThreads - 1) / kRpyThreads, N);
  BD_LAUNCH("rpy_assemble", rpy_assemble_kernel, grid, dim3(kRpyThreads), 0, s, x, D, ld, N, p.hstar,
                     p.a, fill == BD_FILL_FULL ? 1 : 0);
  return hipGetLastError();
}

}  // namespace bd
