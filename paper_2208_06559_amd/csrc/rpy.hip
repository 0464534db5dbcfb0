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

__device__ __forceinline__ void rpy_assemble_body(int bx, int j, const double* __restrict__ x,
                                                  double* __restrict__ D, int64_t ld, int N,
                                                  double hstar, double a, int fill_full) {
  const int i = bx * kRpyThreads + threadIdx.x;  // row bead; j is the column bead
  if (!fill_full && (bx + 1) * kRpyThreads <= j) return;  // block entirely above
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

__global__ __launch_bounds__(kRpyThreads) void rpy_assemble_kernel(
    const double* __restrict__ x, double* __restrict__ D, int64_t ld, int N, double hstar,
    double a, int fill_full) {
  rpy_assemble_body(blockIdx.x, blockIdx.y, x, D, ld, N, hstar, a, fill_full);
}

// Ensembles: lower triangles, one flattened grid; chain c owns
// rpy_batched_blocks(N_c) workgroups, (column bead j, row block bx) each.
__global__ __launch_bounds__(kRpyThreads) void rpy_assemble_batched_kernel(
    const ChainDesc* __restrict__ cd, const int32_t* __restrict__ prefix, int count) {
  const int ci = find_chain(prefix, count, blockIdx.x);
  const ChainDesc& c = cd[ci];
  const int N = c.N;
  const int nbx = (N + kRpyThreads - 1) / kRpyThreads;
  const int local = blockIdx.x - prefix[ci];
  rpy_assemble_body(local % nbx, local / nbx, c.x, c.D, c.ld, N, c.hstar, c.a, 0);
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

int rpy_batched_blocks(int n_beads) {
  return n_beads * ((n_beads + kRpyThreads - 1) / kRpyThreads);
}

hipError_t launch_rpy_assemble_batched(hipStream_t s, const ChainDesc* cd, int count,
                                       const int32_t* prefix, int blocks) {
  BD_LAUNCH("rpy_assemble_batched", rpy_assemble_batched_kernel, dim3(blocks),
            dim3(kRpyThreads), 0, s, cd, prefix, count);
  return hipGetLastError();
}

}  // namespace bd
