// RPY diffusion-tensor assembly (Eqs. 7-9), column-major D with ld.
//
// A workgroup covers kRpyThreads consecutive matrix rows and kRpyJ
// consecutive column beads j.  First its work-items evaluate the pairs
// (i, j) of the beads i of those rows (one sqrt, one divide chain each)
// into LDS; then each work-item takes one row rho = 3i + r and stores row r
// of D_ij, one element in each of the columns 3j .. 3j + 2.  Consecutive
// work-items take consecutive rows, so every store of a wavefront is one
// contiguous 512-byte run of a column.  With BD_FILL_LOWER only blocks with
// i >= j are touched and the diagonal block keeps its lower part only.
#include "common.hpp"
#include "profile.hpp"
#include "rpy_device.hpp"

namespace bd {

namespace {

constexpr int kRpyThreads = 256;

constexpr int kRpyJ = 4;                       // column beads per workgroup
constexpr int kRpyBeads = kRpyThreads / 3 + 2;  // beads a run of kRpyThreads rows touches

__device__ __forceinline__ void rpy_assemble_body(int bx, int by, const double* __restrict__ x,
                                                  double* __restrict__ D, int64_t ld, int N,
                                                  double hstar, double a, int fill_full) {
  // per (bead of the block, column bead): cI, cRR and R = r_i - r_j
  __shared__ double pair[kRpyJ][5][kRpyBeads];
  const int64_t row0 = (int64_t)bx * kRpyThreads;
  const int j0 = by * kRpyJ;
  // rows entirely above the first column bead's diagonal block
  if (!fill_full && row0 + kRpyThreads <= 3 * (int64_t)j0) return;
  const int i0 = (int)(row0 / 3);
  for (int q = threadIdx.x; q < kRpyBeads * kRpyJ; q += kRpyThreads) {
    const int b = q / kRpyJ, u = q - kRpyJ * b, i = i0 + b, j = j0 + u;
    if (i >= N || j >= N || i == j || (!fill_full && i < j)) continue;
    const double R0 = x[3 * i] - x[3 * j];
    const double R1 = x[3 * i + 1] - x[3 * j + 1];
    const double R2c = x[3 * i + 2] - x[3 * j + 2];
    const double R2 = R0 * R0 + R1 * R1 + R2c * R2c;
    double cI, cRR;
    rpy_coeffs(R2, hstar, a, cI, cRR);
    pair[u][0][b] = cI;
    pair[u][1][b] = cRR;
    pair[u][2][b] = R0;
    pair[u][3][b] = R1;
    pair[u][4][b] = R2c;
  }
  __syncthreads();
  const int64_t rho = row0 + threadIdx.x;  // this work-item's row
  if (rho >= 3 * (int64_t)N) return;
  const int i = (int)(rho / 3), r = (int)(rho - 3 * (int64_t)i), b = i - i0;
  for (int u = 0; u < kRpyJ; ++u) {
    const int j = j0 + u;
    if (j >= N || (!fill_full && i < j)) break;  // later beads j lie further right
    double v[3];
    if (i == j) {
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = (r == c) ? 1.0 : 0.0;
    } else {
      const double cI = pair[u][0][b], cRR = pair[u][1][b];
      const double Rv[3] = {pair[u][2][b], pair[u][3][b], pair[u][4][b]};
      const double Rr = pair[u][2 + r][b];
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = (r == c ? cI : 0.0) + cRR * Rr * Rv[c];
    }
    double* col = D + 3 * (int64_t)j * ld + rho;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (!fill_full && i == j && r < c) continue;  // strict upper part of the diagonal block
      col[c * ld] = v[c];
    }
  }
}

__global__ __launch_bounds__(kRpyThreads) void rpy_assemble_kernel(
    const double* __restrict__ x, double* __restrict__ D, int64_t ld, int N, double hstar,
    double a, int fill_full) {
  rpy_assemble_body(blockIdx.x, blockIdx.y, x, D, ld, N, hstar, a, fill_full);
}

// Ensembles: lower triangles, one flattened grid; chain c owns
// rpy_batched_blocks(N_c) workgroups, (group of kRpyJ column beads, row
// block bx) each.
__global__ __launch_bounds__(kRpyThreads) void rpy_assemble_batched_kernel(
    const ChainDesc* __restrict__ cd, const int32_t* __restrict__ prefix, int count) {
  const int ci = find_chain(prefix, count, blockIdx.x);
  const ChainDesc& c = cd[ci];
  const int N = c.N;
  const int nbx = (3 * N + kRpyThreads - 1) / kRpyThreads;
  const int local = blockIdx.x - prefix[ci];
  rpy_assemble_body(local % nbx, local / nbx, c.x, c.D, c.ld, N, c.hstar, c.a, 0);
}

// Adjoint of the assembly: for phi = sum_ij <Dbar_ij, D_ij> (3 x 3 blocks of
// the full n x n matrix Dbar, column-major with ld), bead i receives
// sum_{j != i} g(Dbar_ij + Dbar_ji, R_ij) with, for R = r_i - r_j and
// <B, D_ij> = cI tr B + cRR R^T B R,
//   g(B, R) = cI'(R) tr(B) R/|R| + cRR'(R) (R^T B R) R/|R| + cRR (B + B^T) R,
// and the h* partial sum_j (cI tr Dbar_ij + cRR R^T Dbar_ij R) / h* (D - I
// is linear in h*).
__device__ __forceinline__ void rpy_slopes(double R, double hstar, double a, double& cI,
                                           double& cRR, double& dcI, double& dcRR) {
  if (R >= 2.0 * a) {
    const double pre = 0.75 * hstar, a2 = a * a;
    cI = pre * (1.0 / R + 2.0 * a2 / (3.0 * R * R * R));
    cRR = pre * (1.0 / (R * R * R) - 2.0 * a2 / (R * R * R * R * R));
    dcI = pre * (-1.0 / (R * R) - 2.0 * a2 / (R * R * R * R));
    dcRR = pre * (-3.0 / (R * R * R * R) + 10.0 * a2 / (R * R * R * R * R * R));
  } else {
    const double pre = 3.0 * hstar / (8.0 * a);
    cI = pre * (8.0 / 3.0 - 3.0 * R / (4.0 * a));
    cRR = pre / (4.0 * a * R);
    dcI = -pre * 3.0 / (4.0 * a);
    dcRR = -pre / (4.0 * a * R * R);
  }
}

// One workgroup per kAdjB beads i.  It walks the beads j in tiles of
// kAdjB: the two 3 kAdjB x 3 kAdjB blocks of Dbar it needs, (rows of i,
// columns of j) and (rows of j, columns of i), are staged in LDS by
// consecutive threads reading consecutive rows of one column; then thread
// (li, lj) evaluates the pair (i0 + li, j0 + lj).  Each thread keeps its
// partial sums over its j's; at the end the kAdjB partials of bead i are
// added in lj order.
constexpr int kAdjB = 16;
constexpr int kAdjS = 3 * kAdjB;  // block side in matrix rows

__global__ __launch_bounds__(256) void rpy_adjoint_kernel(
    const double* __restrict__ x, const double* __restrict__ Db, int64_t ld, int N, double a,
    double* __restrict__ xbar, double* __restrict__ hpart, DevState* __restrict__ st) {
  static_assert(kAdjB * kAdjB == 256, "one pair per thread");
  __shared__ double Sij[kAdjS][kAdjS + 1];  // [column (bead j)][row (bead i)]
  __shared__ double Sji[kAdjS][kAdjS + 1];  // [column (bead i)][row (bead j)]
  __shared__ double red[kAdjB][kAdjB][4];
  const int t = threadIdx.x;
  const int li = t % kAdjB, lj = t / kAdjB;
  const int i0 = blockIdx.x * kAdjB;
  const int i = i0 + li;
  const int64_t r0i = 3 * (int64_t)i0;
  const int nrow = 3 * N;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0, hs = 0.0;
  bool coincident = false;
  const double xi0 = (i < N) ? x[3 * i] : 0.0, xi1 = (i < N) ? x[3 * i + 1] : 0.0,
               xi2 = (i < N) ? x[3 * i + 2] : 0.0;
  for (int j0 = 0; j0 < N; j0 += kAdjB) {
    const int64_t r0j = 3 * (int64_t)j0;
    __syncthreads();  // the previous tile's blocks are no longer read
    for (int e = t; e < kAdjS * kAdjS; e += 256) {
      const int row = e % kAdjS, col = e / kAdjS;
      const bool ok_ij = r0i + row < nrow && r0j + col < nrow;
      const bool ok_ji = r0j + row < nrow && r0i + col < nrow;
      Sij[col][row] = ok_ij ? Db[(r0j + col) * ld + r0i + row] : 0.0;
      Sji[col][row] = ok_ji ? Db[(r0i + col) * ld + r0j + row] : 0.0;
    }
    __syncthreads();
    const int j = j0 + lj;
    if (i >= N || j >= N || j == i) continue;
    const double R[3] = {xi0 - x[3 * j], xi1 - x[3 * j + 1], xi2 - x[3 * j + 2]};
    const double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    if (Rn == 0.0) {
      coincident = true;
      continue;
    }
    double B[3][3], Bij[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Bij[r][c] = Sij[3 * lj + c][3 * li + r];
        B[r][c] = Bij[r][c] + Sji[3 * li + c][3 * lj + r];
      }
    double cI, cRR, dcI, dcRR;  // per unit h*
    rpy_slopes(Rn, 1.0, a, cI, cRR, dcI, dcRR);
    double BR[3], BtR[3], BijR[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      BR[r] = B[r][0] * R[0] + B[r][1] * R[1] + B[r][2] * R[2];
      BtR[r] = B[0][r] * R[0] + B[1][r] * R[1] + B[2][r] * R[2];
      BijR[r] = Bij[r][0] * R[0] + Bij[r][1] * R[1] + Bij[r][2] * R[2];
    }
    const double trB = B[0][0] + B[1][1] + B[2][2];
    const double q = R[0] * BR[0] + R[1] * BR[1] + R[2] * BR[2];
    const double sc = (dcI * trB + dcRR * q) / Rn;
    g0 += sc * R[0] + cRR * (BR[0] + BtR[0]);
    g1 += sc * R[1] + cRR * (BR[1] + BtR[1]);
    g2 += sc * R[2] + cRR * (BR[2] + BtR[2]);
    hs += cI * (Bij[0][0] + Bij[1][1] + Bij[2][2]) +
          cRR * (R[0] * BijR[0] + R[1] * BijR[1] + R[2] * BijR[2]);
  }
  red[li][lj][0] = g0;
  red[li][lj][1] = g1;
  red[li][lj][2] = g2;
  red[li][lj][3] = hs;
  if (coincident) st->status = BD_ERR_PARAM;
  __syncthreads();
  if (lj == 0 && i < N) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int k = 0; k < kAdjB; ++k) {
      s0 += red[li][k][0];
      s1 += red[li][k][1];
      s2 += red[li][k][2];
      s3 += red[li][k][3];
    }
    xbar[3 * i] = s0;
    xbar[3 * i + 1] = s1;
    xbar[3 * i + 2] = s2;
    hpart[i] = s3;
  }
}

// d phi / d h* = sum over beads of the partials, in bead order; the
// position gradient is scaled by h* here (the per-bead pass works per unit
// h*).
__global__ __launch_bounds__(kRpyThreads) void rpy_adjoint_finish_kernel(
    const double* __restrict__ hpart, int N, double hstar, double* __restrict__ xbar,
    double* __restrict__ hbar) {
  __shared__ double red[kRpyThreads];
  double s = 0.0;
  const int t = threadIdx.x;
  const int per = (N + kRpyThreads - 1) / kRpyThreads;
  for (int q = 0; q < per; ++q) {
    const int i = t * per + q;
    if (i < N) s += hpart[i];
  }
  red[t] = s;
  for (int e = t; e < 3 * N; e += kRpyThreads) xbar[e] *= hstar;
  __syncthreads();
  if (t == 0) {
    double total = 0.0;
    for (int w = 0; w < kRpyThreads; ++w) total += red[w];
    *hbar = total;
  }
}

}  // namespace

hipError_t launch_rpy_adjoint(hipStream_t s, const bd_params_t& p, const double* x,
                              const double* Dbar, int64_t ld, double* xbar, double* hbar,
                              double* hpart, DevState* st) {
  const int N = p.n_beads;
  BD_LAUNCH("rpy_adjoint", rpy_adjoint_kernel, dim3((N + kAdjB - 1) / kAdjB), dim3(256), 0, s, x,
            Dbar, ld, N, p.a, xbar, hpart, st);
  BD_LAUNCH("rpy_adjoint_finish", rpy_adjoint_finish_kernel, dim3(1), dim3(kRpyThreads), 0, s,
            hpart, N, p.hstar, xbar, hbar);
  return hipGetLastError();
}

hipError_t launch_rpy_assemble(hipStream_t s, const bd_params_t& p, const double* x, double* D,
                               int64_t ld, int fill) {
  const int N = p.n_beads;
  dim3 grid((3 * N + kRpyThreads - 1) / kRpyThreads, (N + kRpyJ - 1) / kRpyJ);
  BD_LAUNCH("rpy_assemble", rpy_assemble_kernel, grid, dim3(kRpyThreads), 0, s, x, D, ld, N, p.hstar,
                     p.a, fill == BD_FILL_FULL ? 1 : 0);
  return hipGetLastError();
}

int rpy_batched_blocks(int n_beads) {
  return ((n_beads + kRpyJ - 1) / kRpyJ) * ((3 * n_beads + kRpyThreads - 1) / kRpyThreads);
}

hipError_t launch_rpy_assemble_batched(hipStream_t s, const ChainDesc* cd, int count,
                                       const int32_t* prefix, int blocks) {
  BD_LAUNCH("rpy_assemble_batched", rpy_assemble_batched_kernel, dim3(blocks),
            dim3(kRpyThreads), 0, s, cd, prefix, count);
  return hipGetLastError();
}

}  // namespace bd
