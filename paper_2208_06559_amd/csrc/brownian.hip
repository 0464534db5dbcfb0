// Correlated Brownian displacement y = c_B * B * xi (the noise term of
// Eq. 6 times dt) and the explicit predictor x* = x + dt kappa.x + y.
//
// xi is drawn in-kernel from Philox4x64-10 (one counter block per four
// elements).  The lower-triangular matrix-vector product reads B once from
// HBM: the lower triangle is cut into 256 x 256 tiles, one workgroup per
// tile, one row per work-item, so every column access of a wavefront is a
// contiguous 512-byte run.  Per-tile partial sums are reduced afterwards in
// a fixed order (no floating-point atomics, bitwise reproducible).  This is
// the noise product of bd_brownian; inside a step the factorisation forms
// y itself (panel by panel, in cholesky.hip), and this file supplies the
// noise and its coefficient.
#include "common.hpp"
#include "profile.hpp"
#include "philox.hpp"

#include <mutex>

namespace bd {

namespace {

constexpr int kTv = 256;  // TRMV tile (rows = cols = threads)

__device__ __forceinline__ void tri_index(int t, int& r, int& c) {
  // t -> (r, c) with r >= c, t = r(r+1)/2 + c
  int rr = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((rr + 1) * (rr + 2) / 2 <= t) ++rr;
  while (rr * (rr + 1) / 2 > t) --rr;
  r = rr;
  c = t - rr * (rr + 1) / 2;
}

__device__ __forceinline__ void noise_body(int bx, double* __restrict__ xi, int64_t n,
                                           uint64_t seed, uint64_t chain, uint64_t step,
                                           int uniform) {
  const int64_t blk = (int64_t)bx * blockDim.x + threadIdx.x;
  if (blk * 4 >= n) return;
  double z[4];
  noise4(seed, chain, step, (uint64_t)blk, uniform, z);
#pragma unroll
  for (int l = 0; l < 4; ++l)
    if (blk * 4 + l < n) xi[blk * 4 + l] = z[l];
}

__global__ __launch_bounds__(256) void noise_kernel(double* __restrict__ xi, int64_t n,
                                                     uint64_t seed, uint64_t chain,
                                                     uint64_t step, int uniform) {
  noise_body(blockIdx.x, xi, n, seed, chain, step, uniform);
}

__device__ __forceinline__ void trmv_tile_body(int t, const double* __restrict__ L, int64_t ld,
                                               int64_t n, const double* __restrict__ xi,
                                               double* __restrict__ part) {
  __shared__ double xs[kTv];
  int rt, ct;
  tri_index(t, rt, ct);
  const int64_t i = (int64_t)rt * kTv + threadIdx.x;
  const int64_t j0 = (int64_t)ct * kTv;
  {
    const int64_t j = j0 + threadIdx.x;
    xs[threadIdx.x] = (j < n) ? xi[j] : 0.0;
  }
  __syncthreads();
  if (i >= n) return;
  int jend = kTv;
  if (j0 + jend > n) jend = (int)(n - j0);
  if (rt == ct) jend = (int)(i - j0) + 1;  // diagonal tile: j <= i
  const double* Lp = L + j0 * ld + i;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  int jj = 0;
  for (; jj + 4 <= jend; jj += 4) {
    acc0 += Lp[(int64_t)(jj + 0) * ld] * xs[jj + 0];
    acc1 += Lp[(int64_t)(jj + 1) * ld] * xs[jj + 1];
    acc2 += Lp[(int64_t)(jj + 2) * ld] * xs[jj + 2];
    acc3 += Lp[(int64_t)(jj + 3) * ld] * xs[jj + 3];
  }
  for (; jj < jend; ++jj) acc0 += Lp[(int64_t)jj * ld] * xs[jj];
  part[(int64_t)ct * n + i] = (acc0 + acc1) + (acc2 + acc3);
}

__global__ __launch_bounds__(kTv) void trmv_tile_kernel(const double* __restrict__ L, int64_t ld,
                                                         int64_t n, const double* __restrict__ xi,
                                                         double* __restrict__ part) {
  trmv_tile_body(blockIdx.x, L, ld, n, xi, part);
}

__device__ __forceinline__ void trmv_reduce_body(int bx, const double* __restrict__ part,
                                                 int64_t n, double c, double* __restrict__ y) {
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int rt = (int)(i / kTv);
  double s = 0.0;
  for (int ct = 0; ct <= rt; ++ct) s += part[(int64_t)ct * n + i];
  y[i] = c * s;
}

__global__ __launch_bounds__(256) void trmv_reduce_kernel(const double* __restrict__ part,
                                                           int64_t n, double c,
                                                           double* __restrict__ y) {
  trmv_reduce_body(blockIdx.x, part, n, c, y);
}

__device__ __forceinline__ void predictor_body(int bx, const double* __restrict__ x,
                                               const double* __restrict__ y,
                                               double* __restrict__ xs, int N, double dt,
                                               double k0, double k1, double k2, double k3,
                                               double k4, double k5, double k6, double k7,
                                               double k8) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double r0 = x[3 * i], r1 = x[3 * i + 1], r2 = x[3 * i + 2];
  // Eq. 5 flow term kappa . r_i, unweighted by D (Eq. 6)
  const double v0 = k0 * r0 + k1 * r1 + k2 * r2;
  const double v1 = k3 * r0 + k4 * r1 + k5 * r2;
  const double v2 = k6 * r0 + k7 * r1 + k8 * r2;
  xs[3 * i] = r0 + dt * v0 + y[3 * i];
  xs[3 * i + 1] = r1 + dt * v1 + y[3 * i + 1];
  xs[3 * i + 2] = r2 + dt * v2 + y[3 * i + 2];
}

__global__ __launch_bounds__(256) void predictor_kernel(const double* __restrict__ x,
                                                         const double* __restrict__ y,
                                                         double* __restrict__ xs, int N, double dt,
                                                         double k0, double k1, double k2,
                                                         double k3, double k4, double k5,
                                                         double k6, double k7, double k8) {
  predictor_body(blockIdx.x, x, y, xs, N, dt, k0, k1, k2, k3, k4, k5, k6, k7, k8);
}

// Ensembles: chain blockIdx.z of the table; grids cover the largest chain.
// d_step non-null: the noise counter from device memory (a captured step
// replays with the plan's counter).
__global__ __launch_bounds__(256) void noise_batched_kernel(const ChainDesc* __restrict__ cd,
                                                             uint64_t step,
                                                             const int64_t* __restrict__ d_step) {
  const ChainDesc& c = cd[blockIdx.z];
  const uint64_t st = d_step ? (uint64_t)*d_step : step;
  noise_body(blockIdx.x, c.xi, c.n, c.seed, c.chain_id, st, c.uniform);
}

__global__ __launch_bounds__(256) void predictor_batched_kernel(const ChainDesc* __restrict__ cd) {
  const ChainDesc& c = cd[blockIdx.z];
  const double* k = c.kappa;
  predictor_body(blockIdx.x, c.x, c.y, c.xs, c.N, c.dt, k[0], k[1], k[2], k[3], k[4], k[5], k[6],
                 k[7], k[8]);
}

// Adjoint of y = c L xi: Lbar(i, j) = c ybar_i xi_j on the lower triangle,
// column-major with ldb.  One workgroup per 64 x 64 tile of the lower
// triangle (tile t = ti (ti + 1)/2 + tj, tj <= ti); lane r of wave w writes
// row r of columns w, w + 4, ... (each column a coalesced 512-byte run).
constexpr int kAdjTile = 64;

__device__ __forceinline__ void tri_tile(int64_t t, int64_t& ti, int64_t& tj) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;           // the estimate may be one off either way
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

__global__ __launch_bounds__(256) void brownian_adjoint_l_kernel(const double* __restrict__ xi,
                                                                  const double* __restrict__ ybar,
                                                                  int64_t n, double c,
                                                                  double* __restrict__ Lbar,
                                                                  int64_t ldb) {
  int64_t ti, tj;
  tri_tile(blockIdx.x, ti, tj);
  const int64_t i = ti * kAdjTile + (threadIdx.x & 63);
  if (i >= n) return;
  const double cy = c * ybar[i];
  for (int q = threadIdx.x >> 6; q < kAdjTile; q += 4) {
    const int64_t j = tj * kAdjTile + q;
    if (j > i) break;  // j grows with q: the rest of this lane's columns lie above the diagonal
    Lbar[j * ldb + i] = cy * xi[j];
  }
}

// xibar_j = c sum_{i >= j} L(i, j) ybar_i: one wave per column j (its rows
// contiguous), lane sums in row order, then a fixed butterfly.
__global__ __launch_bounds__(256) void brownian_adjoint_xi_kernel(const double* __restrict__ L,
                                                                   int64_t ld,
                                                                   const double* __restrict__ ybar,
                                                                   int64_t n, double c,
                                                                   double* __restrict__ xibar) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;  // wave-uniform
  double s = 0.0;
  for (int64_t i = j + lane; i < n; i += 64) s += L[j * ld + i] * ybar[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) xibar[j] = c * s;
}

}  // namespace

static int64_t trmv_tiles(int64_t n) { return (n + kTv - 1) / kTv; }

hipError_t launch_brownian_adjoint(hipStream_t s, const bd_params_t& p, const double* L,
                                   int64_t ld, const double* xi, const double* ybar,
                                   double* Lbar, int64_t ldb, double* xibar) {
  const int64_t n = 3 * (int64_t)p.n_beads;
  const double c = (p.noise == BD_NOISE_UNIFORM_PAPER) ? sqrt(6.0 * p.dt) : sqrt(2.0 * p.dt);
  const int64_t nt = (n + kAdjTile - 1) / kAdjTile;
  BD_LAUNCH("brownian_adjoint_l", brownian_adjoint_l_kernel, dim3((unsigned)(nt * (nt + 1) / 2)),
            dim3(256), 0, s, xi, ybar, n, c, Lbar, ldb);
  BD_LAUNCH("brownian_adjoint_xi", brownian_adjoint_xi_kernel, dim3((unsigned)((n + 3) / 4)),
            dim3(256), 0, s, L, ld, ybar, n, c, xibar);
  return hipGetLastError();
}

hipError_t launch_brownian_adjoint_lbar(hipStream_t s, const bd_params_t& p, const double* xi,
                                        const double* ybar, double* Lbar, int64_t ldb) {
  const int64_t n = 3 * (int64_t)p.n_beads;
  const double c = (p.noise == BD_NOISE_UNIFORM_PAPER) ? sqrt(6.0 * p.dt) : sqrt(2.0 * p.dt);
  const int64_t nt = (n + kAdjTile - 1) / kAdjTile;
  BD_LAUNCH("brownian_adjoint_l", brownian_adjoint_l_kernel, dim3((unsigned)(nt * (nt + 1) / 2)),
            dim3(256), 0, s, xi, ybar, n, c, Lbar, ldb);
  return hipGetLastError();
}

size_t brownian_workspace_bytes(int64_t n) {
  const int64_t nt = trmv_tiles(n);
  return align_up(sizeof(double) * n, 256) + align_up(sizeof(double) * nt * n, 256);
}

// Allocation-free noise product: the workspace of launch_brownian (xi and
// the per-tile partial sums) in a fixed device array sized for matrix order
// n <= kScratchMaxN, one copy per GPU, kept until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr int64_t kScratchMaxN = 12288;
constexpr int64_t kScratchDoubles =
    (int64_t)(((kScratchMaxN * 8 + 255) / 256 * 256 +
               ((kScratchMaxN + kTv - 1) / kTv * kScratchMaxN * 8 + 255) / 256 * 256) / 8);
static __device__ __align__(256) double scratch[kScratchDoubles];
static_assert(kScratchDoubles * 8 >= 8 * kScratchMaxN + 8 * 48 * kScratchMaxN,
              "scratch holds xi and the partial sums at the largest n");

constexpr int kMaxDevices = 64;
static void* g_scratch_addr[kMaxDevices];
static std::mutex g_scratch_mu;

int64_t brownian_scratch_max_n() { return kScratchMaxN; }

hipError_t brownian_scratch_init(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

hipError_t launch_brownian(hipStream_t s, const bd_params_t& p, int64_t step, const double* L,
                           int64_t ld, double* y, double* xi_out, void* ws) {
  const int64_t n = 3 * (int64_t)p.n_beads;
  double* xi = static_cast<double*>(ws);
  double* part = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                           align_up(sizeof(double) * n, 256));
  const int64_t nblk = (n + 3) / 4;
  BD_LAUNCH("noise", noise_kernel, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, s, xi, n,
                     p.seed, p.chain_id, (uint64_t)step, p.noise == BD_NOISE_UNIFORM_PAPER);
  const int64_t nt = trmv_tiles(n);
  const int64_t ntiles = nt * (nt + 1) / 2;
  BD_LAUNCH("trmv_tile", trmv_tile_kernel, dim3((unsigned)ntiles), dim3(kTv), 0, s, L, ld, n, xi, part);
  const double c = (p.noise == BD_NOISE_UNIFORM_PAPER) ? sqrt(6.0 * p.dt) : sqrt(2.0 * p.dt);
  BD_LAUNCH("trmv_reduce", trmv_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                     n, c, y);
  if (xi_out) {
    hipError_t e = hipMemcpyAsync(xi_out, xi, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_predictor(hipStream_t s, const bd_params_t& p, const double* x, const double* y,
                            double* xs) {
  const int N = p.n_beads;
  const double* k = p.kappa;
  BD_LAUNCH("predictor", predictor_kernel, dim3((N + 255) / 256), dim3(256), 0, s, x, y, xs, N, p.dt,
                     k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8]);
  return hipGetLastError();
}

double noise_coeff(const bd_params_t& p) {
  return (p.noise == BD_NOISE_UNIFORM_PAPER) ? sqrt(6.0 * p.dt) : sqrt(2.0 * p.dt);
}

hipError_t launch_noise(hipStream_t s, const bd_params_t& p, int64_t step, double* xi) {
  const int64_t n = 3 * (int64_t)p.n_beads;
  const int64_t nblk = (n + 3) / 4;
  BD_LAUNCH("noise", noise_kernel, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, s, xi, n,
            p.seed, p.chain_id, (uint64_t)step, p.noise == BD_NOISE_UNIFORM_PAPER);
  return hipGetLastError();
}

hipError_t launch_noise_batched(hipStream_t s, const ChainDesc* cd, int count, int64_t max_n,
                                int64_t step, const int64_t* d_step) {
  const int64_t nblk = (max_n + 3) / 4;
  BD_LAUNCH("noise_batched", noise_batched_kernel,
            dim3((unsigned)((nblk + 255) / 256), 1, count), dim3(256), 0, s, cd, (uint64_t)step, d_step);
  return hipGetLastError();
}

hipError_t launch_predictor_batched(hipStream_t s, const ChainDesc* cd, int count, int max_beads) {
  BD_LAUNCH("predictor_batched", predictor_batched_kernel,
            dim3((max_beads + 255) / 256, 1, count), dim3(256), 0, s, cd);
  return hipGetLastError();
}

}  // namespace bd
