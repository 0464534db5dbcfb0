// Chain observables of the paper's flow studies (Section 5): the
// end-to-end vector R_ee = r_{N-1} - r_0 (whose length gives the stretch
// |R_ee| / ((N-1) b) and whose components give R_ee,x/y/z) and the squared
// radius of gyration R_g^2 = (1/N) sum_i |r_i - r_cm|^2, for many chains
// packed one after another.  One workgroup per chain; fixed-order
// reductions (bitwise reproducible).
#include "common.hpp"
#include "profile.hpp"

namespace bd {

namespace {

constexpr int kObThreads = 256;

__device__ double ob_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kObThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kObThreads) void observables_kernel(const double* __restrict__ x,
                                                                 const int64_t* __restrict__ off,
                                                                 double* __restrict__ out) {
  __shared__ double red[kObThreads / 64];
  const int c = blockIdx.x;
  const int64_t b0 = off[c], N = off[c + 1] - off[c];
  const double* xc = x + 3 * b0;
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < N; i += kObThreads)
#pragma unroll
    for (int al = 0; al < 3; ++al) s[al] += xc[3 * i + al];
  double cm[3];
#pragma unroll
  for (int al = 0; al < 3; ++al) cm[al] = ob_block_sum(s[al], red) / (double)N;
  double g = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kObThreads) {
    const double d0 = xc[3 * i] - cm[0], d1 = xc[3 * i + 1] - cm[1], d2 = xc[3 * i + 2] - cm[2];
    g += d0 * d0 + d1 * d1 + d2 * d2;
  }
  g = ob_block_sum(g, red) / (double)N;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int al = 0; al < 3; ++al) out[4 * c + al] = xc[3 * (N - 1) + al] - xc[al];
    out[4 * c + 3] = g;
  }
}

}  // namespace

hipError_t launch_observables(hipStream_t s, int32_t n_chains, const double* x,
                              const int64_t* off, double* out) {
  BD_LAUNCH("observables", observables_kernel, dim3(n_chains), dim3(kObThreads), 0, s, x, off,
            out);
  return hipGetLastError();
}

}  // namespace bd
