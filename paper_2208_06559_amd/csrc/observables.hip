// Chain observables of the paper's flow studies (Section 5): the
// end-to-end vector R_ee = r_{N-1} - r_0 (whose length gives the stretch
// |R_ee| / ((N-1) b) and whose components give R_ee,x/y/z) and the squared
// radius of gyration R_g^2 = (1/N) sum_i |r_i - r_cm|^2, for many chains
// packed one after another.  One workgroup per chain; fixed-order
// reductions (bitwise reproducible).  Also the Kramers stress of the same
// packed chains (Eqs. 28-29).
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

// Kramers stress (Eq. 28) and N1 (Eq. 29) of chain blockIdx.x: tau =
// sum_k c_k Q_k Q_k^T - M I, c_k = F_k / |Q_k| with F_k the connector's
// force along Q_k (the tension T_k of a rigid rod, or K (|Q_k| - b) for a
// Fraenkel spring, Eq. 3).  Six components summed per thread over k, then
// fixed-order block sums.
__global__ __launch_bounds__(kObThreads) void stress_kernel(const double* __restrict__ x,
                                                            const int64_t* __restrict__ off,
                                                            const double* __restrict__ T,
                                                            double K, double b,
                                                            double* __restrict__ out) {
  __shared__ double red[kObThreads / 64];
  const int c = blockIdx.x;
  const int64_t b0 = off[c], M = off[c + 1] - off[c] - 1;
  const double* xc = x + 3 * b0;
  const double* Tc = T ? T + (b0 - c) : nullptr;  // chain c's M tensions
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t k = threadIdx.x; k < M; k += kObThreads) {
    const double q0 = xc[3 * (k + 1)] - xc[3 * k], q1 = xc[3 * (k + 1) + 1] - xc[3 * k + 1],
                 q2 = xc[3 * (k + 1) + 2] - xc[3 * k + 2];
    const double ql = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
    const double mag = Tc ? Tc[k] : K * (ql - b);
    const double ck = mag / ql;
    s[0] += ck * q0 * q0;
    s[1] += ck * q1 * q1;
    s[2] += ck * q2 * q2;
    s[3] += ck * q0 * q1;
    s[4] += ck * q0 * q2;
    s[5] += ck * q1 * q2;
  }
  double t[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) t[e] = ob_block_sum(s[e], red);
  if (threadIdx.x == 0) {
    const double m = (double)M;
    double* o = out + 7 * (int64_t)c;
    o[0] = t[0] - m;
    o[1] = t[1] - m;
    o[2] = t[2] - m;
    o[3] = t[3];
    o[4] = t[4];
    o[5] = t[5];
    o[6] = (t[0] - m) - (t[1] - m);
  }
}

}  // namespace

hipError_t launch_stress(hipStream_t s, int32_t n_chains, const double* x, const int64_t* off,
                         const double* T, double K, double b, double* out) {
  BD_LAUNCH("stress", stress_kernel, dim3(n_chains), dim3(kObThreads), 0, s, x, off, T, K, b,
            out);
  return hipGetLastError();
}

hipError_t launch_observables(hipStream_t s, int32_t n_chains, const double* x,
                              const int64_t* off, double* out) {
  BD_LAUNCH("observables", observables_kernel, dim3(n_chains), dim3(kObThreads), 0, s, x, off,
            out);
  return hipGetLastError();
}

}  // namespace bd
