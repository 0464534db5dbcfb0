// The paper's stiff Fraenkel springs (Eq. 3) with its semi-implicit link
// update (Eqs. 13-17), as an alternative to the rigid-rod tension solve.
//
// Spring k (k = 0..N-2) pulls bead k with F_k = K (|Q_k| - b) Q_k/|Q_k| and
// bead k+1 with -F_k.  With the net bead forces f at t and v = D f (the
// matrix-free product of the tension solve), each link's explicit update is
//   Y_k = Q_k + dt [kappa.Q_k + v_{k+1} - v_k + 2 F_k] + y_{k+1} - y_k,
// where 2 F_k removes the spring's own term (D_kk + D_{k+1,k+1}) F_k from
// the explicit part; that term is taken at t + dt, which gives the closed
// form |Q_k'| = (|Y_k| + 2 dt K b)/(1 + 2 dt K) along Y_k.  Bead 0 moves by
// its explicit equation of motion and the other beads follow the new links.
#include "common.hpp"
#include "profile.hpp"

namespace bd {

namespace {

constexpr int kFrThreads = 1024;  // one workgroup: links k = tid + 1024 q
constexpr int kFrMaxLinks = 8192;
constexpr int kFrPer = kFrMaxLinks / kFrThreads;

__device__ __forceinline__ void spring_force(const double* __restrict__ x, int k, double K,
                                             double b, double F[3]) {
  const double Q0 = x[3 * (k + 1)] - x[3 * k], Q1 = x[3 * (k + 1) + 1] - x[3 * k + 1],
               Q2 = x[3 * (k + 1) + 2] - x[3 * k + 2];
  const double len = sqrt(Q0 * Q0 + Q1 * Q1 + Q2 * Q2);
  F[0] = K * (len - b) * Q0 / len;
  F[1] = K * (len - b) * Q1 / len;
  F[2] = K * (len - b) * Q2 / len;
}

// f_i = F_i - F_{i-1} (zero past the ends), one thread per bead.
__global__ __launch_bounds__(256) void spring_forces_kernel(const double* __restrict__ x, int N,
                                                            double K, double b,
                                                            double* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double Fi[3] = {0.0, 0.0, 0.0}, Fm[3] = {0.0, 0.0, 0.0};
  if (i < N - 1) spring_force(x, i, K, b, Fi);
  if (i > 0) spring_force(x, i - 1, K, b, Fm);
#pragma unroll
  for (int al = 0; al < 3; ++al) f[3 * i + al] = Fi[al] - Fm[al];
}

// The link update and the new positions, in place.  Thread t owns the
// consecutive links t*P .. t*P+P-1 (P = ceil(M / 1024)); their new vectors
// are summed locally, the thread sums are scanned in LDS, and each thread
// writes its beads.
__global__ __launch_bounds__(kFrThreads) void fraenkel_update_kernel(
    double* __restrict__ x, const double* __restrict__ v, const double* __restrict__ y, int N,
    double K, double b, double dt, double k0, double k1, double k2, double k3, double k4,
    double k5, double k6, double k7, double k8, DevState* __restrict__ st) {
  __shared__ double part[3][kFrThreads];
  __shared__ double red[kFrThreads / 64];
  __shared__ double x0s[3];
  if (st->status == BD_ERR_NOT_SPD) return;  // positions stay at t
  const int tid = threadIdx.x;
  const int M = N - 1;
  const int P = (M + kFrThreads - 1) / kFrThreads;
  const int kbeg = tid * P;
  double qn[kFrPer][3];
  double err = 0.0;
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < kFrPer; ++q) {
    const int k = kbeg + q;
    qn[q][0] = qn[q][1] = qn[q][2] = 0.0;
    if (q < P && k < M) {
      double F[3], Q[3], Y[3];
      spring_force(x, k, K, b, F);
#pragma unroll
      for (int al = 0; al < 3; ++al) Q[al] = x[3 * (k + 1) + al] - x[3 * k + al];
      const double kQ[3] = {k0 * Q[0] + k1 * Q[1] + k2 * Q[2], k3 * Q[0] + k4 * Q[1] + k5 * Q[2],
                            k6 * Q[0] + k7 * Q[1] + k8 * Q[2]};
#pragma unroll
      for (int al = 0; al < 3; ++al)
        Y[al] = Q[al] + dt * (kQ[al] + v[3 * (k + 1) + al] - v[3 * k + al] + 2.0 * F[al]) +
                (y[3 * (k + 1) + al] - y[3 * k + al]);
      const double ylen = sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]);
      const double qlen = (ylen + 2.0 * dt * K * b) / (1.0 + 2.0 * dt * K);
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        qn[q][al] = Y[al] * (qlen / ylen);
        s[al] += qn[q][al];
      }
      err = fmax(err, fabs(qlen / b - 1.0));
    }
  }
  if (tid == 0) {  // bead 0 by its explicit equation of motion
    const double r0 = x[0], r1 = x[1], r2 = x[2];
    x0s[0] = r0 + dt * ((k0 * r0 + k1 * r1 + k2 * r2) + v[0]) + y[0];
    x0s[1] = r1 + dt * ((k3 * r0 + k4 * r1 + k5 * r2) + v[1]) + y[1];
    x0s[2] = r2 + dt * ((k6 * r0 + k7 * r1 + k8 * r2) + v[2]) + y[2];
  }
#pragma unroll
  for (int al = 0; al < 3; ++al) part[al][tid] = s[al];
  // wave maxima of the length error
  for (int o = 32; o > 0; o >>= 1) err = fmax(err, __shfl_xor(err, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = err;
  __syncthreads();  // every read of the old x is done
  // inclusive scan of the thread sums (Hillis-Steele)
  for (int off = 1; off < kFrThreads; off <<= 1) {
    double a[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) a[al] = (tid >= off) ? part[al][tid - off] : 0.0;
    __syncthreads();
#pragma unroll
    for (int al = 0; al < 3; ++al) part[al][tid] += a[al];
    __syncthreads();
  }
  double r[3];
#pragma unroll
  for (int al = 0; al < 3; ++al) r[al] = x0s[al] + (tid > 0 ? part[al][tid - 1] : 0.0);
  if (tid == 0) {
#pragma unroll
    for (int al = 0; al < 3; ++al) x[al] = r[al];
  }
#pragma unroll
  for (int q = 0; q < kFrPer; ++q) {
    const int k = kbeg + q;
    if (q < P && k < M) {
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        r[al] += qn[q][al];
        x[3 * (k + 1) + al] = r[al];
      }
    }
  }
  if (tid == 0) {
    double e = 0.0;
    for (int w = 0; w < kFrThreads / 64; ++w) e = fmax(e, red[w]);
    st->max_rod_err = e;
  }
}

}  // namespace

int fraenkel_max_beads() { return kFrMaxLinks + 1; }

hipError_t launch_spring_forces(hipStream_t s, const double* x, int N, double K, double b,
                                double* f) {
  BD_LAUNCH("spring_forces", spring_forces_kernel, dim3((N + 255) / 256), dim3(256), 0, s, x, N,
            K, b, f);
  return hipGetLastError();
}

hipError_t launch_fraenkel_update(hipStream_t s, const bd_params_t& p, double K, double* x,
                                  const double* v, const double* y, DevState* st) {
  const double* k = p.kappa;
  BD_LAUNCH("fraenkel_update", fraenkel_update_kernel, dim3(1), dim3(kFrThreads), 0, s, x, v, y,
            p.n_beads, K, p.b, p.dt, k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8], st);
  return hipGetLastError();
}

}  // namespace bd
