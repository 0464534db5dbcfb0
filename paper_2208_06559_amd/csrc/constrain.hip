// Rigid-rod constraint: tensions T_k (k = 0..N-2) along the rod directions
// u_k at the start of the step such that
//   Q_k(T) = Q*_k + dt (r_{k+1} - r_k),  r = D f(T),  f_i = T_i u_i - T_{i-1} u_{i-1}
// has |Q_k| = b, i.e. g_k(T) = |Q_k|^2 - b^2 = 0 (the infinite-stiffness limit of
// the semi-implicit spring update, Eqs. 13-17, with every tension coupled
// through the full diffusion tensor of Eqs. 7-9).  Then x^{t+dt} = x* + dt r.
//
// Inexact Newton from T = 0; each Newton correction J delta = -g is solved by
// GMRES (modified Gram-Schmidt, Givens) right-preconditioned with the
// tridiagonal part of J, J_kl = -2 dt Q_k . G_kl u_l, G_kl = D_{k+1,l+1} -
// D_{k+1,l} - D_{k,l+1} + D_{k,l}.  Every product with D is matrix-free.
//
// Device work is split in two kernels that the host launches alternately:
//   dmatvec     r = D f over all bead pairs, one workgroup per 16 beads i
//               (no atomics, fixed reduction order);
//   controller  one workgroup of 512 threads: advances the Newton/GMRES state machine by one matrix-vector
//               product (residual check, band Jacobian, Arnoldi step, PCR
//               tridiagonal solve in LDS), then writes the next f.
// Once the iteration has finished both kernels return immediately.
#include "common.hpp"
#include "profile.hpp"
#include "rpy_device.hpp"

namespace bd {

namespace {

constexpr int kKmax = 60;          // GMRES iterations per Newton step
constexpr int kCtlThreads = 512;   // controller workgroup
constexpr int kMaxRods = 4096;     // LDS capacity of the tridiagonal solve
constexpr int kMvI = 16;           // beads i per matvec workgroup

enum { PH_RESID = 0, PH_KRYLOV = 1 };

struct NewtonCtl {
  int32_t phase;
  int32_t j;
  int32_t newton_it;
  int32_t kry;
  double beta;
  double eta;
};

struct Bufs {
  double *u, *Qs, *Q, *Gd, *Gp, *Gm, *T, *lo, *di, *up, *rhs, *z, *f, *r, *V, *H, *cs, *sn, *s, *y;
  NewtonCtl* ctl;
};


Bufs carve(void* ws, int N) {
  const int64_t M = N - 1;
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t count) {
    double* q = reinterpret_cast<double*>(p);
    p += align_up(count * sizeof(double), 256);
    return q;
  };
  Bufs b;
  b.u = take(3 * M);
  b.Qs = take(3 * M);
  b.Q = take(3 * M);
  b.Gd = take(3 * M);
  b.Gp = take(3 * M);
  b.Gm = take(3 * M);
  b.T = take(M);
  b.lo = take(M);
  b.di = take(M);
  b.up = take(M);
  b.rhs = take(M);
  b.z = take(M);
  b.f = take(3 * (size_t)N);
  b.r = take(3 * (size_t)N);
  b.V = take((size_t)(kKmax + 1) * M);
  b.H = take((size_t)(kKmax + 1) * kKmax);
  b.cs = take(kKmax);
  b.sn = take(kKmax);
  b.s = take(kKmax + 1);
  b.y = take(kKmax);
  b.ctl = reinterpret_cast<NewtonCtl*>(take(8));
  return b;
}

size_t carve_bytes(int N) {
  Bufs b = carve(nullptr, N);
  return reinterpret_cast<size_t>(b.ctl) + 256;
}

// RPY coefficients (Eqs. 8-9) for the matrix-free products, without
// divisions: 1/R from the hardware estimate refined by two Newton steps.
struct RpyConst {
  double a2x2;      // (2a)^2, the near/far threshold on R^2
  double far_pre;   // 3 h*/4
  double a2;        // a^2
  double near_pre;  // 3 h*/(8a)
  double near_r;    // 3/(4a)
  double near_rr;   // 3 h*/(8a) / (4a)
};

RpyConst rpy_const(double hstar, double a) {
  RpyConst c;
  c.a2x2 = 4.0 * a * a;
  c.far_pre = 0.75 * hstar;
  c.a2 = a * a;
  c.near_pre = 3.0 * hstar / (8.0 * a);
  c.near_r = 3.0 / (4.0 * a);
  c.near_rr = c.near_pre / (4.0 * a);
  return c;
}

__device__ __forceinline__ void rpy_coeffs_fast(double R2, const RpyConst& k, double& cI,
                                                double& cRR) {
  double y = __builtin_amdgcn_rsq(R2);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double h = 0.5 * R2 * y;
    y = fma(-h, y, 1.5) * y;
  }
  const double inv2 = y * y;
  if (R2 >= k.a2x2) {
    const double pre = k.far_pre * y;
    const double t = k.a2 * inv2;
    cI = pre * (1.0 + (2.0 / 3.0) * t);
    cRR = pre * (1.0 - 2.0 * t) * inv2;
  } else {
    const double R = (R2 > 0.0) ? R2 * y : 0.0;  // coincident beads: the R -> 0 limit
    cI = k.near_pre * (8.0 / 3.0 - k.near_r * R);
    cRR = (R2 > 0.0) ? k.near_rr * y : 0.0;
  }
}

// D_ij applied to v: identity for i == j, RPY block otherwise.
__device__ __forceinline__ void dblock_apply(const double* __restrict__ x, int i, int j,
                                             double hstar, double a, const double v[3],
                                             double out[3]) {
  if (i == j) {
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2];
    return;
  }
  const double R0 = x[3 * i] - x[3 * j], R1 = x[3 * i + 1] - x[3 * j + 1],
               R2c = x[3 * i + 2] - x[3 * j + 2];
  double cI, cRR;
  rpy_coeffs(R0 * R0 + R1 * R1 + R2c * R2c, hstar, a, cI, cRR);
  const double rv = R0 * v[0] + R1 * v[1] + R2c * v[2];
  out[0] = cI * v[0] + cRR * rv * R0;
  out[1] = cI * v[1] + cRR * rv * R1;
  out[2] = cI * v[2] + cRR * rv * R2c;
}

// G_kl v = (D_{k+1,l+1} - D_{k+1,l} - D_{k,l+1} + D_{k,l}) v
__device__ void g_apply(const double* __restrict__ x, int k, int l, double hstar, double a,
                        const double v[3], double out[3]) {
  double t[3];
  out[0] = out[1] = out[2] = 0.0;
  dblock_apply(x, k + 1, l + 1, hstar, a, v, t);
  out[0] += t[0]; out[1] += t[1]; out[2] += t[2];
  dblock_apply(x, k + 1, l, hstar, a, v, t);
  out[0] -= t[0]; out[1] -= t[1]; out[2] -= t[2];
  dblock_apply(x, k, l + 1, hstar, a, v, t);
  out[0] -= t[0]; out[1] -= t[1]; out[2] -= t[2];
  dblock_apply(x, k, l, hstar, a, v, t);
  out[0] += t[0]; out[1] += t[1]; out[2] += t[2];
}

__device__ __forceinline__ void unit_bond(const double* __restrict__ x, int k, double u[3]) {
  const double q0 = x[3 * (k + 1)] - x[3 * k], q1 = x[3 * (k + 1) + 1] - x[3 * k + 1],
               q2 = x[3 * (k + 1) + 2] - x[3 * k + 2];
  const double nq = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
  u[0] = q0 / nq; u[1] = q1 / nq; u[2] = q2 / nq;
}

__global__ __launch_bounds__(256) void constrain_init_kernel(const double* __restrict__ x_old,
                                                              const double* __restrict__ xs,
                                                              Bufs b, int N, double hstar,
                                                              double a, DevState* st) {
  const int M = N - 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < M) {
    const int k = t;
    double u[3];
    unit_bond(x_old, k, u);
    for (int al = 0; al < 3; ++al) {
      b.u[3 * k + al] = u[al];
      b.Qs[3 * k + al] = xs[3 * (k + 1) + al] - xs[3 * k + al];
    }
    b.T[k] = 0.0;
    double o[3];
    g_apply(x_old, k, k, hstar, a, u, o);
    for (int al = 0; al < 3; ++al) b.Gd[3 * k + al] = o[al];
    if (k + 1 < M) {
      double un[3];
      unit_bond(x_old, k + 1, un);
      g_apply(x_old, k, k + 1, hstar, a, un, o);
    } else {
      o[0] = o[1] = o[2] = 0.0;
    }
    for (int al = 0; al < 3; ++al) b.Gp[3 * k + al] = o[al];
    if (k > 0) {
      double um[3];
      unit_bond(x_old, k - 1, um);
      g_apply(x_old, k, k - 1, hstar, a, um, o);
    } else {
      o[0] = o[1] = o[2] = 0.0;
    }
    for (int al = 0; al < 3; ++al) b.Gm[3 * k + al] = o[al];
  }
  for (int64_t e = t; e < 3 * (int64_t)N; e += (int64_t)gridDim.x * blockDim.x) b.r[e] = 0.0;
  if (t == 0) {
    b.ctl->phase = PH_RESID;
    b.ctl->j = 0;
    b.ctl->newton_it = 0;
    b.ctl->kry = 0;
    b.ctl->beta = 0.0;
    b.ctl->eta = 0.0;
    st->done = 0;
  }
}

// r = D f.  A workgroup of 16 waves owns kMvI = 16 beads i and sweeps every
// bead j: lane (il, jp) = (lane % 16, lane / 16) of wave w takes phase
// 4w + jp, i.e. j = phase, phase + 64, ...; the 64 phase sums of each r_i are
// then added in a fixed order (no atomics, no cross-workgroup traffic,
// bitwise reproducible).  16 waves per workgroup keep four waves on each
// SIMD to hide the FP64 latencies.
constexpr int kMvThreads = 1024;
constexpr int kMvWaves = kMvThreads / 64;

__global__ __launch_bounds__(kMvThreads) void dmatvec_kernel(const double* __restrict__ x,
                                                       const double* __restrict__ f,
                                                       double* __restrict__ r, int N, RpyConst kc,
                                                       const DevState* __restrict__ st) {
  if (st->done) return;
  constexpr int kChunk = 512;  // beads j staged in LDS per round
  __shared__ double sx[3 * kChunk], sf[3 * kChunk];
  __shared__ double red[kMvWaves][3][kMvI];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int il = lane & 15, jp = lane >> 4;
  const int i = blockIdx.x * kMvI + il;
  const int ii = (i < N) ? i : N - 1;
  const double xi0 = x[3 * ii], xi1 = x[3 * ii + 1], xi2 = x[3 * ii + 2];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int j0 = 0; j0 < N; j0 += kChunk) {
    const int nj = (N - j0 < kChunk) ? N - j0 : kChunk;
    __syncthreads();
    for (int e = tid; e < 3 * nj; e += kMvThreads) {
      sx[e] = x[3 * j0 + e];
      sf[e] = f[3 * j0 + e];
    }
    __syncthreads();
    for (int jj = 4 * w + jp; jj < nj; jj += 4 * kMvWaves) {
      const int q = 3 * jj;
      const double f0 = sf[q], f1 = sf[q + 1], f2 = sf[q + 2];
      const double R0 = xi0 - sx[q], R1 = xi1 - sx[q + 1], R2c = xi2 - sx[q + 2];
      double cI, cRR;
      rpy_coeffs_fast(R0 * R0 + R1 * R1 + R2c * R2c, kc, cI, cRR);
      if (j0 + jj == ii) {  // D_ii = I
        cI = 1.0;
        cRR = 0.0;
      }
      const double rv = cRR * (R0 * f0 + R1 * f1 + R2c * f2);
      a0 += cI * f0 + rv * R0;
      a1 += cI * f1 + rv * R1;
      a2 += cI * f2 + rv * R2c;
    }
  }
  // phases jp = 0..3 of this wave: lanes il, il+16, il+32, il+48
  a0 += __shfl_xor(a0, 16, 64);
  a1 += __shfl_xor(a1, 16, 64);
  a2 += __shfl_xor(a2, 16, 64);
  a0 += __shfl_xor(a0, 32, 64);
  a1 += __shfl_xor(a1, 32, 64);
  a2 += __shfl_xor(a2, 32, 64);
  if (jp == 0) {
    red[w][0][il] = a0;
    red[w][1][il] = a1;
    red[w][2][il] = a2;
  }
  __syncthreads();
  if (tid < 3 * kMvI) {
    const int al = tid / kMvI, b = tid % kMvI;
    const int ib = blockIdx.x * kMvI + b;
    double acc = 0.0;
    for (int q = 0; q < kMvWaves; ++q) acc += red[q][al][b];
    if (ib < N) r[3 * ib + al] = acc;
  }
}

// ------------------------------------------------------------ controller
struct Ctl {
  double* red;  // LDS, >= 16
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double nanmax(double a, double b) {
  return (a > b || a != a) ? a : b;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = nanmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x, w = tid >> 6;
  v = wave_sum(v);
  if ((tid & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < kCtlThreads / 64; ++q) s += red[q];
  __syncthreads();
  return s;
}
__device__ double block_max(double v, double* red) {
  const int tid = threadIdx.x, w = tid >> 6;
  v = wave_max(v);
  if ((tid & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
  for (int q = 1; q < kCtlThreads / 64; ++q) s = nanmax(s, red[q]);
  __syncthreads();
  return s;
}

// Eight block sums at once (fixed order); every thread gets the results.
__device__ void block_sum8(double v[8], double (*red8)[8]) {
  const int tid = threadIdx.x, w = tid >> 6;
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = wave_sum(v[u]);
  if ((tid & 63) == 0)
#pragma unroll
    for (int u = 0; u < 8; ++u) red8[w][u] = v[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    double s = 0.0;
    for (int q = 0; q < kCtlThreads / 64; ++q) s += red8[q][u];
    v[u] = s;
  }
  __syncthreads();
}

// Parallel cyclic reduction (Hockney) for the tridiagonal system
// (lo, di, up) x = v, M <= kMaxRods, in LDS; result to out (global).
__device__ void pcr_solve(const double* __restrict__ lo, const double* __restrict__ di,
                          const double* __restrict__ up, const double* __restrict__ v,
                          double* __restrict__ out, int M, double* pa, double* pb, double* pc,
                          double* pd) {
  constexpr int R = kMaxRods / kCtlThreads;
  const int tid = threadIdx.x;
  for (int i = tid; i < M; i += kCtlThreads) {
    pa[i] = lo[i];
    pb[i] = di[i];
    pc[i] = up[i];
    pd[i] = v[i];
  }
  __syncthreads();
  for (int s = 1; s < M; s <<= 1) {
    double na[R], nb[R], nc[R], nd[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = tid + q * kCtlThreads;
      if (i < M) {
        double bb = pb[i], dd = pd[i], aa = 0.0, cc = 0.0;
        if (i - s >= 0) {
          const double al = -pa[i] / pb[i - s];
          aa = al * pa[i - s];
          bb += al * pc[i - s];
          dd += al * pd[i - s];
        }
        if (i + s < M) {
          const double ga = -pc[i] / pb[i + s];
          cc = ga * pc[i + s];
          bb += ga * pa[i + s];
          dd += ga * pd[i + s];
        }
        na[q] = aa; nb[q] = bb; nc[q] = cc; nd[q] = dd;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = tid + q * kCtlThreads;
      if (i < M) {
        pa[i] = na[q]; pb[i] = nb[q]; pc[i] = nc[q]; pd[i] = nd[q];
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < M; i += kCtlThreads) out[i] = pd[i] / pb[i];
  __syncthreads();
}

// f_i = z_i u_i - z_{i-1} u_{i-1}
__device__ void rod_forces(const double* __restrict__ z, const double* __restrict__ u,
                           double* __restrict__ f, int N) {
  const int M = N - 1;
  for (int i = threadIdx.x; i < N; i += kCtlThreads) {
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      double v = 0.0;
      if (i < M) v += z[i] * u[3 * i + al];
      if (i > 0) v -= z[i - 1] * u[3 * (i - 1) + al];
      f[3 * i + al] = v;
    }
  }
}

__global__ __launch_bounds__(kCtlThreads) void newton_controller_kernel(
    Bufs b, double* __restrict__ xs, double* __restrict__ T_out, int N, double dt,
    double bl, double tol, int maxit, DevState* __restrict__ st) {
  __shared__ double pa[kMaxRods], pb[kMaxRods], pc[kMaxRods], pd[kMaxRods];
  __shared__ double red[kCtlThreads / 64];
  __shared__ double red8[kCtlThreads / 64][8];
  __shared__ double hcur[kKmax + 1], hsum[kKmax + 1];
  __shared__ int sh_flag;
  if (st->done) return;
  const int tid = threadIdx.x;
  const int M = N - 1;
  const int64_t n3 = 3 * (int64_t)N;
  NewtonCtl* ctl = b.ctl;
  const int phase = ctl->phase;
  if (phase == PH_RESID) {
    double err = 0.0, res = 0.0, g2 = 0.0;
    for (int k = tid; k < M; k += kCtlThreads) {
      double q[3];
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        q[al] = b.Qs[3 * k + al] + dt * (b.r[3 * (k + 1) + al] - b.r[3 * k + al]);
        b.Q[3 * k + al] = q[al];
      }
      const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
      const double e = fabs(sqrt(q2) / bl - 1.0);
      const double g = q2 - bl * bl;
      err = nanmax(err, e);
      res = nanmax(res, fabs(g));
      g2 += g * g;
      b.rhs[k] = -g;
    }
    err = block_max(err, red);
    res = block_max(res, red);
    g2 = block_sum(g2, red);
    const int it = ctl->newton_it;
    if (err <= tol || it >= maxit || !(err == err) || isinf(err)) {
      for (int64_t e = tid; e < n3; e += kCtlThreads) xs[e] += dt * b.r[e];
      if (T_out)
        for (int k = tid; k < M; k += kCtlThreads) T_out[k] = b.T[k];
      if (tid == 0) {
        if (st->status == BD_OK) st->status = (err <= tol) ? BD_OK : BD_ERR_NO_CONVERGE;
        st->newton_iters = it;
        st->krylov_iters = ctl->kry;
        st->max_rod_err = err;
        st->last_newton_res = res;
        st->done = 1;
      }
      return;
    }
    for (int k = tid; k < M; k += kCtlThreads) {
      const double* q = b.Q + 3 * k;
      const double* gd = b.Gd + 3 * k;
      const double* gp = b.Gp + 3 * k;
      const double* gm = b.Gm + 3 * k;
      b.di[k] = -2.0 * dt * (q[0] * gd[0] + q[1] * gd[1] + q[2] * gd[2]);
      b.up[k] = (k + 1 < M) ? -2.0 * dt * (q[0] * gp[0] + q[1] * gp[1] + q[2] * gp[2]) : 0.0;
      b.lo[k] = (k > 0) ? -2.0 * dt * (q[0] * gm[0] + q[1] * gm[1] + q[2] * gm[2]) : 0.0;
    }
    // inexact-Newton forcing term: balance the quadratic term of g against
    // the linear-solve error, never tighter than the final tolerance needs
    const double grms = sqrt(g2 / (double)M) / (bl * bl);
    double eta = 0.25 * grms;
    const double floor_eta = 0.5 * tol / grms;
    if (eta < floor_eta) eta = floor_eta;
    if (eta > 0.1) eta = 0.1;
    const double beta = sqrt(g2);
    for (int k = tid; k < M; k += kCtlThreads) b.V[k] = b.rhs[k] / beta;
    __syncthreads();
    if (tid == 0) {
      b.s[0] = beta;
      ctl->phase = PH_KRYLOV;
      ctl->j = 0;
      ctl->beta = beta;
      ctl->eta = eta;
    }
    pcr_solve(b.lo, b.di, b.up, b.V, b.z, M, pa, pb, pc, pd);
    rod_forces(b.z, b.u, b.f, N);
    return;
  }

  // PH_KRYLOV: r = D f(z_j); w = J z_j into V[j+1]
  const int j = ctl->j;
  const double beta = ctl->beta, eta = ctl->eta;
  double* w = b.V + (int64_t)(j + 1) * M;
  for (int k = tid; k < M; k += kCtlThreads) {
    const double* q = b.Q + 3 * k;
    const double d0 = b.r[3 * (k + 1)] - b.r[3 * k];
    const double d1 = b.r[3 * (k + 1) + 1] - b.r[3 * k + 1];
    const double d2 = b.r[3 * (k + 1) + 2] - b.r[3 * k + 2];
    w[k] = 2.0 * dt * (q[0] * d0 + q[1] * d1 + q[2] * d2);
  }
  __syncthreads();
  // Classical Gram-Schmidt with one re-orthogonalisation: each pass forms
  // every projection h_i = <w, v_i> (block reductions of 8 at a time), then
  // w -= sum_i h_i v_i.
  for (int i = tid; i <= j; i += kCtlThreads) hsum[i] = 0.0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int i0 = 0; i0 <= j; i0 += 8) {
      double pr[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pr[u] = 0.0;
      for (int k = tid; k < M; k += kCtlThreads) {
        const double wk = w[k];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (i0 + u <= j) pr[u] += wk * b.V[(int64_t)(i0 + u) * M + k];
      }
      block_sum8(pr, red8);
      if (tid < 8 && i0 + tid <= j) {
        hcur[i0 + tid] = pr[tid];
        hsum[i0 + tid] += pr[tid];
      }
      __syncthreads();
    }
    for (int k = tid; k < M; k += kCtlThreads) {
      double acc = 0.0;
      for (int i = 0; i <= j; ++i) acc += hcur[i] * b.V[(int64_t)i * M + k];
      w[k] -= acc;
    }
    __syncthreads();
  }
  if (tid <= j) b.H[tid * kKmax + j] = hsum[tid];
  double part = 0.0;
  for (int k = tid; k < M; k += kCtlThreads) part += w[k] * w[k];
  const double hn = sqrt(block_sum(part, red));
  if (hn > 0.0)
    for (int k = tid; k < M; k += kCtlThreads) w[k] /= hn;
  __syncthreads();
  if (tid == 0) {
    double* H = b.H;
    H[(j + 1) * kKmax + j] = hn;
    for (int i = 0; i < j; ++i) {
      const double a0 = H[i * kKmax + j], a1 = H[(i + 1) * kKmax + j];
      H[i * kKmax + j] = b.cs[i] * a0 + b.sn[i] * a1;
      H[(i + 1) * kKmax + j] = -b.sn[i] * a0 + b.cs[i] * a1;
    }
    const double a0 = H[j * kKmax + j], a1 = H[(j + 1) * kKmax + j];
    const double den = sqrt(a0 * a0 + a1 * a1);
    b.cs[j] = (den > 0.0) ? a0 / den : 1.0;
    b.sn[j] = (den > 0.0) ? a1 / den : 0.0;
    H[j * kKmax + j] = den;
    H[(j + 1) * kKmax + j] = 0.0;
    b.s[j + 1] = -b.sn[j] * b.s[j];
    b.s[j] = b.cs[j] * b.s[j];
    ctl->kry += 1;
    const int stop = (fabs(b.s[j + 1]) <= eta * beta) || (hn == 0.0) || (j + 1 == kKmax);
    sh_flag = stop;
    if (stop) {
      const int kk = j + 1;
      for (int i = kk - 1; i >= 0; --i) {
        double t = b.s[i];
        for (int c = i + 1; c < kk; ++c) t -= H[i * kKmax + c] * b.y[c];
        b.y[i] = t / H[i * kKmax + i];
      }
    }
  }
  __syncthreads();
  if (sh_flag) {
    const int kk = j + 1;
    for (int k = tid; k < M; k += kCtlThreads) {
      double acc = 0.0;
      for (int i = 0; i < kk; ++i) acc += b.y[i] * b.V[(int64_t)i * M + k];
      b.rhs[k] = acc;
    }
    __syncthreads();
    pcr_solve(b.lo, b.di, b.up, b.rhs, b.z, M, pa, pb, pc, pd);
    for (int k = tid; k < M; k += kCtlThreads) b.T[k] += b.z[k];
    __syncthreads();
    rod_forces(b.T, b.u, b.f, N);
    if (tid == 0) {
      ctl->newton_it += 1;
      ctl->phase = PH_RESID;
    }
  } else {
    pcr_solve(b.lo, b.di, b.up, w, b.z, M, pa, pb, pc, pd);
    rod_forces(b.z, b.u, b.f, N);
    if (tid == 0) ctl->j = j + 1;
  }
}

}  // namespace

size_t constrain_workspace_bytes(int64_t n_beads) { return carve_bytes((int)n_beads); }

int constrain_max_beads() { return kMaxRods + 1; }

hipError_t launch_constrain(hipStream_t s, const bd_params_t& p, const double* x_old, double* xs,
                            double* T_out, void* ws, DevState* st, DevState* host_state,
                            int* pairs_hint) {
  const int N = p.n_beads;
  const int M = N - 1;
  Bufs b = carve(ws, N);
  const int ithreads = M > 0 ? M : 1;
  int iblk = (ithreads + 255) / 256;
  if (iblk < 16) iblk = 16;
  BD_LAUNCH("constrain_init", constrain_init_kernel, dim3(iblk), dim3(256), 0, s, x_old, xs, b, N,
            p.hstar, p.a, st);
  BD_LAUNCH("newton_controller", newton_controller_kernel, dim3(1), dim3(kCtlThreads), 0, s, b, xs,
            T_out, N, p.dt, p.b, p.newton_tol, p.newton_maxit, st);
  const dim3 mvgrid((N + kMvI - 1) / kMvI);
  const RpyConst kc = rpy_const(p.hstar, p.a);
  // Each (matvec, controller) pair advances the iteration by one product with
  // D.  The first batch is sized from the previous call's count, then the
  // host polls the device flag after every further small batch; launches
  // after convergence return at once.
  const int cap = (p.newton_maxit + 1) * (kKmax + 2);
  int batch = (pairs_hint && *pairs_hint > 0) ? *pairs_hint + 1 : 8;
  int launched = 0;
  while (launched < cap) {
    if (batch > cap - launched) batch = cap - launched;
    for (int c = 0; c < batch; ++c) {
      BD_LAUNCH("dmatvec", dmatvec_kernel, mvgrid, dim3(kMvThreads), 0, s, x_old, b.f, b.r, N, kc,
                st);
      BD_LAUNCH("newton_controller", newton_controller_kernel, dim3(1), dim3(kCtlThreads), 0, s, b,
                xs, T_out, N, p.dt, p.b, p.newton_tol, p.newton_maxit, st);
    }
    launched += batch;
    hipError_t e = hipMemcpyAsync(host_state, st, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (host_state->done) break;
    batch = 4;
  }
  if (pairs_hint && host_state->done)
    *pairs_hint = host_state->newton_iters + host_state->krylov_iters;
  return hipGetLastError();
}

}  // namespace bd
