// Rigid-rod constraint: tensions T_k (k = 0..N-2) along the rod directions
// u_k at the start of the step such that
//   Q_k(T) = Q*_k + dt (r_{k+1} - r_k),  r = D f(T),  f_i = T_i u_i - T_{i-1} u_{i-1}
// has |Q_k| = b, i.e. g_k(T) = |Q_k|^2 - b^2 = 0 (the infinite-stiffness limit of
// the semi-implicit spring update, Eqs. 13-17, with every tension coupled
// through the full diffusion tensor of Eqs. 7-9).  Then x^{t+dt} = x* + dt r.
//
// Inexact Newton from T = 0; each Newton correction J delta = -g is solved by
// GMRES (classical Gram-Schmidt with one re-orthogonalisation, Givens
// rotations) right-preconditioned with the
// tridiagonal part of J, J_kl = -2 dt Q_k . G_kl u_l, G_kl = D_{k+1,l+1} -
// D_{k+1,l} - D_{k,l+1} + D_{k,l}.  Every product with D is matrix-free.
//
// Device work is split in two kernels that the host launches alternately:
//   dmatvec     r = D f over all bead pairs, one workgroup per 16 beads i
//               (no atomics, fixed reduction order);
//   controller  one workgroup of 512 threads: advances the Newton/GMRES
//               state machine by one matrix-vector product (residual check,
//               band Jacobian, Arnoldi step, cyclic-reduction tridiagonal
//               solve in LDS), then writes the next f.
// Once the iteration has finished both kernels return immediately.
#include "common.hpp"
#include "profile.hpp"
#include "rpy_device.hpp"

namespace bd {

namespace {

constexpr int kKmax = 60;          // GMRES iterations per Newton step
constexpr int kCtlThreads = 512;   // controller workgroup
constexpr int kMaxRods = 4096;     // LDS capacity of the tridiagonal solve
constexpr int kMaxRodsBig = 8192;  // longer chains: the tridiagonal system in global memory
constexpr int kMvI = 16;           // beads i per matvec workgroup

enum { PH_RESID = 0, PH_KRYLOV = 1, PH_ADJ_RHS = 2 };

struct NewtonCtl {
  int32_t phase;
  int32_t j;
  int32_t newton_it;
  int32_t kry;
  double beta;
  double eta;
};

// Grid barrier of the one-launch solve: arrival counter, generation and an
// abort flag (a workgroup that waited too long).
struct GridBar {
  uint32_t count, gen, abort, pad;
};

struct Bufs {
  double *u, *Qs, *Q, *Gd, *Gp, *Gm, *T, *lo, *di, *up, *f, *r, *V, *H, *cs, *sn, *s;
  NewtonCtl* ctl;
  GridBar* gb;
  double* tri;  // chains of more than kMaxRods rods: the tridiagonal system (4 x padded M)
};


__host__ __device__ Bufs carve(void* ws, int N) {
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
  b.f = take(3 * (size_t)N);
  b.r = take(3 * (size_t)N);
  b.V = take((size_t)(kKmax + 1) * M);
  b.H = take((size_t)(kKmax + 1) * kKmax);
  b.cs = take(kKmax);
  b.sn = take(kKmax);
  b.s = take(kKmax + 1);
  b.ctl = reinterpret_cast<NewtonCtl*>(take(8));
  b.gb = reinterpret_cast<GridBar*>(take(2));
  b.tri = nullptr;
  if (M > kMaxRods) b.tri = take(4 * (size_t)(M + M / 32 + 1));
  return b;
}

size_t carve_bytes(int N) {
  Bufs b = carve(nullptr, N);
  return (b.tri ? reinterpret_cast<size_t>(b.tri) + sizeof(double) * 4 * (size_t)((N - 1) + (N - 1) / 32 + 1)
                : reinterpret_cast<size_t>(b.gb) + 256);
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

__host__ __device__ RpyConst rpy_const(double hstar, double a) {
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

__device__ __forceinline__ void constrain_init_body(int bx, const double* __restrict__ x_old,
                                                    const double* __restrict__ xs, Bufs b, int N,
                                                    double hstar, double a, DevState* st) {
  const int M = N - 1;
  const int t = bx * blockDim.x + threadIdx.x;
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
    b.gb->count = 0;
    b.gb->abort = 0;
    st->done = 0;
  }
}

__global__ __launch_bounds__(256) void constrain_init_kernel(const double* __restrict__ x_old,
                                                              const double* __restrict__ xs,
                                                              Bufs b, int N, double hstar,
                                                              double a, DevState* st) {
  constrain_init_body(blockIdx.x, x_old, xs, b, N, hstar, a, st);
}

// Far-field coefficients (R >= 2a) of an RPY block, and 1/R; the same
// arithmetic as rpy_coeffs_fast.
__device__ __forceinline__ void rpy_far_coeffs(double R2, const RpyConst& k, double& cI,
                                               double& cRR, double& y) {
  y = __builtin_amdgcn_rsq(R2);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double h = 0.5 * R2 * y;
    y = fma(-h, y, 1.5) * y;
  }
  const double inv2 = y * y;
  const double pre = k.far_pre * y;
  const double t = k.a2 * inv2;
  cI = pre * (1.0 + (2.0 / 3.0) * t);
  cRR = pre * (1.0 - 2.0 * t) * inv2;
}

// Near-field coefficients (R < 2a) from the same 1/R.
__device__ __forceinline__ void rpy_near_coeffs(double R2, double y, const RpyConst& k, double& cI,
                                                double& cRR) {
  const double R = (R2 > 0.0) ? R2 * y : 0.0;  // coincident beads: the R -> 0 limit
  cI = k.near_pre * (8.0 / 3.0 - k.near_r * R);
  cRR = (R2 > 0.0) ? k.near_rr * y : 0.0;
}

// r = D f.  A workgroup of 16 waves owns kMvI = 16 beads i and sweeps every
// bead j: lane (il, jp) = (lane % 16, lane / 16) of wave w takes phase
// 4w + jp, i.e. j = phase, phase + 64, ...; the 64 phase sums of each r_i are
// then added in a fixed order (no atomics, no cross-workgroup traffic,
// bitwise reproducible).  16 waves per workgroup keep four waves on each
// SIMD to hide the FP64 latencies, and each lane takes two of its beads j
// per iteration (two independent chains; far-field coefficients straight
// through, the rare near-field pairs behind a wave-uniform branch), adding
// them in the same order as one at a time.
constexpr int kMvThreads = 1024;
constexpr int kMvWaves = kMvThreads / 64;

// kChunk: beads j staged in LDS per round (2048: 96 KB, one workgroup per
// CU; 1024: two workgroups per CU, for the ensembles' shorter chains).
// kThreads: 1024, or 512 where each wave also does the work of the wave
// eight places on (the two sets of phases kept in separate accumulators,
// so every sum is formed in the same order as with 1024 threads).  LDS,
// from the caller: sxf (6 kChunk doubles, 16-byte aligned: bead j's
// position and force side by side, x0 x1 x2 f0 f1 f2, read as three
// 16-byte words) and red (kMvWaves x 3 x kMvI).
constexpr int kMvLds = 3 * kMvWaves * kMvI;

template <int kChunk, int kThreads>
__device__ __forceinline__ void dmatvec_body(int bx, const double* __restrict__ x,
                                             const double* __restrict__ f, double* __restrict__ r,
                                             int N, const RpyConst& kc,
                                             const DevState* __restrict__ st, double* sxf,
                                             double* redp) {
  static_assert(kThreads == 1024 || kThreads == 512, "one or two phase sets per wave");
  constexpr int kV = kMvThreads / kThreads;  // phase sets per wave
  constexpr int kW = kThreads / 64;          // waves
  if (st && st->done) return;  // st null: always run
  double(*red)[3][kMvI] = reinterpret_cast<double(*)[3][kMvI]>(redp);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int il = lane & 15, jp = lane >> 4;
  const int i = bx * kMvI + il;
  const int ii = (i < N) ? i : N - 1;
  const double xi0 = x[3 * ii], xi1 = x[3 * ii + 1], xi2 = x[3 * ii + 2];
  double a0[kV], a1[kV], a2[kV];
#pragma unroll
  for (int v = 0; v < kV; ++v) a0[v] = a1[v] = a2[v] = 0.0;
  for (int j0 = 0; j0 < N; j0 += kChunk) {
    const int nj = (N - j0 < kChunk) ? N - j0 : kChunk;
    __syncthreads();
    for (int e = tid; e < 3 * nj; e += kThreads) {
      const int jb = e / 3, c = e - 3 * jb;
      sxf[6 * jb + c] = x[3 * j0 + e];
      sxf[6 * jb + 3 + c] = f[3 * j0 + e];
    }
    __syncthreads();
    for (int jt = 4 * w + jp; jt < nj; jt += 8 * kMvWaves) {
#pragma unroll
      for (int v = 0; v < kV; ++v) {
        const int jj = jt + 4 * kW * v;  // phase 4 (w + kW v) + jp
        if (jj >= nj) break;
        const int jb = jj + 4 * kMvWaves;
        const bool hb = jb < nj;
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2* pa = reinterpret_cast<const d2*>(sxf + 6 * jj);
        const d2* pb = reinterpret_cast<const d2*>(sxf + 6 * (hb ? jb : jj));
        const d2 ua0 = pa[0], ua1 = pa[1], ua2 = pa[2];  // x0 x1 | x2 f0 | f1 f2
        const d2 ub0 = pb[0], ub1 = pb[1], ub2 = pb[2];
        const double fa0 = ua1[1], fa1 = ua2[0], fa2 = ua2[1];
        const double fb0 = ub1[1], fb1 = ub2[0], fb2 = ub2[1];
        const double Ra0 = xi0 - ua0[0], Ra1 = xi1 - ua0[1], Ra2 = xi2 - ua1[0];
        const double Rb0 = xi0 - ub0[0], Rb1 = xi1 - ub0[1], Rb2 = xi2 - ub1[0];
        const double R2a = Ra0 * Ra0 + Ra1 * Ra1 + Ra2 * Ra2;
        const double R2b = Rb0 * Rb0 + Rb1 * Rb1 + Rb2 * Rb2;
        double cIa, cRRa, ya, cIb, cRRb, yb;
        rpy_far_coeffs(R2a, kc, cIa, cRRa, ya);
        rpy_far_coeffs(R2b, kc, cIb, cRRb, yb);
        const bool na = !(R2a >= kc.a2x2), nb = !(R2b >= kc.a2x2);
        if (na || nb) {  // rare: pairs closer than 2a
          if (na) rpy_near_coeffs(R2a, ya, kc, cIa, cRRa);
          if (nb) rpy_near_coeffs(R2b, yb, kc, cIb, cRRb);
        }
        if (j0 + jj == ii) {  // D_ii = I
          cIa = 1.0;
          cRRa = 0.0;
        }
        if (j0 + jb == ii) {
          cIb = 1.0;
          cRRb = 0.0;
        }
        if (!hb) {  // past the chunk: no second bead
          cIb = 0.0;
          cRRb = 0.0;
        }
        const double rva = cRRa * (Ra0 * fa0 + Ra1 * fa1 + Ra2 * fa2);
        const double rvb = cRRb * (Rb0 * fb0 + Rb1 * fb1 + Rb2 * fb2);
        a0[v] += cIa * fa0 + rva * Ra0;
        a1[v] += cIa * fa1 + rva * Ra1;
        a2[v] += cIa * fa2 + rva * Ra2;
        a0[v] += cIb * fb0 + rvb * Rb0;
        a1[v] += cIb * fb1 + rvb * Rb1;
        a2[v] += cIb * fb2 + rvb * Rb2;
      }
    }
  }
  // phases jp = 0..3 of a phase set: lanes il, il+16, il+32, il+48
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    double b0 = a0[v], b1 = a1[v], b2 = a2[v];
    b0 += __shfl_xor(b0, 16, 64);
    b1 += __shfl_xor(b1, 16, 64);
    b2 += __shfl_xor(b2, 16, 64);
    b0 += __shfl_xor(b0, 32, 64);
    b1 += __shfl_xor(b1, 32, 64);
    b2 += __shfl_xor(b2, 32, 64);
    if (jp == 0) {
      red[w + kW * v][0][il] = b0;
      red[w + kW * v][1][il] = b1;
      red[w + kW * v][2][il] = b2;
    }
  }
  __syncthreads();
  if (tid < 3 * kMvI) {
    const int al = tid / kMvI, b = tid % kMvI;
    const int ib = bx * kMvI + b;
    double acc = 0.0;
    for (int q = 0; q < kMvWaves; ++q) acc += red[q][al][b];
    if (ib < N) r[3 * ib + al] = acc;
  }
}

__global__ __launch_bounds__(kMvThreads / 2) void dmatvec_kernel(const double* __restrict__ x,
                                                       const double* __restrict__ f,
                                                       double* __restrict__ r, int N, RpyConst kc,
                                                       const DevState* __restrict__ st) {
  __shared__ __attribute__((aligned(16))) double sxf[6 * 2048];
  __shared__ double red[kMvLds];
  dmatvec_body<2048, kMvThreads / 2>(blockIdx.x, x, f, r, N, kc, st, sxf, red);
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

// 1/x from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

// Cyclic reduction (odd-even elimination) for the tridiagonal system
// (pa, pb, pc) x = pd of M <= kMaxRods unknowns, all in LDS and filled by
// the caller; the solution is left in pd.  Forward levels s = 1, 2, 4, ...
// eliminate the couplings of rows i = 2s m + 2s - 1 to rows i -+ s (rows
// read and rows written at one level are disjoint, so one barrier per
// level); backward levels solve rows i = 2s m + s - 1 from rows i -+ s.
// The first row's sub-diagonal and the last row's super-diagonal are zero.
// Every LDS read is unconditional (clamped index, contribution selected)
// so that a level costs one LDS round trip.
constexpr int kR = kMaxRods / kCtlThreads;  // unknowns per thread (k = tid + kCtlThreads q)
constexpr int kRBig = kMaxRodsBig / kCtlThreads;

__device__ __forceinline__ int lp(int i) { return i + (i >> 5); }  // padded LDS index
constexpr int kPadRods = kMaxRods + kMaxRods / 32;

__device__ void cr_solve(int M, double* pa, double* pb, double* pc, double* pd) {
  const int tid = threadIdx.x;
  __syncthreads();
  int s = 1;
  for (; 2 * s - 1 < M; s <<= 1) {
    for (int i = 2 * s - 1 + 2 * s * tid; i < M; i += 2 * s * kCtlThreads) {
      const bool right = i + s < M;
      const int ir = right ? i + s : i;
      const int p = lp(i), pl = lp(i - s), pr = lp(ir);
      const double ai = pa[p], bi = pb[p], ci = pc[p], di = pd[p];
      const double al_ = pa[pl], bl_ = pb[pl], cl_ = pc[pl], dl_ = pd[pl];
      const double ar_ = pa[pr], br_ = pb[pr], cr_ = pc[pr], dr_ = pd[pr];
      const double al = -ai * rcp_refined(bl_);
      const double ga = right ? -ci * rcp_refined(br_) : 0.0;
      pa[p] = al * al_;
      pb[p] = bi + al * cl_ + ga * ar_;
      pc[p] = ga * cr_;
      pd[p] = di + al * dl_ + ga * dr_;
    }
    __syncthreads();
  }
  for (; s >= 1; s >>= 1) {
    for (int i = s - 1 + 2 * s * tid; i < M; i += 2 * s * kCtlThreads) {
      const bool left = i - s >= 0, right = i + s < M;
      const int p = lp(i);
      const double xl = pd[lp(left ? i - s : i)], xr = pd[lp(right ? i + s : i)];
      double t = pd[p];
      if (left) t -= pa[p] * xl;
      if (right) t -= pc[p] * xr;
      pd[p] = t * rcp_refined(pb[p]);
    }
    __syncthreads();
  }
}

// f_i = z_i u_i - z_{i-1} u_{i-1} with z in LDS (z_{-1} = z_{N-1} = 0).  The
// bead loop has a fixed trip count and every load a valid (clamped) index, so
// all loads of u issue together.
template <int kRr = kR>
__device__ void rod_forces(const double* z, const double* __restrict__ u,
                           double* __restrict__ f, int N) {
  const int M = N - 1;
#pragma unroll
  for (int q = 0; q <= kRr; ++q) {
    if (q % 3 == 0) __builtin_amdgcn_sched_barrier(0);  // loads in groups of three beads
    const int i = threadIdx.x + q * kCtlThreads;
    const int ic = (i < M) ? i : M - 1, im = (i > 0 && i - 1 < M) ? i - 1 : 0;
    double ui[3], um[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      ui[al] = u[3 * ic + al];
      um[al] = u[3 * im + al];
    }
    if (i < N) {
      const double zi = (i < M) ? z[lp(i)] : 0.0, zm = (i > 0) ? z[lp(i - 1)] : 0.0;
#pragma unroll
      for (int al = 0; al < 3; ++al) f[3 * i + al] = zi * ui[al] - zm * um[al];
    }
  }
}

// The controller keeps the serial parts of GMRES (rotations, the small
// triangular solve) in LDS and each thread's share of the Krylov vector in
// registers (unknowns k = tid + kCtlThreads q): global memory is touched only
// by batches of independent loads and by the stores of the next state.
//
// kAdj: the same Krylov machinery solves the adjoint system of the tension
// solve, J^T mu = -dt U^T Delta D xbar (see launch_constrain_adjoint): J^T
// is J with the roles of the rod directions u (forces) and the new rod
// vectors Q (contraction) exchanged, the band arrays hold tri(J^T), and the
// first product is D xbar.  xs then receives z = xbar - 2 Delta^T (Q mu).
// The controller's LDS: the tridiagonal system, reduction slots and the
// small GMRES state, carved from one arena of kCtlLds doubles.
constexpr int kCtlLds = 4 * kPadRods + kCtlThreads / 64 + 8 * (kCtlThreads / 64) +
                        2 * (kKmax + 1) + 2 * kKmax + (kKmax + 1) + kKmax + 2;

//
// kRr = kRBig: chains of more than kMaxRods rods, the tridiagonal system in
// global memory (b.tri; the same cyclic reduction, levels separated by the
// workgroup barrier) and kRBig unknowns per thread.
template <bool kAdj, int kRr = kR>
__device__ __forceinline__ void newton_controller_body(
    Bufs b, double* __restrict__ xs, double* __restrict__ T_out, int N, double dt,
    double bl, double tol, int maxit, DevState* __restrict__ st, double* arena,
    const double* __restrict__ xbar = nullptr) {
  constexpr int kR = kRr;
  const int ptri = (kRr == kRBig) ? (N - 1) + (N - 1) / 32 + 1 : kPadRods;
  double* pa = (kRr == kRBig) ? b.tri : arena;
  double* pb = pa + ptri;
  double* pc = pb + ptri;
  double* pd = pc + ptri;
  double* red = arena + 4 * kPadRods;
  double(*red8)[8] = reinterpret_cast<double(*)[8]>(red + kCtlThreads / 64);
  double* hcur = red + kCtlThreads / 64 + 8 * (kCtlThreads / 64);
  double* hsum = hcur + (kKmax + 1);
  double* cs_s = hsum + (kKmax + 1);
  double* sn_s = cs_s + kKmax;
  double* s_s = sn_s + kKmax;
  double* y_s = s_s + (kKmax + 1);
  int& sh_flag = *reinterpret_cast<int*>(y_s + kKmax);
  const int tid = threadIdx.x;
  const int M = N - 1;
  const int64_t n3 = 3 * (int64_t)N;
  NewtonCtl* ctl = b.ctl;
  // state: independent loads, one round trip
  const int done = st->done;
  const int phase = ctl->phase, j = ctl->j, newton_it = ctl->newton_it;
  const double beta_c = ctl->beta, eta = ctl->eta;
  if (done) return;
  if (kAdj && phase == PH_ADJ_RHS) {
    // rhs = -dt U^T Delta (D xbar), with r = D xbar from the first product
    double g2 = 0.0;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      const int kc = (k < M) ? k : M - 1;
      double v = 0.0;
#pragma unroll
      for (int al = 0; al < 3; ++al)
        v += b.u[3 * kc + al] * (b.r[3 * (kc + 1) + al] - b.r[3 * kc + al]);
      const double lo = b.lo[kc], di = b.di[kc], up = b.up[kc];
      if (k < M) {
        const double rhs = -dt * v;
        pd[lp(k)] = rhs;
        g2 += rhs * rhs;
        pa[lp(k)] = lo;
        pb[lp(k)] = di;
        pc[lp(k)] = up;
      }
    }
    const double beta = sqrt(block_sum(g2, red));
    if (!(beta > 0.0)) {  // mu = 0 (or a non-finite right side)
      for (int64_t e = tid; e < n3; e += kCtlThreads) xs[e] = xbar[e];
      if (tid == 0) {
        if (st->status == BD_OK && !(beta == 0.0)) st->status = BD_ERR_NO_CONVERGE;
        st->done = 1;
      }
      return;
    }
    const double rb = 1.0 / beta;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      if (k < M) {
        const double v0 = pd[lp(k)] * rb;
        b.V[k] = v0;
        pd[lp(k)] = v0;
      }
    }
    if (tid == 0) {
      b.s[0] = beta;
      ctl->phase = PH_KRYLOV;
      ctl->j = 0;
      ctl->beta = beta;
      ctl->eta = tol;
    }
    cr_solve(M, pa, pb, pc, pd);
    rod_forces<kRr>(pd, b.Q, b.f, N);
    return;
  }
  if (!kAdj && phase == PH_RESID) {
    double err = 0.0, res = 0.0, g2 = 0.0;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      if (q % 2 == 0) __builtin_amdgcn_sched_barrier(0);  // loads in groups of two rods
      const int k = tid + q * kCtlThreads;
      const int kc = (k < M) ? k : M - 1;  // valid index: loads issue together
      double qv[3], gd[3], gp[3], gm[3];
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        qv[al] = b.Qs[3 * kc + al] + dt * (b.r[3 * (kc + 1) + al] - b.r[3 * kc + al]);
        gd[al] = b.Gd[3 * kc + al];
        gp[al] = b.Gp[3 * kc + al];
        gm[al] = b.Gm[3 * kc + al];
      }
      if (k < M) {
#pragma unroll
        for (int al = 0; al < 3; ++al) b.Q[3 * k + al] = qv[al];
        const double q2 = qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2];
        const double e = fabs(sqrt(q2) / bl - 1.0);
        const double g = q2 - bl * bl;
        err = nanmax(err, e);
        res = nanmax(res, fabs(g));
        g2 += g * g;
        pd[lp(k)] = -g;
        const double di = -2.0 * dt * (qv[0] * gd[0] + qv[1] * gd[1] + qv[2] * gd[2]);
        const double up = (k + 1 < M) ? -2.0 * dt * (qv[0] * gp[0] + qv[1] * gp[1] + qv[2] * gp[2]) : 0.0;
        const double lo = (k > 0) ? -2.0 * dt * (qv[0] * gm[0] + qv[1] * gm[1] + qv[2] * gm[2]) : 0.0;
        b.di[k] = di;
        b.up[k] = up;
        b.lo[k] = lo;
        pa[lp(k)] = lo;
        pb[lp(k)] = di;
        pc[lp(k)] = up;
      }
    }
    err = block_max(err, red);
    res = block_max(res, red);
    g2 = block_sum(g2, red);
    if (err <= tol || newton_it >= maxit || !(err == err) || isinf(err)) {
      for (int64_t e = tid; e < n3; e += kCtlThreads) xs[e] += dt * b.r[e];
      if (T_out)
        for (int k = tid; k < M; k += kCtlThreads) T_out[k] = b.T[k];
      if (tid == 0) {
        if (st->status == BD_OK) st->status = (err <= tol) ? BD_OK : BD_ERR_NO_CONVERGE;
        st->newton_iters = newton_it;
        st->krylov_iters = ctl->kry;
        st->max_rod_err = err;
        st->last_newton_res = res;
        st->done = 1;
      }
      return;
    }
    // inexact-Newton forcing term: balance the quadratic term of g against
    // the linear-solve error, never tighter than the final tolerance needs
    const double grms = sqrt(g2 / (double)M) / (bl * bl);
    double eta_n = 0.25 * grms;
    const double floor_eta = 0.5 * tol / grms;
    if (eta_n < floor_eta) eta_n = floor_eta;
    if (eta_n > 0.1) eta_n = 0.1;
    const double beta = sqrt(g2);
    const double rb = 1.0 / beta;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      if (k < M) {
        const double v0 = pd[lp(k)] * rb;
        b.V[k] = v0;
        pd[lp(k)] = v0;
      }
    }
    if (tid == 0) {
      b.s[0] = beta;
      ctl->phase = PH_KRYLOV;
      ctl->j = 0;
      ctl->beta = beta;
      ctl->eta = eta_n;
    }
    cr_solve(M, pa, pb, pc, pd);
    rod_forces<kRr>(pd, b.u, b.f, N);
    return;
  }

  // PH_KRYLOV: r = D f(z_j); w = J z_j becomes V[j+1]
  const double beta = beta_c;
  // small GMRES state to LDS, and the tridiagonal for the preconditioner
  if (tid < j) {
    cs_s[tid] = b.cs[tid];
    sn_s[tid] = b.sn[tid];
  }
  if (tid <= j) s_s[tid] = b.s[tid];
  double wv[kR];
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    const int k = tid + q * kCtlThreads;
    const int kc = (k < M) ? k : M - 1;  // valid index: loads issue together
    const double* qk = (kAdj ? b.u : b.Q) + 3 * kc;
    const double d0 = b.r[3 * (kc + 1)] - b.r[3 * kc];
    const double d1 = b.r[3 * (kc + 1) + 1] - b.r[3 * kc + 1];
    const double d2 = b.r[3 * (kc + 1) + 2] - b.r[3 * kc + 2];
    const double v = 2.0 * dt * (qk[0] * d0 + qk[1] * d1 + qk[2] * d2);
    const double lo = b.lo[kc], di = b.di[kc], up = b.up[kc];
    wv[q] = (k < M) ? v : 0.0;
    if (k < M) {
      pa[lp(k)] = lo;
      pb[lp(k)] = di;
      pc[lp(k)] = up;
    }
  }
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
      // two halves of four vectors: each half's loads issue together
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < kR; ++q) {
          const int k = tid + q * kCtlThreads;
          const int kc = (k < M) ? k : M - 1;  // wv is 0 past M
#pragma unroll
          for (int u = 4 * h; u < 4 * h + 4; ++u) {
            double v = 0.0;  // wave-uniform condition: the load issues without a wait
            if (i0 + u <= j) v = b.V[(i0 + u) * M + kc];
            pr[u] += wv[q] * v;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      block_sum8(pr, red8);
      if (tid < 8 && i0 + tid <= j) {
        hcur[i0 + tid] = pr[tid];
        hsum[i0 + tid] += pr[tid];
      }
      __syncthreads();
    }
    // w -= sum_i h_i v_i, vectors in batches of 8 so that their loads issue
    // together
    double acc[kR];
#pragma unroll
    for (int q = 0; q < kR; ++q) acc[q] = 0.0;
    for (int i0 = 0; i0 <= j; i0 += 8) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < kR; ++q) {
          const int k = tid + q * kCtlThreads;
          const int kc = (k < M) ? k : M - 1;
#pragma unroll
          for (int u = 4 * h; u < 4 * h + 4; ++u) {
            double v = 0.0, hv = 0.0;
            if (i0 + u <= j) {
              v = b.V[(i0 + u) * M + kc];
              hv = hcur[i0 + u];
            }
            acc[q] += hv * v;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int q = 0; q < kR; ++q)
      if (tid + q * kCtlThreads < M) wv[q] -= acc[q];  // w stays 0 past M
  }
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < kR; ++q) part += wv[q] * wv[q];
  const double hn = sqrt(block_sum(part, red));
  const double rhn = (hn > 0.0) ? 1.0 / hn : 0.0;
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    const int k = tid + q * kCtlThreads;
    if (hn > 0.0) wv[q] *= rhn;
    if (k < M) b.V[(j + 1) * M + k] = wv[q];
  }
  if (tid == 0) {
    // rotate the new Hessenberg column (hsum, hn) by the previous Givens
    // rotations and form the next one; column j of R goes to H
    double hcol_next = hn;
    for (int i = 0; i < j; ++i) {
      const double a0 = hsum[i], a1 = hsum[i + 1];
      hsum[i] = cs_s[i] * a0 + sn_s[i] * a1;
      hsum[i + 1] = -sn_s[i] * a0 + cs_s[i] * a1;
    }
    const double a0 = hsum[j], a1 = hcol_next;
    const double den = sqrt(a0 * a0 + a1 * a1);
    const double csj = (den > 0.0) ? a0 / den : 1.0;
    const double snj = (den > 0.0) ? a1 / den : 0.0;
    hsum[j] = den;
    cs_s[j] = csj;
    sn_s[j] = snj;
    s_s[j + 1] = -snj * s_s[j];
    s_s[j] = csj * s_s[j];
    b.cs[j] = csj;
    b.sn[j] = snj;
    b.s[j] = s_s[j];
    b.s[j + 1] = s_s[j + 1];
    for (int i = 0; i <= j; ++i) b.H[i * kKmax + j] = hsum[i];
    ctl->kry += 1;
    sh_flag = (fabs(s_s[j + 1]) <= eta * beta) || (hn == 0.0) || (j + 1 == kKmax);
  }
  __syncthreads();
  if (sh_flag) {
    // y = R^-1 s on the j+1 columns; R's earlier columns come from H
    const int kk = j + 1;
    double* Rs = pc;  // kk x kk upper triangle, row-major (pc is free here)
    for (int e0 = 0; e0 < kk * kk; e0 += kCtlThreads) {
      const int e = e0 + tid;
      const int ec = (e < kk * kk) ? e : 0;
      const int i = ec / kk, c = ec % kk;
      const double h = b.H[i * kKmax + c];  // any i, c < kKmax is a valid index
      if (e < kk * kk) Rs[e] = (c < j && i <= c) ? h : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i <= j; ++i) Rs[i * kk + j] = hsum[i];
      for (int i = kk - 1; i >= 0; --i) {
        double t = s_s[i];
        for (int c = i + 1; c < kk; ++c) t -= Rs[i * kk + c] * y_s[c];
        y_s[i] = t / Rs[i * kk + i];
      }
    }
    __syncthreads();
    // Newton correction: T += P^-1 (V y), with P the tridiagonal part of J
    double acc[kR];
#pragma unroll
    for (int q = 0; q < kR; ++q) acc[q] = 0.0;
    for (int i0 = 0; i0 < kk; i0 += 8) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < kR; ++q) {
          const int k = tid + q * kCtlThreads;
          const int kc = (k < M) ? k : M - 1;
#pragma unroll
          for (int u = 4 * h; u < 4 * h + 4; ++u) {
            double v = 0.0, yv = 0.0;
            if (i0 + u < kk) {
              v = b.V[(i0 + u) * M + kc];
              yv = y_s[i0 + u];
            }
            acc[q] += yv * v;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      const int kc = (k < M) ? k : M - 1;
      const double lo = b.lo[kc], di = b.di[kc], up = b.up[kc];
      if (k < M) {
        pa[lp(k)] = lo;
        pb[lp(k)] = di;
        pc[lp(k)] = up;
        pd[lp(k)] = acc[q];
      }
    }
    double told[kR];  // loaded before the solve so that its latency is hidden
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      told[q] = b.T[(k < M) ? k : M - 1];
    }
    cr_solve(M, pa, pb, pc, pd);
    if constexpr (kAdj) {
      // mu = P^-1 (V y) is in pd: z_i = xbar_i - 2 (Q_{i-1} mu_{i-1} - Q_i mu_i)
      for (int i = tid; i < N; i += kCtlThreads) {
        const double mm = (i > 0) ? pd[lp(i - 1)] : 0.0, mi = (i < M) ? pd[lp(i)] : 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al) {
          const double qm = (i > 0) ? b.Q[3 * (i - 1) + al] : 0.0;
          const double qi = (i < M) ? b.Q[3 * i + al] : 0.0;
          xs[3 * i + al] = xbar[3 * i + al] - 2.0 * (qm * mm - qi * mi);
        }
      }
      if (tid == 0) {
        const bool ok = fabs(s_s[j + 1]) <= eta * beta;
        if (st->status == BD_OK && !ok) st->status = BD_ERR_NO_CONVERGE;
        st->krylov_iters = ctl->kry;
        st->last_newton_res = fabs(s_s[j + 1]) / beta;
        st->done = 1;
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      if (k < M) {
        const double t = told[q] + pd[lp(k)];
        b.T[k] = t;
        pa[lp(k)] = t;
      }
    }
    __syncthreads();
    rod_forces<kRr>(pa, b.u, b.f, N);
    if (tid == 0) {
      ctl->newton_it = newton_it + 1;
      ctl->phase = PH_RESID;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int k = tid + q * kCtlThreads;
      if (k < M) pd[lp(k)] = wv[q];
    }
    cr_solve(M, pa, pb, pc, pd);
    rod_forces<kRr>(pd, kAdj ? b.Q : b.u, b.f, N);
    if (tid == 0) ctl->j = j + 1;
  }
}

template <int kRr>
__global__ __launch_bounds__(kCtlThreads) void newton_controller_kernel(
    Bufs b, double* __restrict__ xs, double* __restrict__ T_out, int N, double dt,
    double bl, double tol, int maxit, DevState* __restrict__ st) {
  __shared__ double arena[kCtlLds];
  newton_controller_body<false, kRr>(b, xs, T_out, N, dt, bl, tol, maxit, st, arena);
}

// ------------------------------------------------ one launch per solve
// The whole Newton-GMRES iteration in one launch of G <= (compute units)
// workgroups of kCtlThreads, one per compute unit, every one resident at
// once: each product with D is shared out by bead blocks (bx = g, g + G,
// ...), then workgroup 0 runs the controller pass, with a grid barrier after
// each phase.  The results are those of the alternating launches (the same
// bodies; the product with two phase sets per wave sums in the same order).
// Every barrier wait is bounded: a workgroup that waits longer than
// kSpinLimit polls (the GPU did not run every workgroup at once) raises the
// abort flag, every workgroup returns, and the solve reports
// BD_ERR_NO_CONVERGE (positions not committed).
constexpr int kPsLds = (kCtlLds > 6 * 2048 + kMvLds) ? kCtlLds : 6 * 2048 + kMvLds;
constexpr long kSpinLimit = 1L << 21;

__device__ bool grid_sync(GridBar* gb, uint32_t nwg, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's writes, before its arrival
    const uint32_t g = __hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    if (arrived == nwg - 1) {
      __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&gb->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&gb->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&gb->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if (++spins > kSpinLimit) {
          __hip_atomic_store(&gb->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();  // the other workgroups' writes, after the barrier
    *flag = ok;
  }
  __syncthreads();
  return *flag != 0;
}

// The two phases as separate functions, so that each gets its own register
// allocation (inlined together they spill).
__device__ __noinline__ void ps_matvec(int wg, int nwg, const double* __restrict__ x_old, Bufs b,
                                       int N, RpyConst kc, double* arena) {
  const int nblk = (N + kMvI - 1) / kMvI;
  for (int blk = wg; blk < nblk; blk += nwg)
    dmatvec_body<2048, kCtlThreads>(blk, x_old, b.f, b.r, N, kc, nullptr, arena,
                                    arena + 6 * 2048);
}

template <int kRr>
__device__ __noinline__ void ps_controller(Bufs b, double* __restrict__ xs,
                                           double* __restrict__ T_out, int N, double dt, double bl,
                                           double tol, int maxit, DevState* __restrict__ st,
                                           double* arena) {
  newton_controller_body<false, kRr>(b, xs, T_out, N, dt, bl, tol, maxit, st, arena);
}

template <int kRr>
__global__ __launch_bounds__(kCtlThreads) void constrain_persistent_kernel(
    const double* __restrict__ x_old, Bufs b, double* __restrict__ xs,
    double* __restrict__ T_out, int N, double dt, double bl, double tol, int maxit, RpyConst kc,
    DevState* __restrict__ st, int cap) {
  __shared__ __attribute__((aligned(16))) double arena[kPsLds];
  __shared__ int flag;
  const uint32_t nwg = gridDim.x;
  const int wg = blockIdx.x;
  bool ok = true;
  if (wg == 0) ps_controller<kRr>(b, xs, T_out, N, dt, bl, tol, maxit, st, arena);
  ok = grid_sync(b.gb, nwg, &flag);
  for (int it = 0; ok && it < cap; ++it) {
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    ps_matvec(wg, (int)nwg, x_old, b, N, kc, arena);
    if (!(ok = grid_sync(b.gb, nwg, &flag))) break;
    if (wg == 0) ps_controller<kRr>(b, xs, T_out, N, dt, bl, tol, maxit, st, arena);
    ok = grid_sync(b.gb, nwg, &flag);
  }
  if (wg == 0 && threadIdx.x == 0 && (!ok || !st->done)) {
    // a barrier was abandoned, or the launch cap ended the iteration first
    if (st->status == BD_OK) st->status = BD_ERR_NO_CONVERGE;
    st->done = 1;
  }
}

// Adjoint of the tension solve: rod directions u at x_old, the new rod
// vectors Q at x_new, the transposed band of the Jacobian at Q,
// (J^T)_{k,k-1} = J_{k-1,k} = -2 dt Q_{k-1} . G_{k-1,k} u_k,
// (J^T)_kk = -2 dt Q_k . G_kk u_k, (J^T)_{k,k+1} = -2 dt Q_{k+1} . G_{k+1,k} u_k,
// and f = xbar for the first product (r = D xbar).
__global__ __launch_bounds__(256) void constrain_adjoint_init_kernel(
    const double* __restrict__ x_old, const double* __restrict__ x_new,
    const double* __restrict__ xbar, Bufs b, int N, double hstar, double a, double dt,
    DevState* st) {
  const int M = N - 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < M) {
    const int k = t;
    double u[3], qk[3], o[3];
    unit_bond(x_old, k, u);
    for (int al = 0; al < 3; ++al) {
      qk[al] = x_new[3 * (k + 1) + al] - x_new[3 * k + al];
      b.u[3 * k + al] = u[al];
      b.Q[3 * k + al] = qk[al];
    }
    g_apply(x_old, k, k, hstar, a, u, o);
    b.di[k] = -2.0 * dt * (qk[0] * o[0] + qk[1] * o[1] + qk[2] * o[2]);
    double lo = 0.0, up = 0.0;
    if (k > 0) {
      double qm[3];
      for (int al = 0; al < 3; ++al) qm[al] = x_new[3 * k + al] - x_new[3 * (k - 1) + al];
      g_apply(x_old, k - 1, k, hstar, a, u, o);
      lo = -2.0 * dt * (qm[0] * o[0] + qm[1] * o[1] + qm[2] * o[2]);
    }
    if (k + 1 < M) {
      double qp[3];
      for (int al = 0; al < 3; ++al) qp[al] = x_new[3 * (k + 2) + al] - x_new[3 * (k + 1) + al];
      g_apply(x_old, k + 1, k, hstar, a, u, o);
      up = -2.0 * dt * (qp[0] * o[0] + qp[1] * o[1] + qp[2] * o[2]);
    }
    b.lo[k] = lo;
    b.up[k] = up;
  }
  for (int64_t e = t; e < 3 * (int64_t)N; e += (int64_t)gridDim.x * blockDim.x) b.f[e] = xbar[e];
  if (t == 0) {
    b.ctl->phase = PH_ADJ_RHS;
    b.ctl->j = 0;
    b.ctl->newton_it = 0;
    b.ctl->kry = 0;
    b.ctl->beta = 0.0;
    b.ctl->eta = 0.0;
    st->done = 0;
  }
}

template <int kRr>
__global__ __launch_bounds__(kCtlThreads) void adjoint_controller_kernel(
    Bufs b, const double* __restrict__ xbar, double* __restrict__ z, int N, double dt, double tol,
    DevState* __restrict__ st) {
  __shared__ double arena[kCtlLds];
  newton_controller_body<true, kRr>(b, z, nullptr, N, dt, 1.0, tol, 0, st, arena, xbar);
}

// Ensembles: chain blockIdx.z of the table, its workspace carved in place;
// grids cover the largest chain.
__global__ __launch_bounds__(256) void constrain_init_batched_kernel(
    const ChainDesc* __restrict__ cd) {
  const ChainDesc& c = cd[blockIdx.z];
  constrain_init_body(blockIdx.x, c.x, c.xs, carve(c.cons, c.N), c.N, c.hstar, c.a, c.st);
}

// One flattened grid over every chain's bead blocks (no idle workgroups).
__global__ __launch_bounds__(kMvThreads / 2) void dmatvec_batched_kernel(
    const ChainDesc* __restrict__ cd, const int32_t* __restrict__ prefix, int count) {
  const int t = blockIdx.x;
  const int ci = find_chain(prefix, count, t);
  const ChainDesc& c = cd[ci];
  const Bufs b = carve(c.cons, c.N);
  __shared__ __attribute__((aligned(16))) double sxf[6 * 1024];
  __shared__ double red[kMvLds];
  dmatvec_body<1024, kMvThreads / 2>(t - prefix[ci], c.x, b.f, b.r, c.N, rpy_const(c.hstar, c.a),
                                     c.st, sxf, red);
}

__global__ __launch_bounds__(kCtlThreads) void newton_controller_batched_kernel(
    const ChainDesc* __restrict__ cd) {
  const ChainDesc& c = cd[blockIdx.z];
  __shared__ double arena[kCtlLds];
  newton_controller_body<false>(carve(c.cons, c.N), c.xs, nullptr, c.N, c.dt, c.b, c.tol, c.maxit,
                                c.st, arena);
}

// States of `count` chains whose iteration the host stopped launching:
// those not finished report non-convergence (their positions are then not
// committed).
__global__ void constrain_unfinished_kernel(DevState* st, int count) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < count && !st[c].done) {
    if (st[c].status == BD_OK) st[c].status = BD_ERR_NO_CONVERGE;
    st[c].done = 1;
  }
}

}  // namespace

size_t constrain_workspace_bytes(int64_t n_beads) { return carve_bytes((int)n_beads); }

int constrain_max_beads() { return kMaxRodsBig + 1; }

int constrain_batched_max_beads() { return kMaxRods + 1; }

hipError_t launch_constrain(hipStream_t s, const bd_params_t& p, const double* x_old, double* xs,
                            double* T_out, void* ws, DevState* st, DevState* host_state,
                            int* pairs_hint, int n_cu) {
  const int N = p.n_beads;
  const int M = N - 1;
  Bufs b = carve(ws, N);
  const int ithreads = M > 0 ? M : 1;
  int iblk = (ithreads + 255) / 256;
  if (iblk < 16) iblk = 16;
  BD_LAUNCH("constrain_init", constrain_init_kernel, dim3(iblk), dim3(256), 0, s, x_old, xs, b, N,
            p.hstar, p.a, st);
  const bool big = M > kMaxRods;
  if (n_cu > 0) {
    // one launch: no host round trip, asynchronous on the stream
    const int nblk = (N + kMvI - 1) / kMvI;
    const int G = (nblk < n_cu) ? nblk : n_cu;
    const int cap = (p.newton_maxit + 1) * (kKmax + 2);
    auto* ps = big ? constrain_persistent_kernel<kRBig> : constrain_persistent_kernel<kR>;
    BD_LAUNCH("constrain_persistent", ps, dim3(G), dim3(kCtlThreads), 0, s, x_old, b, xs, T_out,
              N, p.dt, p.b, p.newton_tol, p.newton_maxit, rpy_const(p.hstar, p.a), st, cap);
    return hipGetLastError();
  }
  auto* ctl = big ? newton_controller_kernel<kRBig> : newton_controller_kernel<kR>;
  BD_LAUNCH("newton_controller", ctl, dim3(1), dim3(kCtlThreads), 0, s, b, xs, T_out, N, p.dt,
            p.b, p.newton_tol, p.newton_maxit, st);
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
      BD_LAUNCH("dmatvec", dmatvec_kernel, mvgrid, dim3(kMvThreads / 2), 0, s, x_old, b.f, b.r, N, kc,
                st);
      BD_LAUNCH("newton_controller", ctl, dim3(1), dim3(kCtlThreads), 0, s, b, xs, T_out, N,
                p.dt, p.b, p.newton_tol, p.newton_maxit, st);
    }
    launched += batch;
    hipError_t e = hipMemcpyAsync(host_state, st, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (host_state->done) break;
    batch = 4;
  }
  if (!host_state->done) {
    // the launch cap ended the iteration before the device did
    BD_LAUNCH("constrain_unfinished", constrain_unfinished_kernel, dim3(1), dim3(64), 0, s, st, 1);
  } else if (pairs_hint) {
    *pairs_hint = host_state->newton_iters + host_state->krylov_iters;
  }
  return hipGetLastError();
}

hipError_t launch_constrain_adjoint(hipStream_t s, const bd_params_t& p, const double* x_old,
                                    const double* x_new, const double* xbar, double* z, void* ws,
                                    DevState* st, DevState* host_state) {
  const int N = p.n_beads;
  const int M = N - 1;
  Bufs b = carve(ws, N);
  int iblk = (M + 255) / 256;
  if (iblk < 16) iblk = 16;
  BD_LAUNCH("constrain_adjoint_init", constrain_adjoint_init_kernel, dim3(iblk), dim3(256), 0, s,
            x_old, x_new, xbar, b, N, p.hstar, p.a, p.dt, st);
  const dim3 mvgrid((N + kMvI - 1) / kMvI);
  const RpyConst kc = rpy_const(p.hstar, p.a);
  auto* actl = (M > kMaxRods) ? adjoint_controller_kernel<kRBig> : adjoint_controller_kernel<kR>;
  // (matvec, controller) pairs: the first gives D xbar and the right side,
  // each further one a Krylov step; the host polls as for the forward solve
  const int cap = kKmax + 2;
  int batch = 16, launched = 0;
  while (launched < cap) {
    if (batch > cap - launched) batch = cap - launched;
    for (int c = 0; c < batch; ++c) {
      BD_LAUNCH("dmatvec", dmatvec_kernel, mvgrid, dim3(kMvThreads / 2), 0, s, x_old, b.f, b.r, N, kc,
                st);
      BD_LAUNCH("adjoint_controller", actl, dim3(1), dim3(kCtlThreads), 0, s, b, xbar, z, N, p.dt,
                p.newton_tol, st);
    }
    launched += batch;
    hipError_t e = hipMemcpyAsync(host_state, st, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (host_state->done) break;
    batch = 8;
  }
  if (!host_state->done)
    BD_LAUNCH("constrain_unfinished", constrain_unfinished_kernel, dim3(1), dim3(64), 0, s, st, 1);
  return hipGetLastError();
}

int constrain_mv_blocks(int n_beads) { return (n_beads + kMvI - 1) / kMvI; }

hipError_t launch_dmatvec(hipStream_t s, const bd_params_t& p, const double* x, const double* f,
                          double* r, const DevState* st) {
  const int N = p.n_beads;
  BD_LAUNCH("dmatvec", dmatvec_kernel, dim3((N + kMvI - 1) / kMvI), dim3(kMvThreads / 2), 0, s, x, f,
            r, N, rpy_const(p.hstar, p.a), st);
  return hipGetLastError();
}

hipError_t launch_constrain_batched(hipStream_t s, const ChainDesc* cd, int count, int max_beads,
                                    const int32_t* mv_prefix, int mv_blocks, int newton_maxit,
                                    DevState* st, DevState* host_states, int* pairs_hint,
                                    int budget) {
  const int M = max_beads - 1;
  int iblk = (M + 255) / 256;
  if (iblk < 16) iblk = 16;
  BD_LAUNCH("constrain_init_batched", constrain_init_batched_kernel, dim3(iblk, 1, count),
            dim3(256), 0, s, cd);
  BD_LAUNCH("newton_controller_batched", newton_controller_batched_kernel, dim3(1, 1, count),
            dim3(kCtlThreads), 0, s, cd);
  const dim3 mvgrid(mv_blocks);
  if (budget > 0) {
    // a fixed number of pairs, asynchronous (capturable); launches for a
    // finished chain return at once
    for (int q = 0; q < budget; ++q) {
      BD_LAUNCH("dmatvec_batched", dmatvec_batched_kernel, mvgrid, dim3(kMvThreads / 2), 0, s, cd,
                mv_prefix, count);
      BD_LAUNCH("newton_controller_batched", newton_controller_batched_kernel, dim3(1, 1, count),
                dim3(kCtlThreads), 0, s, cd);
    }
    BD_LAUNCH("constrain_unfinished", constrain_unfinished_kernel, dim3((count + 63) / 64),
              dim3(64), 0, s, st, count);
    return hipGetLastError();
  }
  // As for one chain: (matvec, controller) pairs in batches, the first sized
  // from the previous call, until every chain's iteration has finished;
  // launches for a finished chain return at once.
  const int cap = (newton_maxit + 1) * (kKmax + 2);
  int batch = (pairs_hint && *pairs_hint > 0) ? *pairs_hint + 1 : 8;
  int launched = 0;
  bool all_done = false;
  while (launched < cap) {
    if (batch > cap - launched) batch = cap - launched;
    for (int q = 0; q < batch; ++q) {
      BD_LAUNCH("dmatvec_batched", dmatvec_batched_kernel, mvgrid, dim3(kMvThreads / 2), 0, s, cd,
                mv_prefix, count);
      BD_LAUNCH("newton_controller_batched", newton_controller_batched_kernel, dim3(1, 1, count),
                dim3(kCtlThreads), 0, s, cd);
    }
    launched += batch;
    hipError_t e = hipMemcpyAsync(host_states, st, sizeof(DevState) * (size_t)count,
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    all_done = true;
    for (int c = 0; c < count && all_done; ++c) all_done = host_states[c].done != 0;
    if (all_done) break;
    batch = 4;
  }
  if (!all_done) {
    BD_LAUNCH("constrain_unfinished", constrain_unfinished_kernel, dim3((count + 63) / 64),
              dim3(64), 0, s, st, count);
  } else if (pairs_hint) {
    int most = 0;
    for (int c = 0; c < count; ++c) {
      const int p = host_states[c].newton_iters + host_states[c].krylov_iters;
      if (p > most) most = p;
    }
    *pairs_hint = most;
  }
  return hipGetLastError();
}

}  // namespace bd
