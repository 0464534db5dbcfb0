// Reverse-mode derivative of the Cholesky factorisation A = L L^T (Eq. 10),
// in the matrix form of Murray (2016): for a scalar phi with gradient Lbar
// in the lower triangle of L,
//   d phi = <P, dA>,   P = L^-T Phi(L^T Lbar) L^-1,
// Phi taking the lower triangle with the diagonal halved.  For symmetric dA
// the gradient is Abar = (P + P^T)/2 = W^T S W / 2 with W = L^-1 and
// S = Phi(X) + Phi(X)^T, X = L^T Lbar (S_ij = X_ij for i >= j, mirrored).
//
// Everything is FP64 matrix-core work (v_mfma_f64_16x16x4):
//   1. W: the 64 x 64 diagonal blocks of L inverted by substitution (one
//      wave per block), then joined pairwise, block size s = 64, 128, ...:
//      for a pair [[A, 0], [B, C]], W_BA = -W_C (B W_A), two products per
//      level for every pair at once;
//   2. X = L^T Lbar on the lower triangle only (operands masked to their
//      lower triangles, k-range cut to where both are nonzero);
//   3. S by mirroring X's strict lower triangle;
//   4. T = S W, then Abar = alpha W^T T / 2 + beta Abar.
// One general product kernel serves every step: a 64 x 64 tile of
// C = alpha op(A) op(B) + beta C per workgroup, operands staged in LDS
// k-chunks of 16, each wave a 32 x 32 quarter of the tile.  Operands can be
// transposed and masked to the lower triangle of the stored matrix; the
// product can be restricted to C's lower triangle; grid y repeats it along
// the diagonal (the pairs of one level), grid z over matrices of a batch.
#include "common.hpp"
#include "profile.hpp"

namespace bd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;        // C tile per workgroup
constexpr int kGK = 16;        // k per LDS chunk
constexpr int kGThreads = 256;

enum : int32_t { G_TA = 1, G_TB = 2, G_MA = 4, G_MB = 8, G_LOWC = 16 };

struct Kappa {
  double k[9];  // row-major: velocity v = kappa . r
};

// C = alpha op(A) op(B) + beta C on sub-blocks of column-major matrices of
// order nmat.  Origins (row, column) are in stored coordinates; for op(X) =
// X^T the stored block is k x m (A) or n x k (B).  Grid y = pair index: every
// origin moves by `step` along the diagonal and the sizes are clipped to the
// matrix.  A masked operand reads zero above the stored matrix's diagonal.
struct GemmOp {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int64_t sA, sB, sC;  // strides between the matrices of a batch (grid z)
  int32_t a_r, a_c, b_r, b_c, c_r, c_c;
  int32_t step;
  int32_t nmat;
  int32_t m, n, k;
  int32_t flags;
  double alpha, beta;
};

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kGThreads) void gemm_f64_kernel(GemmOp g) {
  __shared__ double sA[kGK][kGT], sB[kGK][kGT];
  const int sh = (int)blockIdx.y * g.step;
  const int ar = g.a_r + sh, ac = g.a_c + sh, br = g.b_r + sh, bc = g.b_c + sh;
  const int cr = g.c_r + sh, cc = g.c_c + sh;
  const bool ta = g.flags & G_TA, tb = g.flags & G_TB;
  const bool ma = g.flags & G_MA, mb = g.flags & G_MB, lowc = g.flags & G_LOWC;
  int m = g.m, n = g.n, K = g.k;
  if (m > g.nmat - cr) m = g.nmat - cr;
  if (n > g.nmat - cc) n = g.nmat - cc;
  const int ka0 = ta ? ar : ac, kb0 = tb ? bc : br;
  if (K > g.nmat - ka0) K = g.nmat - ka0;
  if (K > g.nmat - kb0) K = g.nmat - kb0;
  const int mt = (g.m + kGT - 1) / kGT;
  const int i0 = (int)(blockIdx.x % mt) * kGT, j0 = (int)(blockIdx.x / mt) * kGT;
  if (m <= 0 || n <= 0 || i0 >= m || j0 >= n) return;  // workgroup-uniform
  const int dA = ar - ac, dB = br - bc, dC = cr - cc;
  if (lowc && j0 > i0 + kGT - 1 + dC) return;  // tile above C's diagonal
  // k where both operands can be nonzero
  int kb = 0, ke = K;
  if (ma) {
    if (ta) kb = max(kb, i0 - dA);                       // A(k, i): i <= k + dA
    else ke = min(ke, i0 + kGT + dA);                    // A(i, k): k <= i + dA
  }
  if (mb) {
    if (tb) ke = min(ke, j0 + kGT + dB);                 // B(j, k): k <= j + dB
    else kb = max(kb, j0 - dB);                          // B(k, j): j <= k + dB
  }
  const double* A = g.A + (int64_t)blockIdx.z * g.sA;
  const double* B = g.B + (int64_t)blockIdx.z * g.sB;
  double* C = g.C + (int64_t)blockIdx.z * g.sC;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // op(A)(i, kk): contiguous along i (A) or kk (A^T)
      int i, kk;
      if (ta) { kk = tid & 15; i = (tid >> 4) + 16 * q; }
      else { i = tid & 63; kk = (tid >> 6) + 4 * q; }
      const int gi = i0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < ke) {
        const int sr = ta ? ar + gk : ar + gi, sc = ta ? ac + gi : ac + gk;
        if (!ma || sc <= sr) v = A[(int64_t)sr + (int64_t)sc * g.lda];
      }
      sA[kk][i] = v;
      // op(B)(kk, j): contiguous along kk (B) or j (B^T)
      int j, kj;
      if (tb) { j = tid & 63; kj = (tid >> 6) + 4 * q; }
      else { kj = tid & 15; j = (tid >> 4) + 16 * q; }
      const int gj = j0 + j, gkb = k0 + kj;
      double u = 0.0;
      if (gj < n && gkb < ke) {
        const int sr = tb ? br + gj : br + gkb, sc = tb ? bc + gkb : bc + gj;
        if (!mb || sc <= sr) u = B[(int64_t)sr + (int64_t)sc * g.ldb];
      }
      sB[kj][j] = u;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < kGK / 4; ++kq) {
      const int kr = 4 * kq + lk;
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[kr][wr + 16 * t + lr];
        b[t] = sB[kr][wc + 16 * t + lr];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma64(a[ti], b[tj], acc[ti][tj]);
    }
  }
  // register r of lane (lr, lk) holds row lk + 4 r, column lr of its 16 x 16 tile
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + 16 * ti + lk + 4 * r, j = j0 + wc + 16 * tj + lr;
        if (i < m && j < n && (!lowc || j <= i + dC)) {
          double* c = C + (int64_t)(cr + i) + (int64_t)(cc + j) * g.ldc;
          const double v = g.alpha * acc[ti][tj][r];
          *c = (g.beta != 0.0) ? v + g.beta * *c : v;
        }
      }
}

// W_JJ = (L_JJ)^-1 for the kGT x kGT diagonal block J (the last one ragged)
// of matrix blockIdx.z: lane c solves L_JJ y = e_c by forward substitution
// from LDS.  The block's strict upper triangle of W is set to zero.
__global__ __launch_bounds__(kGT) void trinv_diag_kernel(const double* __restrict__ L, int64_t ld,
                                                         int64_t sL, double* __restrict__ W,
                                                         int64_t ldw, int64_t sW, int n) {
  __shared__ double sLc[kGT][kGT + 1];  // sLc[c][r] = L(r0 + r, r0 + c)
  __shared__ double sY[kGT][kGT + 1];   // sY[c][r] = W(r0 + r, r0 + c)
  const int r0 = (int)blockIdx.x * kGT;
  const int nb = min(kGT, n - r0);
  const double* Lz = L + (int64_t)blockIdx.z * sL;
  double* Wz = W + (int64_t)blockIdx.z * sW;
  const int t = threadIdx.x;
  for (int c = 0; c < nb; ++c)
    sLc[c][t] = (t < nb && t >= c) ? Lz[(int64_t)(r0 + t) + (int64_t)(r0 + c) * ld] : 0.0;
  __syncthreads();
  if (t < nb) {
    const int c = t;
    for (int r = 0; r < c; ++r) sY[c][r] = 0.0;
    sY[c][c] = 1.0 / sLc[c][c];
    for (int r = c + 1; r < nb; ++r) {
      double s = 0.0;
      for (int k = c; k < r; ++k) s += sLc[k][r] * sY[c][k];
      sY[c][r] = -s / sLc[r][r];
    }
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c)
    if (t < nb) Wz[(int64_t)(r0 + t) + (int64_t)(r0 + c) * ldw] = sY[c][t];
}

// S = Phi(X) + Phi(X)^T from X's lower triangle, in place: the strict upper
// triangle receives the mirror of the strict lower one.
__global__ __launch_bounds__(256) void mirror_lower_kernel(double* __restrict__ X, int64_t ld,
                                                           int64_t sX, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);  // element (i, j), i contiguous
  if (i >= j) return;
  double* Xz = X + (int64_t)blockIdx.z * sX;
  Xz[(int64_t)i + (int64_t)j * ld] = Xz[(int64_t)j + (int64_t)i * ld];
}

hipError_t gemm(hipStream_t s, const GemmOp& g, int pairs, int batch) {
  const int mt = (g.m + kGT - 1) / kGT, nt = (g.n + kGT - 1) / kGT;
  if (mt <= 0 || nt <= 0 || pairs <= 0) return hipSuccess;
  BD_LAUNCH("gemm_f64", gemm_f64_kernel, dim3((unsigned)(mt * nt), (unsigned)pairs, (unsigned)batch),
            dim3(kGThreads), 0, s, g);
  return hipGetLastError();
}

GemmOp gemm_op(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
               int64_t ldc, int nmat, int m, int n, int k, int flags, double alpha,
               double beta) {
  GemmOp g;
  g.A = A; g.B = B; g.C = C;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.sA = g.sB = g.sC = 0;
  g.a_r = g.a_c = g.b_r = g.b_c = g.c_r = g.c_c = 0;
  g.step = 0;
  g.nmat = nmat;
  g.m = m; g.n = n; g.k = k;
  g.flags = flags;
  g.alpha = alpha; g.beta = beta;
  return g;
}

int64_t adj_ld(int64_t n) { return (n + 63) / 64 * 64; }

// ---- local parts of the step adjoint (one rigid-rod step, Eq. 6 with the
// constraint tensions): x^{t+dt} = x* + dt D(x) f, f_i = T_i u_i -
// T_{i-1} u_{i-1}, u_k = q_k/|q_k|, q_k = x_{k+1} - x_k, x* = x + dt kappa x
// + y.  z is the tension solve's adjoint (the gradient in x^{t+dt} at fixed
// T, equal to the gradient in x*).

__device__ __forceinline__ void rod_dir(const double* __restrict__ x, int k, double u[3],
                                        double& len) {
  const double q0 = x[3 * (k + 1)] - x[3 * k], q1 = x[3 * (k + 1) + 1] - x[3 * k + 1],
               q2 = x[3 * (k + 1) + 2] - x[3 * k + 2];
  len = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
  u[0] = q0 / len;
  u[1] = q1 / len;
  u[2] = q2 / len;
}

__global__ __launch_bounds__(256) void rod_forces_kernel(const double* __restrict__ x,
                                                         const double* __restrict__ T, int N,
                                                         double* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double ui[3] = {0.0, 0.0, 0.0}, um[3] = {0.0, 0.0, 0.0}, len;
  const double ti = (i < N - 1) ? T[i] : 0.0, tm = (i > 0) ? T[i - 1] : 0.0;
  if (i < N - 1) rod_dir(x, i, ui, len);
  if (i > 0) rod_dir(x, i - 1, um, len);
#pragma unroll
  for (int al = 0; al < 3; ++al) f[3 * i + al] = ti * ui[al] - tm * um[al];
}

// Dbar(a, b) = c z_a f_b, every element (column-major, a contiguous)
__global__ __launch_bounds__(256) void rank1_kernel(const double* __restrict__ z,
                                                    const double* __restrict__ f, double c,
                                                    int64_t n, double* __restrict__ Dbar,
                                                    int64_t ld) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (a >= n) return;
  Dbar[a + b * ld] = c * z[a] * f[b];
}

constexpr int kLocThreads = 256;

// xbar = (u part) + z + dt z kappa; kbar += dt sum_i z_i x_i^T.  Dz = D z
// (matrix-free product), so fbar = dt Dz and ubar_k = T_k (fbar_k -
// fbar_{k+1}); qbar_k = (I - u_k u_k^T) ubar_k / |q_k| moves bead k + 1 by
// +qbar_k and bead k by -qbar_k.  One workgroup; kappa's gradient by
// fixed-order block sums.
__global__ __launch_bounds__(kLocThreads) void step_adjoint_local_kernel(
    const double* __restrict__ x, const double* __restrict__ T, const double* __restrict__ z,
    const double* __restrict__ Dz, int N, double dt, Kappa kap, double* __restrict__ xbar,
    double* __restrict__ kbar) {
  __shared__ double red[kLocThreads / 64][9];
  const int tid = threadIdx.x;
  double kb[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) kb[e] = 0.0;
  for (int i = tid; i < N; i += kLocThreads) {
    double g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // z_i + dt (z_i kappa)_a = z_ia + dt sum_c z_ic kappa_ca
      g[a] = z[3 * i + a] + dt * (z[3 * i] * kap.k[a] + z[3 * i + 1] * kap.k[3 + a] +
                                  z[3 * i + 2] * kap.k[6 + a]);
#pragma unroll
      for (int b = 0; b < 3; ++b) kb[3 * a + b] += z[3 * i + a] * x[3 * i + b];
    }
    // rods i-1 (bead i is its second end) and i (its first end)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int k = (side == 0) ? i - 1 : i;
      if (k < 0 || k >= N - 1) continue;
      double u[3], len;
      rod_dir(x, k, u, len);
      double ub[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) ub[a] = T[k] * dt * (Dz[3 * k + a] - Dz[3 * (k + 1) + a]);
      const double uu = u[0] * ub[0] + u[1] * ub[1] + u[2] * ub[2];
      const double sgn = (side == 0) ? 1.0 : -1.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) g[a] += sgn * (ub[a] - u[a] * uu) / len;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) xbar[3 * i + a] = g[a];
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double v = kb[e];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6][e] = v;
  }
  __syncthreads();
  if (tid < 9) {
    double v = 0.0;
    for (int w = 0; w < kLocThreads / 64; ++w) v += red[w][tid];
    kbar[tid] += dt * v;
  }
}

__global__ __launch_bounds__(256) void step_adjoint_finish_kernel(int64_t n,
                                                                  const double* __restrict__ xbD,
                                                                  const double* __restrict__ hstep,
                                                                  double* __restrict__ xbar,
                                                                  double* __restrict__ hbar) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) xbar[e] += xbD[e];
  if (e == 0) *hbar += *hstep;
}

}  // namespace

hipError_t launch_rod_forces(hipStream_t s, const double* x, const double* T, int N, double* f) {
  BD_LAUNCH("rod_forces", rod_forces_kernel, dim3((N + 255) / 256), dim3(256), 0, s, x, T, N, f);
  return hipGetLastError();
}

hipError_t launch_rank1(hipStream_t s, const double* z, const double* f, double c, int64_t n,
                        double* Dbar, int64_t ld) {
  BD_LAUNCH("rank1", rank1_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0,
            s, z, f, c, n, Dbar, ld);
  return hipGetLastError();
}

hipError_t launch_step_adjoint_local(hipStream_t s, const bd_params_t& p, const double* x,
                                     const double* T, const double* z, const double* Dz,
                                     double* xbar, double* kbar) {
  Kappa kap;
  for (int e = 0; e < 9; ++e) kap.k[e] = p.kappa[e];
  BD_LAUNCH("step_adjoint_local", step_adjoint_local_kernel, dim3(1), dim3(kLocThreads), 0, s, x,
            T, z, Dz, p.n_beads, p.dt, kap, xbar, kbar);
  return hipGetLastError();
}

hipError_t launch_step_adjoint_finish(hipStream_t s, int64_t n, const double* xbD,
                                      const double* hstep, double* xbar, double* hbar) {
  BD_LAUNCH("step_adjoint_finish", step_adjoint_finish_kernel, dim3((unsigned)((n + 255) / 256)),
            dim3(256), 0, s, n, xbD, hstep, xbar, hbar);
  return hipGetLastError();
}

size_t cholesky_adjoint_workspace_bytes(int64_t n) {
  return 3 * align_up(sizeof(double) * (size_t)adj_ld(n) * (size_t)n, 256);
}

// Abar = alpha (P + P^T)/2 + beta Abar for `batch` matrices of order n with
// strides (elements) sL, sLb, sAb between them; ws holds W, X/S and T for
// each (cholesky_adjoint_workspace_bytes(n) per matrix, consecutive).
hipError_t launch_cholesky_adjoint(hipStream_t s, int64_t n64, const double* L, int64_t ld,
                                   int64_t sL, const double* Lbar, int64_t ldb, int64_t sLb,
                                   double* Abar, int64_t lda, int64_t sAb, double alpha,
                                   double beta, int batch, void* ws) {
  const int n = (int)n64;
  const int64_t lw = adj_ld(n64);
  const int64_t mat = (int64_t)(align_up(sizeof(double) * (size_t)lw * (size_t)n, 256) / 8);
  double* W = static_cast<double*>(ws);
  double* X = W + mat;
  double* T = X + mat;
  const int64_t sW = 3 * mat;  // per matrix of the batch
  // 1. W = L^-1: diagonal blocks, then pairs of blocks joined level by level
  const int nbk = (n + kGT - 1) / kGT;
  BD_LAUNCH("trinv_diag", trinv_diag_kernel, dim3((unsigned)nbk, 1, (unsigned)batch), dim3(kGT),
            0, s, L, ld, sL, W, lw, sW, n);
  hipError_t e = hipGetLastError();
  for (int sz = kGT; sz < n && e == hipSuccess; sz *= 2) {
    const int pairs = (n - sz + 2 * sz - 1) / (2 * sz);
    // T[C, A] = L[C, A] W[A, A]
    GemmOp g1 = gemm_op(L, ld, W, lw, T, lw, n, sz, sz, sz, G_MB, 1.0, 0.0);
    g1.sA = sL; g1.sB = sW; g1.sC = sW;
    g1.a_r = sz; g1.a_c = 0; g1.b_r = 0; g1.b_c = 0; g1.c_r = sz; g1.c_c = 0;
    g1.step = 2 * sz;
    e = gemm(s, g1, pairs, batch);
    if (e != hipSuccess) break;
    // W[C, A] = -W[C, C] T[C, A]
    GemmOp g2 = gemm_op(W, lw, T, lw, W, lw, n, sz, sz, sz, G_MA, -1.0, 0.0);
    g2.sA = sW; g2.sB = sW; g2.sC = sW;
    g2.a_r = sz; g2.a_c = sz; g2.b_r = sz; g2.b_c = 0; g2.c_r = sz; g2.c_c = 0;
    g2.step = 2 * sz;
    e = gemm(s, g2, pairs, batch);
  }
  if (e != hipSuccess) return e;
  // 2. X = L^T Lbar, lower triangle
  GemmOp gx = gemm_op(L, ld, Lbar, ldb, X, lw, n, n, n, n, G_TA | G_MA | G_MB | G_LOWC, 1.0, 0.0);
  gx.sA = sL; gx.sB = sLb; gx.sC = sW;
  if ((e = gemm(s, gx, 1, batch)) != hipSuccess) return e;
  // 3. S: mirror the strict lower triangle
  BD_LAUNCH("mirror_lower", mirror_lower_kernel,
            dim3((unsigned)(((int64_t)n * n + 255) / 256), 1, (unsigned)batch), dim3(256), 0, s,
            X, lw, sW, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 4. T = S W, Abar = alpha W^T T / 2 + beta Abar
  GemmOp gt = gemm_op(X, lw, W, lw, T, lw, n, n, n, n, G_MB, 1.0, 0.0);
  gt.sA = sW; gt.sB = sW; gt.sC = sW;
  if ((e = gemm(s, gt, 1, batch)) != hipSuccess) return e;
  GemmOp ga = gemm_op(W, lw, T, lw, Abar, lda, n, n, n, n, G_TA | G_MA, 0.5 * alpha, beta);
  ga.sA = sW; ga.sB = sW; ga.sC = sAb;
  return gemm(s, ga, 1, batch);
}

}  // namespace bd
