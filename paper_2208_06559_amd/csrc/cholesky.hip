// Blocked right-looking Cholesky D = B B^T (Eq. 10), lower, in place,
// column-major with leading dimension ld.
//
// For each panel of width NB starting at column k:
//   1. potrf_diag   one workgroup factors the NB x NB diagonal block in LDS
//                   (FP64) and writes its triangular inverse W = L11^-1;
//   2. panel_solve  L21 = A21 L11^-T = A21 W^T, an MFMA GEMM over row blocks
//                   (FP64); in MIXED mode it also stores an FP32 copy of L21;
//   3. syrk_update  A22 -= L21 L21^T on the lower tiles of the trailing
//                   matrix with MFMA: FP64 operands/accumulators, or (MIXED)
//                   FP32 operands with FP32 accumulation, subtracted into the
//                   FP64 storage.
// The diagonal blocks and panel solves stay FP64 in both modes.
//
// MFMA operand convention (v_mfma_*_16x16x4): operand A holds A[i][k] in
// lane i + 16k, operand B holds B[k][j] in lane j + 16k.  Result register r
// of lane l holds D[i][l%16] with i = 4*(l/16) + r for the FP32 instruction
// and i = l/16 + 4*r for the FP64 one (measured on gfx950).  The "column
// side" rows are fed as operand A and the "row side" rows as operand B, so
// each result register of a wavefront covers 16 consecutive rows of 4
// columns: 128-byte runs in column-major memory.
#include "common.hpp"
#include "profile.hpp"

namespace bd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NB = kNB;       // panel width
constexpr int LDP = NB + 1;   // LDS leading dimension of the diagonal block
constexpr int kTS = kTile;    // trailing-update tile

__device__ __forceinline__ void tri_index(int t, int& r, int& c) {
  int rr = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((rr + 1) * (rr + 2) / 2 <= t) ++rr;
  while (rr * (rr + 1) / 2 > t) --rr;
  r = rr;
  c = t - rr * (rr + 1) / 2;
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of the 16 x 16 result held by register r of a lane with lane/16 = lk.
__device__ __forceinline__ int res_row(d4, int lk, int r) { return lk + 4 * r; }
__device__ __forceinline__ int res_row(f4, int lk, int r) { return 4 * lk + r; }

// ------------------------------------------------------------------------
// 1. Diagonal block: unblocked right-looking Cholesky in LDS, then the
//    in-place inverse of the lower triangle (column j from the last to the
//    first: W_jj = 1/L_jj, W_ij = -W_jj * sum_{j<k<=i} W_ik L_kj).
//    Rows and columns beyond nb are padded with the identity.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int64_t ld,
                                                          int64_t k, int nb,
                                                          double* __restrict__ W,
                                                          DevState* __restrict__ st) {
  __shared__ double S[NB * LDP];
  const int tid = threadIdx.x;
  double* Akk = A + k * ld + k;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int c = idx / NB, r = idx % NB;
    double v = 0.0;
    if (c < nb && r < nb) {
      if (r >= c) v = Akk[(int64_t)c * ld + r];
    } else if (r == c) {
      v = 1.0;
    }
    S[c * LDP + r] = v;
  }
  __syncthreads();

  for (int j = 0; j < nb; ++j) {
    const double d = S[j * LDP + j];
    const double dj = sqrt(d);  // NaN for a non-positive pivot
    if (tid == 0 && !(d > 0.0) && st->potrf_info == 0) {
      st->potrf_info = k + j + 1;
      st->status = BD_ERR_NOT_SPD;
    }
    for (int i = j + 1 + tid; i < nb; i += 256) S[j * LDP + i] = S[j * LDP + i] / dj;
    __syncthreads();
    if (tid == 0) S[j * LDP + j] = dj;
    const int g = tid >> 6, l = tid & 63;
    for (int c = j + 1 + g; c < nb; c += 4) {
      const double ljc = S[j * LDP + c];
      for (int i = c + l; i < nb; i += 64) S[c * LDP + i] -= S[j * LDP + i] * ljc;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int c = idx / nb, r = idx % nb;
    if (r >= c) Akk[(int64_t)c * ld + r] = S[c * LDP + r];
  }
  __syncthreads();

  // in-place inverse of the lower triangle
  for (int j = nb - 1; j >= 0; --j) {
    const double wjj = 1.0 / S[j * LDP + j];
    double x = 0.0;
    const int i = j + 1 + tid;
    if (tid < 128 && i < nb) {
      for (int kk = j + 1; kk <= i; ++kk) x += S[kk * LDP + i] * S[j * LDP + kk];
    }
    __syncthreads();
    if (tid < 128 && i < nb) S[j * LDP + i] = -wjj * x;
    if (tid == 0) S[j * LDP + j] = wjj;
    __syncthreads();
  }
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int c = idx / NB, r = idx % NB;
    W[idx] = (r >= c) ? S[c * LDP + r] : 0.0;
  }
}

// ------------------------------------------------------------------------
// 2. Panel solve X = A21 W^T for a block of 64 rows (all NB columns).
//    The 64 x NB row block is staged in LDS, so the result can overwrite
//    A21 in place.  Wave w computes output columns [32w, 32w+32); W is
//    lower-triangular, so its K loop stops at column 32w+31.
// ------------------------------------------------------------------------
constexpr int kRB = 64;  // rows per panel-solve workgroup

__global__ __launch_bounds__(256) void panel_solve_kernel(double* __restrict__ A, int64_t ld,
                                                           int64_t k, int nb, int64_t m,
                                                           const double* __restrict__ W,
                                                           float* __restrict__ P32,
                                                           int64_t ldp) {
  __shared__ double As[NB][kRB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kRB;
  double* A21 = A + k * ld + k + nb;
  for (int idx = tid; idx < NB * kRB; idx += 256) {
    const int kk = idx / kRB, r = idx % kRB;
    const int64_t row = r0 + r;
    As[kk][r] = (kk < nb && row < m) ? A21[(int64_t)kk * ld + row] : 0.0;
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  d4 acc[2][4];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) acc[bj][bi] = d4{0.0, 0.0, 0.0, 0.0};
  const int kend = 32 * w + 32;
  for (int k0 = 0; k0 < kend; k0 += 4) {
    double af[2], bf[4];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) af[bj] = W[(k0 + lk) * NB + 32 * w + 16 * bj + lr];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) bf[bi] = As[k0 + lk][16 * bi + lr];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) acc[bj][bi] = mfma(af[bj], bf[bi], acc[bj][bi]);
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 16 * bi + lr;
        const int col = 32 * w + 16 * bj + res_row(acc[bj][bi], lk, r);
        if (row < m && col < nb) {
          const double v = acc[bj][bi][r];
          A21[(int64_t)col * ld + row] = v;
          if (P32) P32[(int64_t)col * ldp + row] = (float)v;
        }
      }
}

// ------------------------------------------------------------------------
// 3. Trailing update C -= L L^T on the lower 128 x 128 tiles of the m x m
//    trailing matrix; L is m x NB (column-major, ldl) in FP64 or FP32.
//    Four waves, each a 64 x 64 quadrant (the strictly upper quadrant of a
//    diagonal tile is skipped).  Operands are staged through double-buffered
//    LDS in K-chunks of KC.
// ------------------------------------------------------------------------
template <typename T>
struct SyrkCfg;
template <>
struct SyrkCfg<double> {
  static constexpr int KC = 16;
  typedef d4 acc_t;
};
template <>
struct SyrkCfg<float> {
  static constexpr int KC = 32;
  typedef f4 acc_t;
};

constexpr int kPad = 4;

// Tile sets of one trailing update: every lower tile, only the first tile
// column (the next panel, updated ahead), or every lower tile but the first
// column.
enum { kTilesAll = 0, kTilesNext = 1, kTilesRest = 2 };

template <typename T>
__global__ __launch_bounds__(256) void syrk_update_kernel(double* __restrict__ C, int64_t ld,
                                                           const T* __restrict__ L, int64_t ldl,
                                                           int64_t m, int tiles) {
  constexpr int KC = SyrkCfg<T>::KC;
  typedef typename SyrkCfg<T>::acc_t acc_t;
  constexpr int NLD = KC * kTS / 256;  // elements per thread per operand per chunk
  __shared__ T As[2][KC][kTS + kPad];  // row side
  __shared__ T Bs[2][KC][kTS + kPad];  // column side

  int ti, tj;
  if (tiles == kTilesNext) {
    ti = blockIdx.x;
    tj = 0;
  } else {
    tri_index(blockIdx.x, ti, tj);
    if (tiles == kTilesRest) {
      ++ti;
      ++tj;
    }
  }
  const int64_t row0 = (int64_t)ti * kTS, col0 = (int64_t)tj * kTS;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int wr = w >> 1, wc = w & 1;
  const bool active = !(ti == tj && wr < wc);

  T ra[NLD], rb[NLD];
  auto gload = [&](int kk) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int e = tid + 256 * q;
      const int kc = e / kTS, r = e % kTS;
      const int64_t ia = row0 + r, ib = col0 + r;
      ra[q] = (ia < m) ? L[(int64_t)(kk + kc) * ldl + ia] : T(0);
      rb[q] = (ib < m) ? L[(int64_t)(kk + kc) * ldl + ib] : T(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int e = tid + 256 * q;
      const int kc = e / kTS, r = e % kTS;
      As[buf][kc][r] = ra[q];
      Bs[buf][kc][r] = rb[q];
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bj][bi][r] = 0;

  const int nch = NB / KC;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) gload((ch + 1) * KC);
    if (active) {
#pragma unroll
      for (int kq = 0; kq < KC / 4; ++kq) {
        T af[4], bf[4];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) af[bj] = Bs[buf][4 * kq + lk][64 * wc + 16 * bj + lr];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) bf[bi] = As[buf][4 * kq + lk][64 * wr + 16 * bi + lr];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
          for (int bi = 0; bi < 4; ++bi) acc[bj][bi] = mfma(af[bj], bf[bi], acc[bj][bi]);
      }
    }
    if (ch + 1 < nch) sstore(buf ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = row0 + 64 * wr + 16 * bi + lr;
        const int64_t j = col0 + 64 * wc + 16 * bj + res_row(acc[bj][bi], lk, r);
        if (i < m && j < m && i >= j) C[j * ld + i] -= (double)acc[bj][bi][r];
      }
}

}  // namespace

size_t cholesky_workspace_bytes(int64_t n, bd_precision_t prec) {
  size_t b = align_up(sizeof(double) * NB * NB, 256);
  if (prec == BD_PREC_MIXED) b += 2 * align_up(sizeof(float) * (size_t)n * NB, 256);
  return b;
}

namespace {

struct CholCtx {
  int64_t n, ld;
  double* A;
  double* W;
  float* P32[2];  // FP32 copies of consecutive panels (MIXED), else null
  DevState* st;
};

hipError_t factor_panel(const CholCtx& c, hipStream_t s, int64_t k) {
  const int nb = (int)((c.n - k < NB) ? (c.n - k) : NB);
  BD_LAUNCH("potrf_diag", potrf_diag_kernel, dim3(1), dim3(256), 0, s, c.A, c.ld, k, nb, c.W,
            c.st);
  const int64_t m = c.n - k - nb;
  if (m > 0) {
    float* P = c.P32[(k / NB) & 1];
    BD_LAUNCH("panel_solve", panel_solve_kernel, dim3((unsigned)((m + kRB - 1) / kRB)), dim3(256),
              0, s, c.A, c.ld, k, nb, m, c.W, P, c.n);
  }
  return hipGetLastError();
}

hipError_t trailing(const CholCtx& c, hipStream_t s, int64_t k, int tiles) {
  const int64_t m = c.n - k - NB;
  const int64_t mt = (m + kTS - 1) / kTS;
  unsigned nt = 0;
  if (tiles == kTilesAll) nt = (unsigned)(mt * (mt + 1) / 2);
  if (tiles == kTilesNext) nt = (unsigned)mt;
  if (tiles == kTilesRest) nt = (unsigned)((mt - 1) * mt / 2);
  if (nt == 0) return hipSuccess;
  double* C = c.A + (k + NB) * c.ld + (k + NB);
  const float* P = c.P32[(k / NB) & 1];
  if (P) {
    BD_LAUNCH("syrk_update_f32", syrk_update_kernel<float>, dim3(nt), dim3(256), 0, s, C, c.ld, P,
              c.n, m, tiles);
  } else {
    BD_LAUNCH("syrk_update_f64", syrk_update_kernel<double>, dim3(nt), dim3(256), 0, s, C, c.ld,
              (const double*)(c.A + k * c.ld + k + NB), c.ld, m, tiles);
  }
  return hipGetLastError();
}

}  // namespace

// Right-looking blocked factorisation with depth-1 lookahead: while the
// main stream applies panel k to the trailing matrix (all but the next tile
// column), the auxiliary stream updates the next tile column first, then
// factors the next diagonal block and solves the next panel.  Events order
// the two streams; with aux == nullptr everything runs on `s` in order.
hipError_t launch_cholesky(hipStream_t s, hipStream_t aux, hipEvent_t ev[3], int64_t n, double* A,
                           int64_t ld, bd_precision_t prec, void* ws, DevState* st) {
  CholCtx c;
  c.n = n;
  c.ld = ld;
  c.A = A;
  c.st = st;
  c.W = static_cast<double*>(ws);
  c.P32[0] = c.P32[1] = nullptr;
  if (prec == BD_PREC_MIXED) {
    char* p = static_cast<char*>(ws) + align_up(sizeof(double) * NB * NB, 256);
    c.P32[0] = reinterpret_cast<float*>(p);
    c.P32[1] = reinterpret_cast<float*>(p + align_up(sizeof(float) * (size_t)n * NB, 256));
  }
  hipError_t e;
  if (!aux) {
    for (int64_t k = 0; k < n; k += NB) {
      if ((e = factor_panel(c, s, k)) != hipSuccess) return e;
      if (k + NB < n && (e = trailing(c, s, k, kTilesAll)) != hipSuccess) return e;
    }
    return hipGetLastError();
  }
  hipEvent_t ev_fork = ev[0], ev_panel = ev[1], ev_rest = ev[2];
  if ((e = hipEventRecord(ev_fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(aux, ev_fork, 0)) != hipSuccess) return e;
  if ((e = factor_panel(c, aux, 0)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev_panel, aux)) != hipSuccess) return e;
  for (int64_t k = 0; k + NB < n; k += NB) {
    // main: panel k must be solved before it is applied
    if ((e = hipStreamWaitEvent(s, ev_panel, 0)) != hipSuccess) return e;
    // aux: the next tile column must have every earlier update
    if (k > 0 && (e = hipStreamWaitEvent(aux, ev_rest, 0)) != hipSuccess) return e;
    if ((e = trailing(c, aux, k, kTilesNext)) != hipSuccess) return e;
    if ((e = factor_panel(c, aux, k + NB)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev_panel, aux)) != hipSuccess) return e;
    if ((e = trailing(c, s, k, kTilesRest)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev_rest, s)) != hipSuccess) return e;
  }
  if ((e = hipStreamWaitEvent(s, ev_panel, 0)) != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace bd
