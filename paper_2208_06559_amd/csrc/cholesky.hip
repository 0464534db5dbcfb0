// Blocked right-looking Cholesky D = B B^T (Eq. 10), lower, in place,
// column-major with leading dimension ld.
//
// For each panel of width NB starting at column k:
//   1. potrf_diag   one workgroup factors the NB x NB diagonal block in LDS
//                   (FP64) and writes the inverses of its four 32 x 32
//                   diagonal sub-blocks;
//   2. panel_solve  L21 = A21 L11^-T by blocked forward substitution with
//                   MFMA over row blocks (FP64); in MIXED mode it also stores
//                   an FP32 copy of L21;
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
constexpr int kTS = kTile;    // trailing-update tile

__device__ __forceinline__ void tri_index(int t, int& r, int& c) {
  int rr = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((rr + 1) * (rr + 2) / 2 <= t) ++rr;
  while (rr * (rr + 1) / 2 > t) --rr;
  r = rr;
  c = t - rr * (rr + 1) / 2;
}

__host__ __device__ __forceinline__ int xcd_contiguous(int t, int nwg) {
  const int base = nwg / 8, rem = nwg % 8;
  const int x = t % 8, q = t / 8;
  return x * base + (x < rem ? x : rem) + q;
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
// the FP64 result layout above, as a compile-time fact for register-resident code
constexpr bool res_row_f64_is_lk_plus_4r = true;

// ------------------------------------------------------------------------
// 1. Diagonal block (NB x NB, FP64, one workgroup of 256 threads).
//    Right-looking unblocked factorisation with the matrix in registers:
//    thread (tr, tc) = (t % 16, t / 16) owns the interleaved 8 x 8 tile of
//    rows tr + 16a and columns tc + 16b, so the shrinking trailing triangle
//    stays spread over all threads.  Per column j the owners of column j
//    scale it by 1/sqrt(pivot) and publish it through a 1 KB LDS buffer;
//    every thread then applies the rank-1 update to its tile.  Afterwards
//    four waves invert the four 32 x 32 diagonal blocks of L11 in parallel
//    (forward substitution on the identity) for the panel solve.
//    Writes L11 over A11 and the inverses Winv_p (32 x 32, column-major) to
//    W.  Rows and columns beyond nb are padded with the identity.
// ------------------------------------------------------------------------
constexpr int SB = 32;          // diagonal sub-block of the panel solve
constexpr int NSB = NB / SB;    // sub-blocks per diagonal block
constexpr int SBB = SB * SB;    // doubles per 32 x 32 block
constexpr int TT = NB / 16;     // tile rows/columns per thread (8)

// 1/sqrt(d) to full FP64 accuracy: hardware estimate plus two Newton steps.
__device__ __forceinline__ double rsqrt_refined(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double h = 0.5 * d * y;
    y = fma(-h, y, 1.5) * y;
  }
  return y;
}

// Columns 16 JB .. 16 JB + 15 of the register-tiled factorisation (JB is a
// template parameter so that every register index is a compile-time
// constant).
template <int JB>
__device__ __forceinline__ void chol_block(double (&a)[TT][TT], double* __restrict__ col,
                                           double* __restrict__ piv, double* __restrict__ rdg,
                                           int tr, int tc, int tid, int64_t k,
                                           DevState* __restrict__ st) {
  for (int jr = 0; jr < 16; ++jr) {
    const int j = 16 * JB + jr;
    __syncthreads();  // pivot published; previous column no longer read
    if (tc == jr) {
      const double d = *piv;
      if (tid == jr * 16 + jr && !(d > 0.0) && st->potrf_info == 0) {
        st->potrf_info = k + j + 1;
        st->status = BD_ERR_NOT_SPD;
      }
      const double rs = rsqrt_refined(d);  // NaN for a non-positive pivot
#pragma unroll
      for (int ia = JB; ia < TT; ++ia) {
        const int i = tr + 16 * ia;
        if (i == j) {
          a[ia][JB] = d * rs;
          col[i] = a[ia][JB];
          rdg[j] = rs;  // 1 / L(j,j), used by the diagonal-block inversion
        } else if (i > j) {
          a[ia][JB] *= rs;
          col[i] = a[ia][JB];
        }
      }
    }
    __syncthreads();  // column j of L published
    // Only tiles ib >= JB, ia >= ib can hold live elements: for ia < ib every
    // row is above every column; for ia > ib every row is below; within
    // ia == ib only tr >= tc; and columns c > j need checking only at ib == JB.
    double ci[TT], cc[TT];
#pragma unroll
    for (int ia = JB; ia < TT; ++ia) ci[ia] = col[tr + 16 * ia];
#pragma unroll
    for (int ib = JB; ib < TT; ++ib) cc[ib] = col[tc + 16 * ib];
    const bool lower_diag = tr >= tc;
    const bool col_live = tc > jr;  // column tc + 16 JB is past j
#pragma unroll
    for (int ib = JB; ib < TT; ++ib)
#pragma unroll
      for (int ia = ib; ia < TT; ++ia) {
        bool live = true;
        if (ia == ib) live = lower_diag;
        if (ib == JB) live = live && col_live;
        const double upd = fma(-ci[ia], cc[ib], a[ia][ib]);
        a[ia][ib] = live ? upd : a[ia][ib];
      }
    // publish the next pivot (its owner has just updated it)
    const int jn = j + 1;
    if (tr == (jn & 15) && tc == (jn & 15)) {
      if (jr < 15) {
        *piv = a[JB][JB];
      } else if (JB + 1 < TT) {
        *piv = a[JB + 1 < TT ? JB + 1 : JB][JB + 1 < TT ? JB + 1 : JB];
      }
    }
  }
}

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int64_t ld,
                                                          int64_t k, int nb,
                                                          double* __restrict__ W,
                                                          DevState* __restrict__ st) {
  __shared__ double col[NB];          // the current column of L
  __shared__ double piv;              // the current pivot
  __shared__ double Ld[NSB][SBB];     // diagonal 32 x 32 blocks of L, column-major
  __shared__ double rowb[4][SB];      // per-wave row broadcast of the inversions
  __shared__ double rdg[NB];          // 1 / L(j,j)
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  double* Akk = A + k * ld + k;
  double a[TT][TT];
#pragma unroll
  for (int ia = 0; ia < TT; ++ia)
#pragma unroll
    for (int ib = 0; ib < TT; ++ib) {
      const int i = tr + 16 * ia, c = tc + 16 * ib;
      double v = 0.0;
      if (i < nb && c < nb) {
        if (i >= c) v = Akk[(int64_t)c * ld + i];
      } else if (i == c) {
        v = 1.0;
      }
      a[ia][ib] = v;
    }
  if (tid == 0) piv = a[0][0];
  static_assert(TT == 8, "diagonal block tiling");
  chol_block<0>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<1>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<2>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<3>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<4>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<5>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<6>(a, col, &piv, rdg, tr, tc, tid, k, st);
  chol_block<7>(a, col, &piv, rdg, tr, tc, tid, k, st);
  // L11 to global (lower part) and the diagonal blocks to LDS
#pragma unroll
  for (int ia = 0; ia < TT; ++ia)
#pragma unroll
    for (int ib = 0; ib < TT; ++ib) {
      const int i = tr + 16 * ia, c = tc + 16 * ib;
      if (i < nb && c < nb && i >= c) Akk[(int64_t)c * ld + i] = a[ia][ib];
      if ((i >> 5) == (c >> 5)) Ld[i >> 5][(c & 31) * SB + (i & 31)] = (i >= c) ? a[ia][ib] : 0.0;
    }
  __syncthreads();
  // wave p inverts diagonal block p: lane (r, h) keeps W[r][16h .. 16h+15]
  {
    const int p = tid >> 6, lane = tid & 63, r = lane & 31, h = lane >> 5;
    const double* L = Ld[p];
    double w[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) w[c] = (r == 16 * h + c) ? 1.0 : 0.0;
    for (int q = 0; q < SB; ++q) {
      const double rq = rdg[SB * p + q];
      if (r == q) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          w[c] = w[c] * rq;
          rowb[p][16 * h + c] = w[c];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (r > q) {
        const double lrq = L[q * SB + r];
#pragma unroll
        for (int c = 0; c < 16; ++c) w[c] = fma(-lrq, rowb[p][16 * h + c], w[c]);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    double* Wp = W + p * SBB;
#pragma unroll
    for (int c = 0; c < 16; ++c) Wp[(16 * h + c) * SB + r] = w[c];
  }
}

// ------------------------------------------------------------------------
// 2. Panel solve X L11^T = A21 for a block of 32 rows, by blocked forward
//    substitution over the four 32-column sub-panels:
//      X(:,p) = (A(:,p) - sum_{q<p} X(:,q) L11(p,q)^T) Winv_p^T.
//    Two waves, 16 rows each, and no LDS: with the rows of X as the MFMA
//    B operand, lane (lr, lk) needs exactly the columns c = lk (mod 4) of
//    row lr, which are also the columns the MFMA result leaves in that lane,
//    so the row block stays in registers (x[t] = column 4t + lk).  The L11
//    and Winv operands come straight from global memory (L2-resident).
//    In MIXED mode an FP32 copy of X is stored as well.
// ------------------------------------------------------------------------
constexpr int kRB = 32;          // rows per panel-solve workgroup
constexpr int kPsThreads = 128;  // two waves

template <int P>
__device__ __forceinline__ void solve_subpanel(double (&x)[NB / 4], const double* __restrict__ L11,
                                               int64_t ld, const double* __restrict__ Wp, int lr,
                                               int lk) {
  constexpr int c0 = SB * P;
  // operands first (one round trip), then the MFMA chains
  double la[2][c0 / 4 + 1], wa[2][SB / 4];
#pragma unroll
  for (int jt = 0; jt < 2; ++jt) {
#pragma unroll
    for (int s = 0; s < c0 / 4; ++s) la[jt][s] = L11[(int64_t)(4 * s + lk) * ld + c0 + 16 * jt + lr];
#pragma unroll
    for (int s = 0; s < SB / 4; ++s) wa[jt][s] = Wp[(4 * s + lk) * SB + 16 * jt + lr];
  }
  if (c0 > 0) {
    d4 acc[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
#pragma unroll
    for (int s = 0; s < c0 / 4; ++s)
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) acc[jt] = mfma(la[jt][s], x[s], acc[jt]);
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int q = 0; q < 4; ++q) x[c0 / 4 + 4 * jt + q] -= acc[jt][q];
  }
  d4 y[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
#pragma unroll
  for (int s = 0; s < SB / 4; ++s)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) y[jt] = mfma(wa[jt][s], x[c0 / 4 + s], y[jt]);
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int q = 0; q < 4; ++q) x[c0 / 4 + 4 * jt + q] = y[jt][q];
}

__global__ __launch_bounds__(kPsThreads) void panel_solve_kernel(
    double* __restrict__ A, int64_t ld, int64_t k, int nb, int64_t m, const double* __restrict__ W,
    float* __restrict__ P32, int64_t ldp) {
  static_assert(NSB == 4 && res_row_f64_is_lk_plus_4r, "register layout of the panel solve");
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int64_t row = (int64_t)blockIdx.x * kRB + 16 * w + lr;
  const bool live = row < m;
  double* A21 = A + k * ld + k + nb;
  const double* L11 = A + k * ld + k;
  double x[NB / 4];
#pragma unroll
  for (int t = 0; t < NB / 4; ++t) {
    const int c = 4 * t + lk;
    x[t] = (live && c < nb) ? A21[(int64_t)c * ld + row] : 0.0;
  }
  solve_subpanel<0>(x, L11, ld, W, lr, lk);
  solve_subpanel<1>(x, L11, ld, W + SBB, lr, lk);
  solve_subpanel<2>(x, L11, ld, W + 2 * SBB, lr, lk);
  solve_subpanel<3>(x, L11, ld, W + 3 * SBB, lr, lk);
  if (!live) return;
#pragma unroll
  for (int t = 0; t < NB / 4; ++t) {
    const int c = 4 * t + lk;
    if (c < nb) {
      A21[(int64_t)c * ld + row] = x[t];
      if (P32) P32[(int64_t)c * ldp + row] = (float)x[t];
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

// Pipeline: the C tile is loaded into registers before the K loop (its
// latency hides behind the MFMA work), operand chunks of KC columns go
// global -> registers two chunks ahead and registers -> LDS one chunk
// ahead (LDS double buffer).
template <typename T>
__global__ __launch_bounds__(256) void syrk_update_kernel(double* __restrict__ C, int64_t ld,
                                                           const T* __restrict__ L, int64_t ldl,
                                                           int64_t m, int tiles) {
  constexpr int KC = SyrkCfg<T>::KC;
  typedef typename SyrkCfg<T>::acc_t acc_t;
  constexpr int NLD = KC * kTS / 256;  // elements per thread per operand per chunk
  __shared__ T As[2][KC][kTS + kPad];  // row side
  __shared__ T Bs[2][KC][kTS + kPad];  // column side

  // XCD x receives workgroups x, x+8, ...: cnt(x) = base + (x < rem) of them;
  // the q-th of them takes tile x*base + min(x, rem) + q (a bijection).
  const int t = xcd_contiguous(blockIdx.x, gridDim.x);
  int ti, tj;
  if (tiles == kTilesNext) {
    ti = t;
    tj = 0;
  } else {
    tri_index(t, ti, tj);
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

  acc_t acc[4][4];
  // C tile prefetch (rows i, columns j of this lane's result registers)
  double cv[4][4][4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[bj][bi][r] = 0;
        const int64_t i = row0 + 64 * wr + 16 * bi + lr;
        const int64_t j = col0 + 64 * wc + 16 * bj + res_row(acc[bj][bi], lk, r);
        cv[bj][bi][r] = (active && i < m && j < m && i >= j) ? C[j * ld + i] : 0.0;
      }

  T ra[NLD], rb[NLD];
  auto gload = [&](int kk) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int e = tid + 256 * q;
      const int kc = e / kTS, r = e % kTS;
      // rows past m are clamped (their products only reach masked outputs)
      const int64_t ia = (row0 + r < m) ? row0 + r : m - 1;
      const int64_t ib = (col0 + r < m) ? col0 + r : m - 1;
      ra[q] = L[(int64_t)(kk + kc) * ldl + ia];
      rb[q] = L[(int64_t)(kk + kc) * ldl + ib];
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

  constexpr int nch = NB / KC;
  gload(0);
  sstore(0);
  if (nch > 1) gload(KC);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
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
    if (ch + 1 < nch) {
      sstore(buf ^ 1);                       // chunk ch+1, loaded one iteration ago
      if (ch + 2 < nch) gload((ch + 2) * KC);  // two chunks ahead
    }
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
        if (i < m && j < m && i >= j) C[j * ld + i] = cv[bj][bi][r] - (double)acc[bj][bi][r];
      }
}

}  // namespace

size_t cholesky_workspace_bytes(int64_t n, bd_precision_t prec) {
  size_t b = align_up(sizeof(double) * NB * NB, 256);  // four 32 x 32 inverses (NB*NB/4 used)
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
  if (m > 0) {  // then nb == NB: only the last panel can be narrower
    float* P = c.P32[(k / NB) & 1];
    BD_LAUNCH("panel_solve", panel_solve_kernel, dim3((unsigned)((m + kRB - 1) / kRB)), dim3(kPsThreads),
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
