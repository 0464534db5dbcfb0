// Blocked right-looking Cholesky D = B B^T (Eq. 10), lower, in place,
// column-major with leading dimension ld.
//
// For each panel of width NB starting at column k:
//   1. potrf_tile   one workgroup factors the NB x NB diagonal block (FP64,
//                   16 x 16 tiles in registers, rank-16 updates on matrix
//                   cores; potrf_diag, the register-tiled variant, on
//                   request) and writes the inverses of its four 32 x 32
//                   diagonal sub-blocks;
//   2. panel_solve  L21 = A21 L11^-T by blocked forward substitution with
//                   MFMA over row blocks (FP64); in MIXED mode it also stores
//                   an FP32 copy of L21;
//   3. syrk_update  A22 -= L21 L21^T on the lower tiles of the trailing
//                   matrix with MFMA: FP64 operands/accumulators, or (MIXED)
//                   FP32 operands with FP32 accumulation, subtracted into the
//                   FP64 storage.
// The diagonal blocks and panel solves stay FP64 in both modes.  Panels
// are applied in steps of up to four, with depth-1 lookahead on a second
// stream (launch_cholesky).  Given the noise xi, the call also forms the
// noise product y = c_B L xi: each panel's share of every row below it
// (noise_part_kernel, launched beside the factorisation; for ensembles
// inside the panel solve), then the shares' ordered sums with the
// diagonal blocks' (noise_sum_kernel).
//
// MFMA operand convention (v_mfma_*_16x16x4): operand A holds A[i][k] in
// lane i + 16k, operand B holds B[k][j] in lane j + 16k.  Result register r
// of lane l holds D[i][l%16] with i = 4*(l/16) + r for the FP32 instruction
// and i = l/16 + 4*r for the FP64 one (measured on gfx950).  The "column
// side" rows are fed as operand A and the "row side" rows as operand B, so
// each result register of a wavefront covers 16 consecutive rows of 4
// columns: 128-byte runs in column-major memory.
#include <utility>

#include "common.hpp"
#include "profile.hpp"

namespace bd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NB = kNB;       // panel width
constexpr int kTS = kTile;    // trailing-update tile

// Lower tile (ti, tj) number t of an mt x mt tile triangle in banded order:
// bands of kBand tile rows; within a band, column by column, first the
// band's rows left of its diagonal block, then that block's lower triangle.
// An XCD's run of consecutive tiles then touches kBand row panels and a
// window of column panels, which its L2 can hold, where the row-major
// order touches every column panel up to the current row.
constexpr int kBand = 8;
__host__ __device__ __forceinline__ int64_t band_start(int I) {  // tiles before band I (full bands)
  return (int64_t)kBand * kBand * I * (I - 1) / 2 + (int64_t)I * kBand * (kBand + 1) / 2;
}
__host__ __device__ __forceinline__ void band_index(int t, int mt, int& ti, int& tj) {
  const double a = kBand * kBand * 0.5, b = kBand * (kBand + 1) * 0.5 - a;  // start = a I^2 + b I
  int I = (int)((-b + sqrt(b * b + 4.0 * a * (double)t)) / (2.0 * a));
  const int last = (mt - 1) / kBand;
  if (I > last) I = last;
  while (I > 0 && band_start(I) > t) --I;
  while (I < last && band_start(I + 1) <= t) ++I;
  int o = (int)(t - band_start(I));
  const int rows = (mt - kBand * I < kBand) ? mt - kBand * I : kBand;
  const int rect = kBand * I * rows;
  if (o < rect) {
    tj = o / rows;
    ti = kBand * I + o % rows;
  } else {
    o -= rect;
    int c = 0;
    while (o >= rows - c) {
      o -= rows - c;
      ++c;
    }
    tj = kBand * I + c;
    ti = tj + o;
  }
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

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double shfl_f64(double v, int src_lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Columns j0 .. j0 + 3 (j0 = 16 IB + 4 q) are held by the threads
// tc = 4q .. 4q + 3, which are the four 16-lane groups g = tc & 3 of wave q
// (lane = tr + 16 g); their rows tr + 16 ia sit in a[ia][IB].  With every
// update by columns < j0 applied, that wave factors the four columns on its
// own: per column, the pivot is read across lanes, the column's group
// scales it by 1/sqrt(pivot), and the groups of the later columns apply it
// (its values fetched across lanes by row, the multipliers L(j0+g, j) by
// lane reads).  The four columns then go to the LDS buffer colq[4][NB].
// IB is a template parameter so that every register index is a constant.
template <int IB>
__device__ __forceinline__ void factor_quad(double (&a)[TT][TT], double* __restrict__ colq,
                                            double* __restrict__ rdg, int q, int tr, int tc,
                                            int64_t k, DevState* __restrict__ st) {
  const int g = tc & 3;
  const int j0 = 16 * IB + 4 * q;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + c;
    const double d = readlane_f64(a[IB][IB], (4 * q + c) + 16 * c);  // A(j, j)
    if (g == c && tr == 4 * q + c && !(d > 0.0) && st->potrf_info == 0) {
      st->potrf_info = k + j + 1;
      st->status = BD_ERR_NOT_SPD;
    }
    const double rs = rsqrt_refined(d);  // NaN for a non-positive pivot
    if (g == c) {
#pragma unroll
      for (int ia = IB; ia < TT; ++ia) {
        const int i = tr + 16 * ia;
        if (i == j) {
          a[ia][IB] = d * rs;
          rdg[j] = rs;  // 1 / L(j,j), used by the diagonal-block inversion
        } else if (i > j) {
          a[ia][IB] *= rs;
        }
      }
    }
    if (c < 3) {
      double lv[TT];  // L(tr + 16 ia, j) in every lane
#pragma unroll
      for (int ia = IB; ia < TT; ++ia) lv[ia] = shfl_f64(a[ia][IB], tr + 16 * c);
      // L(j0 + g, j) for the groups g > c: row j0 + g of column j
      const double s1 = readlane_f64(a[IB][IB], (4 * q + c + 1) + 16 * c);
      const double s2 = (c + 2 < 4) ? readlane_f64(a[IB][IB], (4 * q + c + 2) + 16 * c) : 0.0;
      const double s3 = (c + 3 < 4) ? readlane_f64(a[IB][IB], (4 * q + c + 3) + 16 * c) : 0.0;
      const double sv = (g == c + 1) ? s1 : ((g == c + 2) ? s2 : s3);
      if (g > c) {
#pragma unroll
        for (int ia = IB; ia < TT; ++ia) a[ia][IB] = fma(-lv[ia], sv, a[ia][IB]);
      }
    }
  }
#pragma unroll
  for (int ia = IB; ia < TT; ++ia) {
    const int i = tr + 16 * ia;
    if (i >= j0 + g) colq[g * NB + i] = a[ia][IB];
  }
}

// Wave p (of four) inverts diagonal 32 x 32 block p of L11 (column-major in
// Ld, 1/L(j,j) in rdg) column by column: lane c solves L_pp y = e_c by
// forward substitution (y[i] = 0 for i < c falls out of the recursion); the
// upper lanes repeat the work and do not store.  Writes Winv_p (32 x 32,
// column-major) to W + p * SBB.
__device__ __forceinline__ void invert_diag_blocks(const double* __restrict__ Ld,
                                                   const double* __restrict__ rdg,
                                                   double* __restrict__ W, int tid) {
  const int p = tid >> 6, c = tid & 31;
  const double* L = Ld + p * SBB;
  const double* rd = rdg + SB * p;
  double y[SB];
#pragma unroll
  for (int i = 0; i < SB; ++i) {
    double s0 = (i == c) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
    for (int q = 0; q + 1 < i; q += 2) {
      s0 = fma(-L[q * SB + i], y[q], s0);
      s1 = fma(-L[(q + 1) * SB + i], y[q + 1], s1);
    }
    if (i & 1) s0 = fma(-L[(i - 1) * SB + i], y[i - 1], s0);
    y[i] = (s0 + s1) * rd[i];
  }
  if ((tid & 63) < SB) {
    double* Wc = W + p * SBB + c * SB;  // column c of Winv_p (column-major)
#pragma unroll
    for (int i = 0; i < SB; ++i) Wc[i] = y[i];
  }
}

// Rank-4 update by the published columns j0 .. j0 + 3 (j0 = 16 JB + 4 q) of
// the tile columns IB0 <= ib < IB1.  Only tiles ib >= JB, ia >= ib can hold
// live elements: for ia < ib every row is above every column, for ia > ib
// every row is below; within ia == ib only tr >= tc; and at ib == JB only
// the columns past j0 + 3.
template <int JB, int IB0, int IB1>
__device__ __forceinline__ void rank4_tiles(double (&a)[TT][TT], const double* __restrict__ colq,
                                            int q, int tr, int tc) {
  if (IB0 >= IB1) return;
  const bool lower_diag = tr >= tc;
  const bool col_live = tc > 4 * q + 3;
  double ci[4][TT], cc[4][TT];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int ia = IB0; ia < TT; ++ia) ci[u][ia] = colq[u * NB + tr + 16 * ia];
#pragma unroll
    for (int ib = IB0; ib < IB1; ++ib) cc[u][ib] = colq[u * NB + tc + 16 * ib];
  }
#pragma unroll
  for (int ib = IB0; ib < IB1; ++ib)
#pragma unroll
    for (int ia = ib; ia < TT; ++ia) {
      bool live = true;
      if (ia == ib) live = lower_diag;
      if (ib == JB) live = live && col_live;
      double upd = a[ia][ib];
#pragma unroll
      for (int u = 0; u < 4; ++u) upd = fma(-ci[u][ia], cc[u][ib], upd);
      a[ia][ib] = live ? upd : a[ia][ib];
    }
}

// Columns 16 JB .. 16 JB + 15 in four quads.  Quad number qi = 4 JB + q is
// published in colq buffer qi & 1.  Each thread first updates the tile
// column that holds the next quad, whose owning wave then factors and
// publishes it into the other buffer while the remaining tiles are
// updated; one barrier per quad.
template <int JB>
__device__ __forceinline__ void chol_block(double (&a)[TT][TT], double* __restrict__ colq,
                                           double* __restrict__ rdg, int tr, int tc, int w,
                                           int64_t k, DevState* __restrict__ st) {
  constexpr int JN = (JB + 1 < TT) ? JB + 1 : JB;  // tile column of the quad after this block
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qi = 4 * JB + q;
    const double* cur = colq + (qi & 1) * 4 * NB;
    double* nxt = colq + ((qi + 1) & 1) * 4 * NB;
    if (q < 3) {
      rank4_tiles<JB, JB, JB + 1>(a, cur, q, tr, tc);
      if (w == q + 1) factor_quad<JB>(a, nxt, rdg, q + 1, tr, tc, k, st);
      rank4_tiles<JB, JB + 1, TT>(a, cur, q, tr, tc);
    } else if (JB + 1 < TT) {
      // no column of tile column JB is past the last quad of the block
      rank4_tiles<JB, JN, JN + 1>(a, cur, q, tr, tc);
      if (w == 0) factor_quad<JN>(a, nxt, rdg, 0, tr, tc, k, st);
      rank4_tiles<JB, JN + 1, TT>(a, cur, q, tr, tc);
    }
    __syncthreads();  // next quad published; this quad no longer read
  }
}

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int64_t ld,
                                                          int64_t k, int nb,
                                                          double* __restrict__ W,
                                                          DevState* __restrict__ st) {
  __shared__ double colq[2 * 4 * NB]; // two buffers of four columns of L
  __shared__ double Ld[NSB][SBB];     // diagonal 32 x 32 blocks of L, column-major
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
  static_assert(TT == 8, "diagonal block tiling");
  const int w = tid >> 6;
  if (w == 0) factor_quad<0>(a, colq, rdg, 0, tr, tc, k, st);
  __syncthreads();
  chol_block<0>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<1>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<2>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<3>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<4>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<5>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<6>(a, colq, rdg, tr, tc, w, k, st);
  chol_block<7>(a, colq, rdg, tr, tc, w, k, st);
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
  invert_diag_blocks(&Ld[0][0], rdg, W, tid);
}

// ------------------------------------------------------------------------
// 1b. The same diagonal block on matrix cores.  The block is held as 16 x 16
//     tiles in the FP64 MFMA result layout: lane lr + 16 lk, register r
//     holds tile column lr and MFMA row lk + 4r, which stands for tile row
//     tile_row(lk, r) = 2 lk + (r & 1) + 8 (r >> 1) (any fixed row order
//     serves; this one gives each lane row pairs, for 16-byte loads and
//     stores).  Wave w owns tile columns w and w + 4; each diagonal tile is
//     kept whole and symmetric.  The owner of tile column J factors its 16
//     columns alone, without exchanges through LDS: column j's pivot is a
//     lane read, its entries reach the lanes of their row by DPP
//     (row_newbcast), and the multiplier of lane lr is the symmetric entry
//     (j, 16 J + lr) of the diagonal tile, spread over the four lane groups
//     by two lane swaps.  The columns stay unscaled: each rank-1 update
//     carries 1 / A(j,j), whose Newton steps are interleaved with the
//     previous column's update of the tiles below the diagonal, and each
//     column is scaled by 1 / sqrt(A(j,j)) once, when the block is
//     published.  Every wave then applies the published block to its tiles
//     as a rank-16 update (four v_mfma_f64_16x16x4 per tile), the next
//     block's owner first.  One barrier per 16 columns.
// ------------------------------------------------------------------------
constexpr int kLpStride = 17;  // padded LDS row of a published column block

// Inline assembly statements keep their program order (volatile); the
// host build that checks memory accesses defines BD_ASM as a no-op.
#ifndef BD_ASM
#define BD_ASM asm volatile
#endif

__host__ __device__ constexpr int tile_row(int lk, int r) { return 2 * lk + (r & 1) + 8 * (r >> 1); }
// MFMA row i = lk + 4r of a result tile as a tile row
__host__ __device__ constexpr int mfma_row(int i) { return tile_row(i & 3, i >> 2); }
// lane group and register holding tile row p
__host__ __device__ constexpr int row_group(int p) { return (p & 7) >> 1; }
__host__ __device__ constexpr int row_reg(int p) { return (p & 1) + 2 * (p >> 3); }

// 1/x to full FP64 accuracy: hardware estimate plus two Newton steps.
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// Lane (lane & 15) + 16 C's value to every lane of its 16-lane row.
template <int C>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + C, 0xF, 0xF, true);
}

// Lane (lane & 15) + 16 S's value to the lanes (lane & 15) + 16 g, g < 4.
template <int S>
__device__ __forceinline__ uint32_t group_bcast_u32(uint32_t v) {
  const uint32_t h = __builtin_amdgcn_permlane32_swap(v, v, false, false)[S >> 1];
  return __builtin_amdgcn_permlane16_swap(h, h, false, false)[S & 1];
}
template <int S>
__device__ __forceinline__ double group_bcast(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = group_bcast_u32<S>((uint32_t)u), hi = group_bcast_u32<S>((uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Rank-1 update of tiles [TB, TE) by unscaled column C: element (row, lr)
// gains beta(lr) A(row, j).  Lanes with beta = 0 keep their values exactly.
// Column 0 of a block broadcasts with a DPP move and a separate FMA, so that
// the compiler orders these first reads of the matrix-core results; later
// columns use one v_fmac_f64 with the DPP broadcast on its first operand.
// Two wait states must separate a VALU write of a register from a DPP
// instruction reading it, which the compiler does not check inside inline
// assembly: a column's writes of an element and the next column's read of
// it are kept apart by the next pivot's steps (tile 0) or by the next
// column's tile-0 update and first pivot step (other tiles), scheduling
// barriers stop the compiler from moving them closer, the statements are
// volatile so that they keep their program order, and the first
// instruction of each column waits for its coefficient.
template <int C>
__device__ __forceinline__ void fmac_row_bcast(double& x, double beta, bool wait) {
  if (wait)  // beta may have been written by the instruction before (folded when unrolled)
    BD_ASM("s_nop 1\n\tv_fmac_f64_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
        : "+v"(x)
        : "v"(beta), "i"(C));
  else
    BD_ASM("v_fmac_f64_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
        : "+v"(x)
        : "v"(beta), "i"(C));
}

template <int C, int TB, int TE, int NT>
__device__ __forceinline__ void tile_rank1(d4 (&T)[NT], double beta) {
#pragma unroll
  for (int t = TB; t < TE; ++t) {
    if constexpr (C == 0) {
      double v[4];  // all broadcasts first: no temporary is rewritten right after its use
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = row_bcast<C>(T[t][r]);
#pragma unroll
      for (int r = 0; r < 4; ++r) T[t][r] = fma(beta, v[r], T[t][r]);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double x = T[t][r];
        fmac_row_bcast<C>(x, beta, t == 0 && r == 0);
        T[t][r] = x;
      }
    }
  }
}

// Pivot of column j = 16 J + C, in seven dependent parts S = 0 .. 6 that
// the caller interleaves with independent work.  Part 6 yields this lane's
// rank-1 coefficient -A(j, 16 J + lr) / A(j,j) for the columns past j (0
// elsewhere), keeps A(j,j) in the lane of column j (myd) and records the
// first non-positive pivot in `bad`.  The multiplier A(j, 16 J + lr) comes
// from the lane of the same column in the lane group holding tile row j,
// through the LDS crossbar (bsrc: that lane's byte address per group).
struct Pivot {
  double d, m, y, e;
};
template <int J, int C, int S>
__device__ __forceinline__ void pivot_part(const d4& T0, Pivot& p, double& beta, double& myd,
                                           int& bad, int lr, const int (&bsrc)[4]) {
  constexpr int g = row_group(C), q = row_reg(C);
  if constexpr (S == 0) {
    p.d = readlane_f64(T0[q], C + 16 * g);  // A(j, j)
    // the element goes through a scalar first: clang bit-casts a vector
    // element operand as the vector's leading bytes
    const double v = T0[q];
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_ds_bpermute(bsrc[g], (int)(uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_ds_bpermute(bsrc[g], (int)(uint32_t)(u >> 32));
    p.m = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);  // A(j, 16 J + lr)
  } else if constexpr (S == 1) {
    p.y = __builtin_amdgcn_rcp(p.d);  // then two Newton steps
  } else if constexpr (S == 2 || S == 4) {
    p.e = fma(-p.d, p.y, 1.0);
  } else if constexpr (S == 3 || S == 5) {
    p.y = fma(p.y, p.e, p.y);
  } else {
    bad = (bad < 0 && !(p.d > 0.0)) ? 16 * J + C : bad;
    myd = (lr == C) ? p.d : myd;
    beta = (lr > C) ? -p.m * p.y : 0.0;
  }
}

// Column C of block J: tile 0 first, then the next pivot's parts, each
// followed by one tile below the diagonal.
template <int J, int C, int S, int NT>
__device__ __forceinline__ void tile_col_part(d4 (&T)[NT], Pivot& p, double beta, double& bnext,
                                              double& myd, int& bad, int lr,
                                              const int (&bsrc)[4]) {
  pivot_part<J, C + 1, S>(T[0], p, bnext, myd, bad, lr, bsrc);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (1 + S < 8 - J) tile_rank1<C, 1 + S, 2 + S>(T, beta);
  __builtin_amdgcn_sched_barrier(0);
}

template <int J, int C, int NT, int... S>
__device__ __forceinline__ void tile_col_parts(d4 (&T)[NT], Pivot& p, double beta, double& bnext,
                                               double& myd, int& bad, int lr,
                                               const int (&bsrc)[4],
                                               std::integer_sequence<int, S...>) {
  (tile_col_part<J, C, S>(T, p, beta, bnext, myd, bad, lr, bsrc), ...);
}

template <int J, int C, int NT>
__device__ __forceinline__ void tile_col(d4 (&T)[NT], double& beta, double& myd, int& bad,
                                         int lr, const int (&bsrc)[4]) {
  if constexpr (C < 15) {  // column 15 has no columns past it in the block
    tile_rank1<C, 0, 1>(T, beta);
    __builtin_amdgcn_sched_barrier(0);
    Pivot p;
    double bnext;
    tile_col_parts<J, C>(T, p, beta, bnext, myd, bad, lr, bsrc,
                         std::make_integer_sequence<int, 7>{});
    beta = bnext;
  }
}

template <int J, int NT, int... C>
__device__ __forceinline__ void tile_cols(d4 (&T)[NT], double& beta, double& myd, int& bad,
                                          int lr, const int (&bsrc)[4],
                                          std::integer_sequence<int, C...>) {
  (tile_col<J, C>(T, beta, myd, bad, lr, bsrc), ...);
}

template <int J, int... S>
__device__ __forceinline__ void first_pivot(const d4& T0, Pivot& p, double& beta, double& myd,
                                            int& bad, int lr, const int (&bsrc)[4],
                                            std::integer_sequence<int, S...>) {
  (pivot_part<J, 0, S>(T0, p, beta, myd, bad, lr, bsrc), ...);
}

// Owner of tile column J: factor it, scale it, publish its rows below tile
// J to lp and its 1 / L(j,j) to rdg.
template <int J, int NT>
__device__ __forceinline__ void tile_factor_publish(d4 (&T)[NT], double* __restrict__ lp,
                                                    double* __restrict__ rdg, int& bad, int lr,
                                                    int lk) {
  double myd = 1.0, beta = 0.0;
  int bsrc[4];  // byte address of lane lr in each lane group, for the multipliers
#pragma unroll
  for (int g = 0; g < 4; ++g) bsrc[g] = 4 * (lr + 16 * g);
  {
    Pivot p;
    first_pivot<J>(T[0], p, beta, myd, bad, lr, bsrc, std::make_integer_sequence<int, 7>{});
  }
  tile_cols<J>(T, beta, myd, bad, lr, bsrc, std::make_integer_sequence<int, 16>{});
  const double myrs = rsqrt_refined(myd);  // 1 / L(16 J + lr, 16 J + lr); NaN if not positive
#pragma unroll
  for (int t = 0; t < 8 - J; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[t][r] *= myrs;
  if (lk == 0) rdg[16 * J + lr] = myrs;
#pragma unroll
  for (int t = 1; t < 8 - J; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      lp[(16 * (J + t) + tile_row(lk, r)) * kLpStride + lr] = T[t][r];
}

// Rank-16 update of this wave's tiles (K + t, K), t < 8 - K, of tile column
// K by the published column block in lp.
template <int K, int NT>
__device__ __forceinline__ void tile_apply(d4 (&T)[NT], const double* __restrict__ lp, int lr,
                                           int lk) {
  double b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) b[s] = lp[(16 * K + lr) * kLpStride + 4 * s + lk];
  const int ar = mfma_row(lr);
#pragma unroll
  for (int t = 0; t < 8 - K; ++t) {
    double a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = -lp[(16 * (K + t) + ar) * kLpStride + 4 * s + lk];
#pragma unroll
    for (int s = 0; s < 4; ++s) T[t] = mfma(a[s], b[s], T[t]);
  }
}

// Wave W, not the owner of column block J + 1: its tile columns past J.
template <int J, int W>
__device__ __forceinline__ void tile_apply_rest(d4 (&T0)[8], d4 (&T1)[4], const double* lp,
                                                int lr, int lk) {
  if constexpr (W > J) tile_apply<W>(T0, lp, lr, lk);
  if constexpr (W + 4 > J) tile_apply<W + 4>(T1, lp, lr, lk);
}

// After column block J is published in lp_cur: the owner of block J + 1
// updates that tile column first, factors and publishes it into lp_next,
// then updates its other column; every other wave updates its columns
// past J.  Ends with the barrier that publishes block J + 1.  Scheduling
// barriers keep the phases apart, so that no operand of a later phase is
// held in registers through the factorisation.
template <int J>
__device__ __forceinline__ void tile_step(d4 (&T0)[8], d4 (&T1)[4], const double* lp_cur,
                                          double* lp_next, double* rdg, int& bad, int w, int lr,
                                          int lk) {
  constexpr int Jn = J + 1;
  if constexpr (Jn < 8) {
    if (w == Jn % 4) {
      if constexpr (Jn < 4) {
        tile_apply<Jn>(T0, lp_cur, lr, lk);
        __builtin_amdgcn_sched_barrier(0);
        tile_factor_publish<Jn>(T0, lp_next, rdg, bad, lr, lk);
        __builtin_amdgcn_sched_barrier(0);
        tile_apply<Jn + 4>(T1, lp_cur, lr, lk);
      } else {
        tile_apply<Jn>(T1, lp_cur, lr, lk);
        __builtin_amdgcn_sched_barrier(0);
        tile_factor_publish<Jn>(T1, lp_next, rdg, bad, lr, lk);
      }
    } else {
      switch (w) {
        case 0: tile_apply_rest<J, 0>(T0, T1, lp_cur, lr, lk); break;
        case 1: tile_apply_rest<J, 1>(T0, T1, lp_cur, lr, lk); break;
        case 2: tile_apply_rest<J, 2>(T0, T1, lp_cur, lr, lk); break;
        default: tile_apply_rest<J, 3>(T0, T1, lp_cur, lr, lk); break;
      }
    }
    __syncthreads();
  }
}

template <int... J>
__device__ __forceinline__ void tile_steps(d4 (&T0)[8], d4 (&T1)[4], double* lp, double* rdg,
                                           int& bad, int w, int lr, int lk,
                                           std::integer_sequence<int, J...>) {
  (tile_step<J>(T0, T1, lp + (J & 1) * NB * kLpStride, lp + ((J + 1) & 1) * NB * kLpStride, rdg,
                bad, w, lr, lk),
   ...);
}

// Tiles (K + t, K), t < NT, of tile column K from global memory into T,
// rows and columns past nb padded with the identity.  The diagonal tile is
// read whole, its upper part mirrored from the lower one; whole tiles below
// it are read as row pairs (16-byte loads, when ld is even).
template <int NT>
__device__ __forceinline__ void tile_load(d4 (&T)[NT], int K, const double* __restrict__ Akk,
                                          int64_t ld, int nb, int lr, int lk) {
  const int col = 16 * K + lr;
  const bool pairs = (ld & 1) == 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r0 = 16 * (K + t);
    if (t > 0 && pairs && r0 + 16 <= nb && 16 * K + 16 <= nb) {
      if (t < 8 - K) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double2 v = *reinterpret_cast<const double2*>(
              Akk + (int64_t)col * ld + r0 + tile_row(lk, 2 * h));
          T[t][2 * h] = v.x;
          T[t][2 * h + 1] = v.y;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + tile_row(lk, r);
        const bool live = (t < 8 - K) && row < nb && col < nb;
        const int64_t off = (row >= col) ? (int64_t)col * ld + row : (int64_t)row * ld + col;
        double v = (row == col) ? 1.0 : 0.0;
        if (live) v = Akk[off];
        T[t][r] = v;
      }
    }
  }
}

// Tiles of tile column K back to global memory (lower triangle, rows and
// columns below nb; whole tiles below the diagonal as row pairs) and into
// the diagonal 32 x 32 blocks Ld.
template <int NT>
__device__ __forceinline__ void tile_store(const d4 (&T)[NT], int K, double* __restrict__ Akk,
                                           int64_t ld, int nb, double* __restrict__ Ld, int lr,
                                           int lk) {
  const int col = 16 * K + lr;
  const bool pairs = (ld & 1) == 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int I = K + t, r0 = 16 * I;
    if (t < 8 - K) {
      if (t > 0 && pairs && r0 + 16 <= nb && 16 * K + 16 <= nb) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
          *reinterpret_cast<double2*>(Akk + (int64_t)col * ld + r0 + tile_row(lk, 2 * h)) =
              double2{T[t][2 * h], T[t][2 * h + 1]};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + tile_row(lk, r);
          if (row >= col && row < nb && col < nb) Akk[(int64_t)col * ld + row] = T[t][r];
        }
      }
      if ((I >> 1) == (K >> 1))
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + tile_row(lk, r);
          if (row >= col) Ld[(row >> 5) * SBB + (col & 31) * SB + (row & 31)] = T[t][r];
        }
    }
  }
}

// x += bcast_C(l) * b, the DPP broadcast on the multiplicand (see
// fmac_row_bcast for the wait states).
template <int C>
__device__ __forceinline__ void fmac_bcast_src(double& x, double l, double b, bool wait) {
  if (wait)
    BD_ASM("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(x)
        : "v"(l), "v"(b), "i"(C));
  else
    BD_ASM("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(x)
        : "v"(l), "v"(b), "i"(C));
}

// Step K of inverting a lower-triangular 16 x 16 tile L in the tile layout
// by forward elimination: R (initially I) becomes L^-1.  Row K of the
// inverse is R(K, .) / L(K,K); every later row i then loses L(i, K) times
// it.  Lz is L with its diagonal and upper part zeroed, rk = 1 / L(K,K).
template <int K>
__device__ __forceinline__ void tile_inv_step(d4& R, const d4& Lz, double rk, int lk, int lr) {
  constexpr int g = row_group(K), q = row_reg(K);
  R[q] *= (lk == g) ? rk : 1.0;
  if constexpr (K < 15) {
    // -X(K, lr), in every lane group, through the LDS crossbar
    const double v = R[q];
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int src = 4 * (lr + 16 * g);
    const uint32_t lo = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(u >> 32));
    const double xk = -__builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double x = R[r];
      fmac_bcast_src<K>(x, Lz[r], xk, r == 0);
      R[r] = x;
    }
  }
}

// Step K of two independent tiles in one scheduling region, so that their
// dependent chains overlap; the region boundary keeps step K + 1's reads of
// R at least the other tile's step away from step K's writes.
template <int... K>
__device__ __forceinline__ void tile_inv2(d4& R0, const d4& L0, const double (&rd0)[16], d4& R1,
                                          const d4& L1, const double (&rd1)[16], int lk, int lr,
                                          std::integer_sequence<int, K...>) {
  ((tile_inv_step<K>(R0, L0, rd0[K], lk, lr), tile_inv_step<K>(R1, L1, rd1[K], lk, lr),
    __builtin_amdgcn_sched_barrier(0)),
   ...);
}

// Inverses of the four diagonal 32 x 32 blocks of L into W (Winv_p
// column-major at W + p SBB), from the tiles in registers: wave w inverts
// its diagonal tiles (w, w) and (w + 4, w + 4) in place of L's in the
// diagonal blocks Ld; after a barrier wave p forms block p's lower-left
// part -X_c B X_a (B = L(2p+1, 2p), X_a, X_c the inverses of the diagonal
// tiles) with two 16 x 16 x 16 MFMA products and writes the whole block.
__device__ __forceinline__ void invert_diag_tiles(const d4& D0, const d4& D1, double* __restrict__ Ld,
                                                  const double* __restrict__ rdg,
                                                  double* __restrict__ W, int w, int lr, int lk) {
  d4 Lz0, Lz1, R0, R1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = tile_row(lk, r);
    Lz0[r] = (row > lr) ? D0[r] : 0.0;
    Lz1[r] = (row > lr) ? D1[r] : 0.0;
    R0[r] = R1[r] = (row == lr) ? 1.0 : 0.0;
  }
  double rd0[16], rd1[16];  // 1 / L(j,j) of the two tiles, read before the steps
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    rd0[j] = rdg[16 * w + j];
    rd1[j] = rdg[16 * (w + 4) + j];
  }
  tile_inv2(R0, Lz0, rd0, R1, Lz1, rd1, lk, lr, std::make_integer_sequence<int, 16>{});
  // X tiles over the diagonal tiles of the blocks (columns 16 (K & 1) + lr)
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int K = w + 4 * t, o = 16 * (K & 1);
    double* Lp = Ld + (K >> 1) * SBB;
#pragma unroll
    for (int r = 0; r < 4; ++r) Lp[(o + lr) * SB + o + tile_row(lk, r)] = t ? R1[r] : R0[r];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  const double* Lp = Ld + w * SBB;  // block p = w
  d4 Y = {0, 0, 0, 0}, Z = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s)  // Y = B X_a
    Y = mfma(Lp[(4 * s + lk) * SB + 16 + lr], Lp[lr * SB + 4 * s + lk], Y);
#pragma unroll
  for (int s = 0; s < 4; ++s)  // Z = -X_c Y; Y's register s is the B operand of step s
    Z = mfma(-Lp[(16 + 4 * s + lk) * SB + 16 + lr], Y[s], Z);
  double* Wp = W + w * SBB;
#pragma unroll
  for (int r = 0; r < 4; ++r) Wp[lr * SB + 16 + lk + 4 * r] = Z[r];  // rows 16.., columns ..15
  const int lane = lr + 16 * lk;
#pragma unroll
  for (int i = 0; i < 12; ++i) {  // the other three quarters, column-major
    const int qt = i / 4;         // 0: X_a, 1: X_c, 2: upper right (zero)
    const int e = lane + 64 * (i % 4);
    const int col = e / 16, row = e % 16;
    const int oc = (qt == 0) ? 0 : 16, orow = (qt == 1) ? 16 : 0;
    Wp[(oc + col) * SB + orow + row] = (qt == 2) ? 0.0 : Lp[(oc + col) * SB + orow + row];
  }
}

__device__ __forceinline__ void potrf_tile_body(double* __restrict__ A, int64_t ld, int64_t k,
                                                int nb, double* __restrict__ W,
                                                DevState* __restrict__ st) {
  // published column blocks (double buffer); after the last of them has
  // been applied, the diagonal 32 x 32 blocks of L (column-major) for the
  // inversion
  __shared__ double lp[2 * NB * kLpStride];
  static_assert(2 * NB * kLpStride >= NSB * SBB, "diagonal blocks fit the publish buffers");
  double* const Ld = lp;
  __shared__ double rdg[NB];  // 1 / L(j,j)
  __shared__ int first_bad;   // first non-positive pivot (NB: none)
  // the block is on the critical path of the factorisation: its waves take
  // issue priority over trailing-update waves sharing their SIMDs
  __builtin_amdgcn_s_setprio(3);
  const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  double* Akk = A + k * ld + k;
  d4 T0[8], T1[4];  // tile columns w and w + 4
  int bad = -1;     // first non-positive pivot among this wave's columns
  if (tid == 0) first_bad = NB;
  tile_load(T0, w, Akk, ld, nb, lr, lk);
  tile_load(T1, w + 4, Akk, ld, nb, lr, lk);
  if (w == 0) tile_factor_publish<0>(T0, lp, rdg, bad, lr, lk);
  __syncthreads();
  tile_steps(T0, T1, lp, rdg, bad, w, lr, lk, std::make_integer_sequence<int, 7>{});
  tile_store(T0, w, Akk, ld, nb, Ld, lr, lk);
  tile_store(T1, w + 4, Akk, ld, nb, Ld, lr, lk);
  if (lane == 0 && bad >= 0) atomicMin(&first_bad, bad);
  // LDS only: the global stores of L drain during the inversion
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  if (tid == 0 && first_bad < NB && st->potrf_info == 0) {
    st->potrf_info = k + first_bad + 1;
    st->status = BD_ERR_NOT_SPD;
  }
  invert_diag_tiles(T0[0], T1[0], Ld, rdg, W, w, lr, lk);
}

__global__ __launch_bounds__(256) void potrf_tile_kernel(double* __restrict__ A, int64_t ld,
                                                          int64_t k, int nb,
                                                          double* __restrict__ W,
                                                          DevState* __restrict__ st) {
  potrf_tile_body(A, ld, k, nb, W, st);
}

// W bytes of each lane from global memory straight into LDS, at the
// wave-uniform address `lds` plus W times the lane index.
template <int W>
__device__ __forceinline__ void load_to_lds(const void* g, void* lds) {
  static_assert(W == 16 || W == 4, "load width");
  if constexpr (W == 16)
    __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds(g, lds, 4, 0, 0);
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

// With xi non-null (the ensemble's fused noise product) the row block's
// share of the noise product is stored as well: yp(k + nb + row) =
// cB sum_c X(row, c) xi(k + c), yp this panel's row of partial sums (the
// rows below the diagonal block; store only, so no read latency lands on
// the chain of panels).  Each lane sums the columns c = lk (mod 4) in
// order and the four sums are combined pairwise, (s0 + s1) + (s2 + s3);
// noise_part_kernel forms the same sums in the same order.
__device__ __forceinline__ void panel_solve_body(int bx, double* __restrict__ A, int64_t ld,
                                                 int64_t k, int nb, int64_t m,
                                                 const double* __restrict__ W,
                                                 float* __restrict__ P32, int64_t ldp,
                                                 const double* __restrict__ xi,
                                                 double* __restrict__ yp, double cB) {
  static_assert(NSB == 4 && res_row_f64_is_lk_plus_4r, "register layout of the panel solve");
  __builtin_amdgcn_s_setprio(3);  // critical path, like the diagonal block
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int64_t row = (int64_t)bx * kRB + 16 * w + lr;
  const bool live = row < m;
  double* A21 = A + k * ld + k + nb;
  const double* L11 = A + k * ld + k;
  double x[NB / 4];
#pragma unroll
  for (int t = 0; t < NB / 4; ++t) {
    const int c = 4 * t + lk;
    x[t] = (live && c < nb) ? A21[(int64_t)c * ld + row] : 0.0;
  }
  // xi(k .. k + NB - 1) for the noise share, one copy per wave, straight to
  // LDS (no registers), issued after the row block's loads so that waiting
  // for those does not wait for it: it lands while the rows are solved
  __shared__ __attribute__((aligned(16))) double sxi[kPsThreads / 64][NB];
  if (xi) {
#pragma unroll
    for (int u = 0; u < NB * 8 / 256; ++u)
      load_to_lds<4>(reinterpret_cast<const char*>(xi + k) + 256 * u + 4 * lane, &sxi[w][32 * u]);
  }
  solve_subpanel<0>(x, L11, ld, W, lr, lk);
  solve_subpanel<1>(x, L11, ld, W + SBB, lr, lk);
  solve_subpanel<2>(x, L11, ld, W + 2 * SBB, lr, lk);
  solve_subpanel<3>(x, L11, ld, W + 3 * SBB, lr, lk);
  if (xi) {  // lanes lr + 16 lk hold the columns lk (mod 4) of one row
    const double* sxi_w = sxi[w];
    double sxs = 0.0;
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
      const int c = 4 * t + lk;
      if (c < nb) sxs += x[t] * sxi_w[c];
    }
    sxs += __shfl_xor(sxs, 16, 64);
    sxs += __shfl_xor(sxs, 32, 64);
    if (live && lk == 0) yp[k + nb + row] = cB * sxs;
  }
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

__global__ __launch_bounds__(kPsThreads) void panel_solve_kernel(
    double* __restrict__ A, int64_t ld, int64_t k, int nb, int64_t m, const double* __restrict__ W,
    float* __restrict__ P32, int64_t ldp) {
  panel_solve_body(blockIdx.x, A, ld, k, nb, m, W, P32, ldp, nullptr, nullptr, 0.0);
}

// The panels' shares of the noise product y = cB L xi for panels already
// factored (one chain: launched beside the factorisation, after each
// step's trailing update, instead of adding work to each panel solve on
// the chain of diagonal blocks and panel solves).  Block (bx, j) stores,
// for the rows i = i0 + 256 bx + t below panel p = p0 + j,
// ypart(p, i) = cB sum_c L(i, p NB + c) xi(p NB + c), summed exactly as the
// fused panel solve sums it: four running sums over c = q (mod 4) and
// (s0 + s1) + (s2 + s3), so that one chain and an ensemble chain agree to
// the bit.  Lanes read consecutive rows of one column (512 bytes a wave).
constexpr int kNpRows = 256;

__global__ __launch_bounds__(kNpRows) void noise_part_kernel(const double* __restrict__ A,
                                                            int64_t ld, int64_t n, int64_t p0,
                                                            int64_t i0,
                                                            const double* __restrict__ xi,
                                                            double* __restrict__ ypart,
                                                            double cB) {
  const int64_t pn = p0 + blockIdx.y;
  const int64_t k = pn * NB;
  const int64_t i = i0 + (int64_t)blockIdx.x * kNpRows + threadIdx.x;
  if (i < k + NB || i >= n) return;
  const double* Li = A + k * ld + i;
  const double* xk = xi + k;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 8
  for (int t = 0; t < NB / 4; ++t) {
    const int64_t c = 4 * t;
    s0 += Li[c * ld] * xk[c];
    s1 += Li[(c + 1) * ld] * xk[c + 1];
    s2 += Li[(c + 2) * ld] * xk[c + 2];
    s3 += Li[(c + 3) * ld] * xk[c + 3];
  }
  ypart[pn * n + i] = cB * ((s0 + s1) + (s2 + s3));
}

// The noise product's sums, after the factorisation: row i of block b gets
// y(i) = sum_{p < b} ypart(p, i) (the panels' shares, in panel order) +
// cB sum_{c <= r} L(i, bNB + c) xi(bNB + c) (its diagonal block, r = i - bNB).
// Two work-items per row, one per sum; lanes read consecutive rows of one
// column.
__device__ __forceinline__ void noise_sum_body(int blk, const double* __restrict__ A, int64_t ld,
                                               int64_t n, const double* __restrict__ xi,
                                               const double* __restrict__ ypart,
                                               double* __restrict__ y, double cB) {
  // work-items r < NB add the panels' shares of row k + r, work-items NB + r
  // its diagonal block's share, side by side; both sums keep their order
  __shared__ double sdiag[NB];
  const int64_t k = (int64_t)blk * NB;
  const int half = threadIdx.x / NB, r = threadIdx.x - NB * half;
  const bool live = k + r < n;
  // sixteen loads in flight at a time, the sums still in order
  constexpr int U = 16;
  double s = 0.0;
  if (live && half == 0) {
    int p = 0;
    for (; p + U <= blk; p += U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = ypart[(int64_t)(p + u) * n + k + r];
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; p < blk; ++p) s += ypart[(int64_t)p * n + k + r];
  } else if (live) {
    const double* Akk = A + k * ld + k;
    double sxi = 0.0;
    int c = 0;
    for (; c + U <= r + 1; c += U) {
      double a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = Akk[(int64_t)(c + u) * ld + r];
        b[u] = xi[k + c + u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) sxi += a[u] * b[u];
    }
    for (; c <= r; ++c) sxi += Akk[(int64_t)c * ld + r] * xi[k + c];
    sdiag[r] = sxi;
  }
  __syncthreads();
  if (live && half == 0) y[k + r] = s + cB * sdiag[r];
}

__global__ __launch_bounds__(2 * NB) void noise_sum_kernel(const double* __restrict__ A,
                                                           int64_t ld, int64_t n,
                                                           const double* __restrict__ xi,
                                                           const double* __restrict__ ypart,
                                                           double* __restrict__ y, double cB) {
  noise_sum_body(blockIdx.x, A, ld, n, xi, ypart, y, cB);
}

// ------------------------------------------------------------------------
// 3. Trailing update C -= L L^T on the lower TS x TS tiles (TS = 128, or 64
//    for the columns on the lookahead chain) of the m x m trailing matrix; L
//    is m x kdim (column-major, ldl) in FP64 or FP32, kdim a multiple of KC
//    (one to four panels).  Four waves, each a TS/2 x TS/2 quadrant (the
//    strictly upper quadrant of a diagonal tile is skipped).
//    Operands go from HBM straight into LDS (global_load_lds, 16 bytes per
//    lane, no registers), double-buffered in K-chunks of KC: each chunk's
//    loads are issued after the current chunk's LDS reads and complete
//    under its MFMAs.  LDS holds each operand k-major, [k][TS]: the global
//    column segments land contiguously.  Within a quadrant, 16 x 16 block b
//    of NBK = TS/32 takes the rows (columns) NBK i + b, so lane lr reads its
//    NBK consecutive rows at one k in one access, one operand for each
//    block; lane (lr, lk) takes k = 4 kq + lk at step kq for both operands.
//    The row permutation makes each lane's outputs NBK consecutive rows of
//    one column: C is read and written in 16-byte accesses.
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

// Tile sets of one trailing update: every lower tile, only the first nnext
// tile columns (the next step's panels, updated ahead), or every lower tile
// outside those columns.
enum { kTilesAll = 0, kTilesNext = 1, kTilesRest = 2 };

// AL: the operand L and the matrix C start on 16-byte boundaries and their
// column strides are multiples of 16 bytes.  Then each lane moves 16 bytes
// per operand load and C is accessed in 16-byte vectors; otherwise 4 bytes
// per load and scalar C accesses.  A 16-byte operand load may run up to 12
// bytes past a column's last row m - 1 (the group holding it); past the
// last column of an FP32 panel copy that needs the slack of kP32Tail.
template <typename T, int TS, bool AL>
__device__ __forceinline__ void syrk_update_body(int t, double* __restrict__ C, int64_t ld,
                                                 const T* __restrict__ L, int64_t ldl, int64_t m,
                                                 int kdim, int tiles, int nnext) {
  // The FP32 next-column update (TS = 64) takes half-width chunks and 64
  // registers, so that its workgroups fit on a CU beside two bulk ones
  // (448 of 512 registers per SIMD, 128 of 160 KB of LDS) instead of
  // waiting for one of them to finish; same sums in the same order.
  constexpr int KC = (sizeof(T) == 4 && TS == 64) ? 16 : SyrkCfg<T>::KC;
  typedef typename SyrkCfg<T>::acc_t acc_t;
  constexpr int WT = TS / 2;    // each wave owns a WT x WT quadrant
  constexpr int NBK = WT / 16;  // 16 x 16 MFMA blocks per quadrant side
  constexpr int KQ = KC / 4;    // MFMA steps per chunk
  constexpr int SZ = (int)sizeof(T);
  constexpr int W = AL ? 16 : 4;                // bytes per lane per load
  constexpr int RB = TS * SZ;                   // bytes per LDS k-row
  constexpr int BI = 64 * W;                    // bytes per load instruction
  constexpr int NIW = KC * RB / BI / 4;         // loads per wave per operand per chunk
  static_assert(TS == 64 || TS == 128, "tile size");
  static_assert(NIW >= 1 && NIW * BI * 4 == KC * RB, "load split");
  static_assert(BI % RB == 0 || RB % BI == 0, "load shape");
  if constexpr (TS == 64) __builtin_amdgcn_s_setprio(3);  // the lookahead chain's updates
  __shared__ __attribute__((aligned(16))) T As[2][KC][TS];  // row side
  __shared__ __attribute__((aligned(16))) T Bs[2][KC][TS];  // column side

  int ti, tj;
  if (tiles == kTilesNext) {
    // tile column q holds tiles q .. mt-1; columns 0 .. nnext-1 in order
    const int mt = (int)((m + TS - 1) / TS);
    int q = 0, r = t;
    while (q + 1 < nnext && r >= mt - q) {
      r -= mt - q;
      ++q;
    }
    ti = q + r;
    tj = q;
  } else {
    const int mt = (int)((m + TS - 1) / TS) - (tiles == kTilesRest ? nnext : 0);
    band_index(t, mt, ti, tj);
    if (tiles == kTilesRest) {
      ti += nnext;
      tj += nnext;
    }
  }
  const int64_t row0 = (int64_t)ti * TS, col0 = (int64_t)tj * TS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wr = w >> 1, wc = w & 1;
  const bool active = !(ti == tj && wr < wc);

  acc_t acc[NBK][NBK];
#pragma unroll
  for (int bj = 0; bj < NBK; ++bj)
#pragma unroll
    for (int bi = 0; bi < NBK; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[bj][bi][r] = 0;

  // Loads: instruction u of wave w fills bytes [BI (w NIW + u), + BI) of an
  // operand's chunk buffer, lane l the W bytes at W l within them: k-row
  // kr, byte eb of that row, i.e. global row r0 + eb / SZ of column kk + kr.
  // A lane whose group starts at or past m reads the tile's first row
  // instead (in bounds; such rows only reach masked outputs).
  const char* __restrict__ Lb = reinterpret_cast<const char*>(L);
  const int64_t ldb = ldl * SZ;  // column stride in bytes
  auto src = [&](int64_t r0b, int u, int kk) {
    const int B = BI * (w * NIW + u) + W * lane;
    const int kr = B / RB, eb = B % RB;
    const int64_t rb = (r0b + eb < m * SZ) ? r0b + eb : r0b + eb % SZ;
    return Lb + (int64_t)(kk + kr) * ldb + rb;
  };
  auto dma = [&](int buf, int kk) {
#pragma unroll
    for (int u = 0; u < NIW; ++u) {
      char* da = reinterpret_cast<char*>(&As[buf][0][0]) + BI * (w * NIW + u);
      char* db = reinterpret_cast<char*>(&Bs[buf][0][0]) + BI * (w * NIW + u);
      load_to_lds<W>(src(row0 * SZ, u, kk), da);
      load_to_lds<W>(src(col0 * SZ, u, kk), db);
    }
  };
  typedef T vn __attribute__((ext_vector_type(NBK)));
  auto chunk = [&](int buf) {
    vn af[KQ], bf[KQ];
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
      af[kq] = *reinterpret_cast<const vn*>(&Bs[buf][4 * kq + lk][WT * wc + NBK * lr]);
      bf[kq] = *reinterpret_cast<const vn*>(&As[buf][4 * kq + lk][WT * wr + NBK * lr]);
    }
    return [=](acc_t (&a)[NBK][NBK]) {
#pragma unroll
      for (int kq = 0; kq < KQ; ++kq)
#pragma unroll
        for (int bj = 0; bj < NBK; ++bj)
#pragma unroll
          for (int bi = 0; bi < NBK; ++bi) a[bj][bi] = mfma(af[kq][bj], bf[kq][bi], a[bj][bi]);
    };
  };

  // Epilogue addressing.  Output (bj, bi, r) of lane (lr, lk) is C(i, j)
  // with i = qi + NBK lr + bi and j = qj + NBK res_row(lk, r) + bj: for
  // fixed (bj, r) a lane holds NBK consecutive rows of one column.
  const int64_t qi = row0 + WT * wr, qj = col0 + WT * wc;
  typedef double d2v __attribute__((ext_vector_type(2)));
  // a quadrant wholly inside the matrix, on or below the diagonal, with C
  // on 16-byte boundaries: C moves in 16-byte vectors, in batches of EB
  // column blocks, the first batch read under the last chunk's products
  // and each later one read while the previous one is written
  const bool whole = AL && active && qi + WT <= m && qi >= qj + WT - 1;
  double* __restrict__ Cl = C + qj * ld + qi + NBK * lr;
  constexpr int EB = (sizeof(T) == 4) ? NBK / 2 : 1;
  constexpr int NBT = NBK / EB;
  typedef d2v batch_t[EB][4][NBK / 2];
  auto cload = [&](int b0, batch_t& cv) {
#pragma unroll
    for (int e = 0; e < EB; ++e)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double* cc = Cl + (int64_t)(NBK * res_row(acc[0][0], lk, r) + b0 + e) * ld;
#pragma unroll
        for (int h = 0; h < NBK / 2; ++h) cv[e][r][h] = *reinterpret_cast<const d2v*>(cc + 2 * h);
      }
  };
  auto cstore = [&](int b0, const batch_t& cv) {
#pragma unroll
    for (int e = 0; e < EB; ++e)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* cc = Cl + (int64_t)(NBK * res_row(acc[0][0], lk, r) + b0 + e) * ld;
#pragma unroll
        for (int h = 0; h < NBK / 2; ++h) {
          d2v v = cv[e][r][h];
          v[0] -= (double)acc[b0 + e][2 * h][r];
          v[1] -= (double)acc[b0 + e][2 * h + 1][r];
          *reinterpret_cast<d2v*>(cc + 2 * h) = v;
        }
      }
  };

  const int nch = kdim / KC;
  dma(0, 0);
  __syncthreads();
  for (int ch = 0; ch + 1 < nch; ++ch) {
    const int buf = ch & 1;
    if (active) {
      auto run = chunk(buf);
      __builtin_amdgcn_sched_barrier(0);  // the LDS reads go out before the next loads
      dma(buf ^ 1, (ch + 1) * KC);
      run(acc);
    } else {
      dma(buf ^ 1, (ch + 1) * KC);
    }
    __syncthreads();
  }
  if (!active) return;
  if constexpr (sizeof(T) == 4 && TS == 64) {  // 64 registers: one batch at a time
    chunk((nch - 1) & 1)(acc);
    if (whole) {
#pragma unroll
      for (int bt = 0; bt < NBT; ++bt) {
        batch_t cv;
        cload(bt * EB, cv);
        cstore(bt * EB, cv);
      }
      return;
    }
  } else {
  batch_t c0;
  {
    auto run = chunk((nch - 1) & 1);
    if (whole) cload(0, c0);
    run(acc);
  }
  if (whole) {
#pragma unroll
    for (int bt = 0; bt < NBT; bt += 2) {
      batch_t c1;
      if (bt + 1 < NBT) cload((bt + 1) * EB, c1);
      cstore(bt * EB, c0);
      if (bt + 1 < NBT) {
        if (bt + 2 < NBT) cload((bt + 2) * EB, c0);
        cstore((bt + 1) * EB, c1);
      }
    }
    return;
  }
  }
  // other quadrants: element by element, masked
#pragma unroll
  for (int bj = 0; bj < NBK; ++bj) {
    double cv[NBK][4];
#pragma unroll
    for (int bi = 0; bi < NBK; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = qi + NBK * lr + bi;
        const int64_t j = qj + NBK * res_row(acc[bj][bi], lk, r) + bj;
        cv[bi][r] = (i < m && j < m && i >= j) ? C[j * ld + i] : 0.0;
      }
#pragma unroll
    for (int bi = 0; bi < NBK; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = qi + NBK * lr + bi;
        const int64_t j = qj + NBK * res_row(acc[bj][bi], lk, r) + bj;
        if (i < m && j < m && i >= j) C[j * ld + i] = cv[bi][r] - (double)acc[bj][bi][r];
      }
  }
}

// XCD x receives workgroups x, x+8, ...: cnt(x) = base + (x < rem) of them;
// the q-th of them takes tile x*base + min(x, rem) + q (a bijection).
template <typename T, int TS>
constexpr int syrk_min_blocks() { return (sizeof(T) == 4 && TS == 64) ? 8 : 2; }
template <typename T, int TS, bool AL>
__global__ __launch_bounds__(256, (syrk_min_blocks<T, TS>())) void syrk_update_kernel(
    double* __restrict__ C, int64_t ld, const T* __restrict__ L, int64_t ldl, int64_t m, int kdim,
    int tiles, int nnext) {
  syrk_update_body<T, TS, AL>(xcd_contiguous(blockIdx.x, gridDim.x), C, ld, L, ldl, m, kdim, tiles,
                          nnext);
}

// ------------------------------------------------------------------------
// 4. Ensembles: the same kernels over a table of chains, chain blockIdx.z.
//    The host schedule is common to every chain (steps of a fixed number
//    of panels from column 0); each workgroup derives its chain's panel width, row count
//    and tile set from the chain's n and returns at once where the chain
//    has no work.  Grids cover the largest chain still active.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void potrf_tile_batched_kernel(const ChainDesc* __restrict__ cd,
                                                                  int64_t k) {
  const ChainDesc& c = cd[blockIdx.z];
  if (k >= c.n) return;
  potrf_tile_body(c.D, c.ld, k, (c.n - k < NB) ? (int)(c.n - k) : NB, c.W, c.st);
}

// Panel kp of the step starting at k0, whose FP32 copy (MIXED) is P32[pidx];
// one flattened grid over every chain's row blocks.
__global__ __launch_bounds__(kPsThreads) void panel_solve_batched_kernel(
    const ChainDesc* __restrict__ cd, const int32_t* __restrict__ prefix, int z, int64_t k0,
    int64_t kp, int pidx, int noise) {
  const int ci = find_chain(prefix, z, blockIdx.x);
  const ChainDesc& c = cd[ci];
  const int64_t m = c.n - kp - NB;
  float* P = c.P32[pidx];
  if (P) P += (kp - k0) * p32_ld(c.n) + kp + NB;
  panel_solve_body(blockIdx.x - prefix[ci], c.D, c.ld, kp, NB, m, c.W, P, p32_ld(c.n),
                   noise ? c.xi : nullptr, c.ypart + (kp / NB) * c.n, c.cB);
}

// Chain blockIdx.z's rows.
__global__ __launch_bounds__(2 * NB) void noise_sum_batched_kernel(const ChainDesc* __restrict__ cd) {
  const ChainDesc& c = cd[blockIdx.z];
  if ((int64_t)blockIdx.x * NB >= c.n) return;
  noise_sum_body(blockIdx.x, c.D, c.ld, c.n, c.xi, c.ypart, c.y, c.cB);
}

// Tiles of tile set `tiles` in an m x m trailing matrix with TS x TS tiles;
// nnext: the tile columns updated ahead (at most nnext_panels panels).
__host__ __device__ inline int64_t syrk_tile_count(int64_t m, int ts, int tiles,
                                                   int nnext_panels, int64_t* nnext_out) {
  if (m <= 0) {
    *nnext_out = 0;
    return 0;
  }
  const int64_t mt = (m + ts - 1) / ts;
  int64_t np = (m + NB - 1) / NB;
  if (np > nnext_panels) np = nnext_panels;
  int64_t nnext = np * (NB / ts);
  if (nnext > mt) nnext = mt;
  *nnext_out = nnext;
  if (tiles == kTilesAll) return mt * (mt + 1) / 2;
  if (tiles == kTilesNext) return nnext * mt - nnext * (nnext - 1) / 2;
  return (mt - nnext) * (mt - nnext + 1) / 2;
}

// Tile set `tiles` of the update of the trailing matrix from row r0 by the
// kdim columns from k0; nnext_panels caps the panels of the chain's next
// step (the tile columns updated ahead).
// One flattened grid over every chain's tiles, each XCD taking a contiguous
// range of (chain, tile).
template <typename T, int TS, bool AL>
__global__ __launch_bounds__(256, (syrk_min_blocks<T, TS>())) void syrk_update_batched_kernel(
    const ChainDesc* __restrict__ cd, const int32_t* __restrict__ prefix, int z, int64_t k0,
    int64_t r0, int kdim, int tiles, int nnext_panels, int pidx) {
  const int tg = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ci = find_chain(prefix, z, tg);
  const ChainDesc& c = cd[ci];
  const int64_t m = c.n - r0;
  int64_t nnext;
  (void)syrk_tile_count(m, TS, tiles, nnext_panels, &nnext);
  const int t = tg - prefix[ci];
  const T* L;
  int64_t ldl;
  if constexpr (sizeof(T) == 4) {
    L = c.P32[pidx] + r0;
    ldl = p32_ld(c.n);
  } else {
    L = c.D + k0 * c.ld + r0;
    ldl = c.ld;
  }
  syrk_update_body<T, TS, AL>(t, c.D + r0 * c.ld + r0, c.ld, L, ldl, m, kdim, tiles, (int)nnext);
}

}  // namespace

size_t cholesky_batched_workspace_bytes(int64_t n, bd_precision_t prec) {
  size_t b = align_up(sizeof(double) * NB * NB, 256);
  if (prec == BD_PREC_MIXED) b += 2 * p32_copy_bytes(n);
  return b;
}

size_t cholesky_workspace_bytes(int64_t n, bd_precision_t prec) {
  size_t b = align_up(sizeof(double) * NB * NB, 256);  // four 32 x 32 inverses (NB*NB/4 used)
  if (prec == BD_PREC_MIXED) b += 2 * p32_copy_bytes(n);
  return b;
}

namespace {

struct CholCtx {
  int64_t n, ld;
  double* A;
  double* W;
  // MIXED: FP32 copies of the panels of consecutive steps, n x kMaxStep each,
  // indexed by global row (P[c * n + row]); null in FP64
  float* P32[2];
  int max_panels;     // panels per step: 1, 2 or 4
  int64_t wide_rows;  // four-panel steps only while more rows than this remain
  bool tile_potrf;    // diagonal blocks on matrix cores (else register tiles)
  DevState* st;
  // noise product y = cB L xi (xi null: none): each step's panel shares
  // beside the factorisation, their sums at its end; ypart: the panels'
  // partial sums, (n / NB) rows of n
  const double* xi;
  double* y;
  double* ypart;
  double cB;
};

// Columns of the factorisation step starting at column k0: wide steps
// while the trailing matrix is large (its update dominates), narrower ones
// once the chain of diagonal factors is the longer path.
int64_t step_width(const CholCtx& c, int64_t k0) {
  const int panels = (c.n - k0 > c.wide_rows) ? c.max_panels
                                              : (c.max_panels < 2 ? c.max_panels : 2);
  return (c.n - k0 < (int64_t)panels * NB) ? c.n - k0 : (int64_t)panels * NB;
}

// Steps before the one starting at k0; consecutive steps use the two FP32
// panel copies in turn.
int64_t step_index(const CholCtx& c, int64_t k0) {
  int64_t i = 0;
  for (int64_t k = 0; k < k0; k += step_width(c, k)) ++i;
  return i;
}

float* step_copy(const CholCtx& c, int64_t k0) {
  return c.P32[0] ? c.P32[step_index(c, k0) & 1] : nullptr;
}

// Diagonal block and panel solve of the panel at column kp, which is panel
// number (kp - k0) / NB of the step starting at k0.
hipError_t factor_panel(const CholCtx& c, hipStream_t s, int64_t k0, int64_t kp) {
  const int nb = (int)((c.n - kp < NB) ? (c.n - kp) : NB);
  if (c.tile_potrf)
    BD_LAUNCH("potrf_tile", potrf_tile_kernel, dim3(1), dim3(256), 0, s, c.A, c.ld, kp, nb, c.W,
              c.st);
  else
    BD_LAUNCH("potrf_diag", potrf_diag_kernel, dim3(1), dim3(256), 0, s, c.A, c.ld, kp, nb, c.W,
              c.st);
  const int64_t m = c.n - kp - nb;
  if (m > 0) {  // then nb == NB: only the last panel can be narrower
    float* P = step_copy(c, k0);
    if (P) P += (kp - k0) * p32_ld(c.n) + kp + NB;  // column kp - k0 of the step, row kp + NB
    BD_LAUNCH("panel_solve", panel_solve_kernel, dim3((unsigned)((m + kRB - 1) / kRB)),
              dim3(kPsThreads), 0, s, c.A, c.ld, kp, nb, m, c.W, P, p32_ld(c.n));
  }
  return hipGetLastError();
}

// A pointer and a column stride (bytes) that keep every column on a
// 16-byte boundary.
bool aligned16(const void* p, int64_t stride_bytes) {
  return reinterpret_cast<uintptr_t>(p) % 16 == 0 && stride_bytes % 16 == 0;
}

// C -= L L^T on the trailing matrix from row/column r0 with the kdim columns
// k0 .. k0 + kdim - 1 of L, restricted to a tile set.
hipError_t trailing(const CholCtx& c, hipStream_t s, int64_t k0, int64_t r0, int kdim, int tiles,
                    int nnext) {
  // The next-step columns lie on the lookahead chain: 64 x 64 tiles spread
  // them over four times as many CUs; the bulk update keeps 128 x 128 tiles.
  const int ts = (tiles == kTilesNext) ? kTS / 2 : kTS;
  nnext *= NB / ts;  // in tiles
  const int64_t m = c.n - r0;
  const int64_t mt = (m + ts - 1) / ts;
  if (nnext > mt) nnext = (int)mt;
  int64_t nt = 0;
  if (tiles == kTilesAll) nt = mt * (mt + 1) / 2;
  if (tiles == kTilesNext)
    for (int q = 0; q < nnext; ++q) nt += mt - q;
  if (tiles == kTilesRest) nt = (mt - nnext) * (mt - nnext + 1) / 2;
  if (nt <= 0) return hipSuccess;
  double* C = c.A + r0 * c.ld + r0;
  const float* P = step_copy(c, k0);
  const double* L64 = c.A + k0 * c.ld + r0;
  const dim3 grid((unsigned)nt);
  if (P) {
    const int64_t ldp = p32_ld(c.n);
    const bool al = aligned16(P + r0, ldp * 4) && aligned16(C, c.ld * 8);
    if (ts == kTS && al)
      BD_LAUNCH("syrk_update_f32", (syrk_update_kernel<float, kTS, true>), grid, dim3(256), 0, s,
                C, c.ld, P + r0, ldp, m, kdim, tiles, nnext);
    else if (ts == kTS)
      BD_LAUNCH("syrk_update_f32", (syrk_update_kernel<float, kTS, false>), grid, dim3(256), 0, s,
                C, c.ld, P + r0, ldp, m, kdim, tiles, nnext);
    else if (al)
      BD_LAUNCH("syrk_next_f32", (syrk_update_kernel<float, kTS / 2, true>), grid, dim3(256), 0,
                s, C, c.ld, P + r0, ldp, m, kdim, tiles, nnext);
    else
      BD_LAUNCH("syrk_next_f32", (syrk_update_kernel<float, kTS / 2, false>), grid, dim3(256), 0,
                s, C, c.ld, P + r0, ldp, m, kdim, tiles, nnext);
  } else {
    const bool al = aligned16(L64, c.ld * 8) && aligned16(C, c.ld * 8);
    if (ts == kTS && al)
      BD_LAUNCH("syrk_update_f64", (syrk_update_kernel<double, kTS, true>), grid, dim3(256), 0, s,
                C, c.ld, L64, c.ld, m, kdim, tiles, nnext);
    else if (ts == kTS)
      BD_LAUNCH("syrk_update_f64", (syrk_update_kernel<double, kTS, false>), grid, dim3(256), 0,
                s, C, c.ld, L64, c.ld, m, kdim, tiles, nnext);
    else if (al)
      BD_LAUNCH("syrk_next_f64", (syrk_update_kernel<double, kTS / 2, true>), grid, dim3(256), 0,
                s, C, c.ld, L64, c.ld, m, kdim, tiles, nnext);
    else
      BD_LAUNCH("syrk_next_f64", (syrk_update_kernel<double, kTS / 2, false>), grid, dim3(256), 0,
                s, C, c.ld, L64, c.ld, m, kdim, tiles, nnext);
  }
  return hipGetLastError();
}

// The noise product's shares of the panels of the step at columns
// k0 .. k0 + w - 1, once they are factored (the last panel of the matrix
// has no rows below it).
hipError_t noise_parts(const CholCtx& c, hipStream_t s, int64_t k0, int64_t w) {
  if (!c.xi) return hipSuccess;
  const int64_t p0 = k0 / NB;
  const int64_t p1 = (k0 + w + NB - 1) / NB;
  const int64_t np = ((p1 * NB < c.n) ? p1 : (c.n + NB - 1) / NB - 1) - p0;
  const int64_t i0 = (p0 + 1) * NB / kNpRows * kNpRows;  // no row above stores
  if (np > 0)
    BD_LAUNCH("noise_part", noise_part_kernel,
              dim3((unsigned)((c.n - i0 + kNpRows - 1) / kNpRows), (unsigned)np), dim3(kNpRows), 0,
              s, c.A, c.ld, c.n, p0, i0, c.xi, c.ypart, c.cB);
  return hipGetLastError();
}

// The ordered sums of the noise product, once every share is stored (all
// on stream s by then).
hipError_t diag_noise(const CholCtx& c, hipStream_t s) {
  if (!c.xi) return hipSuccess;
  BD_LAUNCH("noise_sum", noise_sum_kernel, dim3((unsigned)((c.n + NB - 1) / NB)), dim3(2 * NB), 0,
            s, c.A, c.ld, c.n, c.xi, c.ypart, c.y, c.cB);
  return hipGetLastError();
}

// The panels of the step starting at k0: each later panel first receives
// the update by the step's earlier panels (one tile column), then is
// factored.  Returns the step width.
hipError_t factor_step(const CholCtx& c, hipStream_t s, int64_t k0, int64_t* width) {
  int64_t kp = k0;
  hipError_t e;
  const int64_t end = k0 + step_width(c, k0);
  for (int p = 0; kp < end; ++p, kp += NB) {
    if (p > 0 && (e = trailing(c, s, k0, kp, (int)(kp - k0), kTilesNext, 1)) != hipSuccess)
      return e;
    if ((e = factor_panel(c, s, k0, kp)) != hipSuccess) return e;
  }
  *width = end - k0;
  return hipSuccess;
}

}  // namespace

// Right-looking blocked factorisation in steps of up to max_panels panels
// (four while more than wide_rows rows remain, two after: a step of p
// panels applies them in one pass over the trailing matrix, dividing its
// HBM traffic per flop by p), with depth-1 lookahead: while the main stream
// applies step k0 to the trailing matrix (all but the next step's tile
// columns), the auxiliary stream updates those tile columns first, then
// factors the next step's panels.  Events order the two streams; with
// aux == nullptr everything runs on `s` in order.
hipError_t launch_cholesky(hipStream_t s, hipStream_t aux, hipEvent_t ev[4], int64_t n, double* A,
                           int64_t ld, bd_precision_t prec, void* ws, DevState* st,
                           int max_panels, int64_t wide_rows, bool tile_potrf, const double* xi,
                           double* y, double cB, double* ypart) {
  CholCtx c;
  c.xi = ypart ? xi : nullptr;
  c.y = y;
  c.ypart = ypart;
  c.cB = cB;
  c.n = n;
  c.ld = ld;
  c.A = A;
  c.st = st;
  c.W = static_cast<double*>(ws);
  c.max_panels = (max_panels >= 4) ? 4 : (max_panels == 2 ? 2 : 1);
  c.wide_rows = wide_rows;
  c.tile_potrf = tile_potrf;
  c.P32[0] = c.P32[1] = nullptr;
  if (prec == BD_PREC_MIXED) {
    char* p = static_cast<char*>(ws) + align_up(sizeof(double) * NB * NB, 256);
    c.P32[0] = reinterpret_cast<float*>(p);
    c.P32[1] = reinterpret_cast<float*>(p + p32_copy_bytes(n));
  }
  hipError_t e;
  int64_t w = 0;
  if (!aux) {
    for (int64_t k = 0; k < n; k += w) {
      if ((e = factor_step(c, s, k, &w)) != hipSuccess) return e;
      if (k + w < n && (e = trailing(c, s, k, k + w, (int)w, kTilesAll, 0)) != hipSuccess) return e;
      if ((e = noise_parts(c, s, k, w)) != hipSuccess) return e;
    }
    return diag_noise(c, s);
  }
  hipEvent_t ev_fork = ev[0], ev_panel = ev[1], ev_rest = ev[2], ev_next = ev[3];
  if ((e = hipEventRecord(ev_fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(aux, ev_fork, 0)) != hipSuccess) return e;
  if ((e = factor_step(c, aux, 0, &w)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev_panel, aux)) != hipSuccess) return e;
  int64_t k = 0;
  for (; k + w < n;) {
    const int64_t r0 = k + w;
    const int nnext = (int)((step_width(c, r0) + NB - 1) / NB);  // panels of the next step
    // main: step k must be factored before it is applied
    if ((e = hipStreamWaitEvent(s, ev_panel, 0)) != hipSuccess) return e;
    // aux: the next step's tile columns must have every earlier update
    if (k > 0 && (e = hipStreamWaitEvent(aux, ev_rest, 0)) != hipSuccess) return e;
    if ((e = trailing(c, aux, k, r0, (int)w, kTilesNext, nnext)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev_next, aux)) != hipSuccess) return e;
    int64_t wn = 0;
    if ((e = factor_step(c, aux, r0, &wn)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev_panel, aux)) != hipSuccess) return e;
    // main: the bulk update starts once the next columns are done, so that
    // they (on the critical path) do not share the GPU with it
    if ((e = hipStreamWaitEvent(s, ev_next, 0)) != hipSuccess) return e;
    if ((e = trailing(c, s, k, r0, (int)w, kTilesRest, nnext)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev_rest, s)) != hipSuccess) return e;
    // main: step k's noise shares, in the time it would wait for the chain
    if ((e = noise_parts(c, s, k, w)) != hipSuccess) return e;
    k = r0;
    w = wn;
  }
  if ((e = hipStreamWaitEvent(s, ev_panel, 0)) != hipSuccess) return e;
  if ((e = noise_parts(c, s, k, w)) != hipSuccess) return e;
  return diag_noise(c, s);
}

namespace {

// The batched schedule: the chains of the table in decreasing order of n,
// so that the chains with work at column k are a prefix of it.
struct BatchCtx {
  const ChainDesc* cd;       // device table
  const ChainDesc* host;     // its host copy
  int count;
  bool mixed;
  int64_t step;  // columns per step, the same for every chain
  BatchTables* tb;
  bool noise;    // fused noise product into each chain's y (xi, cB)
};

// The prefix array of the next launch from the workgroup counts of chains
// 0 .. z-1 (recorded, or checked against the recording); *total: the grid.
// Returns the device copy (null while recording).
template <typename F>
const int32_t* flat_table(const BatchCtx& b, int z, F count, int* total, bool* ok) {
  BatchTables& t = *b.tb;
  const size_t off = t.cur;
  int64_t acc = 0;
  *ok = true;
  if (t.record) t.host.push_back(0);
  else if (off + (size_t)z >= t.host.size() || t.host[off] != 0) *ok = false;
  for (int c = 0; c < z; ++c) {
    acc += count(c);
    if (acc > INT32_MAX) *ok = false;
    if (t.record) t.host.push_back((int32_t)acc);
    else if (*ok && t.host[off + (size_t)c + 1] != (int32_t)acc) *ok = false;
  }
  t.cur += (size_t)z + 1;
  *total = (int)acc;
  return t.record ? nullptr : t.dev + off;
}

// Chains with n > k.
int active(const BatchCtx& b, int64_t k) {
  int a = 0;
  while (a < b.count && b.host[a].n > k) ++a;
  return a;
}

int batch_pidx(const BatchCtx& b, int64_t k0) { return (int)((k0 / b.step) & 1); }

hipError_t batch_trailing(const BatchCtx& b, hipStream_t s, int64_t k0, int64_t r0, int kdim,
                          int tiles, int nnext_panels) {
  const int z = active(b, r0);
  if (z == 0) return hipSuccess;
  const int ts = (tiles == kTilesNext) ? kTS / 2 : kTS;
  int total = 0;
  bool ok = true;
  const int32_t* pre = flat_table(b, z, [&](int c) {
    int64_t nn;
    return syrk_tile_count(b.host[c].n - r0, ts, tiles, nnext_panels, &nn);
  }, &total, &ok);
  if (!ok) return hipErrorInvalidValue;
  if (total == 0 || b.tb->record) return hipSuccess;
  const dim3 grid((unsigned)total);
  const int pidx = batch_pidx(b, k0);
  // every chain's operand and matrix on 16-byte boundaries (the library's
  // own layouts are; a caller's workspace might not be)
  bool al = true;
  for (int c = 0; c < z; ++c) {
    const ChainDesc& h = b.host[c];
    al = al && aligned16(h.D, h.ld * 8) &&
         (!b.mixed || (aligned16(h.P32[0], p32_ld(h.n) * 4) && aligned16(h.P32[1], 16)));
  }
#define BD_SYRK_BATCHED(NAME, T, TSZ)                                                        \
  do {                                                                                       \
    if (al)                                                                                  \
      BD_LAUNCH(NAME, (syrk_update_batched_kernel<T, TSZ, true>), grid, dim3(256), 0, s, b.cd, \
                pre, z, k0, r0, kdim, tiles, nnext_panels, pidx);                            \
    else                                                                                     \
      BD_LAUNCH(NAME, (syrk_update_batched_kernel<T, TSZ, false>), grid, dim3(256), 0, s,      \
                b.cd, pre, z, k0, r0, kdim, tiles, nnext_panels, pidx);                      \
  } while (0)
  if (b.mixed && ts == kTS)
    BD_SYRK_BATCHED("syrk_update_f32_batched", float, kTS);
  else if (b.mixed)
    BD_SYRK_BATCHED("syrk_next_f32_batched", float, kTS / 2);
  else if (ts == kTS)
    BD_SYRK_BATCHED("syrk_update_f64_batched", double, kTS);
  else
    BD_SYRK_BATCHED("syrk_next_f64_batched", double, kTS / 2);
#undef BD_SYRK_BATCHED
  return hipGetLastError();
}

hipError_t batch_factor_step(const BatchCtx& b, hipStream_t s, int64_t k0) {
  hipError_t e;
  for (int64_t kp = k0; kp < k0 + b.step; kp += NB) {
    const int z = active(b, kp);
    if (z == 0) break;
    if (kp > k0 && (e = batch_trailing(b, s, k0, kp, (int)(kp - k0), kTilesNext, 1)) != hipSuccess)
      return e;
    if (!b.tb->record)
      BD_LAUNCH("potrf_tile_batched", potrf_tile_batched_kernel, dim3(1, 1, z), dim3(256), 0, s,
                b.cd, kp);
    const int zp = active(b, kp + NB);  // chains whose panel has rows below it
    if (zp > 0) {
      int total = 0;
      bool ok = true;
      const int32_t* pre = flat_table(b, zp, [&](int c) {
        return (b.host[c].n - kp - NB + kRB - 1) / kRB;
      }, &total, &ok);
      if (!ok) return hipErrorInvalidValue;
      if (!b.tb->record)
        BD_LAUNCH("panel_solve_batched", panel_solve_batched_kernel, dim3((unsigned)total),
                  dim3(kPsThreads), 0, s, b.cd, pre, zp, k0, kp, batch_pidx(b, k0),
                  b.noise ? 1 : 0);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// launch_cholesky's lookahead schedule, `panels` panels per step, over
// every chain of the table at once.
hipError_t launch_cholesky_batched(hipStream_t s, hipStream_t aux, hipEvent_t ev[4],
                                   const ChainDesc* cd, const ChainDesc* cd_host, int count,
                                   bd_precision_t prec, int panels, BatchTables* tb, bool noise) {
  if (count <= 0) return hipSuccess;
  panels = (panels >= 4) ? 4 : 2;
  BatchCtx b{cd, cd_host, count, prec == BD_PREC_MIXED, (int64_t)panels * NB, tb, noise};
  auto diag = [&]() {
    if (noise && !tb->record)
      BD_LAUNCH("noise_sum_batched", noise_sum_batched_kernel,
                dim3((unsigned)((cd_host[0].n + NB - 1) / NB), 1, (unsigned)count), dim3(2 * NB),
                0, s, cd);
    return hipGetLastError();
  };
  tb->cur = 0;
  const int64_t n = cd_host[0].n;  // the largest chain
  const int64_t w = b.step;
  hipError_t e;
  if (!aux) {
    for (int64_t k = 0; k < n; k += w) {
      if ((e = batch_factor_step(b, s, k)) != hipSuccess) return e;
      if (k + w < n && (e = batch_trailing(b, s, k, k + w, (int)w, kTilesAll, 0)) != hipSuccess)
        return e;
    }
    return diag();
  }
  // the recording pass takes the same path without launching anything
  const bool run = !tb->record;
  hipEvent_t ev_fork = ev[0], ev_panel = ev[1], ev_rest = ev[2], ev_next = ev[3];
  auto record = [&](hipEvent_t v, hipStream_t q) { return run ? hipEventRecord(v, q) : hipSuccess; };
  auto wait = [&](hipStream_t q, hipEvent_t v) {
    return run ? hipStreamWaitEvent(q, v, 0) : hipSuccess;
  };
  if ((e = record(ev_fork, s)) != hipSuccess) return e;
  if ((e = wait(aux, ev_fork)) != hipSuccess) return e;
  if ((e = batch_factor_step(b, aux, 0)) != hipSuccess) return e;
  if ((e = record(ev_panel, aux)) != hipSuccess) return e;
  for (int64_t k = 0; k + w < n; k += w) {
    const int64_t r0 = k + w;
    if ((e = wait(s, ev_panel)) != hipSuccess) return e;
    if (k > 0 && (e = wait(aux, ev_rest)) != hipSuccess) return e;
    if ((e = batch_trailing(b, aux, k, r0, (int)w, kTilesNext, panels)) != hipSuccess) return e;
    if ((e = record(ev_next, aux)) != hipSuccess) return e;
    if ((e = batch_factor_step(b, aux, r0)) != hipSuccess) return e;
    if ((e = record(ev_panel, aux)) != hipSuccess) return e;
    if ((e = wait(s, ev_next)) != hipSuccess) return e;
    if ((e = batch_trailing(b, s, k, r0, (int)w, kTilesRest, panels)) != hipSuccess) return e;
    if ((e = record(ev_rest, s)) != hipSuccess) return e;
  }
  if ((e = wait(s, ev_panel)) != hipSuccess) return e;
  return diag();
}

}  // namespace bd
