// Runs the whole Cholesky launch sequence of cholesky.hip on the CPU (see
// hip/hip_runtime.h) with exact-size buffers, so that AddressSanitizer
// reports any out-of-bounds access of a kernel or of the host schedule.  In
// FP64 it also checks the schedule itself from the launch arguments: every
// lower 128 x 128 tile must receive the updates of columns 0 .. 128 J in
// order, each exactly once, before its diagonal block is factored (tracked
// on 64 x 64 sub-tiles, the finest tile a launch uses), and
// every diagonal block is factored exactly once.  In both precisions every
// panel's share of the noise product y = L xi that ends the call must be
// stored for every row below the panel, and every row of y formed from them.
// Usage: chol_emu n ld prec(0 fp64, 1 mixed) max_panels(1|2|4) lookahead(0|1)
//        [tile_potrf(0|1), default 1] [wide_rows, default 0: every step as
//        wide as max_panels allows]
#include <cstring>
#include <map>
#include <utility>

#include "../../paper_2208_06559_amd/csrc/cholesky.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd

namespace {
const double* g_A = nullptr;
int64_t g_n = 0, g_ld = 0;
std::map<std::pair<int64_t, int64_t>, int64_t> g_applied;  // tile -> columns applied
std::map<int64_t, int> g_factored;                          // tile column -> times
int g_errors = 0;

const uint64_t kPartMark = 0x7ff8deadbeef0001ull, kYMark = 0x7ff8deadbeef0002ull;

void fail(const char* what, int64_t a, int64_t b, int64_t c) {
  if (g_errors++ < 10) fprintf(stderr, "schedule error: %s (%lld, %lld, %lld)\n", what,
                               (long long)a, (long long)b, (long long)c);
}

void observe(const void* kernel, dim3 grid, const int64_t* a, int nargs) {
  using namespace bd;
  int64_t ts = 0;
  if (kernel == (const void*)&syrk_update_kernel<double, kTS, true> ||
      kernel == (const void*)&syrk_update_kernel<double, kTS, false>)
    ts = kTS;
  if (kernel == (const void*)&syrk_update_kernel<double, kTS / 2, true> ||
      kernel == (const void*)&syrk_update_kernel<double, kTS / 2, false>)
    ts = kTS / 2;
  if (ts) {
    // (C, ld, L, ldl, m, kdim, tiles, nnext): tile size ts, nnext in tiles
    const int64_t coff = (a[0] - (int64_t)(uintptr_t)g_A) / 8, loff = (a[2] - (int64_t)(uintptr_t)g_A) / 8;
    const int64_t r0 = coff / (g_ld + 1), k0 = (loff - r0) / g_ld;
    const int64_t m = a[4], kdim = a[5], tiles = a[6], nnext = a[7];
    if (coff != r0 * (g_ld + 1) || loff != k0 * g_ld + r0 || m != g_n - r0) fail("syrk args", r0, k0, m);
    const int64_t mt = (m + ts - 1) / ts, nt = grid.x;
    for (int64_t t = 0; t < nt; ++t) {
      int64_t ti, tj;
      if (tiles == kTilesNext) {
        int64_t q = 0, r = t;
        while (q + 1 < nnext && r >= mt - q) {
          r -= mt - q;
          ++q;
        }
        ti = q + r;
        tj = q;
      } else {
        int rr, cc;
        band_index((int)t, (int)(mt - (tiles == kTilesRest ? nnext : 0)), rr, cc);
        ti = rr;
        tj = cc;
        if (tiles == kTilesRest) {
          ti += nnext;
          tj += nnext;
        }
      }
      if (ti >= mt || tj > ti) fail("tile outside region", ti, tj, mt);
      // bookkeeping in 64 x 64 units
      const int64_t f = ts / 64;
      for (int64_t u = 0; u < f; ++u)
        for (int64_t v = 0; v < f; ++v) {
          const int64_t I = (r0 + ti * ts) / 64 + u, J = (r0 + tj * ts) / 64 + v;
          if (I < J || I * 64 >= g_n) continue;
          const std::pair<int64_t, int64_t> key(I, J);
          if (g_applied[key] != k0) fail("update out of order or repeated", I, J, k0);
          g_applied[key] = k0 + kdim;
        }
    }
  } else if (kernel == (const void*)&potrf_diag_kernel ||
             kernel == (const void*)&potrf_tile_kernel) {
    // (A, ld, k, nb, W, st)
    const int64_t kp = a[2], J = kp / NB;
    for (int64_t I = kp / 64; I * 64 < g_n; ++I)
      for (int64_t Jc = kp / 64; Jc < kp / 64 + NB / 64 && Jc <= I && Jc * 64 < g_n; ++Jc)
        if (g_applied[{I, Jc}] != kp) fail("factored before all updates", I, Jc, g_applied[{I, Jc}]);
    if (g_factored[J]++) fail("diagonal block factored twice", J, kp, 0);
  }
}
}  // namespace

int main(int argc, char** argv) {
  if (argc < 6 || argc > 8) return 2;
  const int64_t n = atoll(argv[1]), ld = atoll(argv[2]);
  const int prec = atoi(argv[3]), sp = atoi(argv[4]), use_aux = atoi(argv[5]);
  const bool tile = argc >= 7 ? atoi(argv[6]) != 0 : true;
  const int64_t wide = argc >= 8 ? atoll(argv[7]) : 0;
  double* A = (double*)malloc(sizeof(double) * ((n - 1) * ld + n));
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i < n; ++i) A[c * ld + i] = (i == c) ? 1.0 + n : 0.1;
  g_A = A;
  g_n = n;
  g_ld = ld;
  if (prec == 0) g_emu_observer = observe;
  const size_t wsb = bd::cholesky_workspace_bytes(n, (bd_precision_t)prec);
  void* ws = malloc(wsb);
  memset(ws, 0, wsb);
  bd::DevState* st = (bd::DevState*)calloc(1, sizeof(bd::DevState));
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // the noise product: xi and y of exactly n doubles, the partial sums of
  // exactly noise_part_bytes(n); y and the partial sums start as NaNs with
  // payloads of their own, which no arithmetic on the factor can produce
  double* xi = (double*)malloc(sizeof(double) * n);
  double* y = (double*)malloc(sizeof(double) * n);
  const size_t npb = bd::noise_part_bytes(n);
  double* ypart = (double*)malloc(npb);
  for (size_t i = 0; i < npb / sizeof(double); ++i) memcpy(&ypart[i], &kPartMark, 8);
  for (int64_t i = 0; i < n; ++i) {
    xi[i] = 0.5 + 0.25 * (double)((i * 7) % 13) - 1.5 * (double)(i % 2);
    memcpy(&y[i], &kYMark, 8);
  }
  const hipError_t e = bd::launch_cholesky(nullptr, use_aux ? (hipStream_t)0x1 : nullptr, ev, n, A,
                                           ld, (bd_precision_t)prec, ws, st, sp, wide, tile, xi,
                                           y, 1.0, ypart);
  if (prec == 0)
    for (int64_t J = 0; J * bd::NB < n; ++J)
      if (g_factored[J] != 1) fail("diagonal block not factored once", J, g_factored[J], 0);
  // every panel's share of every row below it stored, and every row of y
  // written without reading a share that was never stored (the emulated
  // arithmetic is not the GPU's, so the values themselves are not checked)
  if (e == hipSuccess) {
    for (int64_t p = 0; (p + 1) * bd::NB < n; ++p)
      for (int64_t i = (p + 1) * bd::NB; i < n; ++i)
        if (memcmp(&ypart[p * n + i], &kPartMark, 8) == 0) fail("noise share not stored", p, i, 0);
    for (int64_t i = 0; i < n; ++i)
      if (memcmp(&y[i], &kYMark, 8) == 0 || memcmp(&y[i], &kPartMark, 8) == 0)
        fail("noise product row not formed from stored shares", i, 0, 0);
  }
  printf("n=%lld ld=%lld prec=%d max_panels=%d lookahead=%d tile_potrf=%d wide_rows=%lld: status %d, %ld launches, %d schedule errors\n",
         (long long)n, (long long)ld, prec, sp, use_aux, (int)tile, (long long)wide, e, g_emu_launches, g_errors);
  free(A);
  free(ws);
  free(st);
  free(xi);
  free(y);
  free(ypart);
  return (e != hipSuccess || g_errors) ? 1 : 0;
}
