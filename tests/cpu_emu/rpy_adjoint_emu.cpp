// Runs the assembly adjoint of rpy.hip (launch_rpy_adjoint: the tiled pair
// pass and the bead-order finish) on the CPU through the stand-in HIP
// runtime, under AddressSanitizer, with buffers of exactly the documented
// sizes: Dbar (n-1)*ld + n doubles for n = 3N, positions 3N, gradient 3N,
// partials N.
// Usage: rpy_adjoint_emu N ld_pad
#include "../../paper_2208_06559_amd/csrc/rpy.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd
int main(int argc, char** argv) {
  if (argc != 3) return 2;
  const int N = atoi(argv[1]);
  const int64_t n = 3 * (int64_t)N, ld = n + atoll(argv[2]);
  const int64_t span = (n - 1) * ld + n;
  double* Db = (double*)malloc(sizeof(double) * span);
  double* x = (double*)malloc(sizeof(double) * n);
  double* xbar = (double*)malloc(sizeof(double) * n);
  double* hpart = (double*)malloc(sizeof(double) * N);
  double* hbar = (double*)malloc(sizeof(double));
  bd::DevState* st = (bd::DevState*)calloc(1, sizeof(bd::DevState));
  for (int64_t e = 0; e < span; ++e) Db[e] = 0.25;
  for (int i = 0; i < N; ++i) {  // a straight chain: no coincident beads
    x[3 * i] = (double)i;
    x[3 * i + 1] = 0.5 * (i % 3);
    x[3 * i + 2] = 0.0;
  }
  bd_params_t p{};
  p.n_beads = N;
  p.a = 0.5;
  p.hstar = 0.25;
  const hipError_t e = bd::launch_rpy_adjoint(nullptr, p, x, Db, ld, xbar, hbar, hpart, st);
  printf("N=%d ld=%ld: status %d (device %d), %ld launches\n", N, (long)ld, e, (int)st->status,
         g_emu_launches);
  const int rc = (e != hipSuccess || st->status != 0) ? 1 : 0;
  free(Db);
  free(x);
  free(xbar);
  free(hpart);
  free(hbar);
  free(st);
  return rc;
}
