// Runs the assembly of rpy.hip (launch_rpy_assemble, and the ensembles'
// launch_rpy_assemble_batched over three chains) on the CPU through the
// stand-in HIP runtime, under AddressSanitizer, with buffers of exactly the
// documented sizes: D (n-1)*ld + n doubles for n = 3N, positions 3N.  Then
// the lower triangle (or the whole matrix with BD_FILL_FULL) must have been
// written, and everything else must keep its NaN fill, the padding rows
// included.  The values are not checked here: the stand-in runtime runs a
// workgroup's work-items one after another, so the pair coefficients that
// the kernel passes between them through LDS across a barrier are not
// reproduced (the GPU tests compare the values with the oracle).
// Usage: rpy_emu N ld_pad fill(0 lower, 1 full)
#include <cmath>
#include <cstring>
#include <vector>

#include "../../paper_2208_06559_amd/csrc/rpy.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd

namespace {
int g_errors = 0;

void positions(int N, int seed, double* x) {  // a bent chain: no coincident beads
  for (int i = 0; i < N; ++i) {
    x[3 * i] = 0.9 * i + 0.05 * ((i * 7 + seed) % 5);
    x[3 * i + 1] = 0.4 * ((i + seed) % 3);
    x[3 * i + 2] = 0.3 * ((i * 3 + seed) % 4) - 0.2;
  }
}

void check(const char* what, const double* D, int64_t ld, int N, bool full) {
  const int64_t n = 3 * (int64_t)N;
  for (int64_t col = 0; col < n; ++col)
    for (int64_t row = 0; row < ld && (col < n - 1 || row < n); ++row) {
      const bool written = row < n && (full || row >= col);
      if (written != !std::isnan(D[col * ld + row]) && g_errors++ < 10)
        fprintf(stderr, "%s: (%ld, %ld) %s\n", what, (long)row, (long)col,
                written ? "not written" : "written");
    }
}
}  // namespace

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const int N = atoi(argv[1]);
  const int64_t pad = atoll(argv[2]);
  const bool full = atoi(argv[3]) != 0;
  const double hstar = 0.25, a = 0.5;
  // one chain through launch_rpy_assemble
  {
    const int64_t n = 3 * (int64_t)N, ld = n + pad, span = (n - 1) * ld + n;
    double* D = (double*)malloc(sizeof(double) * span);
    double* x = (double*)malloc(sizeof(double) * n);
    for (int64_t e = 0; e < span; ++e) D[e] = NAN;
    positions(N, 1, x);
    bd_params_t p{};
    p.n_beads = N;
    p.a = a;
    p.hstar = hstar;
    const hipError_t e = bd::launch_rpy_assemble(nullptr, p, x, D, ld, full ? BD_FILL_FULL : BD_FILL_LOWER);
    if (e != hipSuccess) ++g_errors;
    check("single", D, ld, N, full);
    free(D);
    free(x);
  }
  // three chains (N, N/2 + 1, 1) through the batched kernel, lower triangles
  if (!full) {
    const int Ns[3] = {N, N / 2 + 1, 1};
    std::vector<bd::ChainDesc> cd(3);
    std::vector<double*> Ds(3), xs(3);
    std::vector<int64_t> lds(3);
    std::vector<int32_t> prefix(4, 0);
    for (int c = 0; c < 3; ++c) {
      const int64_t n = 3 * (int64_t)Ns[c], ld = n + pad + c, span = (n - 1) * ld + n;
      Ds[c] = (double*)malloc(sizeof(double) * span);
      xs[c] = (double*)malloc(sizeof(double) * n);
      for (int64_t e = 0; e < span; ++e) Ds[c][e] = NAN;
      positions(Ns[c], 2 + c, xs[c]);
      memset(&cd[c], 0, sizeof(bd::ChainDesc));
      cd[c].N = Ns[c];
      cd[c].n = n;
      cd[c].x = xs[c];
      cd[c].D = Ds[c];
      cd[c].ld = ld;
      cd[c].hstar = hstar;
      cd[c].a = a;
      lds[c] = ld;
      prefix[c + 1] = prefix[c] + bd::rpy_batched_blocks(Ns[c]);
    }
    const hipError_t e =
        bd::launch_rpy_assemble_batched(nullptr, cd.data(), 3, prefix.data(), prefix[3]);
    if (e != hipSuccess) ++g_errors;
    for (int c = 0; c < 3; ++c) {
      check("batched", Ds[c], lds[c], Ns[c], false);
      free(Ds[c]);
      free(xs[c]);
    }
  }
  printf("N=%d pad=%ld fill=%s: %ld launches, %d errors\n", N, (long)pad, full ? "full" : "lower",
         g_emu_launches, g_errors);
  return g_errors ? 1 : 0;
}
