// Runs the noise-product adjoint of brownian.hip (launch_brownian_adjoint:
// Lbar = c tril(ybar xi^T) over the triangular tile grid, and
// xibar = c L^T ybar) on the CPU through the stand-in HIP runtime, under
// AddressSanitizer, with buffers of exactly the documented sizes: L and
// Lbar (n-1)*ld + n doubles at their own leading dimensions, vectors n.
// Usage: brownian_adjoint_emu N ld_pad ldb_pad
#include "../../paper_2208_06559_amd/csrc/brownian.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd
int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const int N = atoi(argv[1]);
  const int64_t n = 3 * (int64_t)N, ld = n + atoll(argv[2]), ldb = n + atoll(argv[3]);
  double* L = (double*)malloc(sizeof(double) * ((n - 1) * ld + n));
  double* Lb = (double*)malloc(sizeof(double) * ((n - 1) * ldb + n));
  double* xi = (double*)malloc(sizeof(double) * n);
  double* yb = (double*)malloc(sizeof(double) * n);
  double* xib = (double*)malloc(sizeof(double) * n);
  for (int64_t e = 0; e < (n - 1) * ld + n; ++e) L[e] = 1.0;
  for (int64_t e = 0; e < n; ++e) xi[e] = yb[e] = 1.0;
  bd_params_t p{};
  p.n_beads = N;
  p.dt = 1e-3;
  const hipError_t e = bd::launch_brownian_adjoint(nullptr, p, L, ld, xi, yb, Lb, ldb, xib);
  printf("N=%d ld=%ld ldb=%ld: status %d, %ld launches\n", N, (long)ld, (long)ldb, e,
         g_emu_launches);
  free(L);
  free(Lb);
  free(xi);
  free(yb);
  free(xib);
  return e;
}
