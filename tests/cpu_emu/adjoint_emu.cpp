// Runs the Cholesky adjoint of adjoint.hip (launch_cholesky_adjoint: the
// diagonal-block inverses, the pairwise joins level by level, the masked
// products and the mirror) on the CPU through the stand-in HIP runtime,
// under AddressSanitizer, for a batch of two matrices in buffers of exactly
// the documented sizes (matrices (n-1)*ld + n doubles at the given strides,
// workspace cholesky_adjoint_workspace_bytes(n) per matrix).
// Usage: adjoint_emu n ld_pad
#include "../../paper_2208_06559_amd/csrc/adjoint.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd
int main(int argc, char** argv) {
  if (argc != 3) return 2;
  const int64_t n = atoll(argv[1]), ld = n + atoll(argv[2]);
  const int batch = 2;
  const int64_t span = (n - 1) * ld + n;  // one matrix
  const int64_t stride = span + 7;        // batch stride, ragged
  const int64_t total = (batch - 1) * stride + span;
  double* L = (double*)malloc(sizeof(double) * total);
  double* Lb = (double*)malloc(sizeof(double) * total);
  double* Ab = (double*)malloc(sizeof(double) * total);
  for (int64_t e = 0; e < total; ++e) {
    L[e] = 1.0;
    Lb[e] = 0.5;
    Ab[e] = 0.0;
  }
  const size_t wsb = bd::cholesky_adjoint_workspace_bytes(n) * batch;
  void* ws = malloc(wsb);
  memset(ws, 0, wsb);
  const hipError_t e = bd::launch_cholesky_adjoint(nullptr, n, L, ld, stride, Lb, ld, stride, Ab,
                                                   ld, stride, 1.0, 1.0, batch, ws);
  printf("n=%ld ld=%ld: status %d, %ld launches\n", (long)n, (long)ld, e, g_emu_launches);
  free(L);
  free(Lb);
  free(Ab);
  free(ws);
  return e;
}
