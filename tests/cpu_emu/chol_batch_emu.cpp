// Runs the batched Cholesky of cholesky.hip (launch_cholesky_batched: every
// chain of an ensemble in shared launches) on the CPU through the stand-in
// HIP runtime, under AddressSanitizer.  Each chain gets its own matrix and
// workspace at exactly the documented sizes (matrix (n-1)*ld + n doubles,
// cholesky_batched_workspace_bytes(n) of workspace), so an access of one
// chain's kernels outside its own buffers is reported.
// Usage: chol_batch_emu prec(0 fp64, 1 mixed) lookahead(0|1) panels(2|4) n_0 n_1 ...
#include <algorithm>
#include <vector>

#include "../../paper_2208_06559_amd/csrc/cholesky.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd

int main(int argc, char** argv) {
  if (argc < 5) return 2;
  const int prec = atoi(argv[1]), use_aux = atoi(argv[2]), panels = atoi(argv[3]);
  const int count = argc - 4;
  std::vector<bd::ChainDesc> cd((size_t)count);
  std::vector<void*> blocks;
  for (int c = 0; c < count; ++c) {
    const int64_t n = atoll(argv[4 + c]), ld = n + c % 3;
    bd::ChainDesc& d = cd[(size_t)c];
    memset(&d, 0, sizeof(d));
    d.n = n;
    d.N = (int)(n / 3);
    d.ld = ld;
    d.index = c;
    d.D = (double*)malloc(sizeof(double) * ((n - 1) * ld + n));
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) d.D[j * ld + i] = (i == j) ? 1.0 + n : 0.1;
    const size_t wsb = bd::cholesky_batched_workspace_bytes(n, (bd_precision_t)prec);
    char* ws = (char*)malloc(wsb);
    memset(ws, 0, wsb);
    d.W = (double*)ws;
    if (prec == 1) {
      char* pc = ws + bd::align_up(sizeof(double) * bd::kNB * bd::kNB, 256);
      d.P32[0] = (float*)pc;
      d.P32[1] = (float*)(pc + bd::p32_copy_bytes(n));
    }
    d.st = (bd::DevState*)calloc(1, sizeof(bd::DevState));
    d.xi = (double*)calloc((size_t)n, sizeof(double));  // the fused noise product
    d.y = (double*)calloc((size_t)n, sizeof(double));
    d.ypart = (double*)calloc(1, bd::noise_part_bytes(n));
    d.cB = 1.0;
    blocks.push_back(d.D);
    blocks.push_back(ws);
    blocks.push_back(d.st);
    blocks.push_back(d.xi);
    blocks.push_back(d.y);
    blocks.push_back(d.ypart);
  }
  std::stable_sort(cd.begin(), cd.end(),
                   [](const bd::ChainDesc& a, const bd::ChainDesc& b) { return a.n > b.n; });
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t aux = use_aux ? (hipStream_t)0x1 : nullptr;
  // recording pass, then the run from an exact-size copy of the tables
  bd::BatchTables tb;
  tb.record = true;
  hipError_t e = bd::launch_cholesky_batched(nullptr, aux, ev, cd.data(), cd.data(), count,
                                             (bd_precision_t)prec, panels, &tb, true);
  const long recorded = g_emu_launches;
  tb.record = false;
  int32_t* tdev = (int32_t*)malloc(sizeof(int32_t) * (tb.host.size() + 1));
  memcpy(tdev, tb.host.data(), sizeof(int32_t) * tb.host.size());
  tb.dev = tdev;
  if (e == hipSuccess)
    e = bd::launch_cholesky_batched(nullptr, aux, ev, cd.data(), cd.data(), count,
                                    (bd_precision_t)prec, panels, &tb, true);
  if (recorded != 0 || tb.cur != tb.host.size()) e = hipErrorInvalidValue;
  free(tdev);
  printf("chains=%d prec=%d lookahead=%d panels=%d: status %d, %ld launches\n", count, prec,
         use_aux, panels, e, g_emu_launches);
  for (void* p : blocks) free(p);
  return e != hipSuccess ? 1 : 0;
}
