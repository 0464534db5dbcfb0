// Runs the batched tension solve of constrain.hip (launch_constrain_batched)
// on the CPU through the stand-in HIP runtime, under AddressSanitizer, with
// each chain's positions and workspace at exactly the documented sizes.
// Values are meaningless there (see constrain_emu.cpp); the iteration runs
// to its caps and every index range of every chain is exercised.
// Usage: constrain_batch_emu newton_maxit N_0 N_1 ...
#include <algorithm>
#include <vector>

#include "../../paper_2208_06559_amd/csrc/constrain.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const int maxit = atoi(argv[1]);
  const int count = argc - 2;
  std::vector<bd::ChainDesc> cd((size_t)count);
  std::vector<void*> blocks;
  bd::DevState* st = (bd::DevState*)calloc((size_t)count, sizeof(bd::DevState));
  bd::DevState* host = (bd::DevState*)calloc((size_t)count, sizeof(bd::DevState));
  int max_beads = 0;
  for (int c = 0; c < count; ++c) {
    const int N = atoi(argv[2 + c]);
    bd::ChainDesc& d = cd[(size_t)c];
    memset(&d, 0, sizeof(d));
    d.N = N;
    d.n = 3 * (int64_t)N;
    d.b = 1.0;
    d.hstar = 0.25;
    d.a = 0.5;
    d.dt = 1e-4;
    d.tol = 1e-13;
    d.maxit = maxit;
    d.index = c;
    d.x = (double*)malloc(sizeof(double) * 3 * N);
    d.xs = (double*)malloc(sizeof(double) * 3 * N);
    for (int i = 0; i < N; ++i)
      for (int al = 0; al < 3; ++al) {
        d.x[3 * i + al] = (al == 0) ? (double)i : 0.01 * ((i * 7 + al * 3) % 5);
        d.xs[3 * i + al] = d.x[3 * i + al] + 1e-3 * ((i + al) % 3);
      }
    const size_t wsb = bd::constrain_workspace_bytes(N);
    d.cons = malloc(wsb);
    memset(d.cons, 0, wsb);
    d.st = st + c;
    blocks.push_back(d.x);
    blocks.push_back(d.xs);
    blocks.push_back(d.cons);
    if (N > max_beads) max_beads = N;
  }
  std::stable_sort(cd.begin(), cd.end(),
                   [](const bd::ChainDesc& a, const bd::ChainDesc& b) { return a.n > b.n; });
  std::vector<int32_t> prefix((size_t)count + 1, 0);
  for (int c = 0; c < count; ++c)
    prefix[(size_t)c + 1] = prefix[(size_t)c] + bd::constrain_mv_blocks(cd[(size_t)c].N);
  int hint = 0;
  const hipError_t e = bd::launch_constrain_batched(nullptr, cd.data(), count, max_beads,
                                                    prefix.data(), prefix[(size_t)count], maxit,
                                                    st, host, &hint);
  int done = 0;
  for (int c = 0; c < count; ++c) done += host[c].done;
  printf("chains=%d maxit=%d: status %d, %ld launches, done %d\n", count, maxit, e,
         g_emu_launches, done);
  for (void* p : blocks) free(p);
  free(st);
  free(host);
  return e != hipSuccess ? 1 : 0;
}
