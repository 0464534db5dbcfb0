// Runs the whole rigid-rod tension solve of constrain.hip (launch_constrain:
// then its adjoint, launch_constrain_adjoint;
// the host's batches of matrix-free products and controller passes) on the
// CPU through the stand-in HIP runtime, under AddressSanitizer, with every
// buffer at exactly the documented size.  Values are meaningless there (no
// barriers or cross-lane exchange), so the Newton-GMRES iteration runs to
// its caps and every index range of the workspace is exercised.
// Usage: constrain_emu n_beads newton_maxit skip_matvec(0|1) [one_launch(0|1)]
// one_launch = 1 runs the one-launch solve with a single workgroup (its grid
// barriers then never wait, so the sequential stand-in can run it).
#include "../../paper_2208_06559_amd/csrc/constrain.hip"
long g_emu_launches = 0;
namespace bd {
thread_local Profiler* g_prof = nullptr;
void prof_mark_begin(hipStream_t, const char*) {}
void prof_mark_end(hipStream_t) {}
}  // namespace bd
int main(int argc, char** argv) {
  if (argc != 4 && argc != 5) return 2;
  const int ncu = (argc == 5) ? atoi(argv[4]) : 0;
  const int N = atoi(argv[1]), maxit = atoi(argv[2]);
  if (atoi(argv[3])) g_emu_skip = (const void*)&bd::dmatvec_kernel;
  bd_params_t p;
  memset(&p, 0, sizeof(p));
  p.n_beads = N;
  p.b = 1.0;
  p.hstar = 0.25;
  p.a = 0.5;
  p.dt = 1e-4;
  p.newton_tol = 1e-13;
  p.newton_maxit = maxit;
  double* x = (double*)malloc(sizeof(double) * 3 * N);
  double* xs = (double*)malloc(sizeof(double) * 3 * N);
  double* T = (double*)malloc(sizeof(double) * (N - 1));
  for (int i = 0; i < N; ++i)
    for (int al = 0; al < 3; ++al) {
      x[3 * i + al] = (al == 0) ? (double)i : 0.01 * ((i * 7 + al * 3) % 5);
      xs[3 * i + al] = x[3 * i + al] + 1e-3 * ((i + al) % 3);
    }
  const size_t wsb = bd::constrain_workspace_bytes(N);
  void* ws = malloc(wsb);
  memset(ws, 0, wsb);
  bd::DevState* st = (bd::DevState*)calloc(1, sizeof(bd::DevState));
  bd::DevState* host = (bd::DevState*)calloc(1, sizeof(bd::DevState));
  int hint = 0;
  const hipError_t e = bd::launch_constrain(nullptr, p, x, xs, T, ws, st, host, &hint, ncu);
  printf("N=%d maxit=%d: status %d, %ld launches, done %d\n", N, maxit, e, g_emu_launches,
         host->done);
  // the adjoint solve on the same workspace: exact-size xbar and z
  double* xbar = (double*)malloc(sizeof(double) * 3 * N);
  double* z = (double*)malloc(sizeof(double) * 3 * N);
  for (int i = 0; i < 3 * N; ++i) xbar[i] = 1.0 + 0.1 * (i % 7);
  const hipError_t ea = bd::launch_constrain_adjoint(nullptr, p, x, xs, xbar, z, ws, st, host);
  printf("adjoint: status %d, %ld launches, done %d\n", ea, g_emu_launches, host->done);
  free(xbar);
  free(z);
  free(x);
  free(xs);
  free(T);
  free(ws);
  free(st);
  free(host);
  return e | ea;
}
