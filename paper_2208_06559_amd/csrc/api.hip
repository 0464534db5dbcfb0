// C ABI of libbdrpy: handle, argument checks, workspace carving and the
// per-step orchestration (assemble -> Cholesky -> noise -> predictor ->
// constraint), all on the handle's stream.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace bd {
int constrain_max_beads();
int constrain_batched_max_beads();
int fraenkel_max_beads();
Profiler* profiler_new();
void profiler_delete(Profiler* p);
int profiler_collect(Profiler* p, hipStream_t s, bd_kernel_stat_t* out, int max_out);
}  // namespace bd

struct bd_handle_s {
  int device;
  hipStream_t stream;
  bd::DevState* st;    // device
  bd::DevState* host;  // pinned host mirror
  bd::Profiler* prof;  // per-kernel timing, or null
  int prof_on;
  int pairs_hint;      // D products the last tension solve needed
  hipStream_t aux;     // lookahead stream of the Cholesky (default priority)
  hipEvent_t ev[4];    // fork / panel-ready / rest-done / next-columns-done events
  int step_panels;     // most Cholesky panels applied per pass over the trailing matrix
  int64_t wide_rows;   // steps of more than two panels while more rows than this remain
  bool tile_potrf;     // Cholesky diagonal blocks on matrix cores
  void* scratch;       // this device's fixed scratch array (bd_brownian_noalloc)
  int ps_cu;           // workgroups of the one-launch tension solve (0: host-polled launches)
  std::vector<bd_schedule_t> sched;  // tuned factorisation schedules (bd_set_schedules)
  int ens_panels[2];   // ensembles' panels per factorisation step, by precision (0: default)
};

namespace {
// The factorisation schedule of a call of matrix order n: the first tuned
// row that covers (n, prec), else the handle's defaults.
void schedule_for(const bd_handle_s* h, int64_t n, bd_precision_t prec, int& panels,
                  int64_t& wide) {
  for (const bd_schedule_t& r : h->sched)
    if (r.prec == (int32_t)prec && n <= r.n_max) {
      panels = r.step_panels;
      wide = r.wide_rows;
      return;
    }
  panels = h->step_panels;
  wide = h->wide_rows;
}
}  // namespace

namespace {

using bd::DevState;

bool params_ok(const bd_params_t* p) {
  if (!p) return false;
  if (p->n_beads < 2) return false;
  if (!(p->b > 0.0) || !isfinite(p->b)) return false;
  if (!(p->a > 0.0) || !isfinite(p->a)) return false;
  if (!(p->dt > 0.0) || !isfinite(p->dt)) return false;
  if (!(p->hstar >= 0.0) || !(p->hstar <= p->a)) return false;
  if (p->noise != BD_NOISE_GAUSSIAN && p->noise != BD_NOISE_UNIFORM_PAPER) return false;
  if (!(p->newton_tol > 0.0) || !isfinite(p->newton_tol)) return false;
  if (p->newton_maxit < 1) return false;
  if (p->reserved != 0) return false;
  for (int e = 0; e < 9; ++e)
    if (!isfinite(p->kappa[e])) return false;
  return true;
}

bool prec_ok(bd_precision_t prec) { return prec == BD_PREC_FP64 || prec == BD_PREC_MIXED; }

// Leading dimension of the internal D in bd_step: a multiple of 64 doubles.
int64_t step_ld(int64_t n) { return (n + 63) / 64 * 64; }

struct StepLayout {
  size_t d, chol, brown, cons, y, xs, total;
};

// The partial sums follow xi in the noise region.
double* step_ypart(char* base, const StepLayout& L, int64_t n) {
  return reinterpret_cast<double*>(base + L.brown + bd::align_up(sizeof(double) * (size_t)n, 256));
}

// batched: the layout of one chain of an ensemble
StepLayout step_layout(int64_t n, bd_precision_t prec, bool batched = false) {
  StepLayout L;
  size_t off = 0;
  L.d = off;
  off += bd::align_up(sizeof(double) * (size_t)step_ld(n) * (size_t)n, 256);
  L.chol = off;
  off += bd::align_up(batched ? bd::cholesky_batched_workspace_bytes(n, prec)
                              : bd::cholesky_workspace_bytes(n, prec),
                      256);
  // the noise xi, then the factorisation's partial sums of c_B L xi
  L.brown = off;
  off += bd::align_up(sizeof(double) * (size_t)n, 256) + bd::noise_part_bytes(n);
  L.cons = off;
  off += bd::align_up(bd::constrain_workspace_bytes(n / 3), 256);
  L.y = off;
  off += bd::align_up(sizeof(double) * n, 256);
  L.xs = off;
  off += bd::align_up(sizeof(double) * n, 256);
  L.total = off;
  return L;
}

// Workspace of bd_step_adjoint: the forward step's own layout (its D
// holds B after the factorisation, its x* the new positions), then Lbar,
// Dbar, the Cholesky adjoint's scratch, and vectors of n: z, xi, T, f,
// D z, the assembly adjoint's gradient, its h* partial sums (N) and h*.
struct StepAdjointLayout {
  size_t fwd, lbar, dbar, cadj, z, xi, T, f, dz, xbd, hpart, hstep, total;
};

StepAdjointLayout step_adjoint_layout(int64_t n) {
  StepAdjointLayout L;
  const size_t mat = bd::align_up(sizeof(double) * (size_t)step_ld(n) * (size_t)n, 256);
  const size_t vec = bd::align_up(sizeof(double) * (size_t)n, 256);
  size_t off = 0;
  L.fwd = off;
  off += step_layout(n, BD_PREC_FP64).total;
  L.lbar = off;
  off += mat;
  L.dbar = off;
  off += mat;
  L.cadj = off;
  off += bd::align_up(bd::cholesky_adjoint_workspace_bytes(n), 256);
  size_t* v[] = {&L.z, &L.xi, &L.T, &L.f, &L.dz, &L.xbd, &L.hpart, &L.hstep};
  for (size_t* p : v) {
    *p = off;
    off += vec;
  }
  L.total = off;
  return L;
}

__global__ void reset_state_kernel(DevState* st) {
  st->status = BD_OK;
  st->newton_iters = 0;
  st->potrf_info = 0;
  st->max_rod_err = 0.0;
  st->last_newton_res = 0.0;
  st->krylov_iters = 0;
  st->done = 0;
}

// x <- xs unless the step failed (non-positive pivot or no converged
// tensions: positions stay at x^t then).
__global__ void commit_positions_kernel(double* x, const double* xs, int64_t n,
                                        const DevState* st) {
  if (st->status != BD_OK) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = xs[e];
}

// Ensembles: every chain's state (count of them, thread c), and the commit
// of chain blockIdx.z of the table.
__global__ void reset_states_kernel(DevState* st, int count) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < count) {
    st[c].status = BD_OK;
    st[c].newton_iters = 0;
    st[c].potrf_info = 0;
    st[c].max_rod_err = 0.0;
    st[c].last_newton_res = 0.0;
    st[c].krylov_iters = 0;
    st[c].done = 0;
  }
}

// *d = v, or *d += 1 (advance): the device noise counter of a captured
// ensemble step.
__global__ void set_step_kernel(int64_t* d, int64_t v, int advance) {
  if (advance) *d += 1;
  else *d = v;
}

__global__ void commit_positions_batched_kernel(const bd::ChainDesc* cd) {
  const bd::ChainDesc& c = cd[blockIdx.z];
  if (c.st->status != BD_OK) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < c.n) c.x[e] = c.xs[e];
}

bd_status_t hip_status(hipError_t e) { return e == hipSuccess ? BD_OK : BD_ERR_HIP; }

// Makes the handle's device current and its profiler (if on) active for the
// calling thread until the end of the call.
struct CallScope {
  explicit CallScope(bd_handle_t h) { bd::g_prof = (h && h->prof_on) ? h->prof : nullptr; }
  ~CallScope() { bd::g_prof = nullptr; }
};

bd_status_t enter(bd_handle_t h) {
  if (!h) return BD_ERR_PARAM;
  return hip_status(hipSetDevice(h->device));
}

hipError_t launch_cholesky_tuned(bd_handle_t h, hipStream_t s, int64_t n, double* A, int64_t ld,
                                 bd_precision_t prec, void* ws, const double* xi = nullptr,
                                 double* y = nullptr, double cB = 0.0, double* ypart = nullptr) {
  int sp;
  int64_t wr;
  schedule_for(h, n, prec, sp, wr);
  return bd::launch_cholesky(s, h->aux, h->ev, n, A, ld, prec, ws, h->st, sp, wr, h->tile_potrf,
                             xi, y, cB, ypart);
}

hipError_t reset(bd_handle_t h) {
  BD_LAUNCH("reset_state", reset_state_kernel, dim3(1), dim3(1), 0, h->stream, h->st);
  return hipGetLastError();
}

}  // namespace

struct bd_ensemble_s {
  bd_handle_t h;
  int count;
  bd_precision_t prec;
  int max_beads;
  int newton_maxit;                  // largest over the chains
  bd::ChainDesc* cd;                 // device table, decreasing n
  std::vector<bd::ChainDesc> host;   // its host copy
  DevState* st;                      // device, one per chain in the caller's order
  DevState* host_st;                 // pinned mirror
  int pairs_hint;
  int step_panels;                   // Cholesky panels per step (2 or 4)
  int32_t* mv_prefix;                // device: flattened grids (matrix-free product,
  int32_t* rpy_prefix;               // assembly)
  int mv_blocks, rpy_blocks;
  bd::BatchTables tb;                // flattened grids of the factorisation
  int32_t* tb_dev;                   // device copy of tb.host
  // a captured step (bd_ensemble_capture): its executable graph, the stream
  // it was captured on, the device noise counter it reads and advances, and
  // the counter the host expects there
  hipGraphExec_t gexec;
  hipStream_t cap;
  int64_t* d_step;
  int64_t next_step;
  int budget;
};

extern "C" {

// Releases whatever a (possibly partially built) handle holds.
static void release(bd_handle_s* h) {
  if (h->aux) (void)hipStreamSynchronize(h->aux);
  for (int i = 0; i < 4; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->st) (void)hipFree(h->st);
  if (h->host) (void)hipHostFree(h->host);
  if (h->prof) bd::profiler_delete(h->prof);
  delete h;
}

bd_status_t bd_create(bd_handle_t* out, int device, void* hip_stream) {
  if (!out) return BD_ERR_PARAM;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return BD_ERR_HIP;
  if (device < 0 || device >= count) return BD_ERR_PARAM;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BD_ERR_HIP;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BD_ERR_UNSUPPORTED;
  if (hipSetDevice(device) != hipSuccess) return BD_ERR_HIP;
  bd_handle_s* h = new (std::nothrow) bd_handle_s;
  if (!h) return BD_ERR_ALLOC;
  h->device = device;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->st = nullptr;
  h->host = nullptr;
  h->prof = nullptr;
  h->prof_on = 0;
  h->pairs_hint = 0;
  h->aux = nullptr;
  h->ev[0] = h->ev[1] = h->ev[2] = h->ev[3] = nullptr;
  h->scratch = nullptr;
  h->ens_panels[0] = h->ens_panels[1] = 0;
  // The tension solve alternates launches of the product with D and the
  // controller, polled by the host; BDRPY_CONSTRAIN=onelaunch runs it as one
  // launch of at most one workgroup per compute unit instead (no host round
  // trip, so that a step can be captured in a HIP graph; slower).
  const char* cm = getenv("BDRPY_CONSTRAIN");
  h->ps_cu = (cm && cm[0] == 'o') ? prop.multiProcessorCount : 0;
  // BDRPY_STEP_PANELS=1 or 2 caps the panels per trailing pass (for
  // comparisons).  By default four panels share each pass while the
  // trailing matrix is large (more than BDRPY_WIDE_ROWS rows, default 4096),
  // halving its HBM traffic per flop, and two once the lookahead chain of
  // diagonal factors and panel solves is the longer path.
  const char* sp = getenv("BDRPY_STEP_PANELS");
  h->step_panels = (sp && sp[0] == '1') ? 1 : (sp && sp[0] == '2') ? 2 : 4;
  const char* wr = getenv("BDRPY_WIDE_ROWS");
  h->wide_rows = wr ? atoll(wr) : 4096;
  // BDRPY_POTRF=reg factors the diagonal blocks with the register-tiled
  // kernel (for comparisons); by default they run on matrix cores.
  const char* pt = getenv("BDRPY_POTRF");
  h->tile_potrf = !(pt && pt[0] == 'r');
  // the device address of this device's scratch array, looked up once per
  // device with the device current
  if (bd::brownian_scratch_init(device, &h->scratch) != hipSuccess) {
    release(h);
    return BD_ERR_HIP;
  }
  if (hipMalloc(&h->st, sizeof(DevState)) != hipSuccess ||
      hipHostMalloc(&h->host, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
    release(h);
    return BD_ERR_ALLOC;
  }
  // BDRPY_LOOKAHEAD=0 runs the factorisation on the caller's stream only
  // (for comparisons); by default the lookahead stream is used.
  const char* la = getenv("BDRPY_LOOKAHEAD");
  const bool lookahead = !(la && la[0] == '0');
  bool ok = !lookahead || hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < 4 && ok && lookahead; ++i)
    ok = hipEventCreateWithFlags(&h->ev[i], hipEventDisableTiming) == hipSuccess;
  memset(h->host, 0, sizeof(DevState));
  if (ok) ok = hipMemcpy(h->st, h->host, sizeof(DevState), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    release(h);
    return BD_ERR_HIP;
  }
  *out = h;
  return BD_OK;
}

bd_status_t bd_destroy(bd_handle_t h) {
  if (!h) return BD_ERR_PARAM;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  release(h);
  return BD_OK;
}

bd_status_t bd_set_stream(bd_handle_t h, void* hip_stream) {
  if (!h) return BD_ERR_PARAM;
  h->stream = static_cast<hipStream_t>(hip_stream);
  return BD_OK;
}

bd_status_t bd_set_schedules(bd_handle_t h, const bd_schedule_t* rows, int32_t count) {
  if (!h || count < 0 || (count > 0 && !rows)) return BD_ERR_PARAM;
  for (int32_t i = 0; i < count; ++i) {
    const bd_schedule_t& r = rows[i];
    if (!prec_ok((bd_precision_t)r.prec) || r.n_max < 1 || r.wide_rows < 0 ||
        (r.step_panels != 1 && r.step_panels != 2 && r.step_panels != 4))
      return BD_ERR_PARAM;
  }
  try {
    h->sched.assign(rows, rows + count);
  } catch (...) {
    return BD_ERR_ALLOC;
  }
  return BD_OK;
}

bd_status_t bd_set_ensemble_panels(bd_handle_t h, bd_precision_t prec, int32_t panels) {
  if (!h || !prec_ok(prec) || (panels != 0 && panels != 2 && panels != 4)) return BD_ERR_PARAM;
  h->ens_panels[prec == BD_PREC_MIXED ? 1 : 0] = panels;
  return BD_OK;
}

bd_status_t bd_workspace_size(bd_op_t op, int64_t n, bd_precision_t prec, size_t* bytes) {
  if (!bytes || n < 1 || !prec_ok(prec)) return BD_ERR_PARAM;
  switch (op) {
    case BD_OP_CHOLESKY:
      *bytes = bd::cholesky_workspace_bytes(n, prec);
      return BD_OK;
    case BD_OP_BROWNIAN:
      if (n % 3) return BD_ERR_PARAM;
      *bytes = bd::brownian_workspace_bytes(n);
      return BD_OK;
    case BD_OP_CONSTRAIN:
      if (n % 3 || n < 6) return BD_ERR_PARAM;
      *bytes = bd::constrain_workspace_bytes(n / 3);
      return BD_OK;
    case BD_OP_STEP:
      if (n % 3 || n < 6) return BD_ERR_PARAM;
      *bytes = step_layout(n, prec).total;
      return BD_OK;
    case BD_OP_CHOLESKY_ADJOINT:
      *bytes = bd::cholesky_adjoint_workspace_bytes(n);
      return BD_OK;
    case BD_OP_STEP_ADJOINT:
      if (n % 3 || n < 6) return BD_ERR_PARAM;
      *bytes = step_adjoint_layout(n).total;
      return BD_OK;
  }
  return BD_ERR_PARAM;
}

bd_status_t bd_rpy_assemble(bd_handle_t h, const bd_params_t* p, const double* d_x, double* d_D,
                            int64_t ld, bd_fill_t fill) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x || !d_D) return BD_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  if (ld < n || (fill != BD_FILL_LOWER && fill != BD_FILL_FULL)) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_rpy_assemble(h->stream, *p, d_x, d_D, ld, fill));
}

bd_status_t bd_cholesky(bd_handle_t h, int64_t n, double* d_A, int64_t ld, bd_precision_t prec,
                        void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (n < 1 || !d_A || ld < n || !prec_ok(prec) || !d_ws) return BD_ERR_PARAM;
  if (ws_bytes < bd::cholesky_workspace_bytes(n, prec)) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  int sp;
  int64_t wr;
  schedule_for(h, n, prec, sp, wr);
  return hip_status(bd::launch_cholesky(h->stream, h->aux, h->ev, n, d_A, ld, prec, d_ws, h->st,
                                        sp, wr, h->tile_potrf));
}

bd_status_t bd_cholesky_adjoint(bd_handle_t h, int64_t n, const double* d_L, int64_t ld,
                                const double* d_Lbar, int64_t ldb, double* d_Abar, int64_t lda,
                                void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (n < 1 || n > 65535 || !d_L || !d_Lbar || !d_Abar || !d_ws) return BD_ERR_PARAM;
  if (ld < n || ldb < n || lda < n) return BD_ERR_PARAM;
  if (ws_bytes < bd::cholesky_adjoint_workspace_bytes(n)) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_cholesky_adjoint(h->stream, n, d_L, ld, 0, d_Lbar, ldb, 0, d_Abar,
                                                lda, 0, 1.0, 0.0, 1, d_ws));
}

bd_status_t bd_brownian(bd_handle_t h, const bd_params_t* p, int64_t step, const double* d_L,
                        int64_t ld, double* d_y, double* d_xi_out, void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_L || !d_y || !d_ws) return BD_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  if (ld < n || ws_bytes < bd::brownian_workspace_bytes(n)) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_brownian(h->stream, *p, step, d_L, ld, d_y, d_xi_out, d_ws));
}

bd_status_t bd_brownian_noalloc(bd_handle_t h, const bd_params_t* p, int64_t step,
                                const double* d_L, int64_t ld, double* d_y, double* d_xi_out) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_L || !d_y) return BD_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  if (ld < n) return BD_ERR_PARAM;
  if (n > bd::brownian_scratch_max_n()) return BD_ERR_UNSUPPORTED;
  if (!h->scratch) return BD_ERR_HIP;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  // the same kernels as bd_brownian, their workspace the fixed array
  return hip_status(bd::launch_brownian(h->stream, *p, step, d_L, ld, d_y, d_xi_out, h->scratch));
}

bd_status_t bd_constrain(bd_handle_t h, const bd_params_t* p, const double* d_x_old,
                         double* d_x_pred_inout, double* d_T_out, void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x_old || !d_x_pred_inout || !d_ws) return BD_ERR_PARAM;
  if (p->n_beads > bd::constrain_max_beads()) return BD_ERR_UNSUPPORTED;
  if (ws_bytes < bd::constrain_workspace_bytes(p->n_beads)) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_constrain(h->stream, *p, d_x_old, d_x_pred_inout, d_T_out, d_ws,
                                         h->st, h->host, &h->pairs_hint, h->ps_cu));
}

bd_status_t bd_step(bd_handle_t h, const bd_params_t* p, int64_t step, double* d_x,
                    bd_precision_t prec, void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x || !d_ws || !prec_ok(prec)) return BD_ERR_PARAM;
  if (p->n_beads > bd::constrain_max_beads()) return BD_ERR_UNSUPPORTED;
  const int64_t n = 3 * (int64_t)p->n_beads;
  const StepLayout L = step_layout(n, prec);
  if (ws_bytes < L.total) return BD_ERR_PARAM;
  char* base = static_cast<char*>(d_ws);
  double* D = reinterpret_cast<double*>(base + L.d);
  double* y = reinterpret_cast<double*>(base + L.y);
  double* xs = reinterpret_cast<double*>(base + L.xs);
  const int64_t ld = step_ld(n);
  hipStream_t s = h->stream;
  hipError_t he = reset(h);
  // the noise first: the factorisation call ends with y = c_B L xi
  double* xi = reinterpret_cast<double*>(base + L.brown);
  if (he == hipSuccess) he = bd::launch_rpy_assemble(s, *p, d_x, D, ld, BD_FILL_LOWER);
  if (he == hipSuccess) he = bd::launch_noise(s, *p, step, xi);
  if (he == hipSuccess)
    he = launch_cholesky_tuned(h, s, n, D, ld, prec, base + L.chol, xi, y, bd::noise_coeff(*p),
                               step_ypart(base, L, n));
  if (he == hipSuccess) he = bd::launch_predictor(s, *p, d_x, y, xs);
  if (he == hipSuccess)
    he = bd::launch_constrain(s, *p, d_x, xs, nullptr, base + L.cons, h->st, h->host,
                               &h->pairs_hint, h->ps_cu);
  if (he == hipSuccess) {
    BD_LAUNCH("commit_positions", commit_positions_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, d_x, xs, n, h->st);
    he = hipGetLastError();
  }
  return hip_status(he);
}

bd_status_t bd_constrain_adjoint(bd_handle_t h, const bd_params_t* p, const double* d_x_old,
                                 const double* d_x_new, const double* d_xbar, double* d_z,
                                 void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x_old || !d_x_new || !d_xbar || !d_z || !d_ws) return BD_ERR_PARAM;
  if (p->n_beads > bd::constrain_max_beads()) return BD_ERR_UNSUPPORTED;
  if (ws_bytes < bd::constrain_workspace_bytes(p->n_beads)) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_constrain_adjoint(h->stream, *p, d_x_old, d_x_new, d_xbar, d_z,
                                                 d_ws, h->st, h->host));
}

bd_status_t bd_step_adjoint(bd_handle_t h, const bd_params_t* p, int64_t step, const double* d_x,
                            double* d_xbar, double* d_hbar, double* d_kbar, void* d_ws,
                            size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x || !d_xbar || !d_hbar || !d_kbar || !d_ws) return BD_ERR_PARAM;
  if (p->n_beads > bd::constrain_max_beads()) return BD_ERR_UNSUPPORTED;
  const int64_t n = 3 * (int64_t)p->n_beads;
  const StepAdjointLayout A = step_adjoint_layout(n);
  if (ws_bytes < A.total) return BD_ERR_PARAM;
  const StepLayout L = step_layout(n, BD_PREC_FP64);
  char* base = static_cast<char*>(d_ws);
  char* fwd = base + A.fwd;
  double* D = reinterpret_cast<double*>(fwd + L.d);
  double* y = reinterpret_cast<double*>(fwd + L.y);
  double* xs = reinterpret_cast<double*>(fwd + L.xs);
  auto vec = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  double *Lbar = vec(A.lbar), *Dbar = vec(A.dbar), *z = vec(A.z), *xi = vec(A.xi), *T = vec(A.T);
  double *f = vec(A.f), *Dz = vec(A.dz), *xbD = vec(A.xbd), *hpart = vec(A.hpart);
  double* hstep = vec(A.hstep);
  const int64_t ld = step_ld(n);
  hipStream_t s = h->stream;
  // the forward step from x, recomputed (FP64): D, B, xi and y, x*, the
  // tensions T and x^{t+dt} (in xs)
  hipError_t he = reset(h);
  if (he == hipSuccess) he = bd::launch_rpy_assemble(s, *p, d_x, D, ld, BD_FILL_LOWER);
  if (he == hipSuccess) he = bd::launch_noise(s, *p, step, xi);
  if (he == hipSuccess)
    he = launch_cholesky_tuned(h, s, n, D, ld, BD_PREC_FP64, fwd + L.chol, xi, y,
                               bd::noise_coeff(*p), step_ypart(fwd, L, n));
  if (he == hipSuccess) he = bd::launch_predictor(s, *p, d_x, y, xs);
  if (he == hipSuccess)
    he = bd::launch_constrain(s, *p, d_x, xs, T, fwd + L.cons, h->st, h->host, &h->pairs_hint,
                              h->ps_cu);
  // the tensions' adjoint: z, the gradient in x^{t+dt} at fixed T
  if (he == hipSuccess)
    he = bd::launch_constrain_adjoint(s, *p, d_x, xs, d_xbar, z, fwd + L.cons, h->st, h->host);
  // x^{t+dt} = x* + dt D(x) f(T, u(x)): Dbar = dt z f^T, the gradient
  // through u and through x* = x + dt kappa x + y (xbar overwritten)
  if (he == hipSuccess) he = bd::launch_rod_forces(s, d_x, T, p->n_beads, f);
  if (he == hipSuccess) he = bd::launch_rank1(s, z, f, p->dt, n, Dbar, ld);
  if (he == hipSuccess) he = bd::launch_dmatvec(s, *p, d_x, z, Dz, nullptr);
  if (he == hipSuccess)
    he = bd::launch_step_adjoint_local(s, *p, d_x, T, z, Dz, d_xbar, d_kbar);
  // y = c_B B xi: Lbar, then the factorisation's adjoint added into Dbar
  if (he == hipSuccess) he = bd::launch_brownian_adjoint_lbar(s, *p, xi, z, Lbar, ld);
  if (he == hipSuccess)
    he = bd::launch_cholesky_adjoint(s, n, D, ld, 0, Lbar, ld, 0, Dbar, ld, 0, 1.0, 1.0, 1,
                                     base + A.cadj);
  // D(x, h*): the assembly's adjoint, then the sums
  if (he == hipSuccess)
    he = bd::launch_rpy_adjoint(s, *p, d_x, Dbar, ld, xbD, hstep, hpart, h->st);
  if (he == hipSuccess) he = bd::launch_step_adjoint_finish(s, n, xbD, hstep, d_xbar, d_hbar);
  return hip_status(he);
}

bd_status_t bd_step_fraenkel(bd_handle_t h, const bd_params_t* p, double k_spring, int64_t step,
                             double* d_x, bd_precision_t prec, void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x || !d_ws || !prec_ok(prec)) return BD_ERR_PARAM;
  if (!(k_spring > 0.0) || !isfinite(k_spring)) return BD_ERR_PARAM;
  if (p->n_beads > bd::fraenkel_max_beads()) return BD_ERR_UNSUPPORTED;
  const int64_t n = 3 * (int64_t)p->n_beads;
  const StepLayout L = step_layout(n, prec);
  if (ws_bytes < L.total) return BD_ERR_PARAM;
  char* base = static_cast<char*>(d_ws);
  double* D = reinterpret_cast<double*>(base + L.d);
  double* y = reinterpret_cast<double*>(base + L.y);
  // bead forces and D f in the tension solve's region
  double* f = reinterpret_cast<double*>(base + L.cons);
  double* v = reinterpret_cast<double*>(base + L.cons + bd::align_up(sizeof(double) * n, 256));
  const int64_t ld = step_ld(n);
  hipStream_t s = h->stream;
  hipError_t he = reset(h);
  double* xi = reinterpret_cast<double*>(base + L.brown);
  if (he == hipSuccess) he = bd::launch_rpy_assemble(s, *p, d_x, D, ld, BD_FILL_LOWER);
  if (he == hipSuccess) he = bd::launch_noise(s, *p, step, xi);
  if (he == hipSuccess)
    he = launch_cholesky_tuned(h, s, n, D, ld, prec, base + L.chol, xi, y, bd::noise_coeff(*p),
                               step_ypart(base, L, n));
  if (he == hipSuccess) he = bd::launch_spring_forces(s, d_x, p->n_beads, k_spring, p->b, f);
  if (he == hipSuccess) he = bd::launch_dmatvec(s, *p, d_x, f, v, h->st);
  if (he == hipSuccess) he = bd::launch_fraenkel_update(s, *p, k_spring, d_x, v, y, h->st);
  return hip_status(he);
}

bd_status_t bd_rpy_assemble_adjoint(bd_handle_t h, const bd_params_t* p, const double* d_x,
                                    const double* d_Dbar, int64_t ld, double* d_xbar,
                                    double* d_hbar, void* d_ws, size_t ws_bytes) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_x || !d_Dbar || !d_xbar || !d_hbar || !d_ws) return BD_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  if (ld < n || ws_bytes < sizeof(double) * (size_t)p->n_beads) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_rpy_adjoint(h->stream, *p, d_x, d_Dbar, ld, d_xbar, d_hbar,
                                           static_cast<double*>(d_ws), h->st));
}

bd_status_t bd_brownian_adjoint(bd_handle_t h, const bd_params_t* p, const double* d_L,
                                int64_t ld, const double* d_xi, const double* d_ybar,
                                double* d_Lbar, int64_t ldb, double* d_xibar) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!params_ok(p) || !d_L || !d_xi || !d_ybar || !d_Lbar || !d_xibar) return BD_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  if (ld < n || ldb < n || n > 65535) return n > 65535 ? BD_ERR_UNSUPPORTED : BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(
      bd::launch_brownian_adjoint(h->stream, *p, d_L, ld, d_xi, d_ybar, d_Lbar, ldb, d_xibar));
}

bd_status_t bd_observables(bd_handle_t h, int32_t n_chains, const double* d_x,
                           const int64_t* d_offsets, double* d_out) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (n_chains < 1 || n_chains > 2147483647 || !d_x || !d_offsets || !d_out) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_observables(h->stream, n_chains, d_x, d_offsets, d_out));
}

bd_status_t bd_stress(bd_handle_t h, int32_t n_chains, const double* d_x,
                      const int64_t* d_offsets, const double* d_T, double k_spring, double b,
                      double* d_out) {
  CallScope scope(h);
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (n_chains < 1 || !d_x || !d_offsets || !d_out) return BD_ERR_PARAM;
  if (!(b > 0.0) || !isfinite(b)) return BD_ERR_PARAM;
  if (!d_T && (!(k_spring > 0.0) || !isfinite(k_spring))) return BD_ERR_PARAM;
  if (reset(h) != hipSuccess) return BD_ERR_HIP;
  return hip_status(bd::launch_stress(h->stream, n_chains, d_x, d_offsets, d_T, k_spring, b,
                                      d_out));
}

bd_status_t bd_get_info(bd_handle_t h, bd_info_t* out) {
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!out) return BD_ERR_PARAM;
  if (hipMemcpyAsync(h->host, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream) !=
      hipSuccess)
    return BD_ERR_HIP;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return BD_ERR_HIP;
  memcpy(out, h->host, sizeof(bd_info_t));
  return BD_OK;
}

bd_status_t bd_profile_begin(bd_handle_t h) {
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!h->prof) h->prof = bd::profiler_new();
  if (!h->prof) return BD_ERR_ALLOC;
  h->prof_on = 1;
  return BD_OK;
}

bd_status_t bd_profile_end(bd_handle_t h, bd_kernel_stat_t* out, int32_t max_out, int32_t* n_out) {
  bd_status_t e = enter(h);
  if (e != BD_OK) return e;
  if (!h->prof || max_out < 0) return BD_ERR_PARAM;
  const int n = bd::profiler_collect(h->prof, h->stream, out, max_out);
  if (n_out) *n_out = n;
  h->prof_on = 0;
  return BD_OK;
}

// ---------------------------------------------------------------- ensembles

static bool ensemble_args_ok(int32_t n_chains, const bd_params_t* p) {
  if (n_chains < 1 || n_chains > 65535 || !p) return false;
  for (int32_t c = 0; c < n_chains; ++c)
    if (!params_ok(&p[c])) return false;
  return true;
}

static bool ensemble_sizes_ok(int32_t n_chains, const bd_params_t* p) {
  for (int32_t c = 0; c < n_chains; ++c)
    if (p[c].n_beads > bd::constrain_batched_max_beads()) return false;
  return true;
}

bd_status_t bd_ensemble_workspace_size(int32_t n_chains, const bd_params_t* p,
                                       bd_precision_t prec, size_t* bytes) {
  if (!bytes || !prec_ok(prec) || !ensemble_args_ok(n_chains, p)) return BD_ERR_PARAM;
  if (!ensemble_sizes_ok(n_chains, p)) return BD_ERR_UNSUPPORTED;
  size_t total = 0;
  for (int32_t c = 0; c < n_chains; ++c) total += step_layout(3 * (int64_t)p[c].n_beads, prec, true).total;
  *bytes = total;
  return BD_OK;
}

static void ensemble_release(bd_ensemble_s* e) {
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  if (e->cap) (void)hipStreamDestroy(e->cap);
  if (e->d_step) (void)hipFree(e->d_step);
  if (e->cd) (void)hipFree(e->cd);
  if (e->mv_prefix) (void)hipFree(e->mv_prefix);
  if (e->rpy_prefix) (void)hipFree(e->rpy_prefix);
  if (e->tb_dev) (void)hipFree(e->tb_dev);
  if (e->st) (void)hipFree(e->st);
  if (e->host_st) (void)hipHostFree(e->host_st);
  delete e;
}

// Releases a partly built ensemble unless disarmed (every error path, and
// a host allocation failure thrown from inside).
struct EnsembleGuard {
  bd_ensemble_s* e;
  ~EnsembleGuard() {
    if (e) ensemble_release(e);
  }
};

static bd_status_t ensemble_create_impl(bd_handle_t h, int32_t n_chains, const bd_params_t* p,
                                        bd_precision_t prec, double* d_x, void* d_ws,
                                        size_t ws_bytes, bd_ensemble_t* out) {
  if (!out) return BD_ERR_PARAM;
  *out = nullptr;
  bd_status_t err = enter(h);
  if (err != BD_OK) return err;
  if (!d_x || !d_ws || !prec_ok(prec) || !ensemble_args_ok(n_chains, p)) return BD_ERR_PARAM;
  if (!ensemble_sizes_ok(n_chains, p)) return BD_ERR_UNSUPPORTED;
  size_t need = 0;
  if (bd_ensemble_workspace_size(n_chains, p, prec, &need) != BD_OK || ws_bytes < need)
    return BD_ERR_PARAM;
  bd_ensemble_s* e = new (std::nothrow) bd_ensemble_s;
  if (!e) return BD_ERR_ALLOC;
  EnsembleGuard guard{e};
  e->h = h;
  e->count = n_chains;
  e->prec = prec;
  e->max_beads = 0;
  e->newton_maxit = 1;
  e->cd = nullptr;
  e->st = nullptr;
  e->host_st = nullptr;
  e->pairs_hint = 0;
  e->mv_prefix = e->rpy_prefix = nullptr;
  e->mv_blocks = e->rpy_blocks = 0;
  e->tb_dev = nullptr;
  e->gexec = nullptr;
  e->cap = nullptr;
  e->d_step = nullptr;
  e->next_step = -1;
  e->budget = 0;
  // BDRPY_ENS_PANELS=2 takes two-panel factorisation steps (for
  // comparisons); by default four: with many chains sharing each launch the
  // trailing updates, not the chain of diagonal blocks, bound the time.
  const char* ep = getenv("BDRPY_ENS_PANELS");
  e->step_panels = (ep && ep[0] == '2') ? 2 : 4;
  if (h->ens_panels[prec == BD_PREC_MIXED ? 1 : 0] > 0)  // tuned (bd_set_ensemble_panels)
    e->step_panels = h->ens_panels[prec == BD_PREC_MIXED ? 1 : 0];
  if (hipMalloc(&e->cd, sizeof(bd::ChainDesc) * (size_t)n_chains) != hipSuccess ||
      hipMalloc(&e->st, sizeof(DevState) * (size_t)n_chains) != hipSuccess ||
      hipHostMalloc(&e->host_st, sizeof(DevState) * (size_t)n_chains, hipHostMallocDefault) !=
          hipSuccess ||
      hipMalloc(&e->mv_prefix, sizeof(int32_t) * ((size_t)n_chains + 1)) != hipSuccess ||
      hipMalloc(&e->rpy_prefix, sizeof(int32_t) * ((size_t)n_chains + 1)) != hipSuccess) {
    return BD_ERR_ALLOC;
  }
  e->host.resize((size_t)n_chains);
  char* base = static_cast<char*>(d_ws);
  int64_t xoff = 0;
  for (int32_t c = 0; c < n_chains; ++c) {
    const bd_params_t& q = p[c];
    const int64_t n = 3 * (int64_t)q.n_beads;
    const StepLayout L = step_layout(n, prec, true);
    bd::ChainDesc& d = e->host[(size_t)c];
    memset(&d, 0, sizeof(d));
    d.N = q.n_beads;
    d.uniform = (q.noise == BD_NOISE_UNIFORM_PAPER) ? 1 : 0;
    d.n = n;
    d.ld = step_ld(n);
    d.hstar = q.hstar;
    d.a = q.a;
    d.b = q.b;
    d.dt = q.dt;
    d.tol = q.newton_tol;
    d.cB = d.uniform ? sqrt(6.0 * q.dt) : sqrt(2.0 * q.dt);
    d.maxit = q.newton_maxit;
    d.index = c;
    for (int k = 0; k < 9; ++k) d.kappa[k] = q.kappa[k];
    d.seed = q.seed;
    d.chain_id = q.chain_id;
    d.x = d_x + xoff;
    d.D = reinterpret_cast<double*>(base + L.d);
    d.W = reinterpret_cast<double*>(base + L.chol);
    if (prec == BD_PREC_MIXED) {
      char* pc = base + L.chol + bd::align_up(sizeof(double) * bd::kNB * bd::kNB, 256);
      d.P32[0] = reinterpret_cast<float*>(pc);
      d.P32[1] = reinterpret_cast<float*>(pc + bd::p32_copy_bytes(n));
    }
    d.xi = reinterpret_cast<double*>(base + L.brown);
    d.ypart = step_ypart(base, L, n);
    d.y = reinterpret_cast<double*>(base + L.y);
    d.xs = reinterpret_cast<double*>(base + L.xs);
    d.cons = base + L.cons;
    d.st = e->st + c;
    base += L.total;
    xoff += n;
    if (q.n_beads > e->max_beads) e->max_beads = q.n_beads;
    if (q.newton_maxit > e->newton_maxit) e->newton_maxit = q.newton_maxit;
  }
  // decreasing n (ties in the caller's order): the chains with work at a
  // given column of the factorisation are a prefix of the table
  std::stable_sort(e->host.begin(), e->host.end(),
                   [](const bd::ChainDesc& a, const bd::ChainDesc& b) { return a.n > b.n; });
  memset(e->host_st, 0, sizeof(DevState) * (size_t)n_chains);
  std::vector<int32_t> prefix((size_t)n_chains + 1, 0), rpre(prefix);
  int64_t pm = 0, pr = 0;  // grids must stay within int32
  for (int32_t c = 0; c < n_chains; ++c) {
    const bd::ChainDesc& d = e->host[(size_t)c];
    pm += bd::constrain_mv_blocks(d.N);
    pr += bd::rpy_batched_blocks(d.N);
    if (pm > INT32_MAX || pr > INT32_MAX) {
        return BD_ERR_UNSUPPORTED;
    }
    prefix[(size_t)c + 1] = (int32_t)pm;
    rpre[(size_t)c + 1] = (int32_t)pr;
  }
  e->mv_blocks = prefix[(size_t)n_chains];
  e->rpy_blocks = rpre[(size_t)n_chains];
  // record the factorisation's flattened grids (no launches), then upload
  e->tb.record = true;
  const hipError_t rec = bd::launch_cholesky_batched(h->stream, h->aux, h->ev, e->cd,
                                                     e->host.data(), n_chains, prec,
                                                     e->step_panels, &e->tb);
  e->tb.record = false;
  if (rec != hipSuccess ||
      hipMalloc(&e->tb_dev, sizeof(int32_t) * (e->tb.host.size() + 1)) != hipSuccess) {
    return rec != hipSuccess ? BD_ERR_PARAM : BD_ERR_ALLOC;
  }
  e->tb.dev = e->tb_dev;
  if (hipMemcpy(e->cd, e->host.data(), sizeof(bd::ChainDesc) * (size_t)n_chains,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(e->mv_prefix, prefix.data(), sizeof(int32_t) * prefix.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(e->rpy_prefix, rpre.data(), sizeof(int32_t) * rpre.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      (!e->tb.host.empty() &&
       hipMemcpy(e->tb_dev, e->tb.host.data(), sizeof(int32_t) * e->tb.host.size(),
                 hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(e->st, e->host_st, sizeof(DevState) * (size_t)n_chains, hipMemcpyHostToDevice) !=
          hipSuccess) {
    return BD_ERR_HIP;
  }
  guard.e = nullptr;
  *out = e;
  return BD_OK;
}

bd_status_t bd_ensemble_create(bd_handle_t h, int32_t n_chains, const bd_params_t* p,
                               bd_precision_t prec, double* d_x, void* d_ws, size_t ws_bytes,
                               bd_ensemble_t* out) {
  try {
    return ensemble_create_impl(h, n_chains, p, prec, d_x, d_ws, ws_bytes, out);
  } catch (...) {  // a host allocation failed: no exception crosses the C ABI
    if (out) *out = nullptr;
    return BD_ERR_ALLOC;
  }
}

// The launches of one ensemble step on stream s: polled tension solves
// (budget 0, noise counter `step`) or, for a captured step, a fixed number
// of products, the noise counter read from d_step and advanced at the end.
static hipError_t ensemble_step_launches(bd_ensemble_s* e, hipStream_t s, int64_t step,
                                         const int64_t* d_step, int budget) {
  bd_handle_t h = e->h;
  const int z = e->count;
  const int64_t max_n = 3 * (int64_t)e->max_beads;
  BD_LAUNCH("reset_states", reset_states_kernel, dim3((unsigned)((z + 255) / 256)), dim3(256), 0,
            s, e->st, z);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess)
    he = bd::launch_rpy_assemble_batched(s, e->cd, z, e->rpy_prefix, e->rpy_blocks);
  if (he == hipSuccess) he = bd::launch_noise_batched(s, e->cd, z, max_n, step, d_step);
  if (he == hipSuccess)
    he = bd::launch_cholesky_batched(s, h->aux, h->ev, e->cd, e->host.data(), z, e->prec,
                                     e->step_panels, &e->tb, true);
  if (he == hipSuccess) he = bd::launch_predictor_batched(s, e->cd, z, e->max_beads);
  if (he == hipSuccess)
    he = bd::launch_constrain_batched(s, e->cd, z, e->max_beads, e->mv_prefix, e->mv_blocks,
                                      e->newton_maxit, e->st, e->host_st, &e->pairs_hint, budget);
  if (he == hipSuccess) {
    BD_LAUNCH("commit_positions_batched", commit_positions_batched_kernel,
              dim3((unsigned)((max_n + 255) / 256), 1, z), dim3(256), 0, s, e->cd);
    he = hipGetLastError();
  }
  if (he == hipSuccess && d_step) {
    BD_LAUNCH("advance_step", set_step_kernel, dim3(1), dim3(1), 0, s,
              const_cast<int64_t*>(d_step), (int64_t)0, 1);
    he = hipGetLastError();
  }
  return he;
}

bd_status_t bd_ensemble_step(bd_ensemble_t e, int64_t step) {
  if (!e) return BD_ERR_PARAM;
  bd_handle_t h = e->h;
  CallScope scope(h);
  bd_status_t err = enter(h);
  if (err != BD_OK) return err;
  if (!e->gexec) return hip_status(ensemble_step_launches(e, h->stream, step, nullptr, 0));
  // replay the captured step; its noise counter lives on the device
  if (step != e->next_step) {
    BD_LAUNCH("set_step", set_step_kernel, dim3(1), dim3(1), 0, h->stream, e->d_step, step, 0);
    if (hipGetLastError() != hipSuccess) return BD_ERR_HIP;
  }
  if (hipGraphLaunch(e->gexec, h->stream) != hipSuccess) return BD_ERR_HIP;
  e->next_step = step + 1;
  return BD_OK;
}

bd_status_t bd_ensemble_capture(bd_ensemble_t e, int32_t max_products) {
  if (!e || max_products < 0) return BD_ERR_PARAM;
  bd_handle_t h = e->h;
  if (h->prof_on) return BD_ERR_PARAM;  // the profiler's events stay out of graphs
  bd_status_t err = enter(h);
  if (err != BD_OK) return err;
  const int budget = max_products > 0 ? max_products
                     : e->pairs_hint > 0 ? e->pairs_hint + e->pairs_hint / 4 + 4
                                         : 2 * 62;
  if (!e->d_step && hipMalloc(&e->d_step, sizeof(int64_t)) != hipSuccess) return BD_ERR_ALLOC;
  if (!e->cap && hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking) != hipSuccess)
    return BD_ERR_HIP;
  // the captured sequence starts after the work already queued on the
  // handle's stream
  if (hipStreamSynchronize(h->stream) != hipSuccess) return BD_ERR_HIP;
  if (hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return BD_ERR_HIP;
  const hipError_t he = ensemble_step_launches(e, e->cap, 0, e->d_step, budget);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(e->cap, &g);
  if (he != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return BD_ERR_HIP;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return BD_ERR_HIP;
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  e->gexec = x;
  e->budget = budget;
  e->next_step = -1;  // the counter is set at the first replay
  return BD_OK;
}

bd_status_t bd_ensemble_get_info(bd_ensemble_t e, bd_info_t* out) {
  if (!e || !out) return BD_ERR_PARAM;
  bd_status_t err = enter(e->h);
  if (err != BD_OK) return err;
  if (hipMemcpyAsync(e->host_st, e->st, sizeof(DevState) * (size_t)e->count,
                     hipMemcpyDeviceToHost, e->h->stream) != hipSuccess)
    return BD_ERR_HIP;
  if (hipStreamSynchronize(e->h->stream) != hipSuccess) return BD_ERR_HIP;
  for (int c = 0; c < e->count; ++c) memcpy(&out[c], &e->host_st[c], sizeof(bd_info_t));
  return BD_OK;
}

bd_status_t bd_ensemble_destroy(bd_ensemble_t e) {
  if (!e) return BD_ERR_PARAM;
  (void)hipSetDevice(e->h->device);
  (void)hipStreamSynchronize(e->h->stream);
  ensemble_release(e);
  return BD_OK;
}

}  // extern "C"
