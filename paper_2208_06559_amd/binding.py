"""ctypes binding of ``libbdrpy.so`` (see ``include/bdrpy.h``).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library.  PyTorch supplies device memory (tensors) and the
current HIP stream.  Calls fail loudly when the library is missing or the
device is not an MI355X (gfx950); there is no CPU fallback.

Matrices are column-major with leading dimension ``ld``: a buffer for an
n x n matrix is a float64 tensor of shape (n, ld) whose row c holds column c
(use :func:`matrix_view` to see it as an ordinary n x n matrix).
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdrpy.so")

OK, ERR_PARAM, ERR_NOT_SPD, ERR_NO_CONVERGE, ERR_HIP, ERR_ALLOC, ERR_UNSUPPORTED = range(7)
PREC_FP64, PREC_MIXED = 0, 1
NOISE_GAUSSIAN, NOISE_UNIFORM_PAPER = 0, 1
FILL_LOWER, FILL_FULL = 0, 1
OP_CHOLESKY, OP_BROWNIAN, OP_CONSTRAIN, OP_STEP = 0, 1, 2, 3
OP_CHOLESKY_ADJOINT, OP_STEP_ADJOINT = 4, 5

STATUS_NAMES = {0: "BD_OK", 1: "BD_ERR_PARAM", 2: "BD_ERR_NOT_SPD", 3: "BD_ERR_NO_CONVERGE",
                4: "BD_ERR_HIP", 5: "BD_ERR_ALLOC", 6: "BD_ERR_UNSUPPORTED"}

EXPORTS = ("bd_create", "bd_destroy", "bd_set_stream", "bd_workspace_size", "bd_rpy_assemble",
           "bd_cholesky", "bd_brownian", "bd_constrain", "bd_step", "bd_get_info",
           "bd_profile_begin", "bd_profile_end", "bd_ensemble_workspace_size",
           "bd_ensemble_create", "bd_ensemble_step", "bd_ensemble_get_info",
           "bd_ensemble_destroy", "bd_step_fraenkel", "bd_observables",
           "bd_rpy_assemble_adjoint", "bd_brownian_adjoint", "bd_brownian_noalloc",
           "bd_stress", "bd_cholesky_adjoint", "bd_constrain_adjoint",
           "bd_step_adjoint", "bd_ensemble_capture", "bd_set_schedules",
           "bd_set_ensemble_panels")


class BdError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")
        self.status = status


class Params(C.Structure):
    """Mirror of bd_params_t."""
    _fields_ = [
        ("n_beads", C.c_int32),
        ("noise", C.c_int32),
        ("b", C.c_double),
        ("hstar", C.c_double),
        ("a", C.c_double),
        ("dt", C.c_double),
        ("kappa", C.c_double * 9),
        ("seed", C.c_uint64),
        ("chain_id", C.c_uint64),
        ("newton_tol", C.c_double),
        ("newton_maxit", C.c_int32),
        ("reserved", C.c_int32),
    ]


class Info(C.Structure):
    """Mirror of bd_info_t."""
    _fields_ = [
        ("status", C.c_int32),
        ("newton_iters", C.c_int32),
        ("potrf_info", C.c_int64),
        ("max_rod_err", C.c_double),
        ("last_newton_res", C.c_double),
        ("krylov_iters", C.c_int32),
        ("reserved", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def make_params(n_beads: int, *, b=1.0, hstar=0.25, a=0.5, dt=1e-4, kappa=None, seed=0,
                chain_id=0, noise=NOISE_GAUSSIAN, newton_tol=1e-13, newton_maxit=20) -> Params:
    p = Params()
    p.n_beads = int(n_beads)
    p.noise = int(noise)
    p.b, p.hstar, p.a, p.dt = float(b), float(hstar), float(a), float(dt)
    k = np.zeros(9) if kappa is None else np.asarray(kappa, dtype=np.float64).reshape(9)
    for e in range(9):
        p.kappa[e] = float(k[e])
    p.seed = int(seed) & (2**64 - 1)
    p.chain_id = int(chain_id) & (2**64 - 1)
    p.newton_tol = float(newton_tol)
    p.newton_maxit = int(newton_maxit)
    p.reserved = 0
    return p


class Schedule(C.Structure):
    """Mirror of bd_schedule_t."""
    _fields_ = [("n_max", C.c_int64), ("prec", C.c_int32), ("step_panels", C.c_int32),
                ("wide_rows", C.c_int64)]


TUNING_PATH = os.path.join(HERE, "tuning.json")


def load_tuning(path: str = TUNING_PATH) -> dict | None:
    """The autotuner's table (tune.py), or None when there is none."""
    import json
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


class KernelStat(C.Structure):
    """Mirror of bd_kernel_stat_t."""
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib = None


def lib():
    """Load libbdrpy.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, pp = C.c_void_p, C.c_void_p, C.POINTER(Params)
        L.bd_create.argtypes = [C.POINTER(vp), C.c_int, vp]
        L.bd_destroy.argtypes = [vp]
        L.bd_set_stream.argtypes = [vp, vp]
        L.bd_workspace_size.argtypes = [C.c_int, C.c_int64, C.c_int, C.POINTER(C.c_size_t)]
        L.bd_rpy_assemble.argtypes = [vp, pp, dp, dp, C.c_int64, C.c_int]
        L.bd_cholesky.argtypes = [vp, C.c_int64, dp, C.c_int64, C.c_int, vp, C.c_size_t]
        L.bd_brownian.argtypes = [vp, pp, C.c_int64, dp, C.c_int64, dp, dp, vp, C.c_size_t]
        L.bd_constrain.argtypes = [vp, pp, dp, dp, dp, vp, C.c_size_t]
        L.bd_step.argtypes = [vp, pp, C.c_int64, dp, C.c_int, vp, C.c_size_t]
        L.bd_get_info.argtypes = [vp, C.POINTER(Info)]
        L.bd_profile_begin.argtypes = [vp]
        L.bd_profile_end.argtypes = [vp, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]
        L.bd_ensemble_workspace_size.argtypes = [C.c_int32, pp, C.c_int, C.POINTER(C.c_size_t)]
        L.bd_ensemble_create.argtypes = [vp, C.c_int32, pp, C.c_int, dp, vp, C.c_size_t,
                                         C.POINTER(vp)]
        L.bd_ensemble_step.argtypes = [vp, C.c_int64]
        L.bd_ensemble_get_info.argtypes = [vp, C.POINTER(Info)]
        L.bd_ensemble_destroy.argtypes = [vp]
        L.bd_ensemble_capture.argtypes = [vp, C.c_int32]
        L.bd_set_schedules.argtypes = [vp, C.POINTER(Schedule), C.c_int32]
        L.bd_set_ensemble_panels.argtypes = [vp, C.c_int, C.c_int32]
        L.bd_step_fraenkel.argtypes = [vp, pp, C.c_double, C.c_int64, dp, C.c_int, vp, C.c_size_t]
        L.bd_observables.argtypes = [vp, C.c_int32, dp, vp, dp]
        L.bd_rpy_assemble_adjoint.argtypes = [vp, pp, dp, dp, C.c_int64, dp, dp, vp, C.c_size_t]
        L.bd_brownian_adjoint.argtypes = [vp, pp, dp, C.c_int64, dp, dp, dp, C.c_int64, dp]
        L.bd_brownian_noalloc.argtypes = [vp, pp, C.c_int64, dp, C.c_int64, dp, dp]
        L.bd_stress.argtypes = [vp, C.c_int32, dp, vp, dp, C.c_double, C.c_double, dp]
        L.bd_cholesky_adjoint.argtypes = [vp, C.c_int64, dp, C.c_int64, dp, C.c_int64, dp,
                                          C.c_int64, vp, C.c_size_t]
        L.bd_constrain_adjoint.argtypes = [vp, pp, dp, dp, dp, dp, vp, C.c_size_t]
        L.bd_step_adjoint.argtypes = [vp, pp, C.c_int64, dp, dp, dp, dp, vp, C.c_size_t]
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != OK:
        raise BdError(st, where)


def _dev_f64(t: torch.Tensor, name: str, numel: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA/HIP tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs {numel} elements, has {t.numel()}")
    return t.data_ptr()


def workspace_size(op: int, n: int, prec: int = PREC_FP64) -> int:
    out = C.c_size_t(0)
    _check(lib().bd_workspace_size(op, n, prec, C.byref(out)), "bd_workspace_size")
    return int(out.value)


def matrix_view(buf: torch.Tensor, n: int) -> torch.Tensor:
    """n x n matrix view of a column-major (n, ld) buffer."""
    return buf[:n, :n].t()


class Handle:
    """One bd_handle_t on the current device, launching on torch's current
    stream at the time of each call."""

    def __init__(self, device: int | None = None, tuned: bool = False):
        """tuned: apply the autotuner's committed table (tuning.json), if any."""
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        h = C.c_void_p()
        with torch.cuda.device(dev):
            stream = torch.cuda.current_stream().cuda_stream
        _check(lib().bd_create(C.byref(h), dev, C.c_void_p(stream)), "bd_create")
        self._h = h
        self._ws = {}
        self._ensembles = weakref.WeakSet()  # destroyed before the handle
        self.tuning = None
        if tuned:
            t = load_tuning()
            if t is not None:
                self.set_schedules(t["schedules"])
                for name, prec in (("fp64", PREC_FP64), ("mixed", PREC_MIXED)):
                    self.set_ensemble_panels(prec, int(t["ensemble_panels"][name]))
                self.tuning = t

    def set_schedules(self, rows):
        """bd_set_schedules from dicts with n_max, prec, step_panels, wide_rows."""
        arr = (Schedule * max(len(rows), 1))()
        for i, r in enumerate(rows):
            arr[i] = Schedule(int(r["n_max"]), int(r["prec"]), int(r["step_panels"]),
                              int(r["wide_rows"]))
        _check(lib().bd_set_schedules(self._h, arr, len(rows)), "bd_set_schedules")

    def set_ensemble_panels(self, prec: int, panels: int):
        _check(lib().bd_set_ensemble_panels(self._h, prec, panels), "bd_set_ensemble_panels")

    def close(self):
        if self._h:
            for e in list(self._ensembles):
                e.close()
            lib().bd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        lib().bd_set_stream(self._h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def workspace(self, op: int, n: int, prec: int = PREC_FP64) -> torch.Tensor:
        nbytes = workspace_size(op, n, prec)
        key = (op, n, prec)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws[key] = ws
        return ws

    def rpy_assemble(self, p: Params, x: torch.Tensor, D: torch.Tensor, ld: int,
                     fill: int = FILL_LOWER):
        n = 3 * p.n_beads
        self._sync_stream()
        _check(lib().bd_rpy_assemble(self._h, C.byref(p), _dev_f64(x, "x", n),
                                     _dev_f64(D, "D", (n - 1) * ld + n), ld, fill),
               "bd_rpy_assemble")

    def cholesky(self, A: torch.Tensor, n: int, ld: int, prec: int = PREC_FP64,
                 ws: torch.Tensor | None = None):
        ws = self.workspace(OP_CHOLESKY, n, prec) if ws is None else ws
        self._sync_stream()
        _check(lib().bd_cholesky(self._h, n, _dev_f64(A, "A", (n - 1) * ld + n), ld, prec,
                                 ws.data_ptr(), ws.numel() * ws.element_size()), "bd_cholesky")

    def brownian(self, p: Params, step: int, L: torch.Tensor, ld: int, y: torch.Tensor,
                 xi_out: torch.Tensor | None = None):
        n = 3 * p.n_beads
        ws = self.workspace(OP_BROWNIAN, n)
        self._sync_stream()
        xi_ptr = _dev_f64(xi_out, "xi_out", n) if xi_out is not None else None
        _check(lib().bd_brownian(self._h, C.byref(p), step, _dev_f64(L, "L", (n - 1) * ld + n), ld,
                                 _dev_f64(y, "y", n), xi_ptr, ws.data_ptr(), ws.numel()),
               "bd_brownian")

    def cholesky_adjoint(self, n: int, L: torch.Tensor, ld: int, Lbar: torch.Tensor, ldb: int,
                         Abar: torch.Tensor, lda: int):
        """bd_cholesky_adjoint: Abar (every element) from B (lower of L) and
        Lbar (lower), all (n, ld) column-major buffers."""
        ws = self.workspace(OP_CHOLESKY_ADJOINT, n)
        self._sync_stream()
        _check(lib().bd_cholesky_adjoint(self._h, n, _dev_f64(L, "L", (n - 1) * ld + n), ld,
                                         _dev_f64(Lbar, "Lbar", (n - 1) * ldb + n), ldb,
                                         _dev_f64(Abar, "Abar", (n - 1) * lda + n), lda,
                                         ws.data_ptr(), ws.numel()), "bd_cholesky_adjoint")

    def constrain_adjoint(self, p: Params, x_old: torch.Tensor, x_new: torch.Tensor,
                          xbar: torch.Tensor, z: torch.Tensor):
        """bd_constrain_adjoint: z = xbar - 2 Delta^T (Q mu) (N x 3)."""
        n = 3 * p.n_beads
        ws = self.workspace(OP_CONSTRAIN, n)
        self._sync_stream()
        _check(lib().bd_constrain_adjoint(self._h, C.byref(p), _dev_f64(x_old, "x_old", n),
                                          _dev_f64(x_new, "x_new", n), _dev_f64(xbar, "xbar", n),
                                          _dev_f64(z, "z", n), ws.data_ptr(), ws.numel()),
               "bd_constrain_adjoint")

    def step_adjoint(self, p: Params, step: int, x: torch.Tensor, xbar: torch.Tensor,
                     hbar: torch.Tensor, kbar: torch.Tensor):
        """bd_step_adjoint: xbar (gradient in x^{t+dt}) becomes the gradient in
        x^t; the gradients in h* and kappa are added to hbar (1) and kbar (9)."""
        n = 3 * p.n_beads
        ws = self.workspace(OP_STEP_ADJOINT, n)
        self._sync_stream()
        _check(lib().bd_step_adjoint(self._h, C.byref(p), step, _dev_f64(x, "x", n),
                                     _dev_f64(xbar, "xbar", n), _dev_f64(hbar, "hbar", 1),
                                     _dev_f64(kbar, "kbar", 9), ws.data_ptr(), ws.numel()),
               "bd_step_adjoint")

    def brownian_noalloc(self, p: Params, step: int, L: torch.Tensor, ld: int, y: torch.Tensor,
                         xi_out: torch.Tensor | None = None):
        """bd_brownian_noalloc: the noise product with the library's fixed
        scratch array in place of a workspace."""
        n = 3 * p.n_beads
        self._sync_stream()
        xi_ptr = _dev_f64(xi_out, "xi_out", n) if xi_out is not None else None
        _check(lib().bd_brownian_noalloc(self._h, C.byref(p), step,
                                         _dev_f64(L, "L", (n - 1) * ld + n), ld,
                                         _dev_f64(y, "y", n), xi_ptr), "bd_brownian_noalloc")

    def constrain(self, p: Params, x_old: torch.Tensor, x_pred: torch.Tensor,
                  T_out: torch.Tensor | None = None):
        n = 3 * p.n_beads
        ws = self.workspace(OP_CONSTRAIN, n)
        self._sync_stream()
        t_ptr = _dev_f64(T_out, "T_out", p.n_beads - 1) if T_out is not None else None
        _check(lib().bd_constrain(self._h, C.byref(p), _dev_f64(x_old, "x_old", n),
                                  _dev_f64(x_pred, "x_pred", n), t_ptr, ws.data_ptr(),
                                  ws.numel()), "bd_constrain")

    def step(self, p: Params, step: int, x: torch.Tensor, prec: int = PREC_FP64,
             ws: torch.Tensor | None = None):
        n = 3 * p.n_beads
        ws = self.workspace(OP_STEP, n, prec) if ws is None else ws
        self._sync_stream()
        _check(lib().bd_step(self._h, C.byref(p), step, _dev_f64(x, "x", n), prec, ws.data_ptr(),
                             ws.numel() * ws.element_size()), "bd_step")

    def step_fraenkel(self, p: Params, k_spring: float, step: int, x: torch.Tensor,
                      prec: int = PREC_FP64, ws: torch.Tensor | None = None):
        n = 3 * p.n_beads
        ws = self.workspace(OP_STEP, n, prec) if ws is None else ws
        self._sync_stream()
        _check(lib().bd_step_fraenkel(self._h, C.byref(p), float(k_spring), step,
                                      _dev_f64(x, "x", n), prec, ws.data_ptr(),
                                      ws.numel() * ws.element_size()), "bd_step_fraenkel")

    def rpy_assemble_adjoint(self, p: Params, x: torch.Tensor, Dbar: torch.Tensor, ld: int):
        """(d phi/d x (N x 3), d phi/d h* (1-element tensor)) for
        phi = <Dbar, D(x)>, Dbar a column-major (n, ld) buffer."""
        n = 3 * p.n_beads
        dev = f"cuda:{self.device}"
        xbar = torch.empty((p.n_beads, 3), dtype=torch.float64, device=dev)
        hbar = torch.empty(1, dtype=torch.float64, device=dev)
        ws = torch.empty(max(p.n_beads, 1), dtype=torch.float64, device=dev)
        self._sync_stream()
        _check(lib().bd_rpy_assemble_adjoint(self._h, C.byref(p), _dev_f64(x, "x", n),
                                             _dev_f64(Dbar, "Dbar", (n - 1) * ld + n), ld,
                                             xbar.data_ptr(), hbar.data_ptr(), ws.data_ptr(),
                                             ws.numel() * 8), "bd_rpy_assemble_adjoint")
        return xbar, hbar

    def brownian_adjoint(self, p: Params, L: torch.Tensor, ld: int, xi: torch.Tensor,
                         ybar: torch.Tensor, Lbar: torch.Tensor, ldb: int, xibar: torch.Tensor):
        n = 3 * p.n_beads
        self._sync_stream()
        _check(lib().bd_brownian_adjoint(self._h, C.byref(p), _dev_f64(L, "L", (n - 1) * ld + n),
                                         ld, _dev_f64(xi, "xi", n), _dev_f64(ybar, "ybar", n),
                                         _dev_f64(Lbar, "Lbar", (n - 1) * ldb + n), ldb,
                                         _dev_f64(xibar, "xibar", n)), "bd_brownian_adjoint")

    def observables(self, x: torch.Tensor, n_beads) -> torch.Tensor:
        """(n_chains, 4) tensor: R_ee (3 components) and R_g^2 per chain of
        the packed positions x (chain c has n_beads[c] beads)."""
        counts = [int(v) for v in n_beads]
        if not counts or min(counts) < 1:
            raise ValueError("n_beads: every chain needs at least one bead")
        off = torch.tensor([0] + list(np.cumsum(counts)), dtype=torch.int64,
                           device=f"cuda:{self.device}")
        out = torch.empty((len(counts), 4), dtype=torch.float64, device=f"cuda:{self.device}")
        self._sync_stream()
        _check(lib().bd_observables(self._h, len(counts), _dev_f64(x, "x", 3 * sum(counts)),
                                    off.data_ptr(), out.data_ptr()), "bd_observables")
        return out

    def stress(self, x: torch.Tensor, n_beads, *, tensions: torch.Tensor | None = None,
               k_spring: float = 0.0, b: float = 1.0) -> torch.Tensor:
        """(n_chains, 7) tensor: tau_xx, tau_yy, tau_zz, tau_xy, tau_xz,
        tau_yz and N1 per chain (bd_stress); rigid rods when ``tensions``
        (packed, N_c - 1 per chain) is given, else springs of stiffness
        ``k_spring``."""
        counts = [int(v) for v in n_beads]
        if not counts or min(counts) < 2:
            raise ValueError("n_beads: every chain needs at least two beads")
        off = torch.tensor([0] + list(np.cumsum(counts)), dtype=torch.int64,
                           device=f"cuda:{self.device}")
        out = torch.empty((len(counts), 7), dtype=torch.float64, device=f"cuda:{self.device}")
        t_ptr = (_dev_f64(tensions, "tensions", sum(counts) - len(counts))
                 if tensions is not None else None)
        self._sync_stream()
        _check(lib().bd_stress(self._h, len(counts), _dev_f64(x, "x", 3 * sum(counts)),
                               off.data_ptr(), t_ptr, float(k_spring), float(b), out.data_ptr()),
               "bd_stress")
        return out

    def profile_begin(self):
        self._sync_stream()
        _check(lib().bd_profile_begin(self._h), "bd_profile_begin")

    def profile_end(self) -> dict:
        """{kernel name: (launches, total_ms)} since profile_begin."""
        buf = (KernelStat * 64)()
        n = C.c_int32(0)
        _check(lib().bd_profile_end(self._h, buf, 64, C.byref(n)), "bd_profile_end")
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                for i in range(min(n.value, 64))}

    def info(self) -> dict:
        out = Info()
        _check(lib().bd_get_info(self._h, C.byref(out)), "bd_get_info")
        return out.as_dict()


def ensemble_workspace_size(params, prec: int = PREC_FP64) -> int:
    arr = (Params * len(params))(*params)
    out = C.c_size_t(0)
    _check(lib().bd_ensemble_workspace_size(len(params), arr, prec, C.byref(out)),
           "bd_ensemble_workspace_size")
    return int(out.value)


class Ensemble:
    """One bd_ensemble_t: chains with parameters `params` (a list of Params)
    whose positions are packed in the float64 tensor `x` (chain c's N_c x 3
    block after those of chains 0..c-1), advanced together by step()."""

    def __init__(self, handle: Handle, params, x: torch.Tensor, prec: int = PREC_FP64):
        self.handle = handle
        self.params = list(params)
        self.count = len(self.params)
        self.prec = prec
        n_tot = 3 * sum(p.n_beads for p in self.params)
        self._arr = (Params * self.count)(*self.params)
        nbytes = ensemble_workspace_size(self.params, prec)
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f"cuda:{handle.device}")
        self.x = x
        e = C.c_void_p()
        handle._sync_stream()
        _check(lib().bd_ensemble_create(handle._h, self.count, self._arr, prec,
                                        _dev_f64(x, "x", n_tot), self.ws.data_ptr(), nbytes,
                                        C.byref(e)), "bd_ensemble_create")
        self._e = e
        handle._ensembles.add(self)

    def step(self, step: int):
        self.handle._sync_stream()
        _check(lib().bd_ensemble_step(self._e, step), "bd_ensemble_step")

    def capture(self, max_products: int = 0):
        """bd_ensemble_capture: later steps replay one captured HIP graph."""
        _check(lib().bd_ensemble_capture(self._e, int(max_products)), "bd_ensemble_capture")

    def info(self) -> list[dict]:
        out = (Info * self.count)()
        _check(lib().bd_ensemble_get_info(self._e, out), "bd_ensemble_get_info")
        return [out[c].as_dict() for c in range(self.count)]

    def close(self):
        if self._e:
            if self.handle._h:  # the handle's close() destroys its ensembles first
                lib().bd_ensemble_destroy(self._e)
            self._e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
