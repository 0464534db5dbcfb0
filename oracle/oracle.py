"""ctypes front end of the CPU FP64 oracle (``oracle/libbdo.so``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the HIP library or its Python binding.

Every function mirrors one routine of ``oracle/bdo.c``, where the equations
each follows are cited (arXiv 2208.06559, Sections 3-4), except
``observables``, ``kramers_stress``, ``rpy_assemble_adjoint``,
``brownian_adjoint``, ``cholesky_adjoint``, ``constrain_adjoint``,
``step_adjoint``, ``mean_stretch`` and ``stretch_gradient``, which are
written here in numpy from their definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdo.so")

OK, ERR_PARAM, ERR_NOT_SPD, ERR_NO_CONVERGE = 0, 1, 2, 3
NOISE_GAUSSIAN, NOISE_UNIFORM_PAPER = 0, 1
FILL_LOWER, FILL_FULL = 0, 1


def build(verbose: bool = False) -> str:
    """Compile ``bdo.c`` into ``libbdo.so`` with gcc (OpenMP, FP64)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", os.path.join(HERE, "bdo.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
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
        ("pad_", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("newton_iters", C.c_int32),
        ("potrf_info", C.c_int64),
        ("max_rod_err", C.c_double),
        ("last_newton_res", C.c_double),
        ("krylov_iters", C.c_int32),
        ("pad_", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        u64p = C.POINTER(C.c_uint64)
        pp = C.POINTER(Params)
        ip = C.POINTER(Info)
        L.bdo_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.bdo_philox4x64_10.restype = None
        L.bdo_noise.argtypes = [pp, C.c_int64, C.c_int64, dp]
        L.bdo_noise.restype = None
        L.bdo_rpy_block.argtypes = [C.c_double, C.c_double, dp, dp]
        L.bdo_rpy_block.restype = None
        L.bdo_rpy_assemble.argtypes = [pp, dp, dp, C.c_int64, C.c_int32]
        L.bdo_rpy_assemble.restype = C.c_int
        L.bdo_cholesky.argtypes = [C.c_int64, dp, C.c_int64]
        L.bdo_cholesky.restype = C.c_int64
        L.bdo_brownian.argtypes = [pp, C.c_int64, dp, C.c_int64, dp, dp]
        L.bdo_brownian.restype = C.c_int
        for name in ("bdo_constrain", "bdo_constrain_dense"):
            f = getattr(L, name)
            f.argtypes = [pp, dp, dp, dp, ip]
            f.restype = C.c_int
        L.bdo_step.argtypes = [pp, C.c_int64, dp, ip]
        L.bdo_step.restype = C.c_int
        L.bdo_step_fraenkel.argtypes = [pp, C.c_double, C.c_int64, dp, ip]
        L.bdo_step_fraenkel.restype = C.c_int
        L.bdo_run.argtypes = [pp, C.c_int64, C.c_int64, dp, ip]
        L.bdo_run.restype = C.c_int
        L.bdo_run_many.argtypes = [pp, C.c_int32, u64p, C.c_int64, C.c_int64, dp,
                                   C.POINTER(C.c_int32)]
        L.bdo_run_many.restype = C.c_int
        L.bdo_num_threads.argtypes = []
        L.bdo_num_threads.restype = C.c_int
        L.bdo_set_num_threads.argtypes = [C.c_int]
        L.bdo_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


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
    return p


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64p = C.POINTER(C.c_uint64)
    lib().bdo_philox4x64_10(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    return out


def noise(p: Params, step: int, n: int) -> np.ndarray:
    xi = np.zeros(n)
    lib().bdo_noise(C.byref(p), step, n, _dp(xi))
    return xi


def rpy_block(hstar: float, a: float, Rvec) -> np.ndarray:
    R = np.ascontiguousarray(Rvec, dtype=np.float64)
    out = np.zeros(9)
    lib().bdo_rpy_block(hstar, a, _dp(R), _dp(out))
    return out.reshape(3, 3)


def rpy_assemble(p: Params, x: np.ndarray, fill: int = FILL_FULL, ld: int | None = None) -> np.ndarray:
    """Returns D as an (n x n) Fortran-ordered array (column-major, ld = n)."""
    n = 3 * p.n_beads
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (p.n_beads, 3)
    D = np.zeros((n, n), dtype=np.float64, order="F")
    st = lib().bdo_rpy_assemble(C.byref(p), _dp(x), _dp(D), n, fill)
    if st != OK:
        raise ValueError(f"bdo_rpy_assemble status {st}")
    return D


def cholesky(A: np.ndarray) -> tuple[np.ndarray, int]:
    """Lower Cholesky of the lower triangle of A; returns (L, info) with
    the strict upper triangle of the input copied through untouched."""
    L = np.array(A, dtype=np.float64, order="F", copy=True)
    n = L.shape[0]
    info = lib().bdo_cholesky(n, _dp(L), n)
    return L, int(info)


def brownian(p: Params, step: int, L: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    n = 3 * p.n_beads
    Lf = np.asfortranarray(L, dtype=np.float64)
    y = np.zeros(n)
    xi = np.zeros(n)
    st = lib().bdo_brownian(C.byref(p), step, _dp(Lf), n, _dp(y), _dp(xi))
    if st != OK:
        raise ValueError(f"bdo_brownian status {st}")
    return y, xi


def constrain(p: Params, x_old: np.ndarray, x_pred: np.ndarray, dense: bool = False):
    xo = np.ascontiguousarray(x_old, dtype=np.float64)
    xs = np.array(x_pred, dtype=np.float64, order="C", copy=True)
    T = np.zeros(max(p.n_beads - 1, 0))
    info = Info()
    f = lib().bdo_constrain_dense if dense else lib().bdo_constrain
    f(C.byref(p), _dp(xo), _dp(xs), _dp(T), C.byref(info))
    return xs, T, info.as_dict()


def step(p: Params, s: int, x: np.ndarray):
    xx = np.array(x, dtype=np.float64, order="C", copy=True)
    info = Info()
    lib().bdo_step(C.byref(p), s, _dp(xx), C.byref(info))
    return xx, info.as_dict()


def step_fraenkel(p: Params, k_spring: float, s: int, x: np.ndarray):
    """One step with stiff Fraenkel springs of stiffness k_spring (Eqs. 3,
    13-17); returns (x', info)."""
    xx = np.array(x, dtype=np.float64, order="C", copy=True)
    info = Info()
    lib().bdo_step_fraenkel(C.byref(p), float(k_spring), s, _dp(xx), C.byref(info))
    return xx, info.as_dict()


def observables(x: np.ndarray) -> np.ndarray:
    """Chain observables of the flow studies (Section 5) for one chain x
    (N x 3): the end-to-end vector R_ee = r_{N-1} - r_0 and the squared
    radius of gyration R_g^2 = (1/N) sum_i |r_i - r_cm|^2, as
    [R_ee,x, R_ee,y, R_ee,z, R_g^2]."""
    x = np.asarray(x, dtype=np.float64)
    ree = x[-1] - x[0]
    rcm = x.mean(axis=0)
    rg2 = np.sum((x - rcm) ** 2) / len(x)
    return np.concatenate([ree, [rg2]])


def kramers_stress(x: np.ndarray, b: float, *, tensions=None, k_spring=None) -> np.ndarray:
    """Kramers stress of one chain (Section 5, Eq. 28) and its first normal
    stress difference (Eq. 29), as [tau_xx, tau_yy, tau_zz, tau_xy, tau_xz,
    tau_yz, N1], in units of kT per chain.

    tau = sum_k F_k Q_k^T - M I over the M = N - 1 connectors Q_k =
    r_{k+1} - r_k, with F_k the connector's force along Q_k: the Fraenkel
    spring force of Eq. 3, K (|Q_k| - b) Q_k / |Q_k| (k_spring = K), or for
    rigid rods the tension T_k times Q_k / |Q_k| (tensions = T, length M).
    The isotropic part enters with the sign that makes tau vanish at
    equilibrium (the virial <Q F^T> = kT I per connector); N1 = tau_xx -
    tau_yy does not depend on it.  Plain loop over connectors."""
    x = np.asarray(x, dtype=np.float64)
    if (tensions is None) == (k_spring is None):
        raise ValueError("give exactly one of tensions (rigid rods) or k_spring (springs)")
    M = len(x) - 1
    S = np.zeros((3, 3))
    for k in range(M):
        q = x[k + 1] - x[k]
        ql = float(np.sqrt(q @ q))
        if tensions is not None:
            mag = float(tensions[k])
        else:
            mag = float(k_spring) * (ql - b)
        F = mag * q / ql
        S += np.outer(F, q)
    tau = S - M * np.eye(3)
    return np.array([tau[0, 0], tau[1, 1], tau[2, 2], tau[0, 1], tau[0, 2], tau[1, 2],
                     tau[0, 0] - tau[1, 1]])


def _rpy_coeffs_and_slopes(hstar: float, a: float, R: float):
    """cI, cRR of D_ij = cI I + cRR R R^T (Eqs. 8-9) and their derivatives
    with respect to R = |r_i - r_j| > 0."""
    if R >= 2 * a:
        pre = 0.75 * hstar
        cI = pre * (1 / R + 2 * a * a / (3 * R ** 3))
        cRR = pre * (1 / R ** 3 - 2 * a * a / R ** 5)
        dcI = pre * (-1 / R ** 2 - 2 * a * a / R ** 4)
        dcRR = pre * (-3 / R ** 4 + 10 * a * a / R ** 6)
    else:
        pre = 3 * hstar / (8 * a)
        cI = pre * (8 / 3 - 3 * R / (4 * a))
        cRR = pre / (4 * a * R)
        dcI = -pre * 3 / (4 * a)
        dcRR = -pre / (4 * a * R * R)
    return cI, cRR, dcI, dcRR


def rpy_assemble_adjoint(p: Params, x: np.ndarray, Dbar: np.ndarray):
    """Adjoint of the assembly (Eqs. 7-9): for phi = sum_ij <Dbar_ij, D_ij>
    (3 x 3 blocks, Dbar a full n x n matrix), returns (d phi/d x (N x 3),
    d phi/d h*).  With R = r_i - r_j, R = |R|, Rh = R/R and B = Dbar_ij,
    <B, D_ij> = cI tr B + cRR R^T B R, so its gradient in R is
    cI' tr(B) Rh + cRR' (R^T B R) Rh + cRR (B + B^T) R, added to bead i and
    subtracted from bead j; D - I is linear in h*.  Coincident beads are
    rejected (the near-field block is not differentiable at R = 0)."""
    x = np.asarray(x, dtype=np.float64)
    N = len(x)
    xbar = np.zeros((N, 3))
    hbar = 0.0
    for i in range(N):
        for j in range(N):
            if i == j:
                continue
            Rv = x[i] - x[j]
            R = float(np.sqrt(Rv @ Rv))
            if R == 0.0:
                raise ValueError("coincident beads")
            B = Dbar[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            cI, cRR, dcI, dcRR = _rpy_coeffs_and_slopes(p.hstar, p.a, R)
            q = Rv @ B @ Rv
            g = dcI * np.trace(B) * Rv / R + dcRR * q * Rv / R + cRR * (B + B.T) @ Rv
            xbar[i] += g
            xbar[j] -= g
            uI, uRR, _, _ = _rpy_coeffs_and_slopes(1.0, p.a, R)  # per unit h*
            hbar += uI * np.trace(B) + uRR * q
    return xbar, hbar


def brownian_adjoint(p: Params, L: np.ndarray, xi: np.ndarray, ybar: np.ndarray):
    """Adjoint of y = c_B L xi (L lower triangular, the noise term of Eq. 6
    times dt): returns (Lbar, xibar) = (c_B tril(ybar xi^T), c_B L^T ybar),
    the gradients of <ybar, y> in L (lower triangle only; L's upper part is
    not a variable) and in xi."""
    c = np.sqrt(6.0 * p.dt) if p.noise == NOISE_UNIFORM_PAPER else np.sqrt(2.0 * p.dt)
    L = np.tril(np.asarray(L, dtype=np.float64))
    return c * np.tril(np.outer(ybar, xi)), c * (L.T @ ybar)


def cholesky_adjoint(L: np.ndarray, Lbar: np.ndarray) -> np.ndarray:
    """Reverse-mode derivative of the Cholesky factorisation A = L L^T
    (Eq. 10) in the matrix form of Murray (2016): for a scalar phi with
    gradient Lbar in the lower-triangular entries of L,
        d phi = <P, dA>,  P = L^-T Phi(L^T Lbar) L^-1,
    Phi taking the lower triangle with the diagonal halved; returned as the
    symmetric Abar = (P + P^T)/2, the gradient for symmetric dA.  The two
    triangular solves are general solves (numpy LU)."""
    L = np.tril(np.asarray(L, dtype=np.float64))
    X = L.T @ np.tril(np.asarray(Lbar, dtype=np.float64))
    Phi = np.tril(X)
    Phi[np.diag_indices_from(Phi)] *= 0.5
    Y = np.linalg.solve(L.T, Phi)        # L^-T Phi
    P = np.linalg.solve(L.T, Y.T).T      # Y L^-1
    return 0.5 * (P + P.T)


def _difference_operator(N: int) -> np.ndarray:
    """(3(N-1) x 3N) matrix of the rod vectors: (Delta x)_k = x_{k+1} - x_k."""
    M = N - 1
    Dl = np.zeros((3 * M, 3 * N))
    for k in range(M):
        for al in range(3):
            Dl[3 * k + al, 3 * (k + 1) + al] = 1.0
            Dl[3 * k + al, 3 * k + al] = -1.0
    return Dl


def constrain_adjoint(p: Params, x_old: np.ndarray, x_new: np.ndarray, xbar: np.ndarray,
                      D: np.ndarray | None = None) -> np.ndarray:
    """Adjoint of the tension solve by the implicit-function theorem.  The
    constraint step maps x* to x^{t+dt} = x* - dt D Delta^T U T with T
    defined by g(T) = |Q_k|^2 - b^2 = 0, Q = Delta x^{t+dt} (U: the rod
    directions at x_old, D = D(x_old)).  For the gradient xbar of a scalar
    in x^{t+dt}, mu solves J^T mu = -dt U^T Delta D xbar with the dense
    Jacobian J = dg/dT = -2 dt diag(Q)^T Delta D Delta^T U (numpy LU), and
    the returned z = xbar - 2 Delta^T (Q mu) (N x 3) is the gradient of that
    scalar in whatever x^{t+dt} depends on at fixed T (in x* it is z
    itself)."""
    N = p.n_beads
    M = N - 1
    dt = p.dt
    x_old = np.asarray(x_old, dtype=np.float64)
    if D is None:
        D = np.array(rpy_assemble(p, x_old, FILL_FULL))
    q = np.diff(x_old, axis=0)
    u = q / np.linalg.norm(q, axis=1)[:, None]
    Q = np.diff(np.asarray(x_new, dtype=np.float64), axis=0)
    xb = np.asarray(xbar, dtype=np.float64).ravel()
    Dl = _difference_operator(N)
    U = np.zeros((3 * M, M))
    Qm = np.zeros((3 * M, M))
    for k in range(M):
        U[3 * k:3 * k + 3, k] = u[k]
        Qm[3 * k:3 * k + 3, k] = Q[k]
    J = -2.0 * dt * Qm.T @ (Dl @ D @ Dl.T) @ U
    rhs = -dt * U.T @ (Dl @ (D @ xb))
    mu = np.linalg.solve(J.T, rhs)
    return (xb - 2.0 * Dl.T @ (Qm @ mu)).reshape(N, 3)


def mean_stretch(X: np.ndarray, b: float) -> float:
    """Ensemble-mean fractional stretch of chains X (C x N x 3): the mean of
    |r_{N-1} - r_0| / ((N - 1) b), the end-to-end length of Section 5 over
    the contour length."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[1]
    return float(np.mean(np.linalg.norm(X[:, -1] - X[:, 0], axis=1)) / ((N - 1) * b))


def stretch_gradient(ps, X0: np.ndarray, nsteps: int, K0: np.ndarray):
    """Pathwise gradient of J = mean_stretch after nsteps rigid-rod steps of
    the chains X0 (C x N x 3; chain c with parameters ps[c], noise fixed by
    their seeds) with respect to h* and to the rate e of kappa = e K0 (each
    ps[c] holds its own kappa; the derivative is taken along K0).  Every
    state is kept; the adjoint runs the steps backwards with step_adjoint.
    Returns (J, dJ/dh*, dJ/de)."""
    X0 = np.asarray(X0, dtype=np.float64)
    C_, N = X0.shape[0], X0.shape[1]
    b = ps[0].b
    Xf = np.zeros_like(X0)
    gh = ge = 0.0
    for c in range(C_):
        states = [X0[c].copy()]
        for s in range(nsteps):
            xn, info = step(ps[c], s, states[-1])
            if info["status"] != OK:
                raise ValueError(f"chain {c} step {s}: status {info['status']}")
            states.append(xn)
        Xf[c] = states[-1]
        R = states[-1][-1] - states[-1][0]
        xbar = np.zeros((N, 3))
        g = R / np.linalg.norm(R) / ((N - 1) * b * C_)
        xbar[-1] += g
        xbar[0] -= g
        for s in range(nsteps - 1, -1, -1):
            xbar, hb, kb = step_adjoint(ps[c], s, states[s], xbar)
            gh += hb
            ge += float(np.sum(kb * K0))
    return mean_stretch(Xf, b), gh, ge


def step_adjoint(p: Params, s: int, x: np.ndarray, xbar_next: np.ndarray):
    """Reverse-mode derivative of one rigid-rod step (``step``, the scheme of
    Eq. 6 with the tensions of the constraint solve) at fixed noise: for the
    gradient xbar_next of a scalar in x^{t+dt}, returns (xbar, hbar, kbar),
    its gradients in x^t (N x 3), h* and kappa (3 x 3).

    The forward parts are recomputed with the oracle's own routines: D(x)
    (Eqs. 7-9), L (Eq. 10), xi and y = c_B L xi, the predictor x* = x +
    dt kappa x + y, the tensions T and x^{t+dt} = x* + dt D f, f_i = T_i u_i
    - T_{i-1} u_{i-1}, u the rod directions at x^t.  T is defined
    implicitly by g_k = |Q_k|^2 - b^2 = 0 with Q = Delta x^{t+dt}; by the
    implicit-function theorem the step's gradient is that of x^{t+dt} at
    fixed T applied to z = xbar_next - 2 Delta^T (Q mu), where mu solves
    J^T mu = (d x^{t+dt}/dT)^T xbar_next with the dense Jacobian
    J = dg/dT = -2 dt diag(Q)^T Delta D Delta^T U (numpy LU).  z is then
    carried through x*, the product D f (in D and in u) and the noise
    product (the Cholesky adjoint above, then the assembly's adjoint)."""
    N = p.n_beads
    M = N - 1
    dt = p.dt
    kap = np.array([p.kappa[e] for e in range(9)]).reshape(3, 3)
    cB = np.sqrt(6.0 * dt) if p.noise == NOISE_UNIFORM_PAPER else np.sqrt(2.0 * dt)
    x = np.asarray(x, dtype=np.float64)
    xb = np.asarray(xbar_next, dtype=np.float64).reshape(N, 3)
    # forward, recomputed
    D = np.array(rpy_assemble(p, x, FILL_FULL))
    L, info = cholesky(D)
    if info != 0:
        raise ValueError(f"bdo_cholesky info {info}")
    L = np.tril(L)
    y, xi = brownian(p, s, L)
    xs = x + dt * x @ kap.T + y.reshape(N, 3)
    xnew, T, inf = constrain(p, x, xs)
    if inf["status"] != OK:
        raise ValueError(f"bdo_constrain status {inf['status']}")
    q = np.diff(x, axis=0)
    ql = np.linalg.norm(q, axis=1)
    u = q / ql[:, None]
    f = np.zeros((N, 3))
    f[:M] += T[:, None] * u
    f[1:] -= T[:, None] * u
    z = constrain_adjoint(p, x, xnew, xb, D=D).ravel()
    # x^{t+dt} = x* + dt D(x) f(T, u(x)) at fixed T
    Dbar = dt * np.outer(z, f.ravel())
    fbar = (dt * D @ z).reshape(N, 3)
    ubar = T[:, None] * (fbar[:M] - fbar[1:])
    qbar = (ubar - u * np.sum(u * ubar, axis=1)[:, None]) / ql[:, None]
    xbar = np.zeros((N, 3))
    xbar[1:] += qbar
    xbar[:M] -= qbar
    # x* = x + dt kappa x + c_B L xi
    zs = z.reshape(N, 3)
    xbar += zs + dt * zs @ kap
    kbar = dt * zs.T @ x
    Lbar = cB * np.tril(np.outer(z, xi))
    Dbar += cholesky_adjoint(L, Lbar)
    xd, hbar = rpy_assemble_adjoint(p, x, Dbar)
    return xbar + xd, float(hbar), kbar


def run(p: Params, step0: int, nsteps: int, x: np.ndarray):
    xx = np.array(x, dtype=np.float64, order="C", copy=True)
    info = Info()
    lib().bdo_run(C.byref(p), step0, nsteps, _dp(xx), C.byref(info))
    return xx, info.as_dict()


def run_many(p: Params, chain_ids, step0: int, nsteps: int, X: np.ndarray):
    """X: (nchains, N, 3), advanced in place on a copy; returns (X, status)."""
    XX = np.array(X, dtype=np.float64, order="C", copy=True)
    ids = np.ascontiguousarray(chain_ids, dtype=np.uint64)
    st = np.zeros(len(ids), dtype=np.int32)
    lib().bdo_run_many(C.byref(p), len(ids), ids.ctypes.data_as(C.POINTER(C.c_uint64)), step0,
                       nsteps, _dp(XX), st.ctypes.data_as(C.POINTER(C.c_int32)))
    return XX, st


def num_threads() -> int:
    return int(lib().bdo_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().bdo_set_num_threads(int(n))
