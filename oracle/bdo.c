/*
 * bdo.c -- plain CPU FP64 oracle for bead-rod Brownian dynamics with RPY
 * hydrodynamic interactions (arXiv 2208.06559).
 *
 * TEST INFRASTRUCTURE ONLY: the HIP library never includes, links or calls
 * this code.  Every routine is written for clarity, not speed: no blocking,
 * no fusion, no reordering beyond what the definition it follows states.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *  - N counts beads; the paper's beads 0..N are our 0..N-1.
 *  - Rods are rigid: the stiff Fraenkel spring of Eq. 3 is replaced by its
 *    infinite-stiffness limit, a tension T_k along the bond direction at the
 *    start of the step, solved implicitly through the full diffusion tensor
 *    (the K* -> infinity limit of the semi-implicit update of Eqs. 13-17).
 *    bdo_step_fraenkel keeps the paper's finite-stiffness springs and its
 *    semi-implicit link update instead; there bead 0 moves by its explicit
 *    equation of motion and the other beads follow along the new links
 *    (the paper integrates link vectors and is silent on positions).
 *  - The bead radius a is a parameter separate from h* (a = b/2 in every
 *    workload); h* <= a keeps D positive definite.
 *  - Noise is Gaussian by default (covariance 2 dt D); the paper's uniform
 *    noise of Eq. 2 (covariance 2 dt D as well) is a flag.
 */
#include "bdo.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x64-10, Salmon et al., "Parallel random numbers: as easy as  */
/* 1, 2, 3", SC'11: 10 rounds of two 64x64->128 multiplies, with the    */
/* Weyl key schedule between rounds.                                    */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL /* golden ratio */
#define PHILOX_W1 0xBB67AE8584CAA73BULL /* sqrt(3) - 1  */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(prod >> 64);
  *lo = (uint64_t)prod;
}

void bdo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(PHILOX_M0, c0, &hi0, &lo0);
    mulhilo64(PHILOX_M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53 random bits to the open interval (0,1): ((w >> 11) + 1/2) * 2^-53. */
static double u01_open(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

void bdo_noise(const bdo_params* p, int64_t step, int64_t n, double* xi) {
  const double two_pi = 6.283185307179586476925286766559;
  uint64_t key[2] = {p->seed, p->chain_id};
  for (int64_t blk = 0; blk * 4 < n; ++blk) {
    uint64_t ctr[4] = {(uint64_t)blk, (uint64_t)step, (uint64_t)BDO_PURPOSE_NOISE, 0};
    uint64_t w[4];
    bdo_philox4x64_10(ctr, key, w);
    double u[4];
    for (int l = 0; l < 4; ++l) u[l] = u01_open(w[l]);
    double z[4];
    if (p->noise == BDO_NOISE_UNIFORM_PAPER) {
      /* Eq. 2: each component uniform on [-1, 1]. */
      for (int l = 0; l < 4; ++l) z[l] = 2.0 * u[l] - 1.0;
    } else {
      /* Box-Muller (1958) on the pairs (u0,u1) and (u2,u3). */
      for (int pr = 0; pr < 2; ++pr) {
        double rad = sqrt(-2.0 * log(u[2 * pr]));
        double ang = two_pi * u[2 * pr + 1];
        z[2 * pr] = rad * cos(ang);
        z[2 * pr + 1] = rad * sin(ang);
      }
    }
    for (int l = 0; l < 4; ++l)
      if (blk * 4 + l < n) xi[blk * 4 + l] = z[l];
  }
}

/* ------------------------------------------------------------------ */
/* RPY tensor, Eqs. 7-9.                                                */
/* ------------------------------------------------------------------ */
void bdo_rpy_block(double hstar, double a, const double Rv[3], double out[9]) {
  double R2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
  double R = sqrt(R2);
  double cI, cRR; /* D_ij = cI * I + cRR * Rvec Rvec^T */
  if (R >= 2.0 * a) {
    /* Eq. 8: (3 hstar/4R) [ (1 + 2a^2/3R^2) I + (1 - 2a^2/R^2) RR/R^2 ] */
    double pre = 3.0 * hstar / (4.0 * R);
    cI = pre * (1.0 + 2.0 * a * a / (3.0 * R2));
    cRR = pre * (1.0 - 2.0 * a * a / R2) / R2;
  } else {
    /* Eq. 9: (3 hstar/4R)(R/2a) [ (8/3 - 3R/4a) I + (R/4a) RR/R^2 ];
     * (3 hstar/4R)(R/2a) = 3 hstar/8a, and (R/4a) RR/R^2 = RR/(4aR), which
     * is taken as 0 at R = 0 (the limit of the I term alone). */
    double pre = 3.0 * hstar / (8.0 * a);
    cI = pre * (8.0 / 3.0 - 3.0 * R / (4.0 * a));
    cRR = (R > 0.0) ? pre / (4.0 * a * R) : 0.0;
  }
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be)
      out[3 * al + be] = (al == be ? cI : 0.0) + cRR * Rv[al] * Rv[be];
}

/* D_ij: identity on the diagonal (Eq. 7), RPY block otherwise. */
static void diffusion_block(const bdo_params* p, const double* x, int64_t i, int64_t j,
                            double out[9]) {
  if (i == j) {
    for (int e = 0; e < 9; ++e) out[e] = (e % 4 == 0) ? 1.0 : 0.0;
    return;
  }
  double Rv[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
  bdo_rpy_block(p->hstar, p->a, Rv, out);
}

static int params_valid(const bdo_params* p) {
  if (!p) return 0;
  if (p->n_beads < 2) return 0;
  if (!(p->b > 0.0) || !isfinite(p->b)) return 0;
  if (!(p->a > 0.0) || !isfinite(p->a)) return 0;
  if (!(p->dt > 0.0) || !isfinite(p->dt)) return 0;
  if (!(p->hstar >= 0.0) || !(p->hstar <= p->a)) return 0;
  if (p->noise != BDO_NOISE_GAUSSIAN && p->noise != BDO_NOISE_UNIFORM_PAPER) return 0;
  if (!(p->newton_tol > 0.0) || !isfinite(p->newton_tol)) return 0;
  if (p->newton_maxit < 1) return 0;
  for (int e = 0; e < 9; ++e)
    if (!isfinite(p->kappa[e])) return 0;
  return 1;
}

int bdo_rpy_assemble(const bdo_params* p, const double* x, double* D, int64_t ld, int32_t fill) {
  if (!params_valid(p) || !x || !D) return BDO_ERR_PARAM;
  const int64_t N = p->n_beads, n = 3 * N;
  if (ld < n || (fill != BDO_FILL_LOWER && fill != BDO_FILL_FULL)) return BDO_ERR_PARAM;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    for (int64_t i = 0; i < N; ++i) {
      double blk[9];
      diffusion_block(p, x, i, j, blk);
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) {
          int64_t row = 3 * i + al, col = 3 * j + be;
          if (fill == BDO_FILL_LOWER && row < col) continue;
          D[col * ld + row] = blk[3 * al + be];
        }
    }
  }
  return BDO_OK;
}

/* ------------------------------------------------------------------ */
/* Cholesky, Eq. 10: D = L L^T with L lower and positive diagonal.      */
/* Crout order, column j = 0..n-1:                                      */
/*   L_jj = sqrt(A_jj - sum_{k<j} L_jk^2)                               */
/*   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj,  i > j                 */
/* The lower triangle is copied to row-major packed storage so that the */
/* sums run over contiguous memory, then copied back.                   */
/* ------------------------------------------------------------------ */
int64_t bdo_cholesky(int64_t n, double* A, int64_t ld) {
  if (n < 0 || ld < n || (n > 0 && !A)) return -1;
  if (n == 0) return 0;
  double* P = (double*)malloc(sizeof(double) * (size_t)(n * (n + 1) / 2));
  if (!P) return -1;
#define ROW(i) (P + (i) * ((i) + 1) / 2)
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k <= i; ++k) ROW(i)[k] = A[k * ld + i];

  int64_t info = 0;
  for (int64_t j = 0; j < n; ++j) {
    double* Lj = ROW(j);
    double s = 0.0;
#pragma omp simd reduction(+ : s)
    for (int64_t k = 0; k < j; ++k) s += Lj[k] * Lj[k];
    double piv = Lj[j] - s;
    if (!(piv > 0.0)) {
      info = j + 1;
      break;
    }
    double d = sqrt(piv);
    Lj[j] = d;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      double* Li = ROW(i);
      double t = 0.0;
#pragma omp simd reduction(+ : t)
      for (int64_t k = 0; k < j; ++k) t += Li[k] * Lj[k];
      Li[j] = (Li[j] - t) / d;
    }
  }
  if (info == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k <= i; ++k) A[k * ld + i] = ROW(i)[k];
  }
#undef ROW
  free(P);
  return info;
}

/* ------------------------------------------------------------------ */
/* Brownian displacement: the noise term of Eq. 6 times dt.             */
/* ------------------------------------------------------------------ */
static double noise_scale(const bdo_params* p) {
  return (p->noise == BDO_NOISE_UNIFORM_PAPER) ? sqrt(6.0 * p->dt) : sqrt(2.0 * p->dt);
}

int bdo_brownian(const bdo_params* p, int64_t step, const double* L, int64_t ld, double* y,
                 double* xi_out) {
  if (!params_valid(p) || !L || !y) return BDO_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  if (ld < n) return BDO_ERR_PARAM;
  double* xi = (double*)malloc(sizeof(double) * (size_t)n);
  if (!xi) return BDO_ERR_PARAM;
  bdo_noise(p, step, n, xi);
  const double c = noise_scale(p);
  /* y_i = c * sum_{j <= i} L_ij xi_j, j ascending (Eq. 6: sigma is lower). */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j <= i; ++j) s += L[j * ld + i] * xi[j];
    y[i] = c * s;
  }
  if (xi_out) memcpy(xi_out, xi, sizeof(double) * (size_t)n);
  free(xi);
  return BDO_OK;
}

/* ------------------------------------------------------------------ */
/* Rigid-rod tension solve.                                             */
/* f = -Delta^T U T (f_i = T_i u_i - T_{i-1} u_{i-1}), r = D f,         */
/* Q_k(T) = Q*_k + dt (r_{k+1} - r_k) = Q*_k - dt sum_l G_kl u_l T_l,   */
/* G_kl = D_{k+1,l+1} - D_{k+1,l} - D_{k,l+1} + D_{k,l}  (the row       */
/* differences of D that Eqs. 11-12 apply to the spring forces).        */
/* Find T with g_k = |Q_k|^2 - b^2 = 0;  dg_k/dT_l = -2 dt Q_k.G_kl u_l. */
/* ------------------------------------------------------------------ */
static void G_times(const bdo_params* p, const double* x, int64_t k, int64_t l, const double v[3],
                    double out[3]) {
  double B[9], acc[9];
  for (int e = 0; e < 9; ++e) acc[e] = 0.0;
  diffusion_block(p, x, k + 1, l + 1, B);
  for (int e = 0; e < 9; ++e) acc[e] += B[e];
  diffusion_block(p, x, k + 1, l, B);
  for (int e = 0; e < 9; ++e) acc[e] -= B[e];
  diffusion_block(p, x, k, l + 1, B);
  for (int e = 0; e < 9; ++e) acc[e] -= B[e];
  diffusion_block(p, x, k, l, B);
  for (int e = 0; e < 9; ++e) acc[e] += B[e];
  for (int al = 0; al < 3; ++al)
    out[al] = acc[3 * al] * v[0] + acc[3 * al + 1] * v[1] + acc[3 * al + 2] * v[2];
}

/* r = D(x) f, matrix-free, j ascending. */
static void D_times(const bdo_params* p, const double* x, const double* f, double* r) {
  const int64_t N = p->n_beads;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      double B[9];
      diffusion_block(p, x, i, j, B);
      s0 += B[0] * f[3 * j] + B[1] * f[3 * j + 1] + B[2] * f[3 * j + 2];
      s1 += B[3] * f[3 * j] + B[4] * f[3 * j + 1] + B[5] * f[3 * j + 2];
      s2 += B[6] * f[3 * j] + B[7] * f[3 * j + 1] + B[8] * f[3 * j + 2];
    }
    r[3 * i] = s0;
    r[3 * i + 1] = s1;
    r[3 * i + 2] = s2;
  }
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Thomas algorithm for sub/diag/super (lo, di, up), rhs overwritten. */
static void thomas(int64_t M, const double* lo, const double* di, const double* up, double* rhs,
                   double* work) {
  double* cp = work;
  double w = di[0];
  cp[0] = (M > 1) ? up[0] / w : 0.0;
  rhs[0] = rhs[0] / w;
  for (int64_t k = 1; k < M; ++k) {
    w = di[k] - lo[k] * cp[k - 1];
    cp[k] = (k < M - 1) ? up[k] / w : 0.0;
    rhs[k] = (rhs[k] - lo[k] * rhs[k - 1]) / w;
  }
  for (int64_t k = M - 2; k >= 0; --k) rhs[k] -= cp[k] * rhs[k + 1];
}

/* Dense LU with partial pivoting, A (M x M row-major) and rhs overwritten. */
static int lu_solve(int64_t M, double* A, double* rhs) {
  for (int64_t c = 0; c < M; ++c) {
    int64_t piv = c;
    for (int64_t r = c + 1; r < M; ++r)
      if (fabs(A[r * M + c]) > fabs(A[piv * M + c])) piv = r;
    if (A[piv * M + c] == 0.0) return 1;
    if (piv != c) {
      for (int64_t k = 0; k < M; ++k) {
        double t = A[c * M + k]; A[c * M + k] = A[piv * M + k]; A[piv * M + k] = t;
      }
      double t = rhs[c]; rhs[c] = rhs[piv]; rhs[piv] = t;
    }
    for (int64_t r = c + 1; r < M; ++r) {
      double m = A[r * M + c] / A[c * M + c];
      for (int64_t k = c; k < M; ++k) A[r * M + k] -= m * A[c * M + k];
      rhs[r] -= m * rhs[c];
    }
  }
  for (int64_t r = M - 1; r >= 0; --r) {
    double s = rhs[r];
    for (int64_t k = r + 1; k < M; ++k) s -= A[r * M + k] * rhs[k];
    rhs[r] = s / A[r * M + r];
  }
  return 0;
}

/* Band part of the Jacobian at the current Q: lo/di/up of J_kl for
 * l = k-1, k, k+1. */
static void band_jacobian(int64_t M, double dt, const double* Q, const double* Gd,
                          const double* Gp, const double* Gm, double* lo, double* di, double* up) {
  for (int64_t k = 0; k < M; ++k) {
    di[k] = -2.0 * dt * dot3(Q + 3 * k, Gd + 3 * k);
    up[k] = (k + 1 < M) ? -2.0 * dt * dot3(Q + 3 * k, Gp + 3 * k) : 0.0;
    lo[k] = (k > 0) ? -2.0 * dt * dot3(Q + 3 * k, Gm + 3 * k) : 0.0;
  }
}

/* f(z)_i = z_i u_i - z_{i-1} u_{i-1}: the bead forces of rod tensions z. */
static void rod_forces(int64_t N, const double* u, const double* z, double* f) {
  const int64_t M = N - 1;
  for (int64_t i = 0; i < N; ++i)
    for (int al = 0; al < 3; ++al) {
      double v = 0.0;
      if (i < M) v += z[i] * u[3 * i + al];
      if (i > 0) v -= z[i - 1] * u[3 * (i - 1) + al];
      f[3 * i + al] = v;
    }
}

/* Jacobian-vector product: (J z)_k = -2 dt Q_k . (G U z)_k with
 * G U z = Delta D Delta^T U z = -Delta D f(z), i.e.
 * (J z)_k = 2 dt Q_k . (r_{k+1} - r_k),  r = D f(z). */
static void jacobian_apply(const bdo_params* p, const double* x_old, const double* u,
                           const double* Q, const double* z, double* f, double* r, double* out) {
  const int64_t N = p->n_beads, M = N - 1;
  rod_forces(N, u, z, f);
  D_times(p, x_old, f, r);
  for (int64_t k = 0; k < M; ++k) {
    double dr[3] = {r[3 * (k + 1)] - r[3 * k], r[3 * (k + 1) + 1] - r[3 * k + 1],
                    r[3 * (k + 1) + 2] - r[3 * k + 2]};
    out[k] = 2.0 * p->dt * dot3(Q + 3 * k, dr);
  }
}

static double dotM(int64_t M, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t k = 0; k < M; ++k) s += a[k] * b[k];
  return s;
}

/* GMRES (Saad & Schultz 1986) for J delta = rhs, right-preconditioned by the
 * tridiagonal band P of J (Thomas), modified Gram-Schmidt Arnoldi, Givens
 * rotations; stops when the residual norm falls below eta * |rhs| or after
 * kmax iterations.  Returns the iterations used; delta is overwritten. */
static int gmres_band(const bdo_params* p, const double* x_old, const double* u, const double* Q,
                      const double* lo, const double* di, const double* up, const double* rhs,
                      double eta, int kmax, double* delta) {
  const int64_t N = p->n_beads, M = N - 1;
  double* V = (double*)calloc((size_t)((kmax + 1) * M), sizeof(double));
  double* H = (double*)calloc((size_t)((kmax + 1) * kmax), sizeof(double)); /* H[i*kmax + j] */
  double* cs = (double*)calloc((size_t)kmax, sizeof(double));
  double* sn = (double*)calloc((size_t)kmax, sizeof(double));
  double* s = (double*)calloc((size_t)(kmax + 1), sizeof(double));
  double* z = (double*)calloc((size_t)M, sizeof(double));
  double* w = (double*)calloc((size_t)M, sizeof(double));
  double* work = (double*)calloc((size_t)M, sizeof(double));
  double* f = (double*)calloc((size_t)(3 * N), sizeof(double));
  double* r = (double*)calloc((size_t)(3 * N), sizeof(double));
  double beta = sqrt(dotM(M, rhs, rhs));
  int k = 0;
  for (int64_t e = 0; e < M; ++e) delta[e] = 0.0;
  if (beta > 0.0) {
    for (int64_t e = 0; e < M; ++e) V[e] = rhs[e] / beta;
    s[0] = beta;
    for (int j = 0; j < kmax; ++j) {
      /* w = J P^{-1} v_j */
      memcpy(z, V + j * M, sizeof(double) * (size_t)M);
      thomas(M, lo, di, up, z, work);
      jacobian_apply(p, x_old, u, Q, z, f, r, w);
      for (int i = 0; i <= j; ++i) {
        double h = dotM(M, w, V + i * M);
        H[i * kmax + j] = h;
        for (int64_t e = 0; e < M; ++e) w[e] -= h * V[i * M + e];
      }
      double hn = sqrt(dotM(M, w, w));
      H[(j + 1) * kmax + j] = hn;
      if (hn > 0.0)
        for (int64_t e = 0; e < M; ++e) V[(j + 1) * M + e] = w[e] / hn;
      for (int i = 0; i < j; ++i) {
        double a0 = H[i * kmax + j], a1 = H[(i + 1) * kmax + j];
        H[i * kmax + j] = cs[i] * a0 + sn[i] * a1;
        H[(i + 1) * kmax + j] = -sn[i] * a0 + cs[i] * a1;
      }
      double a0 = H[j * kmax + j], a1 = H[(j + 1) * kmax + j];
      double den = sqrt(a0 * a0 + a1 * a1);
      cs[j] = (den > 0.0) ? a0 / den : 1.0;
      sn[j] = (den > 0.0) ? a1 / den : 0.0;
      H[j * kmax + j] = den;
      H[(j + 1) * kmax + j] = 0.0;
      s[j + 1] = -sn[j] * s[j];
      s[j] = cs[j] * s[j];
      k = j + 1;
      if (fabs(s[j + 1]) <= eta * beta || hn == 0.0) break;
    }
    /* y = H^{-1} s (upper triangular), delta = P^{-1} V y */
    double* y = (double*)calloc((size_t)k, sizeof(double));
    for (int i = k - 1; i >= 0; --i) {
      double t = s[i];
      for (int c = i + 1; c < k; ++c) t -= H[i * kmax + c] * y[c];
      y[i] = t / H[i * kmax + i];
    }
    for (int i = 0; i < k; ++i)
      for (int64_t e = 0; e < M; ++e) delta[e] += y[i] * V[i * M + e];
    thomas(M, lo, di, up, delta, work);
    free(y);
  }
  free(V); free(H); free(cs); free(sn); free(s); free(z); free(w); free(work); free(f); free(r);
  return k;
}

#define BDO_GMRES_KMAX 60

static int constrain_impl(const bdo_params* p, const double* x_old, double* xs, double* T_out,
                          bdo_info* info, int dense) {
  if (!params_valid(p) || !x_old || !xs) return BDO_ERR_PARAM;
  const int64_t N = p->n_beads, M = N - 1;
  const double dt = p->dt, b = p->b;
  double* u = (double*)calloc((size_t)(3 * M), sizeof(double));
  double* Qs = (double*)calloc((size_t)(3 * M), sizeof(double));
  double* Q = (double*)calloc((size_t)(3 * M), sizeof(double));
  double* T = (double*)calloc((size_t)M, sizeof(double));
  double* f = (double*)calloc((size_t)(3 * N), sizeof(double));
  double* r = (double*)calloc((size_t)(3 * N), sizeof(double));
  double* Gd = (double*)calloc((size_t)(3 * M), sizeof(double)); /* G_kk u_k       */
  double* Gp = (double*)calloc((size_t)(3 * M), sizeof(double)); /* G_k,k+1 u_k+1  */
  double* Gm = (double*)calloc((size_t)(3 * M), sizeof(double)); /* G_k,k-1 u_k-1  */
  double* lo = (double*)calloc((size_t)M, sizeof(double));
  double* di = (double*)calloc((size_t)M, sizeof(double));
  double* up = (double*)calloc((size_t)M, sizeof(double));
  double* rhs = (double*)calloc((size_t)M, sizeof(double));
  double* dlt = (double*)calloc((size_t)M, sizeof(double));
  double* J = dense ? (double*)calloc((size_t)(M * M), sizeof(double)) : NULL;

  for (int64_t k = 0; k < M; ++k) {
    double q[3];
    for (int al = 0; al < 3; ++al) q[al] = x_old[3 * (k + 1) + al] - x_old[3 * k + al];
    double nq = sqrt(dot3(q, q));
    for (int al = 0; al < 3; ++al) {
      u[3 * k + al] = q[al] / nq;
      Qs[3 * k + al] = xs[3 * (k + 1) + al] - xs[3 * k + al];
    }
  }
  if (!dense) {
    for (int64_t k = 0; k < M; ++k) {
      G_times(p, x_old, k, k, u + 3 * k, Gd + 3 * k);
      if (k + 1 < M) G_times(p, x_old, k, k + 1, u + 3 * (k + 1), Gp + 3 * k);
      if (k > 0) G_times(p, x_old, k, k - 1, u + 3 * (k - 1), Gm + 3 * k);
    }
  }

  int status = BDO_ERR_NO_CONVERGE;
  int iters = 0, kry = 0;
  double err = 0.0, res = 0.0;
  for (int it = 0;; ++it) {
    /* residual at T: f(T), r = D f, Q(T) = Q* + dt (r_{k+1} - r_k) */
    rod_forces(N, u, T, f);
    D_times(p, x_old, f, r);
    err = 0.0;
    res = 0.0;
    double g2 = 0.0;
    for (int64_t k = 0; k < M; ++k) {
      for (int al = 0; al < 3; ++al)
        Q[3 * k + al] = Qs[3 * k + al] + dt * (r[3 * (k + 1) + al] - r[3 * k + al]);
      double q2 = dot3(Q + 3 * k, Q + 3 * k);
      double e = fabs(sqrt(q2) / b - 1.0);
      if (e > err || isnan(e)) err = e;
      double g = q2 - b * b;
      rhs[k] = -g;
      g2 += g * g;
      if (fabs(g) > res || isnan(g)) res = fabs(g);
    }
    iters = it;
    if (err <= p->newton_tol) {
      status = BDO_OK;
      break;
    }
    if (it >= p->newton_maxit || !isfinite(err)) break;
    if (!dense) {
      /* Inexact Newton: relative GMRES tolerance eta balances the quadratic
       * term of g against the linear-solve error (g is quadratic in T), and
       * is never tighter than the final tolerance requires. */
      double grms = sqrt(g2 / (double)M) / (b * b);
      double eta = 0.25 * grms;
      double floor_eta = 0.5 * p->newton_tol / grms;
      if (eta < floor_eta) eta = floor_eta;
      if (eta > 0.1) eta = 0.1;
      band_jacobian(M, dt, Q, Gd, Gp, Gm, lo, di, up);
      kry += gmres_band(p, x_old, u, Q, lo, di, up, rhs, eta, BDO_GMRES_KMAX, dlt);
    } else {
      for (int64_t k = 0; k < M; ++k)
        for (int64_t l = 0; l < M; ++l) {
          double gu[3];
          G_times(p, x_old, k, l, u + 3 * l, gu);
          J[k * M + l] = -2.0 * dt * dot3(Q + 3 * k, gu);
        }
      memcpy(dlt, rhs, sizeof(double) * (size_t)M);
      if (lu_solve(M, J, dlt)) break;
    }
    for (int64_t k = 0; k < M; ++k) T[k] += dlt[k];
  }
  /* Corrector: x^{t+dt} = x* + dt D f(T). */
  for (int64_t e = 0; e < 3 * N; ++e) xs[e] += dt * r[e];
  if (T_out) memcpy(T_out, T, sizeof(double) * (size_t)M);
  if (info) {
    info->status = status;
    info->newton_iters = iters;
    info->krylov_iters = kry;
    info->max_rod_err = err;
    info->last_newton_res = res;
  }
  free(u); free(Qs); free(Q); free(T); free(f); free(r); free(Gd); free(Gp); free(Gm);
  free(lo); free(di); free(up); free(rhs); free(dlt); free(J);
  return status;
}

int bdo_constrain(const bdo_params* p, const double* x_old, double* x_pred_inout, double* T_out,
                  bdo_info* info) {
  return constrain_impl(p, x_old, x_pred_inout, T_out, info, 0);
}

int bdo_constrain_dense(const bdo_params* p, const double* x_old, double* x_pred_inout,
                        double* T_out, bdo_info* info) {
  return constrain_impl(p, x_old, x_pred_inout, T_out, info, 1);
}

/* ------------------------------------------------------------------ */
/* One step: D(x) (Eqs. 7-9), L (Eq. 10), y = c L xi (Eq. 6 noise),    */
/* predictor x* = x + dt kappa.x + y (Eqs. 5-6), tension + corrector.    */
/* ------------------------------------------------------------------ */
int bdo_step(const bdo_params* p, int64_t step, double* x, bdo_info* info) {
  bdo_info loc;
  memset(&loc, 0, sizeof loc);
  if (!params_valid(p) || !x) {
    loc.status = BDO_ERR_PARAM;
    if (info) *info = loc;
    return BDO_ERR_PARAM;
  }
  const int64_t N = p->n_beads, n = 3 * N;
  double* D = (double*)malloc(sizeof(double) * (size_t)(n * n));
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  double* xs = (double*)malloc(sizeof(double) * (size_t)n);
  bdo_rpy_assemble(p, x, D, n, BDO_FILL_LOWER);
  loc.potrf_info = bdo_cholesky(n, D, n);
  if (loc.potrf_info != 0) {
    loc.status = BDO_ERR_NOT_SPD;
  } else {
    bdo_brownian(p, step, D, n, y, NULL);
    for (int64_t i = 0; i < N; ++i)
      for (int al = 0; al < 3; ++al) {
        double kx = p->kappa[3 * al] * x[3 * i] + p->kappa[3 * al + 1] * x[3 * i + 1] +
                    p->kappa[3 * al + 2] * x[3 * i + 2];
        xs[3 * i + al] = x[3 * i + al] + p->dt * kx + y[3 * i + al];
      }
    int64_t pinfo = loc.potrf_info;
    bdo_constrain(p, x, xs, NULL, &loc);
    loc.potrf_info = pinfo;
    memcpy(x, xs, sizeof(double) * (size_t)n);
  }
  free(D); free(y); free(xs);
  if (info) *info = loc;
  return loc.status;
}

/* ------------------------------------------------------------------ */
/* Stiff Fraenkel springs, semi-implicit (Eqs. 3, 13-17).               */
/* ------------------------------------------------------------------ */
int bdo_step_fraenkel(const bdo_params* p, double k_spring, int64_t step, double* x,
                      bdo_info* info) {
  bdo_info loc;
  memset(&loc, 0, sizeof loc);
  if (!params_valid(p) || !x || !(k_spring > 0.0) || !isfinite(k_spring)) {
    loc.status = BDO_ERR_PARAM;
    if (info) *info = loc;
    return BDO_ERR_PARAM;
  }
  const int64_t N = p->n_beads, n = 3 * N, M = N - 1;
  const double dt = p->dt, b = p->b, K = k_spring;
  double* D = (double*)malloc(sizeof(double) * (size_t)(n * n));
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  double* F = (double*)malloc(sizeof(double) * (size_t)(3 * M));
  double* f = (double*)malloc(sizeof(double) * (size_t)n);
  double* v = (double*)malloc(sizeof(double) * (size_t)n);
  double* Qn = (double*)malloc(sizeof(double) * (size_t)(3 * M));
  bdo_rpy_assemble(p, x, D, n, BDO_FILL_LOWER);
  loc.potrf_info = bdo_cholesky(n, D, n);
  if (loc.potrf_info != 0) {
    loc.status = BDO_ERR_NOT_SPD;
  } else {
    bdo_brownian(p, step, D, n, y, NULL);
    /* spring forces at t (Eq. 3) and the net force on each bead */
    for (int64_t k = 0; k < M; ++k) {
      const double* q = x + 3 * (k + 1);
      const double Q[3] = {q[0] - x[3 * k], q[1] - x[3 * k + 1], q[2] - x[3 * k + 2]};
      const double len = sqrt(dot3(Q, Q));
      for (int al = 0; al < 3; ++al) F[3 * k + al] = K * (len - b) * Q[al] / len;
    }
    for (int64_t i = 0; i < N; ++i)
      for (int al = 0; al < 3; ++al)
        f[3 * i + al] = (i < M ? F[3 * i + al] : 0.0) - (i > 0 ? F[3 * (i - 1) + al] : 0.0);
    D_times(p, x, f, v);
    /* Eq. 14, then the closed form of Eqs. 15-17 per link */
    double err = 0.0;
    for (int64_t k = 0; k < M; ++k) {
      double Y[3];
      for (int al = 0; al < 3; ++al) {
        const double Q = x[3 * (k + 1) + al] - x[3 * k + al];
        double kQ = 0.0;
        for (int be = 0; be < 3; ++be)
          kQ += p->kappa[3 * al + be] * (x[3 * (k + 1) + be] - x[3 * k + be]);
        Y[al] = Q + dt * (kQ + v[3 * (k + 1) + al] - v[3 * k + al] + 2.0 * F[3 * k + al]) +
                (y[3 * (k + 1) + al] - y[3 * k + al]);
      }
      const double ylen = sqrt(dot3(Y, Y));
      const double qlen = (ylen + 2.0 * dt * K * b) / (1.0 + 2.0 * dt * K);
      for (int al = 0; al < 3; ++al) Qn[3 * k + al] = Y[al] * (qlen / ylen);
      const double e = fabs(qlen / b - 1.0);
      if (e > err) err = e;
    }
    /* bead 0 by its explicit equation of motion, the rest along the links */
    double x0[3];
    for (int al = 0; al < 3; ++al) {
      const double kx = p->kappa[3 * al] * x[0] + p->kappa[3 * al + 1] * x[1] +
                        p->kappa[3 * al + 2] * x[2];
      x0[al] = x[al] + dt * (kx + v[al]) + y[al];
    }
    for (int al = 0; al < 3; ++al) x[al] = x0[al];
    for (int64_t k = 0; k < M; ++k)
      for (int al = 0; al < 3; ++al) x[3 * (k + 1) + al] = x[3 * k + al] + Qn[3 * k + al];
    loc.max_rod_err = err;
  }
  free(D); free(y); free(F); free(f); free(v); free(Qn);
  if (info) *info = loc;
  return loc.status;
}

int bdo_run(const bdo_params* p, int64_t step0, int64_t nsteps, double* x, bdo_info* info) {
  int st = BDO_OK;
  for (int64_t s = 0; s < nsteps; ++s) {
    st = bdo_step(p, step0 + s, x, info);
    if (st != BDO_OK) break;
  }
  return st;
}

int bdo_run_many(const bdo_params* p, int32_t nchains, const uint64_t* chain_ids, int64_t step0,
                 int64_t nsteps, double* x, int32_t* status_out) {
  if (!params_valid(p) || nchains < 0 || !chain_ids || !x) return BDO_ERR_PARAM;
  const int64_t n = 3 * (int64_t)p->n_beads;
  int worst = BDO_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst)
  for (int32_t c = 0; c < nchains; ++c) {
    bdo_params pc = *p;
    pc.chain_id = chain_ids[c];
    bdo_info inf;
    int st = bdo_run(&pc, step0, nsteps, x + c * n, &inf);
    if (status_out) status_out[c] = st;
    if (st > worst) worst = st;
  }
  return worst;
}

int bdo_num_threads(void) { return omp_get_max_threads(); }

/* Threads of the oracle's parallel loops from now on (timing only). */
void bdo_set_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
