/*
 * CPU oracle for the Schur-complement + PCG linear solve of one NMPC step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may call
 * this file; it exists so that tests, the smoke check and the benchmark's CPU
 * baseline can compare the GPU path against a plain, slow, obviously correct
 * implementation.  It shares no code, header or constant with the GPU path.
 *
 * Everything is IEEE double precision, plain loops, no blocking or fusion.
 *
 * Conventions (MPCGPU, Section III "Background"):
 *   N state knots x_0..x_{N-1}, N-1 controls u_0..u_{N-2}.
 *   KKT system  [G C^T; C 0][-dZ; lambda] = [g; c]  with
 *     G = blockdiag(Q_0, R_0, Q_1, ..., R_{N-2}, Q_{N-1}),  g = [q_0, r_0, ..., q_{N-1}],
 *     C block row 0 = [I 0 ...], block row k+1 = [.. -A_k -B_k I ..],
 *     c = [-x0, e_0, ..., e_{N-2}]   (the input x0 is the required value of dx_0).
 *   Schur complement (Section III-B, eq. (5)): the paper writes S = -C G^-1 C^T and
 *   gamma = c - C G^-1 g; the same equation S lambda = gamma is solved here with both
 *   sides negated, S = C G^-1 C^T (positive definite) and gamma = C G^-1 g - c, which
 *   leaves lambda unchanged and matches the positive preconditioner the paper prints.
 *   Blocks (eqs. (6) and (7)):
 *     S_00 = Q_0^-1, S_{k+1,k+1} = theta_k = A_k Q_k^-1 A_k^T + B_k R_k^-1 B_k^T + Q_{k+1}^-1,
 *     S_{k+1,k} = phi_k = -A_k Q_k^-1, S_{k,k+1} = phi_k^T,
 *     gamma_0 = Q_0^-1 q_0 + x0,
 *     gamma_{k+1} = zeta_k - e_k, zeta_k = -A_k Q_k^-1 q_k - B_k R_k^-1 r_k + Q_{k+1}^-1 q_{k+1}.
 *   Preconditioner (Section IV-A, symmetric stair): Phi^-1 = D^-1 - D^-1 E D^-1 with
 *     D the block diagonal of S and E = S - D, i.e. Phi^-1_bb = D_b^-1 and
 *     Phi^-1_{b,b+-1} = -D_b^-1 S_{b,b+-1} D_{b+-1}^-1.
 *   PCG: Algorithm 1, stopped at the first main-loop iteration with eta' < tau, where
 *     tau = eps^2 * eta_ref, eta_ref = gamma^T Phi^-1 gamma (relative preconditioned
 *     residual sqrt(eta'/eta_ref) < eps; stop_abs = 0), or tau = eps (the absolute test
 *     eta' < eps that Algorithm 1 prints; stop_abs = 1).  The initial iterate is also
 *     tested (this only matters when the start already satisfies the rule, e.g. r = 0).
 *   The solve entry points take a mode word: bit 0 (ORC_MODE_STOP_ABS) selects the absolute
 *   rule; bit 1 (ORC_MODE_PHI_FP32) rounds every Phi^-1 entry to the nearest float before
 *   PCG uses it, for comparing unconverged iterates with a solver that stores Phi^-1 in
 *   single precision (the preconditioner changes the Krylov path, never the solution).
 *   Primal step (eq. (5)): dZ = -G^-1 (g - C^T lambda).
 *
 * Storage: row-major, S and Phi^-1 as [N][3][nx][nx] with slot 0 = (b,b-1),
 * slot 1 = (b,b), slot 2 = (b,b+1); slots outside the matrix are zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2, ORC_EINVAL = -1, ORC_ENOMEM = -3 };
enum { ORC_MODE_STOP_ABS = 1, ORC_MODE_PHI_FP32 = 2 };

/* Phi^-1 entries rounded to single precision (mode bit ORC_MODE_PHI_FP32). */
static void round_to_float(double *a, size_t n) {
  for (size_t i = 0; i < n; ++i) a[i] = (double)(float)a[i];
}

/* ---- small dense helpers (n <= 64) ------------------------------------------------ */

/* Inverse of a symmetric positive definite n x n matrix by Cholesky a = L L^T,
 * then inv = L^-T L^-1 column by column.  Returns 0, or -1 if a is not SPD. */
static int spd_inverse(int n, const double *a, double *inv) {
  double *L = calloc((size_t)n * n, sizeof(double));
  double *col = malloc((size_t)n * sizeof(double));
  if (!L || !col) { free(L); free(col); return -1; }
  for (int j = 0; j < n; ++j) {
    double d = a[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) { free(L); free(col); return -1; }
    L[j * n + j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = a[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = s / L[j * n + j];
    }
  }
  for (int c = 0; c < n; ++c) {
    /* solve L y = e_c, then L^T x = y */
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * col[k];
      col[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = col[i];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * col[k];
      col[i] = s / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[i * n + c] = col[i];
  }
  free(L); free(col);
  return 0;
}

/* c[m x n] = a[m x k] * b[k x n] (optionally transposed operands) */
static void matmul(int m, int k, int n, const double *a, int ta, const double *b, int tb, double *c) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int t = 0; t < k; ++t) {
        double av = ta ? a[t * m + i] : a[i * k + t];
        double bv = tb ? b[j * k + t] : b[t * n + j];
        s += av * bv;
      }
      c[i * n + j] = s;
    }
}

/* y[m] = a[m x n] x (or a^T x when ta) */
static void matvec(int m, int n, const double *a, int ta, const double *x, double *y) {
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += (ta ? a[j * m + i] : a[i * n + j]) * x[j];
    y[i] = s;
  }
}

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* y = M x for block-tridiagonal M stored [N][3][nx][nx] */
static void bt_matvec(int nx, int N, const double *M, const double *x, double *y) {
  const size_t bs = (size_t)nx * nx;
  for (int b = 0; b < N; ++b) {
    double *yb = y + (size_t)b * nx;
    for (int i = 0; i < nx; ++i) {
      double s = 0.0;
      for (int slot = 0; slot < 3; ++slot) {
        int c = b + slot - 1;
        if (c < 0 || c >= N) continue;
        const double *blk = M + ((size_t)b * 3 + slot) * bs;
        for (int j = 0; j < nx; ++j) s += blk[i * nx + j] * x[(size_t)c * nx + j];
      }
      yb[i] = s;
    }
  }
}

/* ---- per-knot inverses ------------------------------------------------------------ */

typedef struct {
  int nx, nu, N;
  const double *Q, *R, *A, *B, *q, *r, *x0, *e; /* e may be NULL (zero defects) */
} orc_prob;

/* Q_k^-1 for every knot and R_k^-1 for every control. */
static int knot_inverses(const orc_prob *p, double *Qi, double *Ri) {
  const int nx = p->nx, nu = p->nu, N = p->N;
  for (int k = 0; k < N; ++k)
    if (spd_inverse(nx, p->Q + (size_t)k * nx * nx, Qi + (size_t)k * nx * nx)) return -1;
  for (int k = 0; k + 1 < N; ++k)
    if (spd_inverse(nu, p->R + (size_t)k * nu * nu, Ri + (size_t)k * nu * nu)) return -1;
  return 0;
}

/* ---- Schur complement, right-hand side and preconditioner ------------------------- */

static int form(const orc_prob *p, const double *Qi, const double *Ri, double *S, double *P,
                double *gam) {
  const int nx = p->nx, nu = p->nu, N = p->N;
  const size_t bs = (size_t)nx * nx;
  memset(S, 0, (size_t)N * 3 * bs * sizeof(double));
  memset(P, 0, (size_t)N * 3 * bs * sizeof(double));
  double *T = malloc(bs * sizeof(double)), *U = malloc((size_t)nx * nu * sizeof(double));
  double *V = malloc(bs * sizeof(double)), *v = malloc((size_t)nx * sizeof(double));
  double *w = malloc((size_t)(nx > nu ? nx : nu) * sizeof(double));
  double *Di = malloc((size_t)N * bs * sizeof(double));
  if (!T || !U || !V || !v || !w || !Di) { free(T); free(U); free(V); free(v); free(w); free(Di); return ORC_ENOMEM; }

  /* block row 0: S_00 = Q_0^-1, gamma_0 = Q_0^-1 q_0 + x0 */
  memcpy(S + 1 * bs, Qi, bs * sizeof(double));
  matvec(nx, nx, Qi, 0, p->q, gam);
  for (int i = 0; i < nx; ++i) gam[i] += p->x0[i];

  for (int k = 0; k + 1 < N; ++k) {
    const double *Ak = p->A + (size_t)k * bs, *Bk = p->B + (size_t)k * nx * nu;
    const double *Qik = Qi + (size_t)k * bs, *Qik1 = Qi + (size_t)(k + 1) * bs;
    const double *Rik = Ri + (size_t)k * nu * nu;
    double *theta = S + ((size_t)(k + 1) * 3 + 1) * bs;
    double *phi = S + ((size_t)(k + 1) * 3 + 0) * bs;     /* S_{k+1,k} */
    double *phiT = S + ((size_t)k * 3 + 2) * bs;          /* S_{k,k+1} */
    /* theta_k = A Q^-1 A^T + B R^-1 B^T + Q_{k+1}^-1 */
    matmul(nx, nx, nx, Ak, 0, Qik, 0, T);                 /* T = A_k Q_k^-1 */
    matmul(nx, nx, nx, T, 0, Ak, 1, theta);               /* theta = T A_k^T */
    matmul(nx, nu, nu, Bk, 0, Rik, 0, U);                 /* U = B_k R_k^-1 */
    matmul(nx, nu, nx, U, 0, Bk, 1, V);                   /* V = U B_k^T */
    for (size_t t = 0; t < bs; ++t) theta[t] += V[t] + Qik1[t];
    /* phi_k = -A_k Q_k^-1, and its transpose above the diagonal */
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        phi[i * nx + j] = -T[i * nx + j];
        phiT[j * nx + i] = -T[i * nx + j];
      }
    /* zeta_k = -A_k Q_k^-1 q_k - B_k R_k^-1 r_k + Q_{k+1}^-1 q_{k+1};  gamma_{k+1} = zeta_k - e_k */
    double *g1 = gam + (size_t)(k + 1) * nx;
    matvec(nx, nx, T, 0, p->q + (size_t)k * nx, v);
    matvec(nx, nu, U, 0, p->r + (size_t)k * nu, w);
    for (int i = 0; i < nx; ++i) g1[i] = -v[i] - w[i];
    matvec(nx, nx, Qik1, 0, p->q + (size_t)(k + 1) * nx, v);
    for (int i = 0; i < nx; ++i) g1[i] += v[i] - (p->e ? p->e[(size_t)k * nx + i] : 0.0);
  }

  /* Phi^-1: D_b^-1 on the diagonal (D_0^-1 = Q_0 up to rounding), and
   * -D_b^-1 S_{b,b+-1} D_{b+-1}^-1 off the diagonal. */
  for (int b = 0; b < N; ++b)
    if (spd_inverse(nx, S + ((size_t)b * 3 + 1) * bs, Di + (size_t)b * bs)) {
      free(T); free(U); free(V); free(v); free(w); free(Di); return ORC_BREAKDOWN;
    }
  for (int b = 0; b < N; ++b) {
    memcpy(P + ((size_t)b * 3 + 1) * bs, Di + (size_t)b * bs, bs * sizeof(double));
    for (int slot = 0; slot < 3; slot += 2) {
      int c = b + slot - 1;
      if (c < 0 || c >= N) continue;
      matmul(nx, nx, nx, Di + (size_t)b * bs, 0, S + ((size_t)b * 3 + slot) * bs, 0, T);
      matmul(nx, nx, nx, T, 0, Di + (size_t)c * bs, 0, V);
      double *dst = P + ((size_t)b * 3 + slot) * bs;
      for (size_t t = 0; t < bs; ++t) dst[t] = -V[t];
    }
  }
  free(T); free(U); free(V); free(v); free(w); free(Di);
  return ORC_OK;
}

/* ---- PCG, Algorithm 1 -------------------------------------------------------------- */

/* Solves S lam = gam.  lam holds the start on entry (caller zeroes it for a cold start)
 * and the iterate on exit.  eta_trace (optional, length max_iter+1) receives
 * eta after initialisation and after every main-loop iteration. */
static int pcg(int nx, int N, const double *S, const double *P, const double *gam, double eps,
               int stop_abs, int max_iter, double *lam, int *iters, double *ratio,
               double *eta_trace) {
  const size_t n = (size_t)N * nx;
  double *r = malloc(n * sizeof(double)), *rt = malloc(n * sizeof(double));
  double *p = malloc(n * sizeof(double)), *Sp = malloc(n * sizeof(double));
  if (!r || !rt || !p || !Sp) { free(r); free(rt); free(p); free(Sp); return ORC_ENOMEM; }
  int status = ORC_NOT_CONVERGED, it = 0;

  /* eta_ref = gamma^T Phi^-1 gamma  (reference for the relative stopping rule) */
  bt_matvec(nx, N, P, gam, rt);
  const double eta_ref = dot((int)n, gam, rt);
  const double tau = stop_abs ? eps : eps * eps * eta_ref;

  /* initialisation: r = gamma - S lam; r~ = p = Phi^-1 r; eta = r^T r~ */
  bt_matvec(nx, N, S, lam, Sp);
  for (size_t i = 0; i < n; ++i) r[i] = gam[i] - Sp[i];
  bt_matvec(nx, N, P, r, rt);
  memcpy(p, rt, n * sizeof(double));
  double eta = dot((int)n, r, rt);
  if (eta_trace) eta_trace[0] = eta;
  double eta_new = eta;
  if (!isfinite(eta)) { status = ORC_BREAKDOWN; goto done; }
  if (eta <= tau) { status = ORC_OK; goto done; }

  for (it = 1; it <= max_iter; ++it) {
    bt_matvec(nx, N, S, p, Sp);
    const double pSp = dot((int)n, p, Sp);
    if (!(pSp > 0.0) || !isfinite(pSp)) { status = ORC_BREAKDOWN; break; }
    const double alpha = eta / pSp;
    for (size_t i = 0; i < n; ++i) r[i] -= alpha * Sp[i];
    for (size_t i = 0; i < n; ++i) lam[i] += alpha * p[i];
    bt_matvec(nx, N, P, r, rt);
    eta_new = dot((int)n, r, rt);
    if (eta_trace) eta_trace[it] = eta_new;
    if (!isfinite(eta_new)) { status = ORC_BREAKDOWN; break; }
    if (eta_new < tau) { status = ORC_OK; break; }
    const double beta = eta_new / eta;
    for (size_t i = 0; i < n; ++i) p[i] = rt[i] + beta * p[i];
    eta = eta_new;
  }
  if (it > max_iter) it = max_iter;
done:
  *iters = it;
  *ratio = eta_ref > 0.0 ? sqrt(fmax(eta_new, 0.0) / eta_ref) : 0.0;
  free(r); free(rt); free(p); free(Sp);
  return status;
}

/* ---- primal step: dZ = -G^-1 (g - C^T lam) ------------------------------------------ */

/* With (gx, gu) in place of (q, r) and mu in place of lambda this is also the
 * adjoint's nu_1 = -G^-1 (gbar - C^T mu). */
static void reconstruct(const orc_prob *p, const double *Qi, const double *Ri, const double *gx,
                        const double *gu, const double *lam, double *dx, double *du) {
  const int nx = p->nx, nu = p->nu, N = p->N;
  const size_t bs = (size_t)nx * nx;
  double *t = malloc((size_t)(nx > nu ? nx : nu) * sizeof(double));
  double *s = malloc((size_t)(nx > nu ? nx : nu) * sizeof(double));
  for (int k = 0; k < N; ++k) {
    /* (C^T lam) at x_k = lam_k - A_k^T lam_{k+1} */
    for (int i = 0; i < nx; ++i) t[i] = gx[(size_t)k * nx + i] - lam[(size_t)k * nx + i];
    if (k + 1 < N) {
      matvec(nx, nx, p->A + (size_t)k * bs, 1, lam + (size_t)(k + 1) * nx, s);
      for (int i = 0; i < nx; ++i) t[i] += s[i];
    }
    matvec(nx, nx, Qi + (size_t)k * bs, 0, t, s);
    for (int i = 0; i < nx; ++i) dx[(size_t)k * nx + i] = -s[i];
    if (k + 1 < N) {
      /* (C^T lam) at u_k = -B_k^T lam_{k+1} */
      matvec(nu, nx, p->B + (size_t)k * nx * nu, 1, lam + (size_t)(k + 1) * nx, s);
      for (int i = 0; i < nu; ++i) t[i] = gu[(size_t)k * nu + i] + s[i];
      matvec(nu, nu, Ri + (size_t)k * nu * nu, 0, t, s);
      for (int i = 0; i < nu; ++i) du[(size_t)k * nu + i] = -s[i];
    }
  }
  free(t); free(s);
}

/* ---- exported entry points ---------------------------------------------------------- */

static orc_prob mkprob(int nx, int nu, int N, const double *Q, const double *R, const double *A,
                       const double *B, const double *q, const double *r, const double *x0,
                       const double *e) {
  orc_prob p = {nx, nu, N, Q, R, A, B, q, r, x0, e};
  return p;
}

/* S, Phi^-1 [N][3][nx][nx] and gamma [N][nx]. */
int orc_form(int nx, int nu, int N, const double *Q, const double *R, const double *A,
             const double *B, const double *q, const double *r, const double *x0, const double *e,
             double *S, double *P, double *gam) {
  if (nx < 1 || nu < 1 || N < 1) return ORC_EINVAL;
  orc_prob p = mkprob(nx, nu, N, Q, R, A, B, q, r, x0, e);
  double *Qi = malloc((size_t)N * nx * nx * sizeof(double));
  double *Ri = malloc((size_t)(N > 1 ? N - 1 : 1) * nu * nu * sizeof(double));
  int st = (!Qi || !Ri) ? ORC_ENOMEM : (knot_inverses(&p, Qi, Ri) ? ORC_BREAKDOWN : form(&p, Qi, Ri, S, P, gam));
  free(Qi); free(Ri);
  return st;
}

/* PCG on a given S, Phi^-1, gamma. */
int orc_pcg(int nx, int N, const double *S, const double *P, const double *gam, double eps,
            int stop_abs, int max_iter, double *lam, int *iters, double *ratio, double *eta_trace) {
  if (nx < 1 || N < 1 || max_iter < 0) return ORC_EINVAL;
  return pcg(nx, N, S, P, gam, eps, stop_abs, max_iter, lam, iters, ratio, eta_trace);
}

/* Forward solve: form, PCG, primal step.  lam: start on entry (zeros for cold). */
int orc_solve(int nx, int nu, int N, const double *Q, const double *R, const double *A,
              const double *B, const double *q, const double *r, const double *x0, const double *e,
              double eps, int mode, int max_iter, double *lam, double *dx, double *du,
              int *iters, double *ratio, double *eta_trace) {
  if (nx < 1 || nu < 1 || N < 1) return ORC_EINVAL;
  if (max_iter <= 0) max_iter = N * nx;
  orc_prob p = mkprob(nx, nu, N, Q, R, A, B, q, r, x0, e);
  const size_t bs = (size_t)nx * nx;
  double *Qi = malloc((size_t)N * bs * sizeof(double));
  double *Ri = malloc((size_t)(N > 1 ? N - 1 : 1) * nu * nu * sizeof(double));
  double *S = malloc((size_t)N * 3 * bs * sizeof(double)), *P = malloc((size_t)N * 3 * bs * sizeof(double));
  double *gam = malloc((size_t)N * nx * sizeof(double));
  int st = ORC_ENOMEM;
  *iters = 0; *ratio = 0.0;
  if (Qi && Ri && S && P && gam) {
    st = knot_inverses(&p, Qi, Ri) ? ORC_BREAKDOWN : form(&p, Qi, Ri, S, P, gam);
    if (st == ORC_OK) {
      if (mode & ORC_MODE_PHI_FP32) round_to_float(P, (size_t)N * 3 * bs);
      st = pcg(nx, N, S, P, gam, eps, mode & ORC_MODE_STOP_ABS, max_iter, lam, iters, ratio, eta_trace);
      reconstruct(&p, Qi, Ri, q, r, lam, dx, du);
    }
  }
  free(Qi); free(Ri); free(S); free(P); free(gam);
  return st;
}

/* Adjoint of the forward solve for a scalar loss L(lambda, dx, du).
 *   Inputs: the forward solution (lam, dx, du) and the loss gradients
 *   gl = dL/dlambda, gx = dL/ddx, gu = dL/ddu (gx, gu may be NULL = 0).
 *   The adjoint of K w = b (K symmetric) is K nu = dL/dw with w = [-dZ; lambda]:
 *   eliminating nu_1 gives S mu = gl + C G^-1 gz (mu = -nu_2), solved with the same PCG
 *   and stopping rule, then nu_1 = -G^-1 (gz - C^T mu).  With dL/db = nu and
 *   dL/dK = -nu w^T restricted to the blocks of G and C:
 *     dQ_k = sym(nu1x_k dx_k^T), dR_k = sym(nu1u_k du_k^T),
 *     dA_k = lam_{k+1} nu1x_k^T + mu_{k+1} dx_k^T, dB_k = lam_{k+1} nu1u_k^T + mu_{k+1} du_k^T,
 *     dq_k = nu1x_k, dr_k = nu1u_k, dx0 = mu_0, de_k = -mu_{k+1}, dgamma = mu.
 *   Outputs may be NULL except mu. */
int orc_backward(int nx, int nu, int N, const double *Q, const double *R, const double *A,
                 const double *B, const double *q, const double *r, const double *x0,
                 const double *e, double eps, int mode, int max_iter, const double *lam,
                 const double *dx,
                 const double *du, const double *gl, const double *gx, const double *gu,
                 double *dQ, double *dR, double *dA, double *dB, double *dq, double *dr,
                 double *dx0, double *de, double *mu, int *iters, double *ratio) {
  if (nx < 1 || nu < 1 || N < 1) return ORC_EINVAL;
  if (max_iter <= 0) max_iter = N * nx;
  orc_prob p = mkprob(nx, nu, N, Q, R, A, B, q, r, x0, e);
  const size_t bs = (size_t)nx * nx, n = (size_t)N * nx, m = (size_t)(N > 1 ? N - 1 : 0) * nu;
  double *Qi = malloc((size_t)N * bs * sizeof(double));
  double *Ri = malloc((size_t)(N > 1 ? N - 1 : 1) * nu * nu * sizeof(double));
  double *S = malloc((size_t)N * 3 * bs * sizeof(double)), *P = malloc((size_t)N * 3 * bs * sizeof(double));
  double *gam = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double));
  double *zx = calloc(n, sizeof(double)), *zu = calloc(m + 1, sizeof(double));
  double *n1x = malloc(n * sizeof(double)), *n1u = malloc((m + 1) * sizeof(double));
  double *t = malloc(n * sizeof(double)), *s = malloc((size_t)(nx > nu ? nx : nu) * sizeof(double));
  int st = ORC_ENOMEM;
  *iters = 0; *ratio = 0.0;
  if (!(Qi && Ri && S && P && gam && y && zx && zu && n1x && n1u && t && s)) goto out;
  st = knot_inverses(&p, Qi, Ri) ? ORC_BREAKDOWN : form(&p, Qi, Ri, S, P, gam);
  if (st != ORC_OK) goto out;
  if (mode & ORC_MODE_PHI_FP32) round_to_float(P, (size_t)N * 3 * bs);
  if (gx) memcpy(zx, gx, n * sizeof(double));
  if (gu && m) memcpy(zu, gu, m * sizeof(double));
  /* y = gl + C G^-1 gz:  (C G^-1 gz)_0 = Q_0^-1 zx_0,
   * (C G^-1 gz)_{k+1} = -A_k Q_k^-1 zx_k - B_k R_k^-1 zu_k + Q_{k+1}^-1 zx_{k+1} */
  for (int k = 0; k < N; ++k) matvec(nx, nx, Qi + (size_t)k * bs, 0, zx + (size_t)k * nx, t + (size_t)k * nx);
  for (size_t i = 0; i < n; ++i) y[i] = gl[i];
  for (int i = 0; i < nx; ++i) y[i] += t[i];
  for (int k = 0; k + 1 < N; ++k) {
    double *yk = y + (size_t)(k + 1) * nx;
    matvec(nx, nx, p.A + (size_t)k * bs, 0, t + (size_t)k * nx, s);
    for (int i = 0; i < nx; ++i) yk[i] += -s[i] + t[(size_t)(k + 1) * nx + i];
    double *w = malloc((size_t)nu * sizeof(double)), *v = malloc((size_t)nx * sizeof(double));
    matvec(nu, nu, Ri + (size_t)k * nu * nu, 0, zu + (size_t)k * nu, w);
    matvec(nx, nu, p.B + (size_t)k * nx * nu, 0, w, v);
    for (int i = 0; i < nx; ++i) yk[i] -= v[i];
    free(w); free(v);
  }
  memset(mu, 0, n * sizeof(double));
  st = pcg(nx, N, S, P, y, eps, mode & ORC_MODE_STOP_ABS, max_iter, mu, iters, ratio, NULL);
  /* nu_1 = -G^-1 (gz - C^T mu) */
  reconstruct(&p, Qi, Ri, zx, zu, mu, n1x, n1u);
  for (int k = 0; k < N; ++k) {
    const double *ax = n1x + (size_t)k * nx, *xk = dx + (size_t)k * nx;
    if (dQ)
      for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nx; ++j)
          dQ[(size_t)k * bs + i * nx + j] = 0.5 * (ax[i] * xk[j] + ax[j] * xk[i]);
    if (dq) memcpy(dq + (size_t)k * nx, ax, nx * sizeof(double));
    if (k + 1 < N) {
      const double *au = n1u + (size_t)k * nu, *uk = du + (size_t)k * nu;
      const double *l1 = lam + (size_t)(k + 1) * nx, *m1 = mu + (size_t)(k + 1) * nx;
      if (dR)
        for (int i = 0; i < nu; ++i)
          for (int j = 0; j < nu; ++j)
            dR[(size_t)k * nu * nu + i * nu + j] = 0.5 * (au[i] * uk[j] + au[j] * uk[i]);
      if (dA)
        for (int i = 0; i < nx; ++i)
          for (int j = 0; j < nx; ++j)
            dA[(size_t)k * bs + i * nx + j] = l1[i] * ax[j] + m1[i] * xk[j];
      if (dB)
        for (int i = 0; i < nx; ++i)
          for (int j = 0; j < nu; ++j)
            dB[(size_t)k * nx * nu + i * nu + j] = l1[i] * au[j] + m1[i] * uk[j];
      if (dr) memcpy(dr + (size_t)k * nu, au, nu * sizeof(double));
      if (de)
        for (int i = 0; i < nx; ++i) de[(size_t)k * nx + i] = -m1[i];
    }
  }
  if (dx0) memcpy(dx0, mu, nx * sizeof(double));
out:
  free(Qi); free(Ri); free(S); free(P); free(gam); free(y); free(zx); free(zu);
  free(n1x); free(n1u); free(t); free(s);
  return st;
}

/* Batched forward solve over packed problems (layout of the batched entry point:
 * knot-indexed rows of problem b start at off[b], control-indexed rows at off[b]-b,
 * x0 is [batch][nx]).  Problems are independent; OpenMP spreads them over threads.
 * lam must hold the start (zeros for cold).  iters/status/ratio are [batch]. */
int orc_solve_batch(int nx, int nu, int batch, const int64_t *off, const double *Q,
                    const double *R, const double *A, const double *B, const double *q,
                    const double *r, const double *x0, const double *e, double eps, int mode,
                    int max_iter, double *lam, double *dx, double *du, int *iters, double *ratio,
                    int *status, int nthreads) {
  if (nx < 1 || nu < 1 || batch < 0) return ORC_EINVAL;
  const size_t bs = (size_t)nx * nx, bu = (size_t)nu * nu, bb = (size_t)nx * nu;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int b = 0; b < batch; ++b) {
    const int64_t k0 = off[b], c0 = off[b] - b;
    const int N = (int)(off[b + 1] - off[b]);
    status[b] = orc_solve(nx, nu, N, Q + k0 * bs, R + c0 * bu, A + c0 * bs, B + c0 * bb,
                          q + k0 * nx, r + c0 * nu, x0 + (size_t)b * nx, e ? e + c0 * nx : NULL,
                          eps, mode, max_iter, lam + k0 * nx, dx + k0 * nx, du + c0 * nu, &iters[b],
                          &ratio[b], NULL);
  }
  return ORC_OK;
}

/* Batched adjoint (same packing); gx/gu may be NULL. */
int orc_backward_batch(int nx, int nu, int batch, const int64_t *off, const double *Q,
                       const double *R, const double *A, const double *B, const double *q,
                       const double *r, const double *x0, const double *e, double eps,
                       int mode, int max_iter, const double *lam, const double *dx, const double *du,
                       const double *gl, const double *gx, const double *gu, double *dQ,
                       double *dR, double *dA, double *dB, double *dq, double *dr, double *dx0,
                       double *de, double *mu, int *iters, double *ratio, int *status,
                       int nthreads) {
  if (nx < 1 || nu < 1 || batch < 0) return ORC_EINVAL;
  const size_t bs = (size_t)nx * nx, bu = (size_t)nu * nu, bb = (size_t)nx * nu;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int b = 0; b < batch; ++b) {
    const int64_t k0 = off[b], c0 = off[b] - b;
    const int N = (int)(off[b + 1] - off[b]);
    status[b] = orc_backward(
        nx, nu, N, Q + k0 * bs, R + c0 * bu, A + c0 * bs, B + c0 * bb, q + k0 * nx, r + c0 * nu,
        x0 + (size_t)b * nx, e ? e + c0 * nx : NULL, eps, mode, max_iter, lam + k0 * nx,
        dx + k0 * nx,
        du + c0 * nu, gl + k0 * nx, gx ? gx + k0 * nx : NULL, gu ? gu + c0 * nu : NULL,
        dQ + k0 * bs, dR + c0 * bu, dA + c0 * bs, dB + c0 * bb, dq + k0 * nx, dr + c0 * nu,
        dx0 + (size_t)b * nx, de + c0 * nx, mu + k0 * nx, &iters[b], &ratio[b]);
  }
  return ORC_OK;
}
