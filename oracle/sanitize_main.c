/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the C oracle
 * (schur_pcg.c).  TEST INFRASTRUCTURE ONLY: tests/test_oracle_sanitizers.py compiles it
 * together with schur_pcg.c under -fsanitize=address,undefined and runs it; any invalid
 * access, leak or undefined operation aborts the run.
 *
 * It exercises every entry point on small problems: one, two and several knots, with and
 * without dynamics defects, both stopping rules and both preconditioner precisions, the
 * adjoint with and without loss terms on the primal step, and ragged packed batches.
 * Inputs come from a fixed linear congruential sequence (no arithmetic of the method):
 * Q and R are diagonally dominant symmetric matrices, so positive definite.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_form(int nx, int nu, int N, const double *Q, const double *R, const double *A,
             const double *B, const double *q, const double *r, const double *x0,
             const double *e, double *S, double *P, double *gamma);
int orc_solve(int nx, int nu, int N, const double *Q, const double *R, const double *A,
              const double *B, const double *q, const double *r, const double *x0,
              const double *e, double eps, int mode, int max_iter, double *lam, double *dx,
              double *du, int *iters, double *ratio, double *eta_trace);
int orc_backward(int nx, int nu, int N, const double *Q, const double *R, const double *A,
                 const double *B, const double *q, const double *r, const double *x0,
                 const double *e, double eps, int mode, int max_iter, const double *lam,
                 const double *dx, const double *du, const double *gl, const double *gx,
                 const double *gu, double *dQ, double *dR, double *dA, double *dB, double *dq,
                 double *dr, double *dx0, double *de, double *mu, int *iters, double *ratio);
int orc_solve_batch(int nx, int nu, int batch, const int64_t *off, const double *Q,
                    const double *R, const double *A, const double *B, const double *q,
                    const double *r, const double *x0, const double *e, double eps, int mode,
                    int max_iter, double *lam, double *dx, double *du, int *iters, double *ratio,
                    int *status, int nthreads);
int orc_backward_batch(int nx, int nu, int batch, const int64_t *off, const double *Q,
                       const double *R, const double *A, const double *B, const double *q,
                       const double *r, const double *x0, const double *e, double eps,
                       int mode, int max_iter, const double *lam, const double *dx, const double *du,
                       const double *gl, const double *gx, const double *gu, double *dQ,
                       double *dR, double *dA, double *dB, double *dq, double *dr, double *dx0,
                       double *de, double *mu, int *iters, double *ratio, int *status,
                       int nthreads);

static uint64_t lcg_state = 12345u;
static double uniform(void) { /* in [-1, 1) */
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg_state >> 11) / 4503599627370496.0 - 1.0;
}

/* n x n symmetric, diagonally dominant (hence positive definite) */
static void spd(int n, double *m) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) m[i * n + j] = m[j * n + i] = 0.1 * uniform();
  for (int i = 0; i < n; ++i) m[i * n + i] = 2.0 + (double)n * 0.1 + 0.5 * (uniform() + 1.0);
}

static double *fill(size_t n, double scale) {
  double *a = calloc(n ? n : 1, sizeof(double));
  for (size_t i = 0; i < n; ++i) a[i] = scale * uniform();
  return a;
}

static int failures = 0;
static void expect(int cond, const char *what) {
  if (!cond) {
    fprintf(stderr, "unexpected result: %s\n", what);
    ++failures;
  }
}

/* one packed batch of horizons Ns[0..batch) (nx, nu), solved per problem and batched */
static void run_batch(int nx, int nu, int batch, const int *Ns, int defects) {
  int64_t *off = malloc(sizeof(int64_t) * (size_t)(batch + 1));
  off[0] = 0;
  for (int b = 0; b < batch; ++b) off[b + 1] = off[b] + Ns[b];
  const size_t K = (size_t)off[batch], M = K - (size_t)batch;
  double *Q = malloc(sizeof(double) * K * nx * nx), *R = malloc(sizeof(double) * (M ? M : 1) * nu * nu);
  for (size_t k = 0; k < K; ++k) spd(nx, Q + k * nx * nx);
  for (size_t k = 0; k < M; ++k) spd(nu, R + k * nu * nu);
  double *A = fill(M * nx * nx, 0.3), *B = fill(M * nx * nu, 0.3), *q = fill(K * nx, 1.0);
  double *r = fill(M * nu, 1.0), *x0 = fill((size_t)batch * nx, 1.0);
  double *e = defects ? fill(M * nx, 0.1) : NULL;
  for (size_t k = 0; k < M; ++k)
    for (int i = 0; i < nx; ++i) A[k * nx * nx + i * nx + i] += 1.0;
  double *lam = calloc(K * nx, sizeof(double)), *dx = calloc(K * nx, sizeof(double));
  double *du = calloc(M ? M * nu : 1, sizeof(double));
  int *iters = calloc((size_t)batch, sizeof(int)), *status = calloc((size_t)batch, sizeof(int));
  double *ratio = calloc((size_t)batch, sizeof(double));
  for (int mode = 0; mode < 4; ++mode) {
    const double eps = (mode & 1) ? 1e-8 : 1e-7;
    for (size_t i = 0; i < K * nx; ++i) lam[i] = 0.0;
    expect(orc_solve_batch(nx, nu, batch, off, Q, R, A, B, q, r, x0, e, eps, mode, 0, lam, dx, du, iters,
                           ratio, status, 2) == 0, "orc_solve_batch");
    for (int b = 0; b < batch; ++b) expect(status[b] == 0, "batched solve converges");
  }
  /* the first problem alone, with an eta trace and a form of its blocks */
  {
    const int N = Ns[0];
    double *S = calloc((size_t)N * 3 * nx * nx, sizeof(double)), *P = calloc((size_t)N * 3 * nx * nx, sizeof(double));
    double *g = calloc((size_t)N * nx, sizeof(double)), *tr = calloc((size_t)N * nx + 1, sizeof(double));
    double *l1 = calloc((size_t)N * nx, sizeof(double)), *x1 = calloc((size_t)N * nx, sizeof(double));
    double *u1 = calloc((size_t)(N > 1 ? N - 1 : 1) * nu, sizeof(double));
    int it = 0;
    double ra = 0.0;
    expect(orc_form(nx, nu, N, Q, R, A, B, q, r, x0, e, S, P, g) == 0, "orc_form");
    expect(orc_solve(nx, nu, N, Q, R, A, B, q, r, x0, e, 1e-9, 0, 0, l1, x1, u1, &it, &ra, tr) == 0, "orc_solve");
    expect(orc_solve(nx, nu, N, Q, R, A, B, q, r, x0, e, 1e-9, 0, 1, l1, x1, u1, &it, &ra, NULL) >= 0,
           "orc_solve with one iteration");
    free(S); free(P); free(g); free(tr); free(l1); free(x1); free(u1);
  }
  double *gl = fill(K * nx, 1.0), *gx = fill(K * nx, 1.0), *gu = fill(M * nu, 1.0);
  double *dQ = calloc(K * nx * nx, sizeof(double)), *dR = calloc((M ? M : 1) * nu * nu, sizeof(double));
  double *dA = calloc((M ? M : 1) * nx * nx, sizeof(double)), *dB = calloc((M ? M : 1) * nx * nu, sizeof(double));
  double *dq = calloc(K * nx, sizeof(double)), *dr = calloc((M ? M : 1) * nu, sizeof(double));
  double *dx0 = calloc((size_t)batch * nx, sizeof(double)), *de = calloc((M ? M : 1) * nx, sizeof(double));
  double *mu = calloc(K * nx, sizeof(double));
  expect(orc_backward_batch(nx, nu, batch, off, Q, R, A, B, q, r, x0, e, 1e-8, 0, 0, lam, dx, du, gl, NULL, NULL,
                            dQ, dR, dA, dB, dq, dr, dx0, de, mu, iters, ratio, status, 2) == 0,
         "orc_backward_batch");
  expect(orc_backward_batch(nx, nu, batch, off, Q, R, A, B, q, r, x0, e, 1e-8, 2, 0, lam, dx, du, gl, gx,
                            M ? gu : NULL, dQ, dR, dA, dB, dq, dr, dx0, de, mu, iters, ratio, status, 2) == 0,
         "orc_backward_batch with primal loss terms");
  {
    int it = 0;
    double ra = 0.0;
    expect(orc_backward(nx, nu, Ns[0], Q, R, A, B, q, r, x0, e, 1e-8, 1, 0, lam, dx, du, gl, gx, M ? gu : NULL, dQ,
                        dR, dA, dB, dq, dr, dx0, de, mu, &it, &ra) >= 0,
           "orc_backward");
  }
  free(off); free(Q); free(R); free(A); free(B); free(q); free(r); free(x0); free(e);
  free(lam); free(dx); free(du); free(iters); free(status); free(ratio);
  free(gl); free(gx); free(gu); free(dQ); free(dR); free(dA); free(dB); free(dq); free(dr);
  free(dx0); free(de); free(mu);
}

int main(void) {
  const int one[] = {1}, two[] = {2}, ragged[] = {3, 1, 6, 2, 5};
  run_batch(14, 7, 1, one, 0);
  run_batch(14, 7, 1, two, 1);
  run_batch(14, 7, 5, ragged, 1);
  run_batch(28, 14, 2, ragged + 2, 0);
  run_batch(3, 1, 5, ragged, 1);
  if (failures) {
    fprintf(stderr, "%d unexpected results\n", failures);
    return 1;
  }
  printf("sanitized oracle run ok\n");
  return 0;
}
