/*
 * Banded oracle for the S-MNN weighted least-squares solve (TEST INFRASTRUCTURE:
 * only tests, the smoke check and the benchmark's CPU-baseline leg use this).
 *
 * Computes the same quantity as oracle/dense.py -- the minimiser of
 * || W^{1/2}(A y - b) ||_2 over the constraints of Eqs. 4-7 with the weighting
 * stated before Eq. 9 (App. A.1 gives A, b, W) -- without forming the dense
 * matrix: the weighted rows are taken in time order and reduced by Householder
 * reflections one step at a time (the standard QR of a block-banded matrix).
 * Rows of step t touch only the unknown blocks y_t and y_{t+1}, so after the
 * rows of step t have been reflected, the first R+1 rows of the triangular
 * factor are final and the next R+1 rows carry to step t+1.  Everything is
 * double precision; one instance per OpenMP iteration.
 *
 *  oracle_solve   -- Eq. 9 (the least-squares solution y).
 *  oracle_grad    -- y, the adjoint lam = M^{-1} g of Eq. 14 with M = R^T R,
 *                    and the closed-form per-row gradients (same formulas as
 *                    oracle/dense.py grad_rows).
 *  oracle_cond    -- an estimate of the 2-norm condition number of the normal
 *                    matrix M = A^T W A = R^T R: power iteration on M and on
 *                    M^{-1} (both applied through the triangular factor).
 *
 * Pinned in tests/test_oracle_banded.py against the dense oracle (small T),
 * exact polynomial recovery (any T) and Table 5.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KMAX 6
#define COLS (2 * KMAX + 1)
#define ROWS (3 * KMAX + 1 + KMAX)

static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* Householder QR of the leading ncol columns of a[nrow][COLS] (rhs in column
 * rhs_col is transformed too).  In place; below-diagonal entries become 0. */
static void householder(double a[ROWS][COLS], int nrow, int ncol, int rhs_col) {
  for (int j = 0; j < ncol && j < nrow; ++j) {
    double norm2 = 0.0;
    for (int i = j; i < nrow; ++i) norm2 += a[i][j] * a[i][j];
    if (norm2 == 0.0) continue;
    double alpha = (a[j][j] > 0 ? -1.0 : 1.0) * sqrt(norm2);
    double v[ROWS];
    for (int i = j; i < nrow; ++i) v[i] = a[i][j];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < nrow; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int l = j; l <= rhs_col; ++l) {
      if (l >= ncol && l != rhs_col) continue;
      double dot = 0.0;
      for (int i = j; i < nrow; ++i) dot += v[i] * a[i][l];
      double f = 2.0 * dot / vv;
      for (int i = j; i < nrow; ++i) a[i][l] -= f * v[i];
    }
    a[j][j] = alpha;
    for (int i = j + 1; i < nrow; ++i) a[i][j] = 0.0;
  }
}

/* Weighted smoothness rows between t and t+1 (Eqs. 6-7, weight w_s s^r).
 * row r (forward) / k+r (backward) ; columns 0..k-1 = y_t, k..2k-1 = y_{t+1}. */
static void smooth_rows(int k, double s, double ws, double out[2 * KMAX][2 * KMAX]) {
  memset(out, 0, sizeof(double) * 2 * KMAX * 2 * KMAX);
  for (int r = 0; r < k; ++r) {
    double wr = ws * pow(s, r);
    for (int j = r; j < k; ++j) out[r][j] = wr * pow(s, j - r) / fact(j - r);
    out[r][k + r] = -wr;
    for (int j = r; j < k; ++j) out[k + r][k + j] = wr * pow(-s, j - r) / fact(j - r);
    out[k + r][r] = -wr;
  }
}

/* Factor: Rd[t] (k x k upper), Ro[t] (k x k, coupling y_t -> y_{t+1}), z[t] (k). */
static void factor(int R, int n_init, int t_init, int64_t T, const double* c, const double* d, const double* s,
                   const double* u0, const double* w, double* Rd, double* Ro, double* z) {
  const int k = R + 1;
  double carry[KMAX][KMAX + 1];
  int have_carry = 0;
  for (int64_t t = 0; t < T; ++t) {
    double a[ROWS][COLS];
    memset(a, 0, sizeof(a));
    const int rhs = 2 * k;
    int nrow = 0;
    if (have_carry) {
      for (int i = 0; i < k; ++i) {
        for (int j = 0; j < k; ++j) a[nrow][j] = carry[i][j];
        a[nrow][rhs] = carry[i][k];
        ++nrow;
      }
    }
    for (int j = 0; j < k; ++j) a[nrow][j] = w[0] * c[t * k + j];   /* Eq. 4 */
    a[nrow][rhs] = w[0] * d[t];
    ++nrow;
    if (t < t_init) {                                                  /* Eq. 5 */
      for (int r = 0; r < n_init; ++r) { a[nrow][r] = w[1]; a[nrow][rhs] = w[1] * u0[t * n_init + r]; ++nrow; }
    }
    int ncol = k;
    if (t + 1 < T) {                                                   /* Eqs. 6-7 */
      double sr[2 * KMAX][2 * KMAX];
      smooth_rows(k, s[t], w[2], sr);
      for (int i = 0; i < 2 * k; ++i) {
        for (int j = 0; j < 2 * k; ++j) a[nrow][j] = sr[i][j];
        a[nrow][rhs] = 0.0;
        ++nrow;
      }
      ncol = 2 * k;
    }
    householder(a, nrow, ncol, rhs);
    for (int i = 0; i < k; ++i) {
      for (int j = 0; j < k; ++j) {
        Rd[(t * k + i) * k + j] = a[i][j];
        Ro[(t * k + i) * k + j] = (t + 1 < T) ? a[i][k + j] : 0.0;
      }
      z[t * k + i] = a[i][rhs];
    }
    if (t + 1 < T) {
      for (int i = 0; i < k; ++i) {
        for (int j = 0; j < k; ++j) carry[i][j] = a[k + i][k + j];
        carry[i][k] = a[k + i][rhs];
      }
      have_carry = 1;
    }
  }
}

/* Solve R x = v (block upper bidiagonal). */
static void back_solve(int k, int64_t T, const double* Rd, const double* Ro, const double* v, double* x) {
  for (int64_t t = T - 1; t >= 0; --t) {
    double rhs[KMAX];
    for (int i = 0; i < k; ++i) {
      rhs[i] = v[t * k + i];
      if (t + 1 < T)
        for (int j = 0; j < k; ++j) rhs[i] -= Ro[(t * k + i) * k + j] * x[(t + 1) * k + j];
    }
    for (int i = k - 1; i >= 0; --i) {
      double acc = rhs[i];
      for (int j = i + 1; j < k; ++j) acc -= Rd[(t * k + i) * k + j] * x[t * k + j];
      x[t * k + i] = acc / Rd[(t * k + i) * k + i];
    }
  }
}

/* Solve R^T x = v (block lower bidiagonal). */
static void fwd_solve_T(int k, int64_t T, const double* Rd, const double* Ro, const double* v, double* x) {
  for (int64_t t = 0; t < T; ++t) {
    double rhs[KMAX];
    for (int j = 0; j < k; ++j) {
      rhs[j] = v[t * k + j];
      if (t > 0)
        for (int i = 0; i < k; ++i) rhs[j] -= Ro[((t - 1) * k + i) * k + j] * x[(t - 1) * k + i];
    }
    for (int j = 0; j < k; ++j) {
      double acc = rhs[j];
      for (int i = 0; i < j; ++i) acc -= Rd[(t * k + i) * k + j] * x[t * k + i];
      x[t * k + j] = acc / Rd[(t * k + j) * k + j];
    }
  }
}

static int solve_one(int R, int n_init, int t_init, int64_t T, const double* c, const double* d, const double* s,
                     const double* u0, const double* w, double* y, double* lam, const double* g,
                     double* dc, double* dd, double* ds, double* du0, double* dw) {
  const int k = R + 1;
  double* Rd = (double*)malloc(sizeof(double) * T * k * k);
  double* Ro = (double*)malloc(sizeof(double) * T * k * k);
  double* z = (double*)malloc(sizeof(double) * T * k);
  if (!Rd || !Ro || !z) { free(Rd); free(Ro); free(z); return 1; }
  factor(R, n_init, t_init, T, c, d, s, u0, w, Rd, Ro, z);
  back_solve(k, T, Rd, Ro, z, y);
  if (g) {
    fwd_solve_T(k, T, Rd, Ro, g, z);     /* R^T z = g */
    back_solve(k, T, Rd, Ro, z, lam);    /* R lam = z  => M lam = g (Eq. 14) */
    const double wg = w[0], wi = w[1], ws = w[2];
    dw[0] = dw[1] = dw[2] = 0.0;
    for (int64_t t = 0; t < T; ++t) {     /* governing rows */
      double e = -d[t], f = 0.0;
      for (int j = 0; j < k; ++j) { e += c[t * k + j] * y[t * k + j]; f += c[t * k + j] * lam[t * k + j]; }
      for (int j = 0; j < k; ++j) dc[t * k + j] = -wg * wg * (e * lam[t * k + j] + f * y[t * k + j]);
      dd[t] = wg * wg * f;
      dw[0] += -2.0 * wg * e * f;
      ds[t] = 0.0;
    }
    for (int t = 0; t < t_init; ++t)      /* initial rows (none past the last point) */
      for (int r = 0; r < n_init; ++r) {
        if (t >= T) { du0[t * n_init + r] = 0.0; continue; }
        du0[t * n_init + r] = wi * wi * lam[t * k + r];
        dw[1] += -2.0 * wi * (y[t * k + r] - u0[t * n_init + r]) * lam[t * k + r];
      }
    for (int64_t t = 0; t + 1 < T; ++t) { /* smoothness rows */
      const double st = s[t];
      double sr[2 * KMAX][2 * KMAX], dsr[2 * KMAX][2 * KMAX];
      smooth_rows(k, st, ws, sr);
      memset(dsr, 0, sizeof(dsr));
      for (int r = 0; r < k; ++r) {       /* d/ds of each weighted coefficient */
        for (int j = r; j < k; ++j) {
          dsr[r][j] = (j > 0) ? ws * j * pow(st, j - 1) / fact(j - r) : 0.0;
          double sign = ((j - r) % 2) ? -1.0 : 1.0;
          dsr[k + r][k + j] = (j > 0) ? ws * sign * j * pow(st, j - 1) / fact(j - r) : 0.0;
        }
        dsr[r][k + r] = (r > 0) ? -ws * r * pow(st, r - 1) : 0.0;
        dsr[k + r][r] = (r > 0) ? -ws * r * pow(st, r - 1) : 0.0;
      }
      for (int i = 0; i < 2 * k; ++i) {
        double rho = 0.0, mu = 0.0, dl = 0.0, dy = 0.0;
        for (int j = 0; j < 2 * k; ++j) {
          const double yy = y[t * k + j], ll = lam[t * k + j];
          rho += sr[i][j] * yy; mu += sr[i][j] * ll;
          dl += dsr[i][j] * ll; dy += dsr[i][j] * yy;
        }
        ds[t] += -(dl * rho + mu * dy);
        dw[2] += -2.0 * rho * mu / ws;
      }
    }
  }
  free(Rd); free(Ro); free(z);
  return 0;
}

/* Batched entry points.  off[N+1] = row offsets (instance i owns rows
 * off[i]..off[i+1]-1 of c [.,k], d, s, y [.,k]).  u0 is [N][t_init][n_init]
 * (initial values at the first t_init points), w [N][3].  Returns the number
 * of instances that failed to allocate. */
int oracle_solve(int R, int n_init, int t_init, int64_t N, const int64_t* off, const double* c, const double* d,
                 const double* s, const double* u0, const double* w, double* y) {
  const int k = R + 1;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    const int64_t o = off[i], T = off[i + 1] - off[i];
    fails += solve_one(R, n_init, t_init, T, c + o * k, d + o, s + o, u0 + i * t_init * n_init, w + 3 * i,
                       y + o * k, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
  }
  return fails;
}

int oracle_grad(int R, int n_init, int t_init, int64_t N, const int64_t* off, const double* c, const double* d,
                const double* s, const double* u0, const double* w, const double* g, double* y,
                double* lam, double* dc, double* dd, double* ds, double* du0, double* dw) {
  const int k = R + 1;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    const int64_t o = off[i], T = off[i + 1] - off[i];
    fails += solve_one(R, n_init, t_init, T, c + o * k, d + o, s + o, u0 + i * t_init * n_init, w + 3 * i,
                       y + o * k, lam + o * k, g + o * k, dc + o * k, dd + o, ds + o, du0 + i * t_init * n_init,
                       dw + 3 * i);
  }
  return fails;
}


static void apply_M(int k, int64_t T, const double* Rd, const double* Ro, const double* v, double* tmp, double* out) {
  /* out = R^T (R v) */
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < k; ++i) {
      double acc = 0.0;
      for (int j = i; j < k; ++j) acc += Rd[(t * k + i) * k + j] * v[t * k + j];
      if (t + 1 < T)
        for (int j = 0; j < k; ++j) acc += Ro[(t * k + i) * k + j] * v[(t + 1) * k + j];
      tmp[t * k + i] = acc;
    }
  for (int64_t t = 0; t < T; ++t)
    for (int j = 0; j < k; ++j) {
      double acc = 0.0;
      for (int i = 0; i <= j; ++i) acc += Rd[(t * k + i) * k + j] * tmp[t * k + i];
      if (t > 0)
        for (int i = 0; i < k; ++i) acc += Ro[((t - 1) * k + i) * k + j] * tmp[(t - 1) * k + i];
      out[t * k + j] = acc;
    }
}

static double normalize(int64_t n, double* v) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += v[i] * v[i];
  s = sqrt(s);
  if (s > 0)
    for (int64_t i = 0; i < n; ++i) v[i] /= s;
  return s;
}

static double cond_one(int R, int n_init, int t_init, int64_t T, const double* c, const double* d, const double* s,
                       const double* u0, const double* w, int iters) {
  const int k = R + 1;
  const int64_t n = T * k;
  double* Rd = (double*)malloc(sizeof(double) * n * k);
  double* Ro = (double*)malloc(sizeof(double) * n * k);
  double* z = (double*)malloc(sizeof(double) * n);
  double* v = (double*)malloc(sizeof(double) * n);
  double* t1 = (double*)malloc(sizeof(double) * n);
  double* t2 = (double*)malloc(sizeof(double) * n);
  double kappa = -1.0;
  if (Rd && Ro && z && v && t1 && t2) {
    factor(R, n_init, t_init, T, c, d, s, u0, w, Rd, Ro, z);
    double lmax = 0.0, lmin_inv = 0.0;
    for (int64_t i = 0; i < n; ++i) v[i] = 1.0 + 0.5 * sin(0.7 * (double)i);
    normalize(n, v);
    for (int it = 0; it < iters; ++it) {  /* largest eigenvalue of M */
      apply_M(k, T, Rd, Ro, v, t1, t2);
      lmax = normalize(n, t2);
      memcpy(v, t2, sizeof(double) * n);
    }
    for (int64_t i = 0; i < n; ++i) v[i] = 1.0 + 0.5 * cos(1.3 * (double)i);
    normalize(n, v);
    for (int it = 0; it < iters; ++it) {  /* largest eigenvalue of M^{-1} */
      fwd_solve_T(k, T, Rd, Ro, v, t1);
      back_solve(k, T, Rd, Ro, t1, t2);
      lmin_inv = normalize(n, t2);
      memcpy(v, t2, sizeof(double) * n);
    }
    kappa = lmax * lmin_inv;
  }
  free(Rd); free(Ro); free(z); free(v); free(t1); free(t2);
  return kappa;
}

int oracle_cond(int R, int n_init, int t_init, int64_t N, const int64_t* off, const double* c, const double* d,
                const double* s, const double* u0, const double* w, int iters, double* kappa) {
  const int k = R + 1;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    const int64_t o = off[i], T = off[i + 1] - off[i];
    kappa[i] = cond_one(R, n_init, t_init, T, c + o * k, d + o, s + o, u0 + i * t_init * n_init, w + 3 * i,
                        iters);
    fails += kappa[i] < 0;
  }
  return fails;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
