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
 * rows of step t have been reflected, the first K rows of the triangular
 * factor are final and the next K rows carry to step t+1 (K = V (R+1), the
 * block size of Eq. 10).
 *
 * General form of Sec. 3.1: V variables and Q governing equations per time
 * point.  Unknowns of point t are ordered variable-major, y_t[v (R+1) + r]
 * (the ordering stated before Eq. 10 and in App. A.1); the Q governing rows of
 * point t have coefficients C_t[q][v (R+1) + r] (App. A.2's C_t); initial rows
 * fix y_{t,v,r} = u_{t,v,r} for t < T_init, r < n_init; smoothness rows act on
 * each variable separately.
 *
 * Weights are per row: wg[t][q] for the governing rows of point t,
 * wi[t][v][r] for the initial rows and ws[t] for the 2 V (R+1) smoothness
 * rows between points t and t+1, each of which is further scaled by s_t^r
 * (the weighting paragraph before Eq. 9).  The paper's three scalar weights
 * are the case where every entry of an array holds the same value; their
 * gradients are the sums of the per-row gradients.
 *
 * The arithmetic type `real` is double by default and __float128 (113-bit
 * significand, libquadmath) when compiled with -DORACLE_QUAD.  Inputs and
 * outputs are double either way; the quad build gives the least-squares
 * solution, adjoint and gradients of the double inputs to ~1e-30 relative
 * accuracy for any conditioning met here, which makes it the extended
 * precision reference of the parity tests.
 *
 *  oracle_solve    -- Eq. 9 (the least-squares solution y).
 *  oracle_grad     -- y, the adjoint lam = M^{-1} g of Eq. 14 with M = R^T R,
 *                     and the closed-form per-row gradients (same formulas as
 *                     oracle/dense.py grad_rows).
 *  oracle_cond     -- an estimate of the 2-norm condition number of the normal
 *                     matrix M = A^T W A = R^T R: power iteration on M and on
 *                     M^{-1} (both applied through the triangular factor).
 *  oracle_backward_error -- for a given y, two normal-equation backward
 *                     errors accumulated row by row in `real`: the normwise
 *                     ||beta - M y||_inf / (||M||_inf ||y||_inf + ||beta||_inf)
 *                     and the row-scaled ||A^T W (b - A y)||_inf /
 *                     || |A|^T W (|A||y| + |b|) ||_inf.
 *
 * Pinned in tests/test_oracle_banded.py against the dense oracle (small T),
 * exact polynomial recovery (any T), Table 5 and the exact rational oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_QUAD
#include <quadmath.h>
typedef __float128 real;
#define RSQRT(x) sqrtq(x)
#define RABS(x) fabsq(x)
#else
typedef double real;
#define RSQRT(x) sqrt(x)
#define RABS(x) fabs(x)
#endif

#define KMAX 12                       /* V (R+1) */
#define QMAX 12                       /* governing rows per point */
#define COLS (2 * KMAX + 1)
#define ROWS (KMAX + QMAX + KMAX + 2 * KMAX)

typedef struct {
  int R, V, Q, n_init, t_init;
} oracle_shape;

/* Per-instance views of the inputs (double) */
typedef struct {
  int64_t T;
  const double *c, *d, *s, *u0, *wg, *wi, *ws;
} inst;

static real fact(int n) { real f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
static real ipow(real x, int n) { real p = 1; for (int i = 0; i < n; ++i) p *= x; return p; }

/* Householder QR of the leading ncol columns of a[nrow][COLS] (rhs in column
 * rhs_col is transformed too).  In place; below-diagonal entries become 0. */
static void householder(real a[ROWS][COLS], int nrow, int ncol, int rhs_col) {
  for (int j = 0; j < ncol && j < nrow; ++j) {
    real norm2 = 0;
    for (int i = j; i < nrow; ++i) norm2 += a[i][j] * a[i][j];
    if (norm2 == 0) continue;
    real alpha = (a[j][j] > 0 ? -1 : 1) * RSQRT(norm2);
    real v[ROWS];
    for (int i = j; i < nrow; ++i) v[i] = a[i][j];
    v[j] -= alpha;
    real vv = 0;
    for (int i = j; i < nrow; ++i) vv += v[i] * v[i];
    if (vv == 0) continue;
    for (int l = j; l <= rhs_col; ++l) {
      if (l >= ncol && l != rhs_col) continue;
      real dot = 0;
      for (int i = j; i < nrow; ++i) dot += v[i] * a[i][l];
      real f = 2 * dot / vv;
      for (int i = j; i < nrow; ++i) a[i][l] -= f * v[i];
    }
    a[j][j] = alpha;
    for (int i = j + 1; i < nrow; ++i) a[i][j] = 0;
  }
}

/* Weighted smoothness rows of one variable between t and t+1 (Eqs. 6-7, row
 * weight ws s^r).  Row r (forward) / k+r (backward); columns 0..k-1 = the
 * variable's y_t, k..2k-1 = its y_{t+1}.  dout (optional) = d/ds of each entry. */
static void smooth_rows(int k, real s, real ws, real out[2 * KMAX][2 * KMAX], real dout[2 * KMAX][2 * KMAX]) {
  memset(out, 0, sizeof(real) * 2 * KMAX * 2 * KMAX);
  if (dout) memset(dout, 0, sizeof(real) * 2 * KMAX * 2 * KMAX);
  for (int r = 0; r < k; ++r) {
    /* forward: ws s^r (sum_{j>=r} s^{j-r}/(j-r)! y_{t,j} - y_{t+1,r}) */
    for (int j = r; j < k; ++j) {
      out[r][j] = ws * ipow(s, j) / fact(j - r);
      if (dout && j > 0) dout[r][j] = ws * j * ipow(s, j - 1) / fact(j - r);
    }
    out[r][k + r] = -ws * ipow(s, r);
    if (dout && r > 0) dout[r][k + r] = -ws * r * ipow(s, r - 1);
    /* backward: ws s^r (sum_{j>=r} (-s)^{j-r}/(j-r)! y_{t+1,j} - y_{t,r}) */
    for (int j = r; j < k; ++j) {
      const real sign = ((j - r) % 2) ? -1 : 1;
      out[k + r][k + j] = ws * sign * ipow(s, j) / fact(j - r);
      if (dout && j > 0) dout[k + r][k + j] = ws * sign * j * ipow(s, j - 1) / fact(j - r);
    }
    out[k + r][r] = -ws * ipow(s, r);
    if (dout && r > 0) dout[k + r][r] = -ws * r * ipow(s, r - 1);
  }
}

/* Factor: Rd[t] (K x K upper), Ro[t] (K x K, coupling y_t -> y_{t+1}), z[t] (K). */
static void factor(const oracle_shape* sh, const inst* in, real* Rd, real* Ro, real* z) {
  const int k = sh->R + 1, V = sh->V, Q = sh->Q, K = V * k;
  const int64_t T = in->T;
  real carry[KMAX][KMAX + 1];
  int have_carry = 0;
  for (int64_t t = 0; t < T; ++t) {
    real a[ROWS][COLS];
    memset(a, 0, sizeof(a));
    const int rhs = 2 * K;
    int nrow = 0;
    if (have_carry) {
      for (int i = 0; i < K; ++i) {
        for (int j = 0; j < K; ++j) a[nrow][j] = carry[i][j];
        a[nrow][rhs] = carry[i][K];
        ++nrow;
      }
    }
    for (int q = 0; q < Q; ++q) {                                      /* Eq. 4 */
      const real wq = in->wg[t * Q + q];
      for (int j = 0; j < K; ++j) a[nrow][j] = wq * (real)in->c[(t * Q + q) * K + j];
      a[nrow][rhs] = wq * (real)in->d[t * Q + q];
      ++nrow;
    }
    if (t < sh->t_init) {                                              /* Eq. 5 */
      for (int v = 0; v < V; ++v)
        for (int r = 0; r < sh->n_init; ++r) {
          const int64_t e = (t * V + v) * sh->n_init + r;
          a[nrow][v * k + r] = in->wi[e];
          a[nrow][rhs] = (real)in->wi[e] * (real)in->u0[e];
          ++nrow;
        }
    }
    int ncol = K;
    if (t + 1 < T) {                                                   /* Eqs. 6-7 */
      real sr[2 * KMAX][2 * KMAX];
      smooth_rows(k, in->s[t], in->ws[t], sr, NULL);
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < 2 * k; ++i) {
          for (int j = 0; j < k; ++j) {
            a[nrow][v * k + j] = sr[i][j];
            a[nrow][K + v * k + j] = sr[i][k + j];
          }
          ++nrow;
        }
      ncol = 2 * K;
    }
    householder(a, nrow, ncol, rhs);
    for (int i = 0; i < K; ++i) {
      for (int j = 0; j < K; ++j) {
        Rd[(t * K + i) * K + j] = a[i][j];
        Ro[(t * K + i) * K + j] = (t + 1 < T) ? a[i][K + j] : 0;
      }
      z[t * K + i] = a[i][rhs];
    }
    if (t + 1 < T) {
      for (int i = 0; i < K; ++i) {
        for (int j = 0; j < K; ++j) carry[i][j] = a[K + i][K + j];
        carry[i][K] = a[K + i][rhs];
      }
      have_carry = 1;
    }
  }
}

/* Solve R x = v (block upper bidiagonal). */
static void back_solve(int K, int64_t T, const real* Rd, const real* Ro, const real* v, real* x) {
  for (int64_t t = T - 1; t >= 0; --t) {
    real rhs[KMAX];
    for (int i = 0; i < K; ++i) {
      rhs[i] = v[t * K + i];
      if (t + 1 < T)
        for (int j = 0; j < K; ++j) rhs[i] -= Ro[(t * K + i) * K + j] * x[(t + 1) * K + j];
    }
    for (int i = K - 1; i >= 0; --i) {
      real acc = rhs[i];
      for (int j = i + 1; j < K; ++j) acc -= Rd[(t * K + i) * K + j] * x[t * K + j];
      x[t * K + i] = acc / Rd[(t * K + i) * K + i];
    }
  }
}

/* Solve R^T x = v (block lower bidiagonal). */
static void fwd_solve_T(int K, int64_t T, const real* Rd, const real* Ro, const real* v, real* x) {
  for (int64_t t = 0; t < T; ++t) {
    real rhs[KMAX];
    for (int j = 0; j < K; ++j) {
      rhs[j] = v[t * K + j];
      if (t > 0)
        for (int i = 0; i < K; ++i) rhs[j] -= Ro[((t - 1) * K + i) * K + j] * x[(t - 1) * K + i];
    }
    for (int j = 0; j < K; ++j) {
      real acc = rhs[j];
      for (int i = 0; i < j; ++i) acc -= Rd[(t * K + i) * K + j] * x[t * K + i];
      x[t * K + j] = acc / Rd[(t * K + j) * K + j];
    }
  }
}

/* Outputs of one instance (NULL members are not wanted). */
typedef struct {
  double *y, *lam, *dc, *dd, *ds, *du0, *dwg, *dwi, *dws;
  double* dw3;   /* the three per-row weight gradient sums, accumulated in `real` */
} outs;

static int solve_one(const oracle_shape* sh, const inst* in, const double* g, outs* o) {
  const int k = sh->R + 1, V = sh->V, Q = sh->Q, K = V * k;
  const int64_t T = in->T, n = T * K;
  real* Rd = (real*)malloc(sizeof(real) * n * K);
  real* Ro = (real*)malloc(sizeof(real) * n * K);
  real* z = (real*)malloc(sizeof(real) * n);
  real* y = (real*)malloc(sizeof(real) * n);
  real* lam = (real*)malloc(sizeof(real) * n);
  if (!Rd || !Ro || !z || !y || !lam) { free(Rd); free(Ro); free(z); free(y); free(lam); return 1; }
  factor(sh, in, Rd, Ro, z);
  back_solve(K, T, Rd, Ro, z, y);
  for (int64_t i = 0; i < n; ++i) o->y[i] = (double)y[i];
  if (g) {
    for (int64_t i = 0; i < n; ++i) z[i] = g[i];
    fwd_solve_T(K, T, Rd, Ro, z, lam);   /* R^T x = g */
    memcpy(z, lam, sizeof(real) * n);
    back_solve(K, T, Rd, Ro, z, lam);    /* R lam = x  => M lam = g (Eq. 14) */
    for (int64_t i = 0; i < n; ++i) o->lam[i] = (double)lam[i];
    /* Closed-form per-row gradients: for a weighted row a~.y = b~ with
     * residual rho = a~.y - b~ and mu = a~.lam, a parameter theta of that row
     * receives -[(da~/dtheta . lam) rho + mu (da~/dtheta . y - db~/dtheta)]. */
    real sum_g = 0, sum_i = 0, sum_s = 0;
    for (int64_t t = 0; t < T; ++t) {     /* governing rows, a~ = wg C_t[q], b~ = wg d_{t,q} */
      real dct[KMAX];
      for (int j = 0; j < K; ++j) dct[j] = 0;
      for (int q = 0; q < Q; ++q) {
        const double* cq = in->c + (t * Q + q) * K;
        const real wq = in->wg[t * Q + q];
        real e = -(real)in->d[t * Q + q], f = 0;
        for (int j = 0; j < K; ++j) { e += (real)cq[j] * y[t * K + j]; f += (real)cq[j] * lam[t * K + j]; }
        for (int j = 0; j < K; ++j) o->dc[(t * Q + q) * K + j] = (double)(-wq * wq * (e * lam[t * K + j] + f * y[t * K + j]));
        o->dd[t * Q + q] = (double)(wq * wq * f);
        o->dwg[t * Q + q] = (double)(-2 * wq * e * f);
        sum_g += -2 * wq * e * f;
      }
      o->ds[t] = 0;
    }
    for (int t = 0; t < sh->t_init; ++t)  /* initial rows (none past the last point) */
      for (int v = 0; v < V; ++v)
        for (int r = 0; r < sh->n_init; ++r) {
          const int64_t e = ((int64_t)t * V + v) * sh->n_init + r;
          if (t >= T) { o->du0[e] = 0; o->dwi[e] = 0; continue; }
          const real wv = in->wi[e];
          o->du0[e] = (double)(wv * wv * lam[t * K + v * k + r]);
          const real gi = -2 * wv * (y[t * K + v * k + r] - (real)in->u0[e]) * lam[t * K + v * k + r];
          o->dwi[e] = (double)gi;
          sum_i += gi;
        }
    for (int64_t t = 0; t < T; ++t) o->dws[t] = 0;
    for (int64_t t = 0; t + 1 < T; ++t) { /* smoothness rows, per variable */
      const real wst = in->ws[t];
      real sr[2 * KMAX][2 * KMAX], dsr[2 * KMAX][2 * KMAX];
      smooth_rows(k, in->s[t], wst, sr, dsr);
      real dst = 0, dwt = 0;
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < 2 * k; ++i) {
          real rho = 0, mu = 0, dl = 0, dy = 0;
          for (int j = 0; j < 2 * k; ++j) {
            const int64_t col = (j < k) ? t * K + v * k + j : (t + 1) * K + v * k + (j - k);
            rho += sr[i][j] * y[col]; mu += sr[i][j] * lam[col];
            dl += dsr[i][j] * lam[col]; dy += dsr[i][j] * y[col];
          }
          dst += -(dl * rho + mu * dy);
          dwt += -2 * rho * mu / wst;
        }
      o->ds[t] = (double)dst;
      o->dws[t] = (double)dwt;
      sum_s += dwt;
    }
    o->dw3[0] = (double)sum_g;
    o->dw3[1] = (double)sum_i;
    o->dw3[2] = (double)sum_s;
  }
  free(Rd); free(Ro); free(z); free(y); free(lam);
  return 0;
}

static void view(const oracle_shape* sh, int64_t i, const int64_t* off, const double* c, const double* d,
                 const double* s, const double* u0, const double* wg, const double* wi, const double* ws,
                 inst* in) {
  const int K = sh->V * (sh->R + 1);
  const int64_t o = off[i];
  const int64_t ni = (int64_t)sh->t_init * sh->V * sh->n_init;
  in->T = off[i + 1] - o;
  in->c = c + o * sh->Q * K;
  in->d = d + o * sh->Q;
  in->s = s + o;
  in->u0 = u0 + i * ni;
  in->wg = wg + o * sh->Q;
  in->wi = wi + i * ni;
  in->ws = ws + o;
}

/* Batched entry points.  off[N+1] = point offsets (instance i owns points
 * off[i]..off[i+1]-1).  Per point: c [Q][K], d [Q], s, wg [Q], ws, y [K];
 * per instance: u0 and wi [T_init][V][n_init].  Returns the number of
 * instances that failed to allocate. */
int oracle_solve(const oracle_shape* sh, int64_t N, const int64_t* off, const double* c, const double* d,
                 const double* s, const double* u0, const double* wg, const double* wi, const double* ws,
                 double* y) {
  const int K = sh->V * (sh->R + 1);
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    inst in;
    view(sh, i, off, c, d, s, u0, wg, wi, ws, &in);
    outs o = {y + off[i] * K, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    fails += solve_one(sh, &in, NULL, &o);
  }
  return fails;
}

int oracle_grad(const oracle_shape* sh, int64_t N, const int64_t* off, const double* c, const double* d,
                const double* s, const double* u0, const double* wg, const double* wi, const double* ws,
                const double* g, double* y, double* lam, double* dc, double* dd, double* ds, double* du0,
                double* dwg, double* dwi, double* dws, double* dw3) {
  const int K = sh->V * (sh->R + 1), Q = sh->Q;
  const int64_t ni = (int64_t)sh->t_init * sh->V * sh->n_init;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    inst in;
    view(sh, i, off, c, d, s, u0, wg, wi, ws, &in);
    const int64_t p = off[i];
    outs o = {y + p * K, lam + p * K, dc + p * Q * K, dd + p * Q, ds + p, du0 + i * ni, dwg + p * Q,
              dwi + i * ni, dws + p, dw3 + 3 * i};
    fails += solve_one(sh, &in, g + p * K, &o);
  }
  return fails;
}

/* Accumulate sigma^2 a a^T of one weighted row into the block row t of M
 * held as blk[K][3K] (columns: block t-1, t, t+1), for the rows of M that
 * lie in block t.  cols are global column indices, base = (t-1) K. */
static void add_row_block(int K, int64_t t, int na, const int64_t* cols, const real* a, real blk[KMAX][3 * KMAX]) {
  const int64_t base = (t - 1) * K;
  for (int i = 0; i < na; ++i) {
    if (cols[i] < t * K || cols[i] >= (t + 1) * K) continue;
    for (int j = 0; j < na; ++j) blk[cols[i] - t * K][cols[j] - base] += a[i] * a[j];
  }
}

/* Normal-equation backward errors of a given y (see the header):
 *  *eta_c = ||A^T W (b - A y)||_inf / || |A|^T W (|A||y| + |b|) ||_inf
 *  *eta_n = ||beta - M y||_inf / (||M||_inf ||y||_inf + ||beta||_inf)
 * (beta - M y = A^T W (b - A y)), both accumulated in `real`. */
static int backward_error_one(const oracle_shape* sh, const inst* in, const double* yd, double* eta_c,
                              double* eta_n) {
  const int k = sh->R + 1, V = sh->V, Q = sh->Q, K = V * k;
  const int64_t T = in->T, n = T * K;
  real* gr = (real*)calloc(n, sizeof(real));
  real* sc = (real*)calloc(n, sizeof(real));
  if (!gr || !sc) { free(gr); free(sc); return 1; }
  real mnorm = 0, bnorm = 0, ynorm = 0;
  for (int64_t i = 0; i < n; ++i) if (RABS((real)yd[i]) > ynorm) ynorm = RABS((real)yd[i]);
  for (int64_t t = 0; t < T; ++t) {
    real blk[KMAX][3 * KMAX];          /* block row t of M */
    real beta[KMAX];
    memset(blk, 0, sizeof(blk));
    for (int j = 0; j < K; ++j) beta[j] = 0;
    int64_t cols[2 * KMAX];
    real a[2 * KMAX];
    for (int q = 0; q < Q; ++q) {                 /* governing */
      const double* cq = in->c + (t * Q + q) * K;
      const real wq = in->wg[t * Q + q], w2 = wq * wq;
      real rho = (real)in->d[t * Q + q], mag = RABS((real)in->d[t * Q + q]);
      for (int j = 0; j < K; ++j) { rho -= (real)cq[j] * (real)yd[t * K + j]; mag += RABS((real)cq[j] * (real)yd[t * K + j]); }
      for (int j = 0; j < K; ++j) {
        gr[t * K + j] += w2 * (real)cq[j] * rho;
        sc[t * K + j] += w2 * RABS((real)cq[j]) * mag;
        beta[j] += w2 * (real)cq[j] * (real)in->d[t * Q + q];
        cols[j] = t * K + j;
        a[j] = wq * (real)cq[j];
      }
      add_row_block(K, t, K, cols, a, blk);
    }
    if (t < sh->t_init)                           /* initial */
      for (int v = 0; v < V; ++v)
        for (int r = 0; r < sh->n_init; ++r) {
          const int64_t e = (t * V + v) * sh->n_init + r;
          const real w2 = (real)in->wi[e] * (real)in->wi[e];
          const real yy = yd[t * K + v * k + r];
          gr[t * K + v * k + r] += w2 * ((real)in->u0[e] - yy);
          sc[t * K + v * k + r] += w2 * (RABS(yy) + RABS((real)in->u0[e]));
          beta[v * k + r] += w2 * (real)in->u0[e];
          blk[v * k + r][K + v * k + r] += w2;
        }
    for (int64_t ts = t - 1; ts <= t; ++ts) {     /* smoothness rows of steps t-1 and t */
      if (ts < 0 || ts + 1 >= T) continue;
      real sr[2 * KMAX][2 * KMAX];
      smooth_rows(k, in->s[ts], in->ws[ts], sr, NULL);
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < 2 * k; ++i) {
          real rho = 0, mag = 0;
          for (int j = 0; j < 2 * k; ++j) {
            cols[j] = (j < k) ? ts * K + v * k + j : (ts + 1) * K + v * k + (j - k);
            a[j] = sr[i][j];
            rho -= sr[i][j] * (real)yd[cols[j]];
            mag += RABS(sr[i][j] * (real)yd[cols[j]]);
          }
          if (ts == t)        /* count each smoothness row once in the residual and scale */
            for (int j = 0; j < 2 * k; ++j) { gr[cols[j]] += sr[i][j] * rho; sc[cols[j]] += RABS(sr[i][j]) * mag; }
          add_row_block(K, t, 2 * k, cols, a, blk);
        }
    }
    for (int i = 0; i < K; ++i) {
      real rs = 0;
      for (int j = 0; j < 3 * K; ++j) rs += RABS(blk[i][j]);
      if (rs > mnorm) mnorm = rs;
      if (RABS(beta[i]) > bnorm) bnorm = RABS(beta[i]);
    }
  }
  real gmax = 0, smax = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (RABS(gr[i]) > gmax) gmax = RABS(gr[i]);
    if (sc[i] > smax) smax = sc[i];
  }
  free(gr); free(sc);
  *eta_c = smax > 0 ? (double)(gmax / smax) : 0.0;
  const real den = mnorm * ynorm + bnorm;
  *eta_n = den > 0 ? (double)(gmax / den) : 0.0;
  return 0;
}

int oracle_backward_error(const oracle_shape* sh, int64_t N, const int64_t* off, const double* c,
                          const double* d, const double* s, const double* u0, const double* wg, const double* wi,
                          const double* ws, const double* y, double* eta_c, double* eta_n) {
  const int K = sh->V * (sh->R + 1);
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    inst in;
    view(sh, i, off, c, d, s, u0, wg, wi, ws, &in);
    fails += backward_error_one(sh, &in, y + off[i] * K, eta_c + i, eta_n + i);
  }
  return fails;
}

static void apply_M(int K, int64_t T, const real* Rd, const real* Ro, const real* v, real* tmp, real* out) {
  /* out = R^T (R v) */
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < K; ++i) {
      real acc = 0;
      for (int j = i; j < K; ++j) acc += Rd[(t * K + i) * K + j] * v[t * K + j];
      if (t + 1 < T)
        for (int j = 0; j < K; ++j) acc += Ro[(t * K + i) * K + j] * v[(t + 1) * K + j];
      tmp[t * K + i] = acc;
    }
  for (int64_t t = 0; t < T; ++t)
    for (int j = 0; j < K; ++j) {
      real acc = 0;
      for (int i = 0; i <= j; ++i) acc += Rd[(t * K + i) * K + j] * tmp[t * K + i];
      if (t > 0)
        for (int i = 0; i < K; ++i) acc += Ro[((t - 1) * K + i) * K + j] * tmp[(t - 1) * K + i];
      out[t * K + j] = acc;
    }
}

static real normalize(int64_t n, real* v) {
  real s = 0;
  for (int64_t i = 0; i < n; ++i) s += v[i] * v[i];
  s = RSQRT(s);
  if (s > 0)
    for (int64_t i = 0; i < n; ++i) v[i] /= s;
  return s;
}

static double cond_one(const oracle_shape* sh, const inst* in, int iters) {
  const int K = sh->V * (sh->R + 1);
  const int64_t T = in->T, n = T * K;
  real* Rd = (real*)malloc(sizeof(real) * n * K);
  real* Ro = (real*)malloc(sizeof(real) * n * K);
  real* z = (real*)malloc(sizeof(real) * n);
  real* v = (real*)malloc(sizeof(real) * n);
  real* t1 = (real*)malloc(sizeof(real) * n);
  real* t2 = (real*)malloc(sizeof(real) * n);
  double kappa = -1.0;
  if (Rd && Ro && z && v && t1 && t2) {
    factor(sh, in, Rd, Ro, z);
    real lmax = 0, lmin_inv = 0;
    for (int64_t i = 0; i < n; ++i) v[i] = 1.0 + 0.5 * sin(0.7 * (double)i);
    normalize(n, v);
    for (int it = 0; it < iters; ++it) {  /* largest eigenvalue of M */
      apply_M(K, T, Rd, Ro, v, t1, t2);
      lmax = normalize(n, t2);
      memcpy(v, t2, sizeof(real) * n);
    }
    for (int64_t i = 0; i < n; ++i) v[i] = 1.0 + 0.5 * cos(1.3 * (double)i);
    normalize(n, v);
    for (int it = 0; it < iters; ++it) {  /* largest eigenvalue of M^{-1} */
      fwd_solve_T(K, T, Rd, Ro, v, t1);
      back_solve(K, T, Rd, Ro, t1, t2);
      lmin_inv = normalize(n, t2);
      memcpy(v, t2, sizeof(real) * n);
    }
    kappa = (double)(lmax * lmin_inv);
  }
  free(Rd); free(Ro); free(z); free(v); free(t1); free(t2);
  return kappa;
}

int oracle_cond(const oracle_shape* sh, int64_t N, const int64_t* off, const double* c, const double* d,
                const double* s, const double* u0, const double* wg, const double* wi, const double* ws,
                int iters, double* kappa) {
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int64_t i = 0; i < N; ++i) {
    inst in;
    view(sh, i, off, c, d, s, u0, wg, wi, ws, &in);
    kappa[i] = cond_one(sh, &in, iters);
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
