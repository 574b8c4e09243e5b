// Per-lane arithmetic of the batched S-MNN least-squares solve.
//
// Everything here is a pure function of register arrays, usable from HIP
// device code (the kernels in smnn_kernels.hip) and from host code (the
// CPU emulator in tests/emu).  Notation follows the paper
// (Scalable Mechanistic Neural Networks):
//   * one instance = V coupled variables (Sec. 3.1) with QE governing
//     equations per time point, block size K = V (R + 1) (Form below; the
//     common case is one (batch, variable) pair, V = QE = 1); initial rows
//     (Eq. 5) at the first T_init nodes;
//   * node t carries the unknowns y_t (K values);
//   * M is block tridiagonal (Eq. 10): diagonal blocks A_t ("M_t"),
//     block (t+1, t) = B_t ("N_t"), right-hand side f_t ("beta_t");
//   * the blocks come from App. A.2: governing term w_g^2 C_t^T C_t, initial
//     term w_i^2 U_t, and the smoothness terms of the rows of Eqs. 6-7
//     weighted by w_s s_t^r (the weighting before Eq. 9), one k x k block
//     per variable; the weights are scalars or per row (App. A.1's W).
//
// Elimination follows the block Cholesky recurrence of Alg. 3 and the
// substitutions of Alg. 4 (Cholesky form, Eqs. 11-13) inside a chunk of
// consecutive nodes; chunks are coupled through separator nodes whose Schur
// complement is again block tridiagonal (see smnn_kernels.hip).
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define SMNN_HD __host__ __device__ __forceinline__
#else
#define SMNN_HD inline
#endif

namespace smnn {

template <int K>
struct Dim {
  static constexpr int Q = K * (K + 1) / 2;  // packed lower triangle
  static constexpr int KK = K * K;
  static constexpr int P = 2 * K - 1;        // powers s^0 .. s^{2R}
};

SMNN_HD constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Compile-time coefficients of the smoothness blocks.  With S+ = diag(s^r),
// F_{ij} = 1/(j-i)! (j >= i) as in App. A.2, every entry of the three blocks
// a pair of neighbouring nodes contributes is w_s^2 s^{i+j} times a constant:
//   left node  (S+ F^T F S+ + S^2)_{ij}      = s^{i+j} (alpha_ij + [i=j])
//   right node (S- F^T F S- + S^2)_{ij}      = s^{i+j} ((-1)^{i+j} alpha_ij + [i=j])
//   coupling   (-S+ F S+ - S- F^T S-)_{ij}   = s^{i+j} nu_ij      (block (t+1, t))
// alpha_ij = sum_{r <= min(i,j)} 1/((i-r)!(j-r)!),
// nu_ij    = -([j >= i]/(j-i)! + [i >= j] (-1)^{i-j}/(i-j)!).
template <int K>
struct Coef {
  double inv_fact[K];
  double alpha[K][K];
  double nu[K][K];
  constexpr Coef() : inv_fact(), alpha(), nu() {
    double f = 1.0;
    for (int n = 0; n < K; ++n) {
      if (n > 0) f *= n;
      inv_fact[n] = 1.0 / f;
    }
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        double s = 0.0;
        const int m = i < j ? i : j;
        for (int r = 0; r <= m; ++r) s += inv_fact[i - r] * inv_fact[j - r];
        alpha[i][j] = s;
        double v = 0.0;
        if (j >= i) v += inv_fact[j - i];
        if (i >= j) v += (((i - j) & 1) ? -1.0 : 1.0) * inv_fact[i - j];
        nu[i][j] = -v;
      }
  }
};

// ---------------------------------------------------------------- algebra
// 1/sqrt(d).  On the GPU: the hardware reciprocal square root estimate
// refined by two Newton steps y <- y (3 - d y^2) / 2 (each roughly doubles the
// number of correct bits), a short dependency chain instead of a correctly
// rounded square root followed by a correctly rounded division.  Non-positive
// d gives NaN or Inf, as 1/sqrt does.
SMNN_HD double rsqrt_pivot(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(d);
  double t = d * y;
  double e = fma(-t, y, 1.0);
  y = fma(0.5 * y, e, y);
  t = d * y;
  e = fma(-t, y, 1.0);
  return fma(0.5 * y, e, y);
#else
  return 1.0 / sqrt(d);
#endif
}

// In-place Cholesky of the packed symmetric matrix D.  On return the strict
// lower part holds L and the diagonal holds 1/L_jj.  Returns false when a
// pivot is not > 0 (or is NaN); the NaN then propagates to the results.
template <int K>
SMNN_HD bool chol(double (&D)[Dim<K>::Q]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double d = D[tri(j, j)];
#pragma unroll
    for (int m = 0; m < j; ++m) d -= D[tri(j, m)] * D[tri(j, m)];
    ok = ok && (d > 0.0);
    const double inv = rsqrt_pivot(d);
    D[tri(j, j)] = inv;
#pragma unroll
    for (int i = j + 1; i < K; ++i) {
      double v = D[tri(i, j)];
#pragma unroll
      for (int m = 0; m < j; ++m) v -= D[tri(i, m)] * D[tri(j, m)];
      D[tri(i, j)] = v * inv;
    }
  }
  return ok;
}

// v <- L^{-1} v
template <int K>
SMNN_HD void lsolve(const double (&L)[Dim<K>::Q], double (&v)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double t = v[j];
#pragma unroll
    for (int m = 0; m < j; ++m) t -= L[tri(j, m)] * v[m];
    v[j] = t * L[tri(j, j)];
  }
}

// v <- L^{-T} v
template <int K>
SMNN_HD void usolve(const double (&L)[Dim<K>::Q], double (&v)[K]) {
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    double t = v[j];
#pragma unroll
    for (int m = j + 1; m < K; ++m) t -= L[tri(m, j)] * v[m];
    v[j] = t * L[tri(j, j)];
  }
}

// W <- W L^{-T}   (W row-major K x K)
template <int K>
SMNN_HD void rsolve_t(const double (&L)[Dim<K>::Q], double (&W)[Dim<K>::KK]) {
#pragma unroll
  for (int r = 0; r < K; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double t = W[r * K + j];
#pragma unroll
      for (int m = 0; m < j; ++m) t -= W[r * K + m] * L[tri(j, m)];
      W[r * K + j] = t * L[tri(j, j)];
    }
}

// X <- L^{-1} X   (column by column)
template <int K>
SMNN_HD void lsolve_cols(const double (&L)[Dim<K>::Q], double (&X)[Dim<K>::KK]) {
#pragma unroll
  for (int c = 0; c < K; ++c)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double t = X[j * K + c];
#pragma unroll
      for (int m = 0; m < j; ++m) t -= L[tri(j, m)] * X[m * K + c];
      X[j * K + c] = t * L[tri(j, j)];
    }
}

// D <- A - W W^T  (packed lower)
template <int K>
SMNN_HD void sym_minus_wwt(const double (&A)[Dim<K>::Q], const double (&W)[Dim<K>::KK],
                           double (&D)[Dim<K>::Q]) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double t = A[tri(i, j)];
#pragma unroll
      for (int m = 0; m < K; ++m) t -= W[i * K + m] * W[j * K + m];
      D[tri(i, j)] = t;
    }
}

// y <- y - W x
template <int K>
SMNN_HD void sub_matvec(const double (&W)[Dim<K>::KK], const double (&x)[K], double (&y)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double t = y[i];
#pragma unroll
    for (int m = 0; m < K; ++m) t -= W[i * K + m] * x[m];
    y[i] = t;
  }
}

// y <- y - B^T x
template <int K>
SMNN_HD void sub_matvec_t(const double (&B)[Dim<K>::KK], const double (&x)[K], double (&y)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double t = y[i];
#pragma unroll
    for (int m = 0; m < K; ++m) t -= B[m * K + i] * x[m];
    y[i] = t;
  }
}

// Z <- -W X
template <int K>
SMNN_HD void neg_matmul(const double (&W)[Dim<K>::KK], const double (&X)[Dim<K>::KK],
                        double (&Z)[Dim<K>::KK]) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double t = 0.0;
#pragma unroll
      for (int m = 0; m < K; ++m) t -= W[i * K + m] * X[m * K + j];
      Z[i * K + j] = t;
    }
}

// S += X^T X (packed), r += X^T g
template <int K>
SMNN_HD void acc_xtx(const double (&X)[Dim<K>::KK], const double (&g)[K], double (&S)[Dim<K>::Q],
                     double (&r)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double t = S[tri(i, j)];
#pragma unroll
      for (int m = 0; m < K; ++m) t += X[m * K + i] * X[m * K + j];
      S[tri(i, j)] = t;
    }
    double t = r[i];
#pragma unroll
    for (int m = 0; m < K; ++m) t += X[m * K + i] * g[m];
    r[i] = t;
  }
}

// ------------------------------------------------------- smoothness blocks
template <int K>
SMNN_HD void powers(double s, double (&pw)[Dim<K>::P]) {
  pw[0] = 1.0;
#pragma unroll
  for (int e = 1; e < Dim<K>::P; ++e) pw[e] = pw[e - 1] * s;
}

// The smoothness rows of Eqs. 6-7 act on one variable's k = R+1 unknowns
// (App. A.2: S_t = Diag(S_t^*, ..., S_t^*) over the V variables).  The
// functions below add one variable's k x k block into the K x K block of a
// node (K = V k), at unknowns off .. off+k-1.

// A += w_s^2 * (smoothness block of the LEFT node of a pair with step s)
template <int k, int K = k>
SMNN_HD void add_left_block(const double (&pw)[Dim<k>::P], double ws2, double (&A)[Dim<K>::Q], int off = 0) {
  constexpr Coef<k> C{};
#pragma unroll
  for (int i = 0; i < k; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      A[tri(off + i, off + j)] += ws2 * pw[i + j] * (C.alpha[i][j] + (i == j ? 1.0 : 0.0));
}

// A += w_s^2 * (smoothness block of the RIGHT node of a pair with step s)
template <int k, int K = k>
SMNN_HD void add_right_block(const double (&pw)[Dim<k>::P], double ws2, double (&A)[Dim<K>::Q], int off = 0) {
  constexpr Coef<k> C{};
#pragma unroll
  for (int i = 0; i < k; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      A[tri(off + i, off + j)] += ws2 * pw[i + j] *
                                  ((((i + j) & 1) ? -C.alpha[i][j] : C.alpha[i][j]) + (i == j ? 1.0 : 0.0));
}

// B = w_s^2 * coupling block (row = right node, column = left node), at
// rows and columns off .. off+k-1 of the K x K block (the rest untouched)
template <int k, int K = k>
SMNN_HD void coupling_block(const double (&pw)[Dim<k>::P], double ws2, double (&B)[Dim<K>::KK], int off = 0) {
  constexpr Coef<k> C{};
#pragma unroll
  for (int i = 0; i < k; ++i)
#pragma unroll
    for (int j = 0; j < k; ++j) B[(off + i) * K + off + j] = ws2 * pw[i + j] * C.nu[i][j];
}

// Row residuals of the 2K weighted smoothness rows of a pair (Eqs. 6-7 scaled
// by w_s s^r) at (v_t, v_{t+1}): rho = -(a . v); returns the contributions
// a^T rho to the left node (cl) and to the right node (cr).
//
// The residual of an iterate near the solution is a small difference of
// large terms, so its rounding noise is a sizeable part of its value.  That
// noise is harmless only if every kernel that evaluates the residual of a
// node (the reduce and the back-substitution passes) rounds it identically,
// so contraction into FMAs -- which the compiler may decide differently in
// different kernels -- is switched off here and in residual_rhs below.
template <int K>
SMNN_HD void pair_residual(const double (&pw)[Dim<K>::P], double ws, const double (&vt)[K],
                           const double (&vn)[K], double (&cl)[K], double (&cr)[K]) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
  constexpr Coef<K> C{};
  double wp[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    wp[j] = ws * pw[j];
    cl[j] = 0.0;
    cr[j] = 0.0;
  }
#pragma unroll
  for (int r = 0; r < K; ++r) {
    // weighted coefficients of forward row r on v_{t,j} (and, with sign
    // (-1)^{j-r}, of backward row r on v_{t+1,j}): w_s s^j/(j-r)!
    double cf[K];
#pragma unroll
    for (int j = r; j < K; ++j) cf[j] = (j == r) ? wp[j] : wp[j] * C.inv_fact[j - r];
    // forward row r: sum_{j>=r} cf_j v_{t,j} - w_s s^r v_{t+1,r};  rho = -(row . v)
    double af = -(wp[r] * vn[r]);
#pragma unroll
    for (int j = r; j < K; ++j) af = fma(cf[j], vt[j], af);
    // backward row r: sum_{j>=r} (-1)^{j-r} cf_j v_{t+1,j} - w_s s^r v_{t,r}
    double ab = -(wp[r] * vt[r]);
#pragma unroll
    for (int j = r; j < K; ++j) ab = fma(((j - r) & 1) ? -cf[j] : cf[j], vn[j], ab);
#pragma unroll
    for (int j = r; j < K; ++j) {
      cl[j] = fma(cf[j], -af, cl[j]);
      cr[j] = fma(((j - r) & 1) ? -cf[j] : cf[j], -ab, cr[j]);
    }
    cr[r] = fma(wp[r], af, cr[r]);     // (-w_s s^r) * rho_f, rho_f = -af
    cl[r] = fma(wp[r], ab, cl[r]);     // (-w_s s^r) * rho_b
  }
}

// Gradient contributions of the 2K smoothness rows of a pair.  For a weighted
// row a~ (depends on s and w_s) with rho = a~.y and mu = a~.lam the loss
// gradient is -( (da~.lam) rho + mu (da~.y) ) for s and -2 rho mu / w_s for
// w_s.  Rows are evaluated without the w_s factor (hat) to avoid dividing.
template <int K>
SMNN_HD void pair_grad(double s, double ws, const double (&yt)[K], const double (&yn)[K],
                       const double (&lt)[K], const double (&ln)[K], double& ds, double& dws) {
  constexpr Coef<K> C{};
  double pw[K];
  pw[0] = 1.0;
#pragma unroll
  for (int e = 1; e < K; ++e) pw[e] = pw[e - 1] * s;
  double acc_s = 0.0, acc_w = 0.0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    // forward row r
    double rho = -pw[r] * yn[r], mu = -pw[r] * ln[r];
    double dy = (r > 0) ? -r * pw[r - 1] * yn[r] : 0.0;
    double dl = (r > 0) ? -r * pw[r - 1] * ln[r] : 0.0;
#pragma unroll
    for (int j = r; j < K; ++j) {
      const double cf = C.inv_fact[j - r];
      rho += pw[j] * cf * yt[j];
      mu += pw[j] * cf * lt[j];
      if (j > 0) {
        dy += j * pw[j - 1] * cf * yt[j];
        dl += j * pw[j - 1] * cf * lt[j];
      }
    }
    acc_s += dl * rho + mu * dy;
    acc_w += rho * mu;
    // backward row r
    rho = -pw[r] * yt[r];
    mu = -pw[r] * lt[r];
    dy = (r > 0) ? -r * pw[r - 1] * yt[r] : 0.0;
    dl = (r > 0) ? -r * pw[r - 1] * lt[r] : 0.0;
#pragma unroll
    for (int j = r; j < K; ++j) {
      const double cf = ((j - r) & 1) ? -C.inv_fact[j - r] : C.inv_fact[j - r];
      rho += pw[j] * cf * yn[j];
      mu += pw[j] * cf * ln[j];
      if (j > 0) {
        dy += j * pw[j - 1] * cf * yn[j];
        dl += j * pw[j - 1] * cf * ln[j];
      }
    }
    acc_s += dl * rho + mu * dy;
    acc_w += rho * mu;
  }
  ds = -ws * ws * acc_s;
  dws = -2.0 * ws * acc_w;
}

// Chunk geometry at one level.  Chunks have L nodes; chunk j of an instance
// with n nodes owns nodes jL .. min(jL+L, n)-1.  Every chunk but the last
// ends in a separator (its last owned node); the last chunk has no separator
// and may hold up to L interior nodes.  n <= L gives a single chunk.
struct ChunkGeom {
  int64_t a, b;       // interior nodes a..b
  bool has_left, has_right;
};

SMNN_HD ChunkGeom chunk_geom(int64_t j, int64_t n, int L) {
  ChunkGeom g;
  g.a = j * L;
  const bool last = g.a + L >= n;
  g.b = last ? n - 1 : g.a + L - 2;
  g.has_left = j > 0;
  g.has_right = !last;
  return g;
}

// ------------------------------------------------------------ chunk cores
// A chunk covers nodes a..b of one instance's block-tridiagonal system.  The
// node at a-1 (if has_left) and b+1 (if has_right) are separators.  Src
// supplies   load(i, A, f, Bp)  diagonal block, right-hand side and (for
//                               i > 0) block (i, i-1) of node i,
//            coupling(i, B)     block (i+1, i).

// Result of eliminating a chunk's interior (Schur complement pieces).
template <int K>
struct Reduced {
  double rA[Dim<K>::Q];   // right separator: A_{b+1} - B_b D_b^{-1} B_b^T
  double rf[K];           //                  f_{b+1} - B_b D_b^{-1} g_b
  double lA[Dim<K>::Q];   // left separator contribution: -E_L^T A_I^{-1} E_L
  double lf[K];           //                              -E_L^T A_I^{-1} f_I
  double lB[Dim<K>::KK];  // coupling (b+1, a-1): -B_b [A_I^{-1}]_{b,a} B_{a-1}
  int fail;               // chunk-relative node + 1 of the first non-positive pivot, 0 if none
};

template <int K, int L, class Src>
SMNN_HD void reduce_chunk(const Src& src, int64_t a, int64_t b, bool has_left, bool has_right,
                          Reduced<K>& out) {
  constexpr int Q = Dim<K>::Q, KK = Dim<K>::KK;
  double Lc[Q], gh[K], Xh[KK];
#pragma unroll
  for (int e = 0; e < Q; ++e) out.lA[e] = 0.0;
#pragma unroll
  for (int e = 0; e < K; ++e) out.lf[e] = 0.0;
#pragma unroll
  for (int e = 0; e < KK; ++e) { out.lB[e] = 0.0; Xh[e] = 0.0; }
  out.fail = 0;
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int64_t i = a + u;
    if (i > b) break;
    double A[Q], f[K], Bp[KK];
    src.load(i, A, f, Bp);                     // Bp = B_{i-1} (block (i, i-1)) when i > 0
    double D[Q], X[KK];
    if (u == 0) {
#pragma unroll
      for (int e = 0; e < Q; ++e) D[e] = A[e];
      if (has_left) {
#pragma unroll
        for (int e = 0; e < KK; ++e) X[e] = Bp[e];   // E_L block: (a, a-1) = B_{a-1}
      }
    } else {
      double (&W)[KK] = Bp;
      rsolve_t<K>(Lc, W);                      // W = B_{i-1} L_{i-1}^{-T}
      sym_minus_wwt<K>(A, W, D);               // D_i = A_i - W W^T
      sub_matvec<K>(W, gh, f);                 // g_i = f_i - W ghat_{i-1}
      if (has_left) neg_matmul<K>(W, Xh, X);   // X_i = -W Xhat_{i-1}
    }
    const bool ok = chol<K>(D);
    if (!ok && out.fail == 0) out.fail = u + 1;
#pragma unroll
    for (int e = 0; e < Q; ++e) Lc[e] = D[e];
#pragma unroll
    for (int e = 0; e < K; ++e) gh[e] = f[e];
    lsolve<K>(Lc, gh);                         // ghat_i = L_i^{-1} g_i
    if (has_left) {
#pragma unroll
      for (int e = 0; e < KK; ++e) Xh[e] = X[e];
      lsolve_cols<K>(Lc, Xh);                  // Xhat_i = L_i^{-1} X_i
      acc_xtx<K>(Xh, gh, out.lA, out.lf);      // sum Xhat^T Xhat, sum Xhat^T ghat
    }
  }
  if (has_left) {
#pragma unroll
    for (int e = 0; e < Q; ++e) out.lA[e] = -out.lA[e];
#pragma unroll
    for (int e = 0; e < K; ++e) out.lf[e] = -out.lf[e];
  }
  if (has_right) {
    double V[KK], A[Q], f[K];
    src.load(b + 1, A, f, V);                  // V = B_b
    rsolve_t<K>(Lc, V);                        // V = B_b L_b^{-T}
    sym_minus_wwt<K>(A, V, out.rA);
    sub_matvec<K>(V, gh, f);
#pragma unroll
    for (int e = 0; e < K; ++e) out.rf[e] = f[e];
    if (has_left) neg_matmul<K>(V, Xh, out.lB);
  }
}

// The right-hand-side half of reduce_chunk for a chunk whose factor is
// already known (Ls[u] = Cholesky factor of node a+u's reduced diagonal
// block, as backsub_forward leaves it for the same nodes and matrix): the
// forward substitution of Alg. 4 over the interior and the separators'
// right-hand-side pieces rf and lf.  The matrix pieces rA, lA, lB and the
// pivots are not formed (a right-hand-side-only solve reuses the separator
// records of the first one).  Bitwise equal to reduce_chunk's rf, lf.
template <int K, int L, class Src>
SMNN_HD void reduce_chunk_rhs(const Src& src, int64_t a, int64_t b, bool has_left, bool has_right,
                              const double (&Ls)[L][Dim<K>::Q], Reduced<K>& out) {
  constexpr int Q = Dim<K>::Q, KK = Dim<K>::KK;
  double gh[K], Xh[KK], Lb[Q];
#pragma unroll
  for (int e = 0; e < K; ++e) out.lf[e] = 0.0;
#pragma unroll
  for (int e = 0; e < KK; ++e) Xh[e] = 0.0;
  out.fail = 0;
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int64_t i = a + u;
    if (i > b) break;
#pragma unroll
    for (int e = 0; e < Q; ++e) Lb[e] = Ls[u][e];   // the last node's factor after the loop
    double A[Q], f[K], Bp[KK];
    src.load(i, A, f, Bp);                     // A unused
    double X[KK];
    if (u == 0) {
      if (has_left) {
#pragma unroll
        for (int e = 0; e < KK; ++e) X[e] = Bp[e];
      }
    } else {
      double (&W)[KK] = Bp;
      rsolve_t<K>(Ls[u > 0 ? u - 1 : 0], W);   // W = B_{i-1} L_{i-1}^{-T}
      sub_matvec<K>(W, gh, f);
      if (has_left) neg_matmul<K>(W, Xh, X);
    }
#pragma unroll
    for (int e = 0; e < K; ++e) gh[e] = f[e];
    lsolve<K>(Ls[u], gh);
    if (has_left) {
#pragma unroll
      for (int e = 0; e < KK; ++e) Xh[e] = X[e];
      lsolve_cols<K>(Ls[u], Xh);
#pragma unroll
      for (int r = 0; r < K; ++r) {
        double t = out.lf[r];
#pragma unroll
        for (int m = 0; m < K; ++m) t += Xh[m * K + r] * gh[m];
        out.lf[r] = t;
      }
    }
  }
  if (has_left) {
#pragma unroll
    for (int e = 0; e < K; ++e) out.lf[e] = -out.lf[e];
  }
  if (has_right) {
    double V[KK], A[Q], f[K];
    src.load(b + 1, A, f, V);                  // V = B_b; A unused
    rsolve_t<K>(Lb, V);                        // V = B_b L_b^{-T}
    sub_matvec<K>(V, gh, f);
#pragma unroll
    for (int e = 0; e < K; ++e) out.rf[e] = f[e];
  }
}

// Receives nothing: the caller reads x afterwards.
struct NoSink {
  template <int K>
  SMNN_HD void node(int64_t, const double (&)[K]) {}
};

// Solve the chunk interior a..b with the separator values xl (node a-1) and
// xr (node b+1) known, in two sweeps.  The forward sweep factors the interior
// (Ls[u] = Cholesky factor of node a+u's reduced diagonal block) and leaves
// the forward-substituted right-hand sides in x; the backward sweep turns x
// into the solution, x[u] = node a+u for u = 0..b-a, and calls sink.node(i,
// x_i) as each node is finished, in decreasing order of i.  Returns the
// chunk-relative node + 1 of the first non-positive pivot, 0 if none.
template <int K, int L, class Src>
SMNN_HD int backsub_forward(const Src& src, int64_t a, int64_t b, bool has_left, bool has_right,
                            const double (&xl)[K], const double (&xr)[K], double (&Ls)[L][Dim<K>::Q],
                            double (&x)[L][K]) {
  constexpr int Q = Dim<K>::Q, KK = Dim<K>::KK;
  int fail = 0;
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int64_t i = a + u;
    if (i > b) break;
    double A[Q], f[K], Bp[KK];
    src.load(i, A, f, Bp);                     // Bp = B_{i-1} when i > 0
    if (u == 0 && has_left) sub_matvec<K>(Bp, xl, f);   // f_a -= B_{a-1} x_{a-1}
    if (i == b && has_right) {
      double B[KK];
      src.coupling(b, B);
      sub_matvec_t<K>(B, xr, f);               // f_b -= B_b^T x_{b+1}
    }
    double D[Q];
    if (u == 0) {
#pragma unroll
      for (int e = 0; e < Q; ++e) D[e] = A[e];
    } else {
      double (&W)[KK] = Bp;
      rsolve_t<K>(Ls[u > 0 ? u - 1 : 0], W);   // W = B_{i-1} L_{i-1}^{-T}
      sym_minus_wwt<K>(A, W, D);               // D_i = A_i - W W^T
      sub_matvec<K>(W, x[u > 0 ? u - 1 : 0], f);
    }
    const bool ok = chol<K>(D);
    if (!ok && fail == 0) fail = u + 1;
#pragma unroll
    for (int e = 0; e < Q; ++e) Ls[u][e] = D[e];
    lsolve<K>(Ls[u], f);                       // ghat_i = L_i^{-1} g_i
#pragma unroll
    for (int e = 0; e < K; ++e) x[u][e] = f[e];
  }
  return fail;
}

template <int K, int L, class Src, class Sink = NoSink>
SMNN_HD void backsub_backward(const Src& src, int64_t a, int64_t b, const double (&Ls)[L][Dim<K>::Q],
                              double (&x)[L][K], Sink&& sink = Sink()) {
  constexpr int KK = Dim<K>::KK;
#pragma unroll
  for (int u = L - 1; u >= 0; --u) {
    const int64_t i = a + u;
    if (i > b) continue;
    if (i < b) {
      double B[KK], t[K];
      src.coupling(i, B);
#pragma unroll
      for (int e = 0; e < K; ++e) t[e] = 0.0;
      sub_matvec_t<K>(B, x[u + 1 < L ? u + 1 : u], t);   // t = -B_i^T x_{i+1}
      lsolve<K>(Ls[u], t);
#pragma unroll
      for (int e = 0; e < K; ++e) x[u][e] += t[e];
    }
    usolve<K>(Ls[u], x[u]);                    // x_i = L^{-T}(ghat_i - L^{-1} B_i^T x_{i+1})
    sink.template node<K>(i, x[u]);
  }
}

template <int K, int L, class Src, class Sink = NoSink>
SMNN_HD int backsub_chunk(const Src& src, int64_t a, int64_t b, bool has_left, bool has_right,
                          const double (&xl)[K], const double (&xr)[K], double (&x)[L][K],
                          Sink&& sink = Sink()) {
  double Ls[L][Dim<K>::Q];
  const int fail = backsub_forward<K, L>(src, a, b, has_left, has_right, xl, xr, Ls, x);
  backsub_backward<K, L>(src, a, b, Ls, x, static_cast<Sink&&>(sink));
  return fail;
}

// ----------------------------------------------------------- level-0 source
// Shape of one instance's constraint rows (Sec. 3.1, Eq. 4; App. A.1-A.2):
// V variables with k = K / V unknowns each (orders 0..R of that variable;
// block size K = V (R+1)), QE governing equations per time point over all K
// unknowns (App. A.2's C_t is QE x K), and weights either three scalars per
// instance (WROW false: w_gov, w_init, w_smooth) or one per row (WROW true:
// App. A.1's W = diag(w) with a governing weight per (point, equation), an
// initial weight per (point, variable, order) and a smoothness weight per
// step, which scales that step's Taylor rows of every variable and order
// together with s_t^r).
template <int V_, int QE_, bool WROW_>
struct Form {
  static constexpr int V = V_, QE = QE_;
  static constexpr bool WROW = WROW_;
};
using FormScalar = Form<1, 1, false>;

// Per-instance parameters: scalar weights (unsquared; unused with per-row
// weights), and the shape of the initial rows (Eq. 5): orders < n_init of
// every variable at each of the first t_init points.  The initial values
// themselves are read from memory at those nodes only.
template <int K>
struct Inst {
  double wg, wi, ws;
  int n_init;
  int t_init = 1;
};

enum RhsMode : int {
  RHS_BETA = 0,   // f = beta (Eq. 9's A^T W b, App. A.2)
  RHS_RESID = 1,  // f = A^T W (b - A v)         (refinement of the solution)
  RHS_G = 2,      // f = g = dl/dy                (adjoint, Eq. 14)
  RHS_GRESID = 3  // f = g - A^T W A v            (refinement of the adjoint)
};

// Where element e of a per-step array with W elements per row lives: the
// identity for arrays in global memory (and on the host); the GPU kernels
// pass a policy that places the rows they stage in LDS (smnn_kernels.hip).
struct IxPlain {
  template <int W>
  SMNN_HD static int64_t at(int64_t e) { return e; }
};

// Node data assembled on the fly from the per-step inputs of one instance.
// TIO is the element type of the arrays in memory (double or float); IX
// maps the element indices of c, d, s, g, v and the per-row weights.
template <int K, class TIO, int RHS, class F = FormScalar, class IX = IxPlain>
struct Src0 {
  static constexpr int V = F::V, QE = F::QE, k = K / F::V;
  static_assert(k * V == K, "block size is V (R+1)");
  const TIO* c;      // [..][QE][K] node i of this instance is row o + i
  const TIO* d;      // [..][QE]
  const TIO* s;      // [..]  (s of the last node unused)
  const TIO* g;      // [..][K]  dl/dy (RHS_G, RHS_GRESID)
  const TIO* v;      // [..][K]  previous iterate (RHS_RESID, RHS_GRESID)
  const TIO* wg = nullptr;   // [..][QE] governing weights (per-row weights)
  const TIO* wsm = nullptr;  // [..]     smoothness weight of the pair (i, i+1) (per-row weights)
  const TIO* u = nullptr;    // initial values of every instance, [N][t_init][V][n_init]
  const TIO* wi = nullptr;   // initial weights, same layout as u (per-row weights)
  int uo = 0;                // element offset of this instance's block in u (and wi)
  int64_t n;
  int64_t o = 0;     // row of node 0 in the arrays above
  Inst<K> p;
  // residual modes: contribution of pair (next_node-1, next_node) to next_node,
  // computed with the previous node (nodes are visited in increasing order)
  mutable double carry[K];
  mutable int64_t carry_node = -1;

  SMNN_HD double ld(const TIO* ptr, int64_t i) const {
    return static_cast<double>(ptr[IX::template at<1>(o + i)]);
  }
  SMNN_HD double ldk(const TIO* ptr, int64_t i, int r) const {
    return static_cast<double>(ptr[IX::template at<K>((o + i) * K + r)]);
  }
  // coefficient j of governing equation q at node i; its right-hand side
  SMNN_HD double ldc(int64_t i, int q, int j) const {
    return static_cast<double>(c[IX::template at<QE * K>(((o + i) * QE + q) * K + j)]);
  }
  SMNN_HD double ldd(int64_t i, int q) const { return static_cast<double>(d[IX::template at<QE>((o + i) * QE + q)]); }
  // weights (unsquared) of governing row (i, q), of the pair (i, i+1) and of
  // initial row (i, variable vv, order r)
  SMNN_HD double gov_w(int64_t i, int q) const {
    if constexpr (F::WROW) return static_cast<double>(wg[IX::template at<QE>((o + i) * QE + q)]);
    else return p.wg;
  }
  SMNN_HD double smooth_w(int64_t i) const {
    if constexpr (F::WROW) return ld(wsm, i);
    else return p.ws;
  }
  SMNN_HD int uidx(int64_t i, int vv, int r) const {
    return uo + (static_cast<int>(i) * V + vv) * p.n_init + r;
  }
  SMNN_HD double init_w(int64_t i, int vv, int r) const {
    if constexpr (F::WROW) return static_cast<double>(wi[uidx(i, vv, r)]);
    else return p.wi;
  }
  // initial value of order r of variable vv at node i < t_init
  SMNN_HD double uval(int64_t i, int vv, int r) const { return static_cast<double>(u[uidx(i, vv, r)]); }

  SMNN_HD void coupling(int64_t i, double (&B)[Dim<K>::KK]) const {
    double pw[Dim<k>::P];
    powers<k>(ld(s, i), pw);
    const double w = smooth_w(i);
    if (V > 1) {
#pragma unroll
      for (int e = 0; e < Dim<K>::KK; ++e) B[e] = 0.0;
    }
#pragma unroll
    for (int vv = 0; vv < V; ++vv) coupling_block<k, K>(pw, w * w, B, vv * k);
  }

  // f = A^T W (b - A v) (RHS_RESID) or g - A^T W A v (RHS_GRESID) at node i,
  // evaluated row by row from the constraint rows touching the node.  ci is
  // governing row 0 of the node (the caller has it loaded).
  SMNN_HD void residual_rhs(int64_t i, const double (&ci)[K], bool has_next, bool has_prev,
                            const double (&pl)[Dim<k>::P], const double (&pr)[Dim<k>::P], double (&f)[K]) const {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    double vi[K];
#pragma unroll
    for (int r = 0; r < K; ++r) vi[r] = ldk(v, i, r);
#pragma unroll
    for (int q = 0; q < QE; ++q) {
      double cq[K];
#pragma unroll
      for (int r = 0; r < K; ++r) cq[r] = q == 0 ? ci[r] : ldc(i, q, r);
      const double w = gov_w(i, q);
      double e = (RHS == RHS_RESID) ? ldd(i, q) : 0.0;
#pragma unroll
      for (int r = 0; r < K; ++r) e = fma(-cq[r], vi[r], e);
      const double we = (w * w) * e;
#pragma unroll
      for (int r = 0; r < K; ++r) {
        if (q == 0) f[r] = (RHS == RHS_GRESID) ? fma(cq[r], we, ldk(g, i, r)) : cq[r] * we;
        else f[r] = fma(cq[r], we, f[r]);
      }
    }
    if (i < p.t_init) {
#pragma unroll
      for (int vv = 0; vv < V; ++vv)
#pragma unroll
        for (int r = 0; r < k; ++r)
          if (r < p.n_init) {
            const double w = init_w(i, vv, r);
            f[vv * k + r] += (w * w) * ((RHS == RHS_RESID ? uval(i, vv, r) : 0.0) - vi[vv * k + r]);
          }
    }
    if (has_prev) {
      double cr[K];
      if (carry_node == i) {
#pragma unroll
        for (int r = 0; r < K; ++r) cr[r] = carry[r];
      } else {
        const double w = smooth_w(i - 1);
#pragma unroll
        for (int vv = 0; vv < V; ++vv) {
          double vp[k], vc[k], cl[k], crv[k];
#pragma unroll
          for (int r = 0; r < k; ++r) { vp[r] = ldk(v, i - 1, vv * k + r); vc[r] = vi[vv * k + r]; }
          pair_residual<k>(pl, w, vp, vc, cl, crv);
#pragma unroll
          for (int r = 0; r < k; ++r) cr[vv * k + r] = crv[r];
        }
      }
#pragma unroll
      for (int r = 0; r < K; ++r) f[r] += cr[r];
    }
    if (has_next) {
      const double w = smooth_w(i);
#pragma unroll
      for (int vv = 0; vv < V; ++vv) {
        double vc[k], vn[k], cl[k], crv[k];
#pragma unroll
        for (int r = 0; r < k; ++r) { vc[r] = vi[vv * k + r]; vn[r] = ldk(v, i + 1, vv * k + r); }
        pair_residual<k>(pr, w, vc, vn, cl, crv);
#pragma unroll
        for (int r = 0; r < k; ++r) {
          carry[vv * k + r] = crv[r];
          f[vv * k + r] += cl[r];
        }
      }
      carry_node = i + 1;
    }
  }

  SMNN_HD void load(int64_t i, double (&A)[Dim<K>::Q], double (&f)[K], double (&Bp)[Dim<K>::KK]) const {
    double ci[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ci[r] = ldc(i, 0, r);
    // governing rows: w_q^2 c_q c_q^T (App. A.2's C_t^T C_t, weighted per row)
#pragma unroll
    for (int q = 0; q < QE; ++q) {
      double cq[K];
#pragma unroll
      for (int r = 0; r < K; ++r) cq[r] = q == 0 ? ci[r] : ldc(i, q, r);
      const double w = gov_w(i, q), wg2 = w * w;
#pragma unroll
      for (int r = 0; r < K; ++r)
#pragma unroll
        for (int j = 0; j <= r; ++j) {
          if (q == 0) A[tri(r, j)] = wg2 * cq[r] * cq[j];
          else A[tri(r, j)] += wg2 * cq[r] * cq[j];
        }
      if (RHS == RHS_BETA) {
        const double dq = ldd(i, q);
#pragma unroll
        for (int r = 0; r < K; ++r) {
          if (q == 0) f[r] = wg2 * cq[r] * dq;
          else f[r] += wg2 * cq[r] * dq;
        }
      }
    }
    if (i < p.t_init) {
#pragma unroll
      for (int vv = 0; vv < V; ++vv)
#pragma unroll
        for (int r = 0; r < k; ++r)
          if (r < p.n_init) {
            const double w = init_w(i, vv, r), wi2 = w * w;
            A[tri(vv * k + r, vv * k + r)] += wi2;
            if (RHS == RHS_BETA) f[vv * k + r] += wi2 * uval(i, vv, r);
          }
    }
    double pl[Dim<k>::P], pr[Dim<k>::P];
    const bool has_next = i + 1 < n, has_prev = i > 0;
    if (has_next) {
      powers<k>(ld(s, i), pr);
      const double w = smooth_w(i);
#pragma unroll
      for (int vv = 0; vv < V; ++vv) add_left_block<k, K>(pr, w * w, A, vv * k);
    }
    if (has_prev) {
      powers<k>(ld(s, i - 1), pl);
      const double w = smooth_w(i - 1);
      if (V > 1) {
#pragma unroll
        for (int e = 0; e < Dim<K>::KK; ++e) Bp[e] = 0.0;
      }
#pragma unroll
      for (int vv = 0; vv < V; ++vv) {
        add_right_block<k, K>(pl, w * w, A, vv * k);
        coupling_block<k, K>(pl, w * w, Bp, vv * k);
      }
    }
    if (RHS == RHS_G) {
#pragma unroll
      for (int r = 0; r < K; ++r) f[r] = ldk(g, i, r);
    } else if (RHS != RHS_BETA) {
      residual_rhs(i, ci, has_next, has_prev, pl, pr, f);
    }
  }
};

// Level-0 solution sink: out_i = (v_i +) x_i in the I/O type.  Rows of out
// are RS elements apart (0: K, dense); IX maps element indices as in Src0.
template <class TIO, bool ADD, int RS = 0, class IX = IxPlain>
struct StoreSink {
  TIO* out;        // [..][RS]: node i is row oo + i, its first K elements
  const TIO* v;    // previous iterate (ADD): node i is row vo + i
  int64_t vo = 0;
  int64_t oo = 0;
  template <int K>
  SMNN_HD void node(int64_t i, const double (&x)[K]) {
    constexpr int W = RS ? RS : K;
#pragma unroll
    for (int e = 0; e < K; ++e) {
      double val = x[e];
      if (ADD) val += static_cast<double>(v[IX::template at<K>((vo + i) * K + e)]);
      out[IX::template at<W>((oo + i) * W + e)] = static_cast<TIO>(val);
    }
  }
};

// Level-0 gradient sink.  As the back-substitution finishes node i (in
// decreasing order) with lam_i = (v_i +) x_i it forms the gradients of the
// rows the chunk owns: the governing rows of node i, the initial rows when
// i < t_init, and the smoothness pair (i, i+1), using the node finished just
// before.  Per weighted row a~.y = b~ with rho = a~.y - b~ and mu = a~.lam,
// dl/dtheta = -[(da~.lam) rho + mu (da~.y - db~)] (Eq. 14 chained through the
// row); for the row's own weight sigma, dl/dsigma = -2 rho mu / sigma.  With
// scalar weights dw accumulates this chunk's partial sums of the three
// weight gradients; with per-row weights every row's is written (dwg, dws
// like dd, ds; dwi like du0).  IX maps the element indices of the per-step
// arrays as in Src0 (not those of du0, dwi, u, wi).
template <int K, class TIO, bool ADD, class F = FormScalar, class IX = IxPlain>
struct GradSink {
  static constexpr int V = F::V, QE = F::QE, k = K / F::V;
  const TIO *c, *d, *s, *y, *v;   // inputs: node i is row o + i
  const TIO *wg = nullptr, *wsm = nullptr;   // per-row weights, rows as d and s
  TIO *dc, *dd, *ds;              // outputs: node i is row oo + i
  TIO *dwg = nullptr, *dws = nullptr;        // per-row weight gradients, rows as dd and ds
  TIO* du0;                       // this instance's [t_init][V][n_init]
  TIO* dwi = nullptr;             // this instance's initial-weight gradients, as du0
  const TIO* u = nullptr;         // initial values of every instance, [N][t_init][V][n_init]
  const TIO* wi = nullptr;        // initial weights, as u (per-row weights)
  int uo = 0;                     // element offset of this instance's block in u (and wi)
  int64_t o = 0, oo = 0;
  Inst<K> p;
  double lam_n[K], y_n[K];   // node i+1 (the one finished before)
  bool have_next = false;
  double dw[3] = {0.0, 0.0, 0.0};

  SMNN_HD double gov_w(int64_t i, int q) const {
    if constexpr (F::WROW) return static_cast<double>(wg[IX::template at<QE>((o + i) * QE + q)]);
    else return p.wg;
  }
  SMNN_HD double smooth_w(int64_t i) const {
    if constexpr (F::WROW) return static_cast<double>(wsm[IX::template at<1>(o + i)]);
    else return p.ws;
  }
  SMNN_HD void lam_y(int64_t i, const double (&x)[K], double (&lam)[K], double (&yi)[K]) const {
#pragma unroll
    for (int e = 0; e < K; ++e) {
      lam[e] = x[e] + (ADD ? static_cast<double>(v[IX::template at<K>((o + i) * K + e)]) : 0.0);
      yi[e] = static_cast<double>(y[IX::template at<K>((o + i) * K + e)]);
    }
  }
  SMNN_HD void governing(int64_t i, const double (&lam)[K], const double (&yi)[K]) {
#pragma unroll
    for (int q = 0; q < QE; ++q) {
      const double w = gov_w(i, q), wg2 = w * w;
      double e = -static_cast<double>(d[IX::template at<QE>((o + i) * QE + q)]), f = 0.0;
#pragma unroll
      for (int r = 0; r < K; ++r) {
        const double cr = static_cast<double>(c[IX::template at<QE * K>(((o + i) * QE + q) * K + r)]);
        e = fma(cr, yi[r], e);
        f = fma(cr, lam[r], f);
      }
#pragma unroll
      for (int r = 0; r < K; ++r)
        dc[IX::template at<QE * K>(((oo + i) * QE + q) * K + r)] = static_cast<TIO>(-wg2 * (e * lam[r] + f * yi[r]));
      dd[IX::template at<QE>((oo + i) * QE + q)] = static_cast<TIO>(wg2 * f);
      if constexpr (F::WROW) dwg[IX::template at<QE>((oo + i) * QE + q)] = static_cast<TIO>(-2.0 * w * e * f);
      else dw[0] += -2.0 * p.wg * e * f;
    }
    if (i < p.t_init) {
#pragma unroll
      for (int vv = 0; vv < V; ++vv)
#pragma unroll
        for (int r = 0; r < k; ++r)
          if (r < p.n_init) {
            const int ui = (static_cast<int>(i) * V + vv) * p.n_init + r;
            const double ur = static_cast<double>(u[uo + ui]);
            const double w = F::WROW ? static_cast<double>(wi[uo + ui]) : p.wi;
            const double l = lam[vv * k + r];
            du0[ui] = static_cast<TIO>(w * w * l);
            if constexpr (F::WROW) dwi[ui] = static_cast<TIO>(-2.0 * w * (yi[vv * k + r] - ur) * l);
            else dw[1] += -2.0 * p.wi * (yi[vv * k + r] - ur) * l;
          }
    }
  }
  SMNN_HD void pair(int64_t i, const double (&lam)[K], const double (&yi)[K]) {
    const double si = static_cast<double>(s[IX::template at<1>(o + i)]), w = smooth_w(i);
    double g_s = 0.0, g_w = 0.0;
#pragma unroll
    for (int vv = 0; vv < V; ++vv) {
      double yt[k], yn[k], lt[k], ln[k], gs, gw;
#pragma unroll
      for (int r = 0; r < k; ++r) {
        yt[r] = yi[vv * k + r]; yn[r] = y_n[vv * k + r];
        lt[r] = lam[vv * k + r]; ln[r] = lam_n[vv * k + r];
      }
      pair_grad<k>(si, w, yt, yn, lt, ln, gs, gw);
      g_s += gs;
      g_w += gw;
    }
    ds[IX::template at<1>(oo + i)] = static_cast<TIO>(g_s);
    if constexpr (F::WROW) dws[IX::template at<1>(oo + i)] = static_cast<TIO>(g_w);
    else dw[2] += g_w;
  }
  // the chunk's right separator (owned; finished by the level above)
  SMNN_HD void start(int64_t i, const double (&x)[K]) {
    double lam[K], yi[K];
    lam_y(i, x, lam, yi);
    governing(i, lam, yi);
#pragma unroll
    for (int e = 0; e < K; ++e) { lam_n[e] = lam[e]; y_n[e] = yi[e]; }
    have_next = true;
  }
  template <int KK>
  SMNN_HD void node(int64_t i, const double (&x)[KK]) {
    double lam[K], yi[K];
    lam_y(i, x, lam, yi);
    governing(i, lam, yi);
    if (have_next) pair(i, lam, yi);
#pragma unroll
    for (int e = 0; e < K; ++e) { lam_n[e] = lam[e]; y_n[e] = yi[e]; }
    have_next = true;
  }
  // the instance's last point: its step slot enters no row
  SMNN_HD void last_point(int64_t n) {
    ds[IX::template at<1>(oo + n - 1)] = static_cast<TIO>(0.0);
    if constexpr (F::WROW) dws[IX::template at<1>(oo + n - 1)] = static_cast<TIO>(0.0);
  }
  // initial points past the instance's last node (n < t_init) have no row:
  // their gradient is zero (called by the lane owning the instance's end)
  SMNN_HD void zero_past_end(int64_t n) {
    for (int64_t t = n; t < p.t_init; ++t)
      for (int e = 0; e < V * p.n_init; ++e) {
        du0[t * V * p.n_init + e] = static_cast<TIO>(0.0);
        if constexpr (F::WROW) dwi[t * V * p.n_init + e] = static_cast<TIO>(0.0);
      }
  }
  // the chunk's left separator: only the smoothness pair (i, i+1) is owned here
  SMNN_HD void left(int64_t i, const double (&x)[K]) {
    double lam[K], yi[K];
    lam_y(i, x, lam, yi);
    pair(i, lam, yi);
  }
};

// Node data of a reduced (separator) level in the natural layout: one
// record per node, as the CPU emulator in tests/emu and the upper-level
// kernel's LDS keep them (the other kernels use the interleaved layout of
// SrcT).  rec[node] = {A packed (Q), B = block (node+1, node) (K*K)}.
template <int K>
struct SrcN {
  const double* rec;  // [n][Q + KK] of this instance
  const double* rhs;  // [n][K]
  SMNN_HD void load(int64_t i, double (&A)[Dim<K>::Q], double (&f)[K], double (&Bp)[Dim<K>::KK]) const {
    constexpr int R = Dim<K>::Q + Dim<K>::KK;
#pragma unroll
    for (int e = 0; e < Dim<K>::Q; ++e) A[e] = rec[i * R + e];
#pragma unroll
    for (int e = 0; e < K; ++e) f[e] = rhs[i * K + e];
    if (i > 0) {
#pragma unroll
      for (int e = 0; e < Dim<K>::KK; ++e) Bp[e] = rec[(i - 1) * R + Dim<K>::Q + e];
    }
  }
  SMNN_HD void coupling(int64_t i, double (&B)[Dim<K>::KK]) const {
    constexpr int R = Dim<K>::Q + Dim<K>::KK;
#pragma unroll
    for (int e = 0; e < Dim<K>::KK; ++e) B[e] = rec[i * R + Dim<K>::Q + e];
  }
};

// Separator levels store node records interleaved by groups of W = 8
// chunks: field e (of F) of node u of chunk C (global chunk index at that
// level, chunk length L) sits at ((C / W) L + u) F W + W e + C % W.  The
// lanes of a wave own consecutive chunks, so one field of their u-th nodes
// is 64 doubles in whole 64-byte runs, and the reduce below, which writes a
// few consecutive chunks' records, writes whole 64-byte runs too.  An
// instance's last chunk may leave slots unused.
constexpr int TILE_W = 8;
SMNN_HD int64_t tpos(int64_t C, int64_t u, int L, int F, int e) {
  return ((C / TILE_W) * L + u) * (TILE_W * F) + TILE_W * e + (C % TILE_W);
}

// Node data of a separator level in the interleaved layout, seen from
// the lane that owns chunk C (first node a, instance-relative): nodes a..a+L-1
// are in chunk C, node a-1 is the last node of chunk C-1.
template <int K>
struct SrcT {
  const double* rec;  // records, F = Q + KK: {A packed, B = block (node+1, node)}
  const double* rhs;  // right-hand sides, F = K
  int64_t C, a;
  int L;
  SMNN_HD void where(int64_t i, int64_t& c, int64_t& u) const {
    c = i >= a ? C : C - 1;
    u = i >= a ? i - a : L - 1;
  }
  SMNN_HD void load(int64_t i, double (&A)[Dim<K>::Q], double (&f)[K], double (&Bp)[Dim<K>::KK]) const {
    constexpr int R = Dim<K>::Q + Dim<K>::KK;
    int64_t c, u;
    where(i, c, u);
#pragma unroll
    for (int e = 0; e < Dim<K>::Q; ++e) A[e] = rec[tpos(c, u, L, R, e)];
#pragma unroll
    for (int e = 0; e < K; ++e) f[e] = rhs[tpos(c, u, L, K, e)];
    if (i > 0) {
      int64_t cp, up;
      where(i - 1, cp, up);
#pragma unroll
      for (int e = 0; e < Dim<K>::KK; ++e) Bp[e] = rec[tpos(cp, up, L, R, Dim<K>::Q + e)];
    }
  }
  SMNN_HD void coupling(int64_t i, double (&B)[Dim<K>::KK]) const {
    constexpr int R = Dim<K>::Q + Dim<K>::KK;
    int64_t c, u;
    where(i, c, u);
#pragma unroll
    for (int e = 0; e < Dim<K>::KK; ++e) B[e] = rec[tpos(c, u, L, R, Dim<K>::Q + e)];
  }
};

// combine_separator for the interleaved layout: the node is node u of
// chunk C of its level (chunk length L).
template <int K>
SMNN_HD void combine_separator_t(const double (&rA)[Dim<K>::Q], const double (&rf)[K], const Reduced<K>& lh,
                                 double* rec, double* rhs, int64_t C, int64_t u, int L, bool write_rec) {
  constexpr int Q = Dim<K>::Q, KK = Dim<K>::KK;
  if (write_rec) {
#pragma unroll
    for (int e = 0; e < Q; ++e) rec[tpos(C, u, L, Q + KK, e)] = rA[e] + lh.lA[e];
#pragma unroll
    for (int e = 0; e < KK; ++e) rec[tpos(C, u, L, Q + KK, Q + e)] = lh.lB[e];
  }
#pragma unroll
  for (int e = 0; e < K; ++e) rhs[tpos(C, u, L, K, e)] = rf[e] + lh.lf[e];
}

// Record of a separator node combined from the two chunks that share it
// (natural layout): rh = reduction of the chunk on its left (which owns it),
// lh = reduction of the chunk on its right.
template <int K>
SMNN_HD void combine_separator(const double (&rA)[Dim<K>::Q], const double (&rf)[K],
                               const Reduced<K>& lh, double* rec, double* rhs, bool write_rec) {
  constexpr int Q = Dim<K>::Q, KK = Dim<K>::KK;
  if (write_rec) {
#pragma unroll
    for (int e = 0; e < Q; ++e) rec[e] = rA[e] + lh.lA[e];
#pragma unroll
    for (int e = 0; e < KK; ++e) rec[Q + e] = lh.lB[e];
  }
#pragma unroll
  for (int e = 0; e < K; ++e) rhs[e] = rf[e] + lh.lf[e];
}

}  // namespace smnn
