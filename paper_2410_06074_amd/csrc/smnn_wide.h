// Row-distributed block algebra for wide blocks (K = V (R+1) > 5 unknowns
// per time point, e.g. three coupled second-order variables: K = 9).
//
// A block that size does not fit one lane's registers, so here a group of
// 16 lanes works on one chunk: lane r of the group holds row r of every
// K x K block (A_t, B_t, the Cholesky factor, the Schur-complement pieces)
// and element r of every K-vector.  Rows travel between the lanes of a group
// by broadcasts (Grp::bcast); lanes r >= K take part in every broadcast but
// hold nothing that an active row reads.  The elimination is the same as the
// one-lane form in smnn_core.h: the block Cholesky recurrence of Alg. 3 with
// the forward substitution of Alg. 4 over a chunk interior, the fill that
// couples it to its left separator, and the back-substitution, written row
// by row.
//
// Every routine takes the group context G, whose bcast(v, j) returns the
// value v of row j of the calling lane's group.  Every lane of a group must
// reach every bcast in the same order (the routines keep group-uniform
// control flow).  On the GPU the context is a lane shuffle; the CPU emulator
// in tests/emu runs the 16 rows as threads.
#pragma once

#include "smnn_core.h"

namespace smnn {

constexpr int GROUP = 16;   // lanes per chunk (a DPP row of the wave)

// ------------------------------------------------------------- row algebra
// In-place Cholesky of the symmetric D, row-distributed (row r in d[]).  On
// return row r holds L[r][0..r] with the diagonal as 1/L_rr, zeros above.
// Returns false on this row's lane when a pivot was not > 0 (NaN follows).
template <int K, class G>
SMNN_HD bool wchol(const G& g, double (&d)[K]) {
  const int r = g.r;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    // row j's pivot, on its own lane (its entries < j are final)
    double p = d[j];
#pragma unroll
    for (int m = 0; m < j; ++m) p -= d[m] * d[m];
    const double inv = rsqrt_pivot(p);
    if (r == j) {
      ok = p > 0.0;
      d[j] = inv;
    }
    // rows below: L[r][j] = (D[r][j] - sum_m L[r][m] L[j][m]) / L[j][j]
    double lj[K];
#pragma unroll
    for (int m = 0; m <= j; ++m) lj[m] = g.bcast(d[m], j);
    if (r > j) {
      double t = d[j];
#pragma unroll
      for (int m = 0; m < j; ++m) t -= d[m] * lj[m];
      d[j] = t * lj[j];
    }
  }
  if (r < K) {
#pragma unroll
    for (int m = 0; m < K; ++m)
      if (m > r) d[m] = 0.0;
  }
  return ok;
}

// row r of W = B L^{-T}  (b: row r of B; l: row r of L)
template <int K, class G>
SMNN_HD void wrsolve_t(const G& g, const double (&l)[K], const double (&b)[K], double (&w)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double t = b[j];
#pragma unroll
    for (int m = 0; m < j; ++m) t -= w[m] * g.bcast(l[m], j);
    w[j] = t * g.bcast(l[j], j);
  }
}

// row r of D = A - W W^T
template <int K, class G>
SMNN_HD void wsym_minus_wwt(const G& g, const double (&a)[K], const double (&w)[K], double (&d)[K]) {
#pragma unroll
  for (int c = 0; c < K; ++c) {
    double t = a[c];
#pragma unroll
    for (int m = 0; m < K; ++m) t -= w[m] * g.bcast(w[m], c);
    d[c] = t;
  }
}

// element r of y - W x  (x distributed: element m on row m)
template <int K, class G>
SMNN_HD double wsub_matvec(const G& g, const double (&w)[K], double x, double y) {
#pragma unroll
  for (int m = 0; m < K; ++m) y -= w[m] * g.bcast(x, m);
  return y;
}

// row r of Z = -W X  (x: row r of X)
template <int K, class G>
SMNN_HD void wneg_matmul(const G& g, const double (&w)[K], const double (&x)[K], double (&z)[K]) {
#pragma unroll
  for (int c = 0; c < K; ++c) z[c] = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) {
#pragma unroll
    for (int c = 0; c < K; ++c) z[c] -= w[m] * g.bcast(x[c], m);
  }
}

// element r of L^{-1} f (forward substitution, a chain over the rows)
template <int K, class G>
SMNN_HD double wlsolve(const G& g, const double (&l)[K], double f) {
  const int r = g.r;
  double acc = 0.0, out = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double v = (f - acc) * l[j];          // final on row j
    if (r == j) out = v;
    const double xj = g.bcast(v, j);
    if (r > j) acc += l[j] * xj;
  }
  return out;
}

// Rows of Xh = L^{-1} X (x, xh: row r), and, as each row j of Xh is
// finished, la += Xh[j][r] Xh[j][:] and lf += Xh[j][r] gh[j] (the
// left-separator accumulators: row r of Xh^T Xh and element r of Xh^T gh).
template <int K, class G>
SMNN_HD void wlsolve_rows_acc(const G& g, const double (&l)[K], const double (&x)[K], double gh,
                              double (&xh)[K], double (&la)[K], double& lf) {
  const int r = g.r;
  double acc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) acc[c] = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double row[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double v = (x[c] - acc[c]) * l[j];   // final on row j
      if (r == j) xh[c] = v;
      row[c] = g.bcast(v, j);
    }
    const double gj = g.bcast(gh, j);
    if (r > j) {
#pragma unroll
      for (int c = 0; c < K; ++c) acc[c] += l[j] * row[c];
    }
    double mine = 0.0;   // row[r]: this row's column of Xh row j
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (c == r) mine = row[c];
#pragma unroll
    for (int c = 0; c < K; ++c) la[c] += mine * row[c];
    lf += mine * gj;
  }
}

// element r of L^{-T} x (back substitution, a chain over the rows downward):
// x_j = (x_j - sum_{m>j} L[m][j] x_m) / L[j][j]; row m holds L[m][j].
template <int K, class G>
SMNN_HD double wusolve(const G& g, const double (&l)[K], double x) {
  const int r = g.r;
  double out = 0.0;
  // acc on row j: sum_{m>j} L[m][j] x_m, gathered as the rows below finish
  double acc = 0.0;
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const double v = (x - acc) * l[j];          // final on row j (l[j] = 1/L_jj there)
    if (r == j) out = v;
    const double xj = g.bcast(v, j);
    // row r < j needs L[j][r] x_j: L[j][r] lives on row j, column r
    double ljr = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double t = g.bcast(l[c], j);
      if (c == r) ljr = t;
    }
    if (r < j) acc += ljr * xj;
  }
  return out;
}

// element r of y - B^T x for B given by columns (bc: column r of B, i.e.
// B[m][r] for m = 0..K-1; x distributed)
template <int K, class G>
SMNN_HD double wsub_matvec_t(const G& g, const double (&bc)[K], double x, double y) {
#pragma unroll
  for (int m = 0; m < K; ++m) y -= bc[m] * g.bcast(x, m);
  return y;
}

// ----------------------------------------------------------- chunk routines
// Result of eliminating a chunk interior, row r of each piece.
template <int K>
struct WReduced {
  double rA[K];   // right separator: A_{b+1} - B_b D_b^{-1} B_b^T
  double rf;      //                  f_{b+1} - B_b D_b^{-1} g_b
  double lA[K];   // left separator contribution: -E_L^T A_I^{-1} E_L
  double lf;      //                              -E_L^T A_I^{-1} f_I
  double lB[K];   // coupling (b+1, a-1): -B_b [A_I^{-1}]_{b,a} B_{a-1}
  int fail;       // chunk-relative node + 1 of the first non-positive pivot (this row), 0 if none
};

// Src supplies, for the calling row r:
//   load(i, a, f, bp)   row r of A_i, element r of the right-hand side, and
//                       (i > 0) row r of B_{i-1} = block (i, i-1);
//   coupling_col(i, bc) column r of B_i = block (i+1, i).
template <int K, int L, class G, class Src>
SMNN_HD void wreduce_chunk(const G& g, const Src& src, int64_t a, int64_t b, bool has_left, bool has_right,
                           WReduced<K>& out) {
  double lc[K], xh[K];
  double gh = 0.0;
#pragma unroll
  for (int e = 0; e < K; ++e) { out.lA[e] = 0.0; out.lB[e] = 0.0; xh[e] = 0.0; lc[e] = 0.0; }
  out.lf = 0.0;
  out.rf = 0.0;
  out.fail = 0;
#pragma unroll 1
  for (int u = 0; u < L; ++u) {
    const int64_t i = a + u;
    if (i > b) break;
    double av[K], bp[K], d[K], x[K];
    double f;
    src.load(i, av, f, bp);
    if (u == 0) {
#pragma unroll
      for (int e = 0; e < K; ++e) { d[e] = av[e]; x[e] = has_left ? bp[e] : 0.0; }
    } else {
      double w[K];
      wrsolve_t<K>(g, lc, bp, w);               // W = B_{i-1} L_{i-1}^{-T}
      wsym_minus_wwt<K>(g, av, w, d);           // D_i = A_i - W W^T
      f = wsub_matvec<K>(g, w, gh, f);          // g_i = f_i - W ghat_{i-1}
      if (has_left) wneg_matmul<K>(g, w, xh, x);   // X_i = -W Xhat_{i-1}
    }
    const bool ok = wchol<K>(g, d);
    if (!ok && out.fail == 0) out.fail = u + 1;
#pragma unroll
    for (int e = 0; e < K; ++e) lc[e] = d[e];
    gh = wlsolve<K>(g, lc, f);                  // ghat_i = L_i^{-1} g_i
    if (has_left) wlsolve_rows_acc<K>(g, lc, x, gh, xh, out.lA, out.lf);
  }
  if (has_left) {
#pragma unroll
    for (int e = 0; e < K; ++e) out.lA[e] = -out.lA[e];
    out.lf = -out.lf;
  }
  if (has_right) {
    double av[K], vb[K], w[K];
    double f;
    src.load(b + 1, av, f, vb);                 // vb = row r of B_b
    wrsolve_t<K>(g, lc, vb, w);                 // W = B_b L_b^{-T}
    wsym_minus_wwt<K>(g, av, w, out.rA);
    out.rf = wsub_matvec<K>(g, w, gh, f);
    if (has_left) wneg_matmul<K>(g, w, xh, out.lB);
  }
}

// Solve the chunk interior a..b with the separator values xl (node a-1) and
// xr (node b+1) known (distributed: element r on row r).  Forward sweep:
// ls[u] = row r of the Cholesky factor of node a+u's reduced block, x[u] =
// element r of its forward-substituted right-hand side.  Returns the
// chunk-relative node + 1 of the first non-positive pivot on this row.
template <int K, int L, class G, class Src>
SMNN_HD int wbacksub_forward(const G& g, const Src& src, int64_t a, int64_t b, bool has_left, bool has_right,
                             double xl, double xr, double (&ls)[L][K], double (&x)[L]) {
  int fail = 0;
#pragma unroll
  for (int u = 0; u < L; ++u) {
    const int64_t i = a + u;
    if (i > b) break;
    double av[K], bp[K], d[K];
    double f;
    src.load(i, av, f, bp);
    if (u == 0 && has_left) f = wsub_matvec<K>(g, bp, xl, f);   // f_a -= B_{a-1} x_{a-1}
    if (i == b && has_right) {
      double bc[K];
      src.coupling_col(b, bc);
      f = wsub_matvec_t<K>(g, bc, xr, f);      // f_b -= B_b^T x_{b+1}
    }
    if (u == 0) {
#pragma unroll
      for (int e = 0; e < K; ++e) d[e] = av[e];
    } else {
      double w[K];
      wrsolve_t<K>(g, ls[u > 0 ? u - 1 : 0], bp, w);
      wsym_minus_wwt<K>(g, av, w, d);
      f = wsub_matvec<K>(g, w, x[u > 0 ? u - 1 : 0], f);
    }
    const bool ok = wchol<K>(g, d);
    if (!ok && fail == 0) fail = u + 1;
#pragma unroll
    for (int e = 0; e < K; ++e) ls[u][e] = d[e];
    x[u] = wlsolve<K>(g, ls[u], f);
  }
  return fail;
}

// Backward sweep: x[u] becomes element r of node a+u's solution; sink.node
// is called as each node is finished, in decreasing order.
template <int K, int L, class G, class Src, class Sink>
SMNN_HD void wbacksub_backward(const G& g, const Src& src, int64_t a, int64_t b, const double (&ls)[L][K],
                               double (&x)[L], Sink& sink) {
#pragma unroll
  for (int u = L - 1; u >= 0; --u) {
    const int64_t i = a + u;
    if (i > b) continue;
    if (i < b) {
      double bc[K];
      src.coupling_col(i, bc);
      double t = wsub_matvec_t<K>(g, bc, x[u + 1 < L ? u + 1 : u], 0.0);   // -B_i^T x_{i+1}
      t = wlsolve<K>(g, ls[u], t);
      x[u] += t;
    }
    x[u] = wusolve<K>(g, ls[u], x[u]);          // x_i = L^{-T}(ghat_i - L^{-1} B_i^T x_{i+1})
    sink.node(i, x[u]);
  }
}

struct WNoSink {
  SMNN_HD void node(int64_t, double) {}
};

// ------------------------------------------------------------ level sources
// Separator levels keep node records in the natural layout, full K x K
// blocks: the two halves of the diagonal block (from the chunk on the
// node's left and the one on its right), the coupling block (node+1, node),
// and the two halves of the right-hand side.  Each half is written by one
// chunk only, so a reduce writes no location another chunk writes.
template <int K>
struct WRec {
  static constexpr int F = 3 * K * K;   // Ar, Al, B
  static constexpr int AR = 0, AL = K * K, BB = 2 * K * K;
};

template <int K>
struct WSrcN {
  const double* rec;   // [n][3 K K] of this instance
  const double* rhs;   // [n][2 K]: fr, fl
  int r;
  SMNN_HD void load(int64_t i, double (&av)[K], double& f, double (&bp)[K]) const {
    const double* p = rec + i * WRec<K>::F;
#pragma unroll
    for (int c = 0; c < K; ++c) av[c] = r < K ? p[WRec<K>::AR + r * K + c] + p[WRec<K>::AL + r * K + c] : 0.0;
    f = r < K ? rhs[i * 2 * K + r] + rhs[i * 2 * K + K + r] : 0.0;
    if (i > 0) {
      const double* q = rec + (i - 1) * WRec<K>::F + WRec<K>::BB;
#pragma unroll
      for (int c = 0; c < K; ++c) bp[c] = r < K ? q[r * K + c] : 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < K; ++c) bp[c] = 0.0;
    }
  }
  SMNN_HD void coupling_col(int64_t i, double (&bc)[K]) const {
    const double* q = rec + i * WRec<K>::F + WRec<K>::BB;
#pragma unroll
    for (int m = 0; m < K; ++m) bc[m] = r < K ? q[m * K + r] : 0.0;
  }
};

// Write a chunk's reduction into the next level's records: the right pieces
// to its right separator (node m = the chunk's index j at the next level),
// the left pieces to its left separator (node j - 1), and the coupling
// between them as block (j, j - 1) (stored with node j - 1).
template <int K>
SMNN_HD void wwrite_reduced(const WReduced<K>& red, int r, double* rec, double* rhs, int64_t j, bool has_left,
                            bool has_right, bool write_rec) {
  if (r >= K) return;
  if (has_right) {
    if (write_rec) {
#pragma unroll
      for (int c = 0; c < K; ++c) rec[j * WRec<K>::F + WRec<K>::AR + r * K + c] = red.rA[c];
    }
    rhs[j * 2 * K + r] = red.rf;
  }
  if (has_left) {
    if (write_rec) {
#pragma unroll
      for (int c = 0; c < K; ++c) {
        rec[(j - 1) * WRec<K>::F + WRec<K>::AL + r * K + c] = red.lA[c];
        if (has_right) rec[(j - 1) * WRec<K>::F + WRec<K>::BB + r * K + c] = red.lB[c];
      }
    }
    rhs[(j - 1) * 2 * K + K + r] = red.lf;
  }
}

// Level-0 rows assembled on the fly (App. A.2), for the calling row r:
// variable v = r / k, order rr = r % k.
template <int K, class TIO, int RHS, class F>
struct WSrc0 {
  static constexpr int V = F::V, QE = F::QE, k = K / F::V;
  static_assert(k * V == K, "block size is V (R+1)");
  const TIO *c, *d, *s, *g, *v;   // node i is row o + i ([QE][K], [QE], 1, [K], [K] per row)
  const TIO *wg = nullptr, *wsm = nullptr, *u = nullptr, *wi = nullptr;
  int uo = 0;
  int64_t n, o = 0;
  Inst<K> p;
  int r;

  SMNN_HD double ld(const TIO* ptr, int64_t idx) const { return static_cast<double>(ptr[idx]); }
  SMNN_HD double ldc(int64_t i, int q, int j) const { return ld(c, ((o + i) * QE + q) * K + j); }
  SMNN_HD double gov_w(int64_t i, int q) const {
    if constexpr (F::WROW) return ld(wg, (o + i) * QE + q);
    else return p.wg;
  }
  SMNN_HD double smooth_w(int64_t i) const {
    if constexpr (F::WROW) return ld(wsm, o + i);
    else return p.ws;
  }
  SMNN_HD int uidx(int64_t i, int vv, int rr) const { return uo + (static_cast<int>(i) * V + vv) * p.n_init + rr; }
  SMNN_HD double init_w(int64_t i, int vv, int rr) const {
    if constexpr (F::WROW) return ld(wi, uidx(i, vv, rr));
    else return p.wi;
  }

  // row r of the smoothness blocks of the pair (i, i+1) (step s_i, weight
  // ws): left node (i), right node (i+1), coupling (i+1, i) and its column r
  SMNN_HD void smooth_rows(double s_i, double ws2, double (&left)[K], double (&right)[K], double (&cpl)[K],
                           double (&cplc)[K]) const {
    constexpr Coef<k> C{};
    double pw[2 * k - 1];
    pw[0] = 1.0;
#pragma unroll
    for (int e = 1; e < 2 * k - 1; ++e) pw[e] = pw[e - 1] * s_i;
    const int vv = r / k, rr = r % k;
#pragma unroll
    for (int cc = 0; cc < K; ++cc) { left[cc] = 0.0; right[cc] = 0.0; cpl[cc] = 0.0; cplc[cc] = 0.0; }
    if (r >= K) return;
#pragma unroll
    for (int j = 0; j < k; ++j) {
      const double e = ws2 * pw[rr + j];
      left[vv * k + j] = e * (C.alpha[rr][j] + (rr == j ? 1.0 : 0.0));
      right[vv * k + j] = e * ((((rr + j) & 1) ? -C.alpha[rr][j] : C.alpha[rr][j]) + (rr == j ? 1.0 : 0.0));
      cpl[vv * k + j] = e * C.nu[rr][j];      // row rr of block (i+1, i) within variable vv
      cplc[vv * k + j] = e * C.nu[j][rr];     // column rr
    }
  }

  SMNN_HD void coupling_col(int64_t i, double (&bc)[K]) const {
    double l[K], rt[K], cp[K];
    const double w = smooth_w(i);
    smooth_rows(ld(s, o + i), w * w, l, rt, cp, bc);
  }

  // element r of A^T W (b - A v) (RHS_RESID) or g - A^T W A v (RHS_GRESID),
  // row by row from the constraints touching node i
  SMNN_HD double residual(int64_t i) const {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    const int vv = r / k, rr = r % k;
    double vi[K];
#pragma unroll
    for (int j = 0; j < K; ++j) vi[j] = ld(v, (o + i) * K + j);
    double f = (RHS == RHS_GRESID && r < K) ? ld(g, (o + i) * K + r) : 0.0;
    if (r >= K) return 0.0;
#pragma unroll
    for (int q = 0; q < QE; ++q) {
      double e = (RHS == RHS_RESID) ? ld(d, (o + i) * QE + q) : 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) e = fma(-ldc(i, q, j), vi[j], e);
      const double w = gov_w(i, q);
      f = fma(ldc(i, q, r), (w * w) * e, f);
    }
    if (i < p.t_init && rr < p.n_init) {
      const double w = init_w(i, vv, rr);
      f += (w * w) * ((RHS == RHS_RESID ? ld(u, uidx(i, vv, rr)) : 0.0) - vi[r]);
    }
    // smoothness rows of variable vv with the neighbours
    if (i > 0) {
      double pw[Dim<k>::P], vp[k], vc[k], cl[k], cr[k];
      powers<k>(ld(s, o + i - 1), pw);
#pragma unroll
      for (int j = 0; j < k; ++j) { vp[j] = ld(v, (o + i - 1) * K + vv * k + j); vc[j] = vi[vv * k + j]; }
      pair_residual<k>(pw, smooth_w(i - 1), vp, vc, cl, cr);
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < k; ++j)
        if (j == rr) t = cr[j];
      f += t;
    }
    if (i + 1 < n) {
      double pw[Dim<k>::P], vc[k], vn[k], cl[k], cr[k];
      powers<k>(ld(s, o + i), pw);
#pragma unroll
      for (int j = 0; j < k; ++j) { vc[j] = vi[vv * k + j]; vn[j] = ld(v, (o + i + 1) * K + vv * k + j); }
      pair_residual<k>(pw, smooth_w(i), vc, vn, cl, cr);
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < k; ++j)
        if (j == rr) t = cl[j];
      f += t;
    }
    return f;
  }

  SMNN_HD void load(int64_t i, double (&av)[K], double& f, double (&bp)[K]) const {
    const int vv = r / k, rr = r % k;
#pragma unroll
    for (int cc = 0; cc < K; ++cc) { av[cc] = 0.0; bp[cc] = 0.0; }
    f = 0.0;
    if (r < K) {
#pragma unroll
      for (int q = 0; q < QE; ++q) {
        const double w = gov_w(i, q), wg2 = w * w, cr = ldc(i, q, r);
#pragma unroll
        for (int cc = 0; cc < K; ++cc) av[cc] += wg2 * cr * ldc(i, q, cc);
        if (RHS == RHS_BETA) f += wg2 * cr * ld(d, (o + i) * QE + q);
      }
      if (i < p.t_init && rr < p.n_init) {
        const double w = init_w(i, vv, rr), wi2 = w * w;
        av[r] += wi2;
        if (RHS == RHS_BETA) f += wi2 * ld(u, uidx(i, vv, rr));
      }
    }
    double l[K], rt[K], cp[K], cc2[K];
    if (i + 1 < n) {
      const double w = smooth_w(i);
      smooth_rows(ld(s, o + i), w * w, l, rt, cp, cc2);
#pragma unroll
      for (int cc = 0; cc < K; ++cc) av[cc] += l[cc];
    }
    if (i > 0) {
      const double w = smooth_w(i - 1);
      smooth_rows(ld(s, o + i - 1), w * w, l, rt, cp, cc2);
#pragma unroll
      for (int cc = 0; cc < K; ++cc) { av[cc] += rt[cc]; bp[cc] = cp[cc]; }
    }
    if (RHS == RHS_G) f = r < K ? ld(g, (o + i) * K + r) : 0.0;
    else if (RHS != RHS_BETA) f = residual(i);
  }
};

// Level-0 solution sink: out_i[r] = (v_i[r] +) x[r].
template <int K, class TIO, bool ADD>
struct WStoreSink {
  TIO* out;
  const TIO* v;
  int64_t o = 0;
  int r;
  SMNN_HD void node(int64_t i, double x) {
    if (r >= K) return;
    double val = x;
    if (ADD) val += static_cast<double>(v[(o + i) * K + r]);
    out[(o + i) * K + r] = static_cast<TIO>(val);
  }
};

// Level-0 gradient sink (the rows a chunk owns, as GradSink in smnn_core.h):
// lam and y of each node are gathered to every row; each row writes its own
// elements of dc, row 0 the per-point values (dd, ds, per-row weight
// gradients) and accumulates the chunk's scalar-weight partial sums.
template <int K, class TIO, bool ADD, class F, class G>
struct WGradSink {
  static constexpr int V = F::V, QE = F::QE, k = K / F::V;
  const G& g;
  const TIO *c, *d, *s, *y, *v, *wg, *wsm, *u, *wi;
  TIO *dc, *dd, *ds, *dwg, *dws, *du0, *dwi;   // du0, dwi: this instance's
  int uo = 0;
  int64_t o = 0;
  Inst<K> p;
  double lam_n[K], y_n[K];
  bool have_next = false;
  double dw[3] = {0.0, 0.0, 0.0};

  SMNN_HD WGradSink(const G& grp) : g(grp) {}
  SMNN_HD double gov_w(int64_t i, int q) const {
    if constexpr (F::WROW) return static_cast<double>(wg[(o + i) * QE + q]);
    else return p.wg;
  }
  SMNN_HD double smooth_w(int64_t i) const {
    if constexpr (F::WROW) return static_cast<double>(wsm[o + i]);
    else return p.ws;
  }
  SMNN_HD void gather(int64_t i, double x, double (&lam)[K], double (&yi)[K]) const {
    const int r = g.r;
    const double mine = x + ((ADD && r < K) ? static_cast<double>(v[(o + i) * K + r]) : 0.0);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      lam[m] = g.bcast(mine, m);
      yi[m] = static_cast<double>(y[(o + i) * K + m]);
    }
  }
  SMNN_HD void governing(int64_t i, const double (&lam)[K], const double (&yi)[K]) {
    const int r = g.r;
#pragma unroll
    for (int q = 0; q < QE; ++q) {
      const double w = gov_w(i, q), wg2 = w * w;
      double e = -static_cast<double>(d[(o + i) * QE + q]), f = 0.0;
#pragma unroll
      for (int m = 0; m < K; ++m) {
        const double cm = static_cast<double>(c[((o + i) * QE + q) * K + m]);
        e = fma(cm, yi[m], e);
        f = fma(cm, lam[m], f);
      }
      double lr = 0.0, yr = 0.0;
#pragma unroll
      for (int m = 0; m < K; ++m)
        if (m == r) { lr = lam[m]; yr = yi[m]; }
      if (r < K) dc[((o + i) * QE + q) * K + r] = static_cast<TIO>(-wg2 * (e * lr + f * yr));
      if (r == 0) {
        dd[(o + i) * QE + q] = static_cast<TIO>(wg2 * f);
        if constexpr (F::WROW) dwg[(o + i) * QE + q] = static_cast<TIO>(-2.0 * w * e * f);
        else dw[0] += -2.0 * p.wg * e * f;
      }
    }
    if (i < p.t_init && r < K) {
      const int vv = r / k, rr = r % k;
      if (rr < p.n_init) {
        const int ui = (static_cast<int>(i) * V + vv) * p.n_init + rr;
        const double ur = static_cast<double>(u[uo + ui]);
        const double w = F::WROW ? static_cast<double>(wi[uo + ui]) : p.wi;
        double lr = 0.0, yr = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m)
          if (m == r) { lr = lam[m]; yr = yi[m]; }
        du0[ui] = static_cast<TIO>(w * w * lr);
        if constexpr (F::WROW) dwi[ui] = static_cast<TIO>(-2.0 * w * (yr - ur) * lr);
        else dw[1] += -2.0 * p.wi * (yr - ur) * lr;   // summed over the rows at the end
      }
    }
  }
  SMNN_HD void pair(int64_t i, const double (&lam)[K], const double (&yi)[K]) {
    const double si = static_cast<double>(s[o + i]), w = smooth_w(i);
    double g_s = 0.0, g_w = 0.0;
#pragma unroll
    for (int vv = 0; vv < V; ++vv) {
      double yt[k], yn[k], lt[k], ln[k], gs, gw;
#pragma unroll
      for (int rr = 0; rr < k; ++rr) {
        yt[rr] = yi[vv * k + rr]; yn[rr] = y_n[vv * k + rr];
        lt[rr] = lam[vv * k + rr]; ln[rr] = lam_n[vv * k + rr];
      }
      pair_grad<k>(si, w, yt, yn, lt, ln, gs, gw);
      g_s += gs;
      g_w += gw;
    }
    if (g.r == 0) {
      ds[o + i] = static_cast<TIO>(g_s);
      if constexpr (F::WROW) dws[o + i] = static_cast<TIO>(g_w);
      else dw[2] += g_w;
    }
  }
  SMNN_HD void keep(const double (&lam)[K], const double (&yi)[K]) {
#pragma unroll
    for (int e = 0; e < K; ++e) { lam_n[e] = lam[e]; y_n[e] = yi[e]; }
    have_next = true;
  }
  SMNN_HD void start(int64_t i, double x) {   // the chunk's right separator
    double lam[K], yi[K];
    gather(i, x, lam, yi);
    governing(i, lam, yi);
    keep(lam, yi);
  }
  SMNN_HD void node(int64_t i, double x) {
    double lam[K], yi[K];
    gather(i, x, lam, yi);
    governing(i, lam, yi);
    if (have_next) pair(i, lam, yi);
    keep(lam, yi);
  }
  SMNN_HD void left(int64_t i, double x) {   // the chunk's left separator: only the pair (i, i+1)
    double lam[K], yi[K];
    gather(i, x, lam, yi);
    pair(i, lam, yi);
  }
  SMNN_HD void last_point(int64_t n) {
    if (g.r == 0) {
      ds[o + n - 1] = static_cast<TIO>(0.0);
      if constexpr (F::WROW) dws[o + n - 1] = static_cast<TIO>(0.0);
    }
  }
  SMNN_HD void zero_past_end(int64_t n) {
    if (g.r != 0) return;
    for (int64_t t = n; t < p.t_init; ++t)
      for (int e = 0; e < V * p.n_init; ++e) {
        du0[t * V * p.n_init + e] = static_cast<TIO>(0.0);
        if constexpr (F::WROW) dwi[t * V * p.n_init + e] = static_cast<TIO>(0.0);
      }
  }
};

}  // namespace smnn
