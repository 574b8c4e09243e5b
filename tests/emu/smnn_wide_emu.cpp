// Host build of the row-distributed wide-block routines of
// paper_2410_06074_amd/csrc/smnn_wide.h, run through the same level / chunk
// schedule as the wide kernels: the 16 rows of a group are 16 threads that
// meet at every broadcast, so the code under test is the device code itself.
// Test tool only; the product library never uses it.
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "../../paper_2410_06074_amd/csrc/smnn_levels.h"
#include "../../paper_2410_06074_amd/csrc/smnn_wide.h"

using namespace smnn;

namespace {

int g_init_points = 1;

// Reusable barrier for the 16 row threads.
class Barrier {
 public:
  explicit Barrier(int n) : n_(n) {}
  void wait() {
    std::unique_lock<std::mutex> lk(m_);
    const long gen = gen_;
    if (++count_ == n_) {
      count_ = 0;
      ++gen_;
      cv_.notify_all();
    } else {
      cv_.wait(lk, [&] { return gen != gen_; });
    }
  }

 private:
  std::mutex m_;
  std::condition_variable cv_;
  int n_, count_ = 0;
  long gen_ = 0;
};

struct Board {
  double val[GROUP];
  Barrier bar{GROUP};
};

struct CpuGrp {
  int r;
  Board* bd;
  double bcast(double v, int j) const {
    bd->val[r] = v;
    bd->bar.wait();
    const double out = bd->val[j];
    bd->bar.wait();
    return out;
  }
};

// Run fn(chunk, group) for every chunk of a level on 16 row threads.
template <class Fn>
void for_chunks(int64_t chunks, Fn fn) {
  Board bd;
  std::vector<std::thread> th;
  for (int r = 0; r < GROUP; ++r)
    th.emplace_back([&, r] {
      const CpuGrp G{r, &bd};
      for (int64_t ch = 0; ch < chunks; ++ch) fn(ch, G);
    });
  for (auto& t : th) t.join();
}

template <int K, int L0, int L1, class F>
struct WEmu {
  static constexpr int REC = WRec<K>::F;
  int n_init = 0, t_init = 1;
  std::vector<Level> lv;
  std::vector<std::vector<double>> rec, rhs, x;
  const double *c, *d, *s, *u0, *w, *wg = nullptr, *wi = nullptr, *wsm = nullptr;

  void alloc() {
    rec.assign(lv.size(), {}); rhs.assign(lv.size(), {}); x.assign(lv.size(), {});
    for (size_t l = 1; l < lv.size(); ++l) {
      rec[l].assign(lv[l].nodes * REC, 0.0);
      rhs[l].assign(lv[l].nodes * 2 * K, 0.0);
      x[l].assign(lv[l].nodes * K, 0.0);
    }
  }
  Inst<K> inst(int64_t i) const {
    Inst<K> p{};
    if (w) { p.wg = w[3 * i]; p.wi = w[3 * i + 1]; p.ws = w[3 * i + 2]; }
    p.n_init = n_init;
    p.t_init = t_init;
    return p;
  }
  template <int RHS>
  WSrc0<K, double, RHS, F> src0(int64_t i, const double* g, const double* v, int r) const {
    WSrc0<K, double, RHS, F> S;
    S.c = c; S.d = d; S.s = s; S.g = g; S.v = v;
    S.wg = wg; S.wsm = wsm; S.u = u0; S.wi = wi;
    S.uo = static_cast<int>(i * t_init * F::V * n_init);
    S.o = lv[0].node_off[i];
    S.n = lv[0].n[i];
    S.p = inst(i);
    S.r = r;
    return S;
  }
  template <int RHS>
  void reduce(int l, bool wrec, const double* g, const double* v) {
    const Level& lvl = lv[l];
    for_chunks(lvl.chunks, [&](int64_t ch, const CpuGrp& G) {
      const int64_t i = lvl.chunk_inst[ch];
      const int64_t j = ch - lvl.chunk_off[i];
      const ChunkGeom geo = chunk_geom(j, lvl.n[i], l == 0 ? L0 : L1);
      if (!geo.has_left && !geo.has_right) return;
      WReduced<K> red;
      if (l == 0) {
        wreduce_chunk<K, L0>(G, src0<RHS>(i, g, v, G.r), geo.a, geo.b, geo.has_left, geo.has_right, red);
      } else {
        const WSrcN<K> S{rec[l].data() + lvl.node_off[i] * REC, rhs[l].data() + lvl.node_off[i] * 2 * K, G.r};
        wreduce_chunk<K, L1>(G, S, geo.a, geo.b, geo.has_left, geo.has_right, red);
      }
      const int64_t o1 = lv[l + 1].node_off[i];
      wwrite_reduced<K>(red, G.r, rec[l + 1].data() + o1 * REC, rhs[l + 1].data() + o1 * 2 * K, j, geo.has_left,
                        geo.has_right, wrec);
    });
  }
  void backsubN(int l) {
    const Level& lvl = lv[l];
    const bool has_next = l + 1 < static_cast<int>(lv.size());
    for_chunks(lvl.chunks, [&](int64_t ch, const CpuGrp& G) {
      const int r = G.r;
      const int64_t i = lvl.chunk_inst[ch];
      const int64_t j = ch - lvl.chunk_off[i];
      const ChunkGeom geo = chunk_geom(j, lvl.n[i], L1);
      const int64_t up = has_next ? lv[l + 1].node_off[i] : 0;
      const double xl = (geo.has_left && r < K) ? x[l + 1][(up + j - 1) * K + r] : 0.0;
      const double xr = (geo.has_right && r < K) ? x[l + 1][(up + j) * K + r] : 0.0;
      const int64_t o = lvl.node_off[i];
      const WSrcN<K> S{rec[l].data() + o * REC, rhs[l].data() + o * 2 * K, r};
      double ls[L1][K], xs[L1];
      wbacksub_forward<K, L1>(G, S, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, ls, xs);
      WNoSink sink;
      wbacksub_backward<K, L1>(G, S, geo.a, geo.b, ls, xs, sink);
      if (r < K) {
        for (int64_t t = geo.a; t <= geo.b; ++t) x[l][(o + t) * K + r] = xs[t - geo.a];
        if (geo.has_right) x[l][(o + geo.b + 1) * K + r] = xr;
      }
    });
  }
  // level-0 back-substitution: out (OUT_STORE) or the gradients
  template <int RHS, bool GRAD>
  void backsub0(const double* g, const double* v, double* out, const double* y, double* dc, double* dd,
                double* ds, double* du0, double* dwg, double* dwi, double* dws, std::vector<double>* dwp) {
    constexpr bool ADD = (RHS == RHS_RESID || RHS == RHS_GRESID);
    const Level& lvl = lv[0];
    if (dwp) dwp->assign(lvl.chunks * 3, 0.0);
    for_chunks(lvl.chunks, [&](int64_t ch, const CpuGrp& G) {
      const int r = G.r;
      const int64_t i = lvl.chunk_inst[ch];
      const int64_t j = ch - lvl.chunk_off[i];
      const ChunkGeom geo = chunk_geom(j, lvl.n[i], L0);
      const bool nx = lv.size() > 1;
      const int64_t up = nx ? lv[1].node_off[i] : 0;
      const double xl = (nx && geo.has_left && r < K) ? x[1][(up + j - 1) * K + r] : 0.0;
      const double xr = (nx && geo.has_right && r < K) ? x[1][(up + j) * K + r] : 0.0;
      const auto S = src0<RHS>(i, g, v, r);
      double ls[L0][K], xs[L0];
      wbacksub_forward<K, L0>(G, S, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, ls, xs);
      if (!GRAD) {
        WStoreSink<K, double, ADD> sink{out, v, S.o, r};
        if (geo.has_right) sink.node(geo.b + 1, xr);
        wbacksub_backward<K, L0>(G, S, geo.a, geo.b, ls, xs, sink);
      } else {
        WGradSink<K, double, ADD, F, CpuGrp> sink(G);
        sink.c = c; sink.d = d; sink.s = s; sink.y = y; sink.v = v;
        sink.wg = wg; sink.wsm = wsm; sink.u = u0; sink.wi = wi;
        sink.dc = dc; sink.dd = dd; sink.ds = ds; sink.dwg = dwg; sink.dws = dws;
        const int ni = t_init * F::V * n_init;
        sink.du0 = du0 + i * ni;
        sink.dwi = dwi ? dwi + i * ni : nullptr;
        sink.uo = S.uo;
        sink.o = S.o;
        sink.p = S.p;
        if (geo.has_right) sink.start(geo.b + 1, xr);
        wbacksub_backward<K, L0>(G, S, geo.a, geo.b, ls, xs, sink);
        if (geo.has_left) sink.left(geo.a - 1, xl);
        if (!geo.has_right) {
          sink.last_point(lvl.n[i]);
          sink.zero_past_end(lvl.n[i]);
        }
        double dw1 = 0.0;
        for (int m = 0; m < K; ++m) dw1 += G.bcast(sink.dw[1], m);
        if (r == 0 && dwp) {
          (*dwp)[ch * 3] = sink.dw[0];
          (*dwp)[ch * 3 + 1] = dw1;
          (*dwp)[ch * 3 + 2] = sink.dw[2];
        }
      }
    });
  }
  template <int RHS>
  void upper(bool wrec, const double* g, const double* v) {
    const int nl = static_cast<int>(lv.size());
    for (int l = 0; l + 1 < nl; ++l) {
      if (l == 0) reduce<RHS>(0, wrec, g, v);
      else reduce<RHS_BETA>(l, wrec, nullptr, nullptr);
    }
    for (int l = nl - 1; l >= 1; --l) backsubN(l);
  }
};

template <int K, int L, class F>
struct WRunner {
  using E_t = WEmu<K, L, L, F>;
  static void setup(E_t& E, int n_init, int64_t N, const int64_t* T, const double* c, const double* d,
                    const double* s, const double* u0, const double* w, const double* wg, const double* wi,
                    const double* ws) {
    E.n_init = n_init;
    E.t_init = g_init_points;
    E.lv = build_levels(std::vector<int64_t>(T, T + N), L, L);
    E.c = c; E.d = d; E.s = s; E.u0 = u0; E.w = w; E.wg = wg; E.wi = wi; E.wsm = ws;
    E.alloc();
  }
  static int forward(int n_init, int64_t N, const int64_t* T, const double* c, const double* d, const double* s,
                     const double* u0, const double* w, const double* wg, const double* wi, const double* ws,
                     double* y, int refine) {
    E_t E;
    setup(E, n_init, N, T, c, d, s, u0, w, wg, wi, ws);
    const int64_t S = E.lv[0].nodes;
    std::vector<double> b0(S * K), b1(S * K);
    double* bufs[2] = {b0.data(), b1.data()};
    double* dst = refine == 0 ? y : bufs[0];
    E.template upper<RHS_BETA>(true, nullptr, nullptr);
    E.template backsub0<RHS_BETA, false>(nullptr, nullptr, dst, nullptr, nullptr, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, nullptr, nullptr);
    for (int m = 1; m <= refine; ++m) {
      double* prev = dst;
      dst = (m == refine) ? y : bufs[m % 2];
      E.template upper<RHS_RESID>(false, nullptr, prev);
      E.template backsub0<RHS_RESID, false>(nullptr, prev, dst, nullptr, nullptr, nullptr, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, nullptr);
    }
    return 0;
  }
  static int backward(int n_init, int64_t N, const int64_t* T, const double* c, const double* d, const double* s,
                      const double* u0, const double* w, const double* wg, const double* wi, const double* ws,
                      const double* y, const double* gy, double* dc, double* dd, double* ds, double* du0,
                      double* dw, double* dwg, double* dwi, double* dws, int refine) {
    E_t E;
    setup(E, n_init, N, T, c, d, s, u0, w, wg, wi, ws);
    const int64_t S = E.lv[0].nodes;
    std::vector<double> b0(S * K), b1(S * K), tmp(S * K);
    double* bufs[2] = {b0.data(), b1.data()};
    std::vector<double> dwp;
    E.template upper<RHS_BETA>(true, nullptr, nullptr);   // the factor records of the forward pass
    E.template backsub0<RHS_BETA, false>(nullptr, nullptr, tmp.data(), nullptr, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, nullptr, nullptr, nullptr);
    if (refine == 0) {
      E.template upper<RHS_G>(false, gy, nullptr);
      E.template backsub0<RHS_G, true>(gy, nullptr, nullptr, y, dc, dd, ds, du0, dwg, dwi, dws, &dwp);
    } else {
      double* dst = bufs[0];
      E.template upper<RHS_G>(false, gy, nullptr);
      E.template backsub0<RHS_G, false>(gy, nullptr, dst, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                        nullptr, nullptr, nullptr);
      for (int m = 1; m < refine; ++m) {
        double* nd = bufs[m % 2];
        E.template upper<RHS_GRESID>(false, gy, dst);
        E.template backsub0<RHS_GRESID, false>(gy, dst, nd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                               nullptr, nullptr, nullptr);
        dst = nd;
      }
      E.template upper<RHS_GRESID>(false, gy, dst);
      E.template backsub0<RHS_GRESID, true>(gy, dst, nullptr, y, dc, dd, ds, du0, dwg, dwi, dws, &dwp);
    }
    if (!F::WROW)
      for (int64_t i = 0; i < N; ++i) {
        double acc[3] = {0, 0, 0};
        for (int64_t ch = E.lv[0].chunk_off[i]; ch < E.lv[0].chunk_off[i + 1]; ++ch)
          for (int e = 0; e < 3; ++e) acc[e] += dwp[ch * 3 + e];
        for (int e = 0; e < 3; ++e) dw[i * 3 + e] = acc[e];
      }
    return 0;
  }
};

}  // namespace

#define DISPATCH_W(KV, LV, VV, QV, WV, FN, ...)                                              \
  if (K == KV && L == LV && V == VV && QE == QV && wrow == WV)                                 \
    return WRunner<KV, LV, Form<VV, QV, (WV != 0)>>::FN(__VA_ARGS__);

extern "C" {

void emu_wide_set_init_points(int t) { g_init_points = t > 0 ? t : 1; }

int emu_wide_forward(int K, int L, int V, int QE, int wrow, int n_init, int64_t N, const int64_t* T, const double* c,
                     const double* d, const double* s, const double* u0, const double* w, const double* wg,
                     const double* wi, const double* ws, double* y, int refine) {
  DISPATCH_W(6, 4, 2, 2, 0, forward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, refine)
  DISPATCH_W(6, 4, 3, 3, 0, forward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, refine)
  DISPATCH_W(9, 4, 3, 3, 0, forward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, refine)
  DISPATCH_W(9, 4, 3, 3, 1, forward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, refine)
  return -1;
}

int emu_wide_backward(int K, int L, int V, int QE, int wrow, int n_init, int64_t N, const int64_t* T,
                      const double* c, const double* d, const double* s, const double* u0, const double* w,
                      const double* wg, const double* wi, const double* ws, const double* y, const double* gy,
                      double* dc, double* dd, double* ds, double* du0, double* dw, double* dwg, double* dwi,
                      double* dws, int refine) {
  DISPATCH_W(6, 4, 2, 2, 0, backward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, gy, dc, dd, ds, du0, dw, dwg,
             dwi, dws, refine)
  DISPATCH_W(6, 4, 3, 3, 0, backward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, gy, dc, dd, ds, du0, dw, dwg,
             dwi, dws, refine)
  DISPATCH_W(9, 4, 3, 3, 0, backward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, gy, dc, dd, ds, du0, dw, dwg,
             dwi, dws, refine)
  DISPATCH_W(9, 4, 3, 3, 1, backward, n_init, N, T, c, d, s, u0, w, wg, wi, ws, y, gy, dc, dd, ds, du0, dw, dwg,
             dwi, dws, refine)
  return -1;
}
}
