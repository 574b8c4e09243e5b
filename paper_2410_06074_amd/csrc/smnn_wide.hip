// HIP kernels of the solve for wide blocks (K = V (R+1) > 5): the same
// partition into chunks and separator levels as smnn_kernels.hip, with one
// 16-lane group per chunk instead of one lane (four chunks per wavefront),
// each lane holding one row of the chunk's blocks (smnn_wide.h).  Separator
// records are full K x K blocks in the natural layout, each half written by
// the one chunk that owns it, so no two groups write the same location and
// no exchange between groups is needed.  Inputs are read straight from
// global memory (the rows of a group read the same coefficients, which the
// caches serve once).
#include <hip/hip_runtime.h>

#include "smnn_internal.h"
#include "smnn_wide.h"

#ifndef SMNN_TU_K
#error "compile with -DSMNN_TU_K=<block size>"
#endif

namespace smnn {
namespace {

constexpr int WAVE = 64;
constexpr int GPW = WAVE / GROUP;   // chunks (groups) per wavefront
// One wave per SIMD: the rows of a 9 x 9 block step need ~450 registers;
// held to two waves per SIMD the kernels spill ~1 KB per lane to scratch and
// measured 2.9x slower (27.3 vs 9.4 ms per fp64r step, 512 x 1000, V = 3).
#ifndef SMNN_WIDE_MIN_BLOCKS
#define SMNN_WIDE_MIN_BLOCKS 1
#endif

// Row J of the lane's 16-lane group (a DPP row of the wave): a
// row_newbcast data-parallel move, one VALU instruction per 32-bit half.
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x150 + J, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x150 + J, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// The lane's group: its row r and a broadcast within the 16 lanes.  j is a
// compile-time constant at every call (unrolled loops), so the switch folds
// to the one move.
struct GpuGrp {
  int r;
  __device__ __forceinline__ double bcast(double v, int j) const {
    switch (j) {
      case 0: return row_bcast<0>(v);
      case 1: return row_bcast<1>(v);
      case 2: return row_bcast<2>(v);
      case 3: return row_bcast<3>(v);
      case 4: return row_bcast<4>(v);
      case 5: return row_bcast<5>(v);
      case 6: return row_bcast<6>(v);
      case 7: return row_bcast<7>(v);
      case 8: return row_bcast<8>(v);
      case 9: return row_bcast<9>(v);
      case 10: return row_bcast<10>(v);
      case 11: return row_bcast<11>(v);
      case 12: return row_bcast<12>(v);
      case 13: return row_bcast<13>(v);
      case 14: return row_bcast<14>(v);
      default: return row_bcast<15>(v);
    }
  }
};

__device__ __forceinline__ GpuGrp grp() {
  const int lane = threadIdx.x & (WAVE - 1);
  return GpuGrp{lane & (GROUP - 1)};
}

// Wave index (XCD-aware, as in smnn_kernels.hip) and the static tile schedule.
constexpr int XCDS = 8;
__device__ __forceinline__ int64_t wave_id(const Level0Args& a) {
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / WAVE);
  const int64_t nb = a.nwaves / a.wpb;
  const int64_t b = blockIdx.x;
  const int64_t q = nb / XCDS, r = nb % XCDS, x = b % XCDS, k = b / XCDS;
  const int64_t vb = x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
  return vb * a.wpb + w;
}

__device__ __forceinline__ void report_fail(const Level0Args& a, int64_t inst, int level, int64_t node) {
  uint32_t* info = a.info;
  if (!info) return;
  int64_t step = node;
  for (int l = level; l > 0; --l) step = (step + 1) * (l == 1 ? a.L0 : a.L1) - 1;
  const uint64_t v = static_cast<uint64_t>(step) + 1;
  atomicMin(info + inst, v > 0xFFFFFFFEull ? 0xFFFFFFFEu : static_cast<uint32_t>(v));
}

template <int K, class TIO>
__device__ __forceinline__ Inst<K> load_inst(const Level0Args& a, int64_t i) {
  Inst<K> p;
  if (a.w) {
    const TIO* w = static_cast<const TIO*>(a.w);
    p.wg = static_cast<double>(w[3 * i]);
    p.wi = static_cast<double>(w[3 * i + 1]);
    p.ws = static_cast<double>(w[3 * i + 2]);
  } else {
    p.wg = p.wi = p.ws = 0.0;
  }
  p.n_init = a.n_init;
  p.t_init = a.t_init;
  return p;
}

template <int K, class TIO, int RHS, class F>
__device__ __forceinline__ WSrc0<K, TIO, RHS, F> make_src0(const Level0Args& a, int64_t inst, int64_t off,
                                                           int64_t n, int r) {
  WSrc0<K, TIO, RHS, F> S;
  S.c = static_cast<const TIO*>(a.c);
  S.d = static_cast<const TIO*>(a.d);
  S.s = static_cast<const TIO*>(a.s);
  S.g = static_cast<const TIO*>(a.g);
  S.v = static_cast<const TIO*>(a.v);
  S.wg = static_cast<const TIO*>(a.wg);
  S.wsm = static_cast<const TIO*>(a.ws);
  S.u = static_cast<const TIO*>(a.u0);
  S.wi = static_cast<const TIO*>(a.wi);
  S.uo = static_cast<int>(inst) * a.t_init * F::V * a.n_init;
  S.o = off;
  S.n = n;
  S.p = load_inst<K, TIO>(a, inst);
  S.r = r;
  return S;
}

// Chunk of this group in the tile: tiles hold GPW consecutive chunks.
struct Where {
  int64_t g, inst, j, off, n;
  bool valid;
};

__device__ __forceinline__ Where where(const LevelDev& lv, int64_t tile) {
  Where w;
  const int grp_in_wave = (threadIdx.x & (WAVE - 1)) / GROUP;
  w.g = tile * GPW + grp_in_wave;
  w.valid = w.g < lv.chunks;
  const int64_t gg = w.valid ? w.g : lv.chunks - 1;
  w.inst = lv.chunk_inst[gg];
  w.j = gg - lv.chunk_off[w.inst];
  w.off = lv.node_off[w.inst];
  w.n = lv.node_off[w.inst + 1] - w.off;
  return w;
}

// ------------------------------------------------------------------ reduces
template <int K, int L, class TIO, int RHS, bool WREC, class F>
__global__ void __launch_bounds__(256, SMNN_WIDE_MIN_BLOCKS) wk_reduce0(LevelDev l0, LevelDev l1, Level0Args a) {
  const GpuGrp G = grp();
  const int64_t tiles = (l0.chunks + GPW - 1) / GPW;
  for (int64_t tw = wave_id(a); tw < tiles; tw += a.nwaves) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const Where w = where(l0, tile);
    const ChunkGeom geo = chunk_geom(w.j, w.n, L);
    if (w.valid && (geo.has_left || geo.has_right)) {
      const auto src = make_src0<K, TIO, RHS, F>(a, w.inst, w.off, w.n, G.r);
      WReduced<K> red;
      wreduce_chunk<K, L>(G, src, geo.a, geo.b, geo.has_left, geo.has_right, red);
      if (red.fail) report_fail(a, w.inst, 0, geo.a + red.fail - 1);
      const int64_t o1 = l1.node_off[w.inst];
      wwrite_reduced<K>(red, G.r, l1.rec + o1 * WRec<K>::F, l1.rhs + o1 * 2 * K, w.j, geo.has_left,
                        geo.has_right, WREC);
    }
  }
}

template <int K, int L, bool WREC>
__global__ void __launch_bounds__(256, SMNN_WIDE_MIN_BLOCKS) wk_reduceN(LevelDev lv, LevelDev nx, Level0Args a, int level) {
  const GpuGrp G = grp();
  const int64_t tiles = (lv.chunks + GPW - 1) / GPW;
  for (int64_t tw = wave_id(a); tw < tiles; tw += a.nwaves) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const Where w = where(lv, tile);
    const ChunkGeom geo = chunk_geom(w.j, w.n, L);
    if (w.valid && (geo.has_left || geo.has_right)) {
      const WSrcN<K> src{lv.rec + w.off * WRec<K>::F, lv.rhs + w.off * 2 * K, G.r};
      WReduced<K> red;
      wreduce_chunk<K, L>(G, src, geo.a, geo.b, geo.has_left, geo.has_right, red);
      if (red.fail) report_fail(a, w.inst, level, geo.a + red.fail - 1);
      const int64_t o1 = nx.node_off[w.inst];
      wwrite_reduced<K>(red, G.r, nx.rec + o1 * WRec<K>::F, nx.rhs + o1 * 2 * K, w.j, geo.has_left,
                        geo.has_right, WREC);
    }
  }
}

// ----------------------------------------------------- back-substitutions
template <int K, int L>
__global__ void __launch_bounds__(256, SMNN_WIDE_MIN_BLOCKS) wk_backsubN(LevelDev lv, LevelDev nx, bool has_next, Level0Args a,
                                                      int level) {
  const GpuGrp G = grp();
  const int r = G.r;
  const int64_t tiles = (lv.chunks + GPW - 1) / GPW;
  for (int64_t tw = wave_id(a); tw < tiles; tw += a.nwaves) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const Where w = where(lv, tile);
    if (!w.valid) continue;   // group-uniform: the group's lanes share the chunk
    const ChunkGeom geo = chunk_geom(w.j, w.n, L);
    const int64_t up = has_next ? nx.node_off[w.inst] : 0;
    const double xl = (geo.has_left && r < K) ? nx.x[(up + w.j - 1) * K + r] : 0.0;
    const double xr = (geo.has_right && r < K) ? nx.x[(up + w.j) * K + r] : 0.0;
    const WSrcN<K> src{lv.rec + w.off * WRec<K>::F, lv.rhs + w.off * 2 * K, r};
    double ls[L][K], xs[L];
    const int fail = wbacksub_forward<K, L>(G, src, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, ls, xs);
    WNoSink sink;
    wbacksub_backward<K, L>(G, src, geo.a, geo.b, ls, xs, sink);
    if (fail) report_fail(a, w.inst, level, geo.a + fail - 1);
    if (r < K) {
      double* x = lv.x + w.off * K;
#pragma unroll
      for (int u = 0; u < L; ++u) {
        const int64_t t = geo.a + u;
        if (t > geo.b) break;
        x[t * K + r] = xs[u];
      }
      if (geo.has_right) x[(geo.b + 1) * K + r] = xr;
    }
  }
}

template <int K, int L, class TIO, int RHS, int OUT, class F>
__global__ void __launch_bounds__(256, SMNN_WIDE_MIN_BLOCKS) wk_backsub0(LevelDev l0, LevelDev l1, bool has_next, Level0Args a) {
  constexpr bool ADD = (RHS == RHS_RESID || RHS == RHS_GRESID);
  const GpuGrp G = grp();
  const int r = G.r;
  const int64_t tiles = (l0.chunks + GPW - 1) / GPW;
  for (int64_t tw = wave_id(a); tw < tiles; tw += a.nwaves) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const Where w = where(l0, tile);
    if (!w.valid) continue;   // group-uniform
    const ChunkGeom geo = chunk_geom(w.j, w.n, L);
    const int64_t up = has_next ? l1.node_off[w.inst] : 0;
    const double xl = (geo.has_left && r < K) ? l1.x[(up + w.j - 1) * K + r] : 0.0;
    const double xr = (geo.has_right && r < K) ? l1.x[(up + w.j) * K + r] : 0.0;
    const auto src = make_src0<K, TIO, RHS, F>(a, w.inst, w.off, w.n, r);
    double ls[L][K], xs[L];
    const int fail = wbacksub_forward<K, L>(G, src, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, ls, xs);
    if (OUT == OUT_STORE) {
      WStoreSink<K, TIO, ADD> sink{static_cast<TIO*>(a.out), static_cast<const TIO*>(a.v), w.off, r};
      if (geo.has_right) sink.node(geo.b + 1, xr);   // owned right separator
      wbacksub_backward<K, L>(G, src, geo.a, geo.b, ls, xs, sink);
    } else {
      WGradSink<K, TIO, ADD, F, GpuGrp> sink(G);
      sink.c = src.c; sink.d = src.d; sink.s = src.s;
      sink.y = static_cast<const TIO*>(a.y);
      sink.v = static_cast<const TIO*>(a.v);
      sink.wg = src.wg; sink.wsm = src.wsm; sink.u = src.u; sink.wi = src.wi;
      sink.dc = static_cast<TIO*>(a.dc);
      sink.dd = static_cast<TIO*>(a.dd);
      sink.ds = static_cast<TIO*>(a.ds);
      sink.dwg = static_cast<TIO*>(a.dwg);
      sink.dws = static_cast<TIO*>(a.dws);
      const int ni = a.t_init * F::V * a.n_init;
      sink.du0 = static_cast<TIO*>(a.du0) + w.inst * ni;
      sink.dwi = a.dwi ? static_cast<TIO*>(a.dwi) + w.inst * ni : nullptr;
      sink.uo = src.uo;
      sink.o = w.off;
      sink.p = src.p;
      if (geo.has_right) sink.start(geo.b + 1, xr);
      wbacksub_backward<K, L>(G, src, geo.a, geo.b, ls, xs, sink);
      if (geo.has_left) sink.left(geo.a - 1, xl);
      if (!geo.has_right) {
        sink.last_point(w.n);
        sink.zero_past_end(w.n);
      }
      if constexpr (!F::WROW) {
        // the initial-row weight partials sit on the rows that own them
        double dw1 = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m) dw1 += G.bcast(sink.dw[1], m);
        if (r == 0) {
          a.dw_part[w.g * 3 + 0] = sink.dw[0];
          a.dw_part[w.g * 3 + 1] = dw1;
          a.dw_part[w.g * 3 + 2] = sink.dw[2];
        }
      }
    }
    if (fail) report_fail(a, w.inst, 0, geo.a + fail - 1);
  }
}

// ------------------------------------------------------------ launchers
int64_t grid_for(int64_t tiles, const Launch& cfg) {
  const int64_t waves_per_block = cfg.block / WAVE;
  int64_t blocks = (tiles + waves_per_block - 1) / waves_per_block;
  if (cfg.max_blocks > 0 && blocks > cfg.max_blocks) blocks = cfg.max_blocks;
  return blocks < 1 ? 1 : blocks;
}

Level0Args shape(const Level0Args& a, const Launch& cfg, dim3 grid) {
  Level0Args b = a;
  b.wpb = cfg.block / WAVE;
  b.nwaves = static_cast<int64_t>(grid.x) * b.wpb;
  return b;
}

template <int K, int L, class TIO, class F>
hipError_t reduce0_t(int rhs, bool wrec, const LevelDev& l0, const LevelDev& l1, const Level0Args& a,
                     const Launch& cfg, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(grid_for((l0.chunks + GPW - 1) / GPW, cfg))), block(cfg.block);
  const Level0Args b = shape(a, cfg, grid);
  switch (rhs) {
    case RHS_BETA:
      if (wrec) hipLaunchKernelGGL((wk_reduce0<K, L, TIO, RHS_BETA, true, F>), grid, block, 0, st, l0, l1, b);
      else hipLaunchKernelGGL((wk_reduce0<K, L, TIO, RHS_BETA, false, F>), grid, block, 0, st, l0, l1, b);
      break;
    case RHS_RESID: hipLaunchKernelGGL((wk_reduce0<K, L, TIO, RHS_RESID, false, F>), grid, block, 0, st, l0, l1, b); break;
    case RHS_G: hipLaunchKernelGGL((wk_reduce0<K, L, TIO, RHS_G, false, F>), grid, block, 0, st, l0, l1, b); break;
    case RHS_GRESID: hipLaunchKernelGGL((wk_reduce0<K, L, TIO, RHS_GRESID, false, F>), grid, block, 0, st, l0, l1, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K, int L, class TIO, class F>
hipError_t backsub0_t(int rhs, int out, const LevelDev& l0, const LevelDev* l1, const Level0Args& a,
                      const Launch& cfg, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(grid_for((l0.chunks + GPW - 1) / GPW, cfg))), block(cfg.block);
  const Level0Args b = shape(a, cfg, grid);
  const LevelDev nx = l1 ? *l1 : LevelDev{};
  const bool hn = l1 != nullptr;
  if (out == OUT_STORE) {
    switch (rhs) {
      case RHS_BETA: hipLaunchKernelGGL((wk_backsub0<K, L, TIO, RHS_BETA, OUT_STORE, F>), grid, block, 0, st, l0, nx, hn, b); break;
      case RHS_RESID: hipLaunchKernelGGL((wk_backsub0<K, L, TIO, RHS_RESID, OUT_STORE, F>), grid, block, 0, st, l0, nx, hn, b); break;
      case RHS_G: hipLaunchKernelGGL((wk_backsub0<K, L, TIO, RHS_G, OUT_STORE, F>), grid, block, 0, st, l0, nx, hn, b); break;
      case RHS_GRESID: hipLaunchKernelGGL((wk_backsub0<K, L, TIO, RHS_GRESID, OUT_STORE, F>), grid, block, 0, st, l0, nx, hn, b); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (rhs) {
      case RHS_G: hipLaunchKernelGGL((wk_backsub0<K, L, TIO, RHS_G, OUT_GRAD, F>), grid, block, 0, st, l0, nx, hn, b); break;
      case RHS_GRESID: hipLaunchKernelGGL((wk_backsub0<K, L, TIO, RHS_GRESID, OUT_GRAD, F>), grid, block, 0, st, l0, nx, hn, b); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int K, int L>
hipError_t reduceN_t(bool wrec, int level, const LevelDev& l, const LevelDev& nx, const Level0Args& a,
                     const Launch& cfg, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(grid_for((l.chunks + GPW - 1) / GPW, cfg))), block(cfg.block);
  const Level0Args b = shape(a, cfg, grid);
  if (wrec) hipLaunchKernelGGL((wk_reduceN<K, L, true>), grid, block, 0, st, l, nx, b, level);
  else hipLaunchKernelGGL((wk_reduceN<K, L, false>), grid, block, 0, st, l, nx, b, level);
  return hipGetLastError();
}

template <int K, int L>
hipError_t backsubN_t(int level, const LevelDev& l, const LevelDev* nx, const Level0Args& a, const Launch& cfg,
                      hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(grid_for((l.chunks + GPW - 1) / GPW, cfg))), block(cfg.block);
  const Level0Args b = shape(a, cfg, grid);
  const LevelDev n2 = nx ? *nx : LevelDev{};
  hipLaunchKernelGGL((wk_backsubN<K, L>), grid, block, 0, st, l, n2, nx != nullptr, b, level);
  return hipGetLastError();
}

}  // namespace

// What this translation unit compiles in: (K, L, instance form, form id).
#if SMNN_TU_K == 6
#define SMNN_WIDE_L(X) X(6, 4)
#define SMNN_WIDE_KLF(X) X(6, 4, Form<2 SMNN_COMMA 2 SMNN_COMMA false>, SMNN_FORM_V2) \
                         X(6, 4, Form<3 SMNN_COMMA 3 SMNN_COMMA false>, SMNN_FORM_V3)
#elif SMNN_TU_K == 9
#define SMNN_WIDE_L(X) X(9, 4)
#define SMNN_WIDE_KLF(X) X(9, 4, Form<3 SMNN_COMMA 3 SMNN_COMMA false>, SMNN_FORM_V3) \
                         X(9, 4, Form<3 SMNN_COMMA 3 SMNN_COMMA true>, SMNN_FORM_V3_ROWS)
#else
#error "wide block sizes built: 6, 9"
#endif
#define SMNN_COMMA ,

bool SMNN_WFN(wide_supported)(int K, int L, int form) {
#define X(KV, LV, FT, FID) if (K == KV && L == LV && form == FID) return true;
  SMNN_WIDE_KLF(X)
#undef X
  return false;
}

hipError_t SMNN_WFN(launch_wreduce0)(int K, int L, int form, bool f32, int rhs, bool wrec, const LevelDev& l0,
                                     const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV, FT, FID)                                                               \
  if (K == KV && L == LV && form == FID)                                                 \
    return f32 ? reduce0_t<KV, LV, float, FT>(rhs, wrec, l0, l1, a, cfg, st)            \
               : reduce0_t<KV, LV, double, FT>(rhs, wrec, l0, l1, a, cfg, st);
  SMNN_WIDE_KLF(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_WFN(launch_wbacksub0)(int K, int L, int form, bool f32, int rhs, int out, const LevelDev& l0,
                                      const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV, FT, FID)                                                               \
  if (K == KV && L == LV && form == FID)                                                 \
    return f32 ? backsub0_t<KV, LV, float, FT>(rhs, out, l0, l1, a, cfg, st)            \
               : backsub0_t<KV, LV, double, FT>(rhs, out, l0, l1, a, cfg, st);
  SMNN_WIDE_KLF(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_WFN(launch_wreduceN)(int K, int L, bool wrec, int level, const LevelDev& l, const LevelDev& nx,
                                     const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV) \
  if (K == KV && L == LV) return reduceN_t<KV, LV>(wrec, level, l, nx, a, cfg, st);
  SMNN_WIDE_L(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_WFN(launch_wbacksubN)(int K, int L, int level, const LevelDev& l, const LevelDev* nx,
                                      const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV) \
  if (K == KV && L == LV) return backsubN_t<KV, LV>(level, l, nx, a, cfg, st);
  SMNN_WIDE_L(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace smnn
