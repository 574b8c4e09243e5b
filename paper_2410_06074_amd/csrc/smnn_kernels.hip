// HIP kernels (gfx950) of the batched S-MNN least-squares solve.
//
// The normal equations M y = beta of Eq. 9 are block tridiagonal (Eq. 10).
// Instead of the paper's single sequential sweep over t (Alg. 3/4, which
// the paper names as its parallelism limit), every level of this solver cuts
// each instance's nodes into chunks of L consecutive nodes; one lane owns one
// chunk.  The last node of every chunk but the instance's last is a
// separator.  A reduce kernel eliminates every chunk interior with the block
// Cholesky recurrence of Alg. 3 (and the forward substitution of Alg. 4),
// accumulating the Schur complement on the two neighbouring separators; the
// separators of neighbouring lanes are combined through a lane shuffle and
// written as the (again block tridiagonal, SPD) system of the next level.
// Back-substitution kernels then solve every chunk interior given its
// separator values, from the top level down.  Per-step factors are never
// stored: each pass recomputes the cheap 3x3..5x5 FP64 recurrence from the
// inputs, so HBM carries only the inputs, the solution and the small
// separator systems.
//
// Lanes map to consecutive chunks, and the per-step arrays are instance-major
// and time-contiguous, so a wavefront's chunks are one contiguous range of
// memory.  Reduce tiles hold 63 new chunks per wave (lane 0 repeats the
// previous tile's last chunk so that every separator has both of its chunks
// in one wave); back-substitution tiles hold 64 chunks.
#include <hip/hip_runtime.h>

#include "smnn_core.h"
#include "smnn_internal.h"

// This file is compiled once per block size K (-DSMNN_TU_K=2..5); each
// translation unit instantiates the chunk lengths listed for its K and
// exports launchers suffixed _k<K> (see smnn_internal.h).
#ifndef SMNN_TU_K
#error "compile with -DSMNN_TU_K=<block size>"
#endif

namespace smnn {
namespace {

constexpr int WAVE = 64;
#ifndef SMNN_MIN_WAVES
#define SMNN_MIN_WAVES 1
#endif

__device__ __forceinline__ int64_t wave_id() {
  return (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
}
__device__ __forceinline__ int64_t wave_count() {
  return static_cast<int64_t>(gridDim.x) * blockDim.x / WAVE;
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

template <int K, class TIO>
__device__ __forceinline__ Inst<K> load_inst(const Level0Args& a, int64_t i) {
  const TIO* w = static_cast<const TIO*>(a.w);
  const TIO* u0 = static_cast<const TIO*>(a.u0);
  Inst<K> p;
  p.wg = static_cast<double>(w[3 * i]);
  p.wi = static_cast<double>(w[3 * i + 1]);
  p.ws = static_cast<double>(w[3 * i + 2]);
  p.n_init = a.n_init;
#pragma unroll
  for (int r = 0; r < K; ++r) p.u0[r] = (r < a.n_init) ? static_cast<double>(u0[i * a.n_init + r]) : 0.0;
  return p;
}

template <int K, class TIO, int RHS>
__device__ __forceinline__ Src0<K, TIO, RHS> make_src0(const Level0Args& a, int64_t i, int64_t off, int64_t n) {
  Src0<K, TIO, RHS> S;
  S.c = static_cast<const TIO*>(a.c) + off * K;
  S.d = static_cast<const TIO*>(a.d) + off;
  S.s = static_cast<const TIO*>(a.s) + off;
  S.g = a.g ? static_cast<const TIO*>(a.g) + off * K : nullptr;
  S.v = a.v ? static_cast<const TIO*>(a.v) + off * K : nullptr;
  S.n = n;
  S.p = load_inst<K, TIO>(a, i);
  return S;
}

__device__ __forceinline__ void report_fail(const Level0Args& a, int64_t inst, int level, int64_t node) {
  uint32_t* info = a.info;
  if (!info) return;
  int64_t step = node;
  for (int l = level; l > 0; --l) step = (step + 1) * (l == 1 ? a.L0 : a.L1) - 1;
  const uint64_t v = static_cast<uint64_t>(step) + 1;
  atomicMin(info + inst, v > 0xFFFFFFFEull ? 0xFFFFFFFEu : static_cast<uint32_t>(v));
}

// Exchange the right-separator reduction of lane-1 and write the combined
// separator record.  All 64 lanes must call this.
template <int K>
__device__ __forceinline__ void exchange_and_write(const Reduced<K>& red, bool writer, double* rec, double* rhs,
                                                   bool write_rec) {
  constexpr int Q = Dim<K>::Q;
  double rA[Q], rf[K];
#pragma unroll
  for (int e = 0; e < Q; ++e) rA[e] = __shfl_up(red.rA[e], 1, WAVE);
#pragma unroll
  for (int e = 0; e < K; ++e) rf[e] = __shfl_up(red.rf[e], 1, WAVE);
  if (writer) combine_separator<K>(rA, rf, red, rec, rhs, write_rec);
}

// ------------------------------------------------------------ level 0 reduce
template <int K, int L, class TIO, int RHS, bool WREC>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_reduce0(LevelDev l0, LevelDev l1, Level0Args a) {
  constexpr int REC = Dim<K>::Q + Dim<K>::KK;
  const int lane = lane_id();
  const int64_t G = l0.chunks;
  const int64_t tiles = G > 1 ? (G - 2) / (WAVE - 1) + 1 : 1;
  for (int64_t tile = wave_id(); tile < tiles; tile += wave_count()) {
    const int64_t g = tile * (WAVE - 1) + lane;
    const bool valid = g < G;
    const int64_t gg = valid ? g : G - 1;
    const int64_t inst = l0.chunk_inst[gg];
    const int64_t j = gg - l0.chunk_off[inst];
    const int64_t off = l0.node_off[inst];
    const int64_t n = l0.node_off[inst + 1] - off;
    const ChunkGeom geo = chunk_geom(j, n, L);
    Reduced<K> red;
#pragma unroll
    for (int e = 0; e < Dim<K>::Q; ++e) { red.rA[e] = 0.0; red.lA[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < K; ++e) { red.rf[e] = 0.0; red.lf[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < Dim<K>::KK; ++e) red.lB[e] = 0.0;
    red.fail = 0;
    if (valid && (geo.has_left || geo.has_right)) {
      const auto S = make_src0<K, TIO, RHS>(a, inst, off, n);
      reduce_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, red);
      if (red.fail) report_fail(a, inst, 0, geo.a + red.fail - 1);
    }
    const bool writer = valid && lane > 0 && geo.has_left;
    const int64_t node = writer ? l1.node_off[inst] + j - 1 : 0;
    exchange_and_write<K>(red, writer, l1.rec + node * REC, l1.rhs + node * K, WREC);
  }
}

// -------------------------------------------------------- level >= 1 reduce
template <int K, int L, bool WREC>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_reduceN(LevelDev lv, LevelDev nx, Level0Args a, int level) {
  constexpr int REC = Dim<K>::Q + Dim<K>::KK;
  const int lane = lane_id();
  const int64_t G = lv.chunks;
  const int64_t tiles = G > 1 ? (G - 2) / (WAVE - 1) + 1 : 1;
  for (int64_t tile = wave_id(); tile < tiles; tile += wave_count()) {
    const int64_t g = tile * (WAVE - 1) + lane;
    const bool valid = g < G;
    const int64_t gg = valid ? g : G - 1;
    const int64_t inst = lv.chunk_inst[gg];
    const int64_t j = gg - lv.chunk_off[inst];
    const int64_t off = lv.node_off[inst];
    const int64_t n = lv.node_off[inst + 1] - off;
    const ChunkGeom geo = chunk_geom(j, n, L);
    Reduced<K> red;
#pragma unroll
    for (int e = 0; e < Dim<K>::Q; ++e) { red.rA[e] = 0.0; red.lA[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < K; ++e) { red.rf[e] = 0.0; red.lf[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < Dim<K>::KK; ++e) red.lB[e] = 0.0;
    red.fail = 0;
    if (valid && (geo.has_left || geo.has_right)) {
      SrcN<K> S;
      S.rec = lv.rec + off * REC;
      S.rhs = lv.rhs + off * K;
      reduce_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, red);
      if (red.fail) report_fail(a, inst, level, geo.a + red.fail - 1);
    }
    const bool writer = valid && lane > 0 && geo.has_left;
    const int64_t node = writer ? nx.node_off[inst] + j - 1 : 0;
    exchange_and_write<K>(red, writer, nx.rec + node * REC, nx.rhs + node * K, WREC);
  }
}

// --------------------------------------------------- level >= 1 back-subst.
template <int K, int L>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_backsubN(LevelDev lv, LevelDev nx, bool has_next, Level0Args a,
                                                 int level) {
  constexpr int REC = Dim<K>::Q + Dim<K>::KK;
  const int lane = lane_id();
  const int64_t G = lv.chunks;
  const int64_t tiles = (G + WAVE - 1) / WAVE;
  for (int64_t tile = wave_id(); tile < tiles; tile += wave_count()) {
    const int64_t g = tile * WAVE + lane;
    if (g >= G) continue;
    const int64_t inst = lv.chunk_inst[g];
    const int64_t j = g - lv.chunk_off[inst];
    const int64_t off = lv.node_off[inst];
    const int64_t n = lv.node_off[inst + 1] - off;
    const ChunkGeom geo = chunk_geom(j, n, L);
    double xl[K], xr[K], xs[L][K];
    const int64_t up = has_next ? nx.node_off[inst] : 0;
#pragma unroll
    for (int e = 0; e < K; ++e) {
      xl[e] = geo.has_left ? nx.x[(up + j - 1) * K + e] : 0.0;
      xr[e] = geo.has_right ? nx.x[(up + j) * K + e] : 0.0;
    }
    SrcN<K> S;
    S.rec = lv.rec + off * REC;
    S.rhs = lv.rhs + off * K;
    const int fail = backsub_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, xs);
    if (fail) report_fail(a, inst, level, geo.a + fail - 1);
    double* x = lv.x + off * K;
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int64_t t = geo.a + u;
      if (t > geo.b) break;
#pragma unroll
      for (int e = 0; e < K; ++e) x[t * K + e] = xs[u][e];
    }
    if (geo.has_right) {
#pragma unroll
      for (int e = 0; e < K; ++e) x[(geo.b + 1) * K + e] = xr[e];
    }
  }
}

// ------------------------------------------------------- level 0 back-subst.
template <int K, int L, class TIO, int RHS, int OUT>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_backsub0(LevelDev l0, LevelDev l1, bool has_next, Level0Args a) {
  constexpr bool ADD = (RHS == RHS_RESID || RHS == RHS_GRESID);
  const int lane = lane_id();
  const int64_t G = l0.chunks;
  const int64_t tiles = (G + WAVE - 1) / WAVE;
  for (int64_t tile = wave_id(); tile < tiles; tile += wave_count()) {
    const int64_t g = tile * WAVE + lane;
    if (g >= G) continue;
    const int64_t inst = l0.chunk_inst[g];
    const int64_t j = g - l0.chunk_off[inst];
    const int64_t off = l0.node_off[inst];
    const int64_t n = l0.node_off[inst + 1] - off;
    const ChunkGeom geo = chunk_geom(j, n, L);
    double xl[K], xr[K], xs[L][K];
    const int64_t up = has_next ? l1.node_off[inst] : 0;
#pragma unroll
    for (int e = 0; e < K; ++e) {
      xl[e] = geo.has_left ? l1.x[(up + j - 1) * K + e] : 0.0;
      xr[e] = geo.has_right ? l1.x[(up + j) * K + e] : 0.0;
    }
    const auto S = make_src0<K, TIO, RHS>(a, inst, off, n);
    const TIO* v = ADD ? static_cast<const TIO*>(a.v) + off * K : nullptr;
    int fail;
    if (OUT == OUT_STORE) {
      StoreSink<TIO, ADD> sink{static_cast<TIO*>(a.out) + off * K, v};
      if (geo.has_right) sink.template node<K>(geo.b + 1, xr);   // owned right separator
      fail = backsub_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, xs, sink);
    } else {
      GradSink<K, TIO, ADD> sink;
      sink.c = S.c; sink.d = S.d; sink.s = S.s;
      sink.y = static_cast<const TIO*>(a.y) + off * K;
      sink.v = v;
      sink.dc = static_cast<TIO*>(a.dc) + off * K;
      sink.dd = static_cast<TIO*>(a.dd) + off;
      sink.ds = static_cast<TIO*>(a.ds) + off;
      sink.du0 = static_cast<TIO*>(a.du0) + inst * a.n_init;
      sink.p = S.p;
      if (geo.has_right) sink.start(geo.b + 1, xr);
      fail = backsub_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, xs, sink);
      if (geo.has_left) sink.left(geo.a - 1, xl);
      if (!geo.has_right) sink.ds[n - 1] = static_cast<TIO>(0.0);   // s of the last point is unused
#pragma unroll
      for (int e = 0; e < 3; ++e) a.dw_part[g * 3 + e] = sink.dw[e];
    }
    if (fail) report_fail(a, inst, 0, geo.a + fail - 1);
  }
}

int64_t grid_for(int64_t tiles, const Launch& cfg) {
  const int64_t waves_per_block = cfg.block / WAVE;
  int64_t blocks = (tiles + waves_per_block - 1) / waves_per_block;
  if (cfg.max_blocks > 0 && blocks > cfg.max_blocks) blocks = cfg.max_blocks;
  return blocks < 1 ? 1 : blocks;
}

// ------------------------------------------------------------- dispatchers
template <int K, int L, class TIO>
hipError_t reduce0_t(int rhs, bool wrec, const LevelDev& l0, const LevelDev& l1, const Level0Args& a,
                     const Launch& cfg, hipStream_t st) {
  const int64_t tiles = l0.chunks > 1 ? (l0.chunks - 2) / (WAVE - 1) + 1 : 1;
  const dim3 grid(static_cast<unsigned>(grid_for(tiles, cfg))), block(cfg.block);
  switch (rhs) {
    case RHS_BETA:
      if (wrec) hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS_BETA, true>), grid, block, 0, st, l0, l1, a);
      else hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS_BETA, false>), grid, block, 0, st, l0, l1, a);
      break;
    case RHS_RESID: hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS_RESID, false>), grid, block, 0, st, l0, l1, a); break;
    case RHS_G:
      if (wrec) hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS_G, true>), grid, block, 0, st, l0, l1, a);
      else hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS_G, false>), grid, block, 0, st, l0, l1, a);
      break;
    case RHS_GRESID: hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS_GRESID, false>), grid, block, 0, st, l0, l1, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K, int L, class TIO>
hipError_t backsub0_t(int rhs, int out, const LevelDev& l0, const LevelDev* l1, const Level0Args& a,
                      const Launch& cfg, hipStream_t st) {
  const int64_t tiles = (l0.chunks + WAVE - 1) / WAVE;
  const dim3 grid(static_cast<unsigned>(grid_for(tiles, cfg))), block(cfg.block);
  const LevelDev nx = l1 ? *l1 : LevelDev{};
  const bool hn = l1 != nullptr;
  if (out == OUT_STORE) {
    switch (rhs) {
      case RHS_BETA: hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS_BETA, OUT_STORE>), grid, block, 0, st, l0, nx, hn, a); break;
      case RHS_RESID: hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS_RESID, OUT_STORE>), grid, block, 0, st, l0, nx, hn, a); break;
      case RHS_G: hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS_G, OUT_STORE>), grid, block, 0, st, l0, nx, hn, a); break;
      case RHS_GRESID: hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS_GRESID, OUT_STORE>), grid, block, 0, st, l0, nx, hn, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (rhs) {
      case RHS_G: hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS_G, OUT_GRAD>), grid, block, 0, st, l0, nx, hn, a); break;
      case RHS_GRESID: hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS_GRESID, OUT_GRAD>), grid, block, 0, st, l0, nx, hn, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int K, int L>
hipError_t reduceN_t(bool wrec, int level, const LevelDev& l, const LevelDev& nx, const Level0Args& a,
                     const Launch& cfg, hipStream_t st) {
  const int64_t tiles = l.chunks > 1 ? (l.chunks - 2) / (WAVE - 1) + 1 : 1;
  const dim3 grid(static_cast<unsigned>(grid_for(tiles, cfg))), block(cfg.block);
  if (wrec) hipLaunchKernelGGL((k_reduceN<K, L, true>), grid, block, 0, st, l, nx, a, level);
  else hipLaunchKernelGGL((k_reduceN<K, L, false>), grid, block, 0, st, l, nx, a, level);
  return hipGetLastError();
}

template <int K, int L>
hipError_t backsubN_t(int level, const LevelDev& l, const LevelDev* nx, const Level0Args& a, const Launch& cfg,
                      hipStream_t st) {
  const int64_t tiles = (l.chunks + WAVE - 1) / WAVE;
  const dim3 grid(static_cast<unsigned>(grid_for(tiles, cfg))), block(cfg.block);
  const LevelDev n2 = nx ? *nx : LevelDev{};
  hipLaunchKernelGGL((k_backsubN<K, L>), grid, block, 0, st, l, n2, nx != nullptr, a, level);
  return hipGetLastError();
}

}  // namespace

// (K, L) pairs compiled in: L is the chunk length of every level.
#ifdef SMNN_FOR_EACH_KL
#elif SMNN_TU_K == 2
#define SMNN_FOR_EACH_KL(X) X(2, 8) X(2, 16)
#elif SMNN_TU_K == 3
#define SMNN_FOR_EACH_KL(X) X(3, 4) X(3, 8) X(3, 16)
#elif SMNN_TU_K == 4
#define SMNN_FOR_EACH_KL(X) X(4, 4) X(4, 8)
#elif SMNN_TU_K == 5
#define SMNN_FOR_EACH_KL(X) X(5, 4)
#endif

bool SMNN_KFN(supported)(int K, int L) {
#define X(KV, LV) if (K == KV && L == LV) return true;
  SMNN_FOR_EACH_KL(X)
#undef X
  return false;
}

hipError_t SMNN_KFN(launch_reduce0)(int K, int L, bool f32, int rhs_mode, bool write_rec, const LevelDev& l0,
                          const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV)                                                                                    \
  if (K == KV && L == LV)                                                                            \
    return f32 ? reduce0_t<KV, LV, float>(rhs_mode, write_rec, l0, l1, a, cfg, st)                  \
               : reduce0_t<KV, LV, double>(rhs_mode, write_rec, l0, l1, a, cfg, st);
  SMNN_FOR_EACH_KL(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_KFN(launch_backsub0)(int K, int L, bool f32, int rhs_mode, int out_mode, const LevelDev& l0,
                           const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV)                                                                                    \
  if (K == KV && L == LV)                                                                            \
    return f32 ? backsub0_t<KV, LV, float>(rhs_mode, out_mode, l0, l1, a, cfg, st)                  \
               : backsub0_t<KV, LV, double>(rhs_mode, out_mode, l0, l1, a, cfg, st);
  SMNN_FOR_EACH_KL(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_KFN(launch_reduceN)(int K, int L, bool write_rec, int level, const LevelDev& l, const LevelDev& lnext,
                          const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV) \
  if (K == KV && L == LV) return reduceN_t<KV, LV>(write_rec, level, l, lnext, a, cfg, st);
  SMNN_FOR_EACH_KL(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_KFN(launch_backsubN)(int K, int L, int level, const LevelDev& l, const LevelDev* lnext,
                           const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV) \
  if (K == KV && L == LV) return backsubN_t<KV, LV>(level, l, lnext, a, cfg, st);
  SMNN_FOR_EACH_KL(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace smnn
