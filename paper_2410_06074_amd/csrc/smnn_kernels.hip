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
//
// Level-0 kernels first copy that range (plus one step on either side) of
// every per-step array they read into the wave's slice of LDS, with
// direct global-to-LDS loads that all lanes issue at once; the chunk
// recurrences then read LDS.  A wave thus waits on HBM about once per tile
// rather than once per node step.  The level-0 back-substitution writes its
// results into the slice and stores them as whole rows.  In the refined
// modes the back-substitution of the first solve also performs the level-0
// reduce of the refinement solve (k_backsub_reduce0), from the iterate it
// leaves in LDS.  Separator levels keep their records interleaved by groups
// of chunks (tpos in smnn_core.h), so their per-lane node loads are
// contiguous across the lanes of a wave.

#include <hip/hip_runtime.h>

#include "smnn_core.h"
#include "smnn_internal.h"

// This file is compiled once per block size K (-DSMNN_TU_K=2..5) and group
// of instance forms (-DSMNN_TU_FORMS=0..2, see the lists at the end); each
// translation unit instantiates the chunk lengths listed for its K and
// exports launchers suffixed _k<K> (forms group 0) or _k<K>f<group> (see
// smnn_internal.h).
#ifndef SMNN_TU_K
#error "compile with -DSMNN_TU_K=<block size>"
#endif

namespace smnn {
namespace {

constexpr int WAVE = 64;
#ifndef SMNN_MIN_WAVES
#define SMNN_MIN_WAVES 1
#endif

// Wave index and wave count of the launch (wave-uniform values; the launch
// shape comes in through the arguments so no dispatch-packet loads precede
// the first memory requests).  Workgroups are dispatched round-robin over
// the 8 XCDs (workgroup b runs on XCD b % 8); the wave index gives each
// XCD a contiguous range of tiles, so that neighbouring tiles, which share
// boundary rows and write the two halves of some 64-byte runs, meet in the
// same L2.  The map is a bijection of [0, nwaves).  Launches alternate
// the direction in which the tiles are taken (Level0Args::rev), so that a
// kernel starts with the data the previous one touched last, which the
// device's last-level (memory-side) cache still holds.
constexpr int XCDS = 8;
__device__ __forceinline__ int64_t wave_id(const Level0Args& a) {
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / WAVE);
  const int64_t nb = a.nwaves / a.wpb;
  const int64_t b = blockIdx.x;
  const int64_t q = nb / XCDS, r = nb % XCDS, x = b % XCDS, k = b / XCDS;
  const int64_t vb = x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
  return vb * a.wpb + w;
}
__device__ __forceinline__ int64_t wave_count(const Level0Args& a) { return a.nwaves; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// Tile schedule of a launch.  Without a queue the tiles are dealt out
// statically: wave w takes tiles w, w + waves, ...  Persistent launches
// (a capped grid) carry a device work queue instead, a counter that every
// wave increments to claim its next tile until the tiles run out, so waves
// that finish early take more.  Every lane of a wave calls these at the
// same point (wave-uniform control flow), lane 0 claims for the wave and
// the claim is read back into a scalar register (readfirstlane, not a lane
// shuffle), so that the tile index stays wave-uniform to the compiler as in
// the static schedule: addresses derived from it stay scalar and the tile
// loop is not treated as divergent.
__device__ __forceinline__ int64_t claim_tile(const Level0Args& a) {
  int v = 0;
  if (lane_id() == 0) v = static_cast<int>(atomicAdd(a.queue, 1u));
  return static_cast<int64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(v)));
}
__device__ __forceinline__ int64_t first_tile(const Level0Args& a) {
  return a.queue ? claim_tile(a) : wave_id(a);
}
__device__ __forceinline__ int64_t next_tile(const Level0Args& a, int64_t tw) {
  return a.queue ? claim_tile(a) : tw + wave_count(a);
}

// ---------------------------------------------------------- LDS staging
// Per-step arrays a level-0 kernel variant reads (c and s always; the
// per-row governing and smoothness weights with per-row weights).
template <int RHS, int OUT>
struct Reads {
  static constexpr bool d = RHS == RHS_BETA || RHS == RHS_RESID || OUT == OUT_GRAD;
  static constexpr bool g = RHS == RHS_G || RHS == RHS_GRESID;
  static constexpr bool v = RHS == RHS_RESID || RHS == RHS_GRESID;
  static constexpr bool y = OUT == OUT_GRAD;   // staged after the forward sweep, over g
};

// ------------------------------------------------------------ LDS placement
// A lane reads the rows of its own chunk, so in one LDS instruction the 64
// lanes touch addresses W L elements apart (W elements per row, L rows per
// chunk): 12 doubles for the 3 x 3 blocks of c at chunk 4, 4 for the step
// sizes.  Both are multiples of 8 dwords, which puts the 64 addresses on 4
// bank groups of the LDS.  A bank model (32 and 64 banks, 4 bytes wide; 16
// or 32 lanes per cycle for 8-byte reads, 32 or 64 for 4-byte ones) puts
// strides that are multiples of 8 elements at 8- to 32-way conflicts and the
// others (4, 12, 20) at 4-way.  Arrays of the first kind are stored swizzled
// within 256-byte blocks: element e sits at e XOR ((e >> (log2(elements per
// block) + SH)) mod elements per block), its slot within the block XORed
// with the block index shifted by SH (chosen per A with the same model;
// 2-way at most).  A block holds 256 contiguous input bytes whichever the
// swizzle, so the staging loads stay coalesced: each lane of a load fetches
// the element its LDS position holds (the map is its own inverse).  The
// 4-way arrays (among them all of 3 x 3 blocks at chunk 4 in FP64) stay in
// the plain layout: measured there, the swizzle cut the conflict stalls 5x
// but cost 15 % more VALU and 25 % more LDS instructions (each element needs
// its own address, where the plain layout reads a row at immediate offsets
// from one), and those kernels ran 2-9 % slower.  Where it pays is 3 x 3
// blocks with float I/O at chunk 8 (8-way): 1-2 % faster steps on every
// such workload measured (the 10,000-step batch, the 1,460-step AR(1)
// batch, the long-T batch).  Other block sizes keep the plain layout: the
// order-1 batch (2 x 2, chunk 8) ran 3-4 % slower with it and the order-3
// ragged batch (4 x 4, whose kernels fill the register file at one wave
// per SIMD) 3 % slower.
constexpr int swz_shift(int A, int esz) {   // -1: plain layout
  return A % 8 != 0 ? -1 : esz == 8 ? (A == 24 || A == 64 ? 1 : 0) : (A == 24 || A == 40 || A == 48 ? 1 : 0);
}
template <int K, int L, class TIO>
struct LdsSwz {
  static constexpr int EB = 256 / static_cast<int>(sizeof(TIO));   // elements per 256-byte block
  static constexpr int LOG_EB = sizeof(TIO) == 8 ? 5 : 6;
  template <int W>
  static constexpr bool on() { return K == 3 && swz_shift(W * L, static_cast<int>(sizeof(TIO))) >= 0; }
  template <int W>
  __host__ __device__ __forceinline__ static int64_t at(int64_t e) {
    if constexpr (!on<W>()) {
      return e;
    } else {
      constexpr int SH = LOG_EB + swz_shift(W * L, static_cast<int>(sizeof(TIO)));
      const int x = static_cast<int>(e);
      return x ^ ((x >> SH) & (EB - 1));
    }
  }
};

// Byte layout of one wave's LDS slice: ROWS steps of each array read, every
// array 16-byte aligned, swizzled arrays a whole number of 256-byte blocks
// (their staging writes whole blocks).  A tile spans at most CH chunks (one per lane, 64
// unless TileChunks below says fewer) of L steps plus the step before and
// the step after.  Rows of c hold QE K values, rows of b and of the
// governing weights QE.
template <int K, int L, class TIO, int RHS, int OUT, class F = FormScalar, int CH = WAVE>
struct Stage {
  using RD = Reads<RHS, OUT>;
  static constexpr size_t al(size_t b, bool swz) { return swz ? (b + 255) / 256 * 256 : (b + 15) / 16 * 16; }
  using SW = LdsSwz<K, L, TIO>;
  struct Layout {
    size_t C, S, D, G, V, WG, WS, BYTES;
  };
  // slot offsets of a slice of `rows` rows
  static constexpr Layout layout(int rows) {
    const size_t row_k = al(sizeof(TIO) * K * rows, SW::template on<K>());
    const size_t row_1 = al(sizeof(TIO) * rows, SW::template on<1>());
    const size_t row_c = al(sizeof(TIO) * F::QE * K * rows, SW::template on<F::QE * K>());
    const size_t row_d = al(sizeof(TIO) * F::QE * rows, SW::template on<F::QE>());
    Layout o{};
    o.C = 0;
    o.S = o.C + row_c;
    o.D = o.S + row_1;
    o.G = o.D + (RD::d ? row_d : 0);
    o.V = o.G + (RD::g ? row_k : 0);
    o.WG = o.V + (RD::v ? row_k : 0);
    o.WS = o.WG + (F::WROW ? row_d : 0);
    o.BYTES = o.WS + (F::WROW ? row_1 : 0);
    return o;
  }
  static constexpr int ROWS = CH * L + 2;
  static constexpr size_t C = layout(ROWS).C;
  static constexpr size_t S = layout(ROWS).S;
  static constexpr size_t D = layout(ROWS).D;
  static constexpr size_t G = layout(ROWS).G;
  static constexpr size_t V = layout(ROWS).V;
  static constexpr size_t Y = G;   // dl/dy is read by the forward sweep only
  static constexpr size_t WG = layout(ROWS).WG;
  static constexpr size_t WS = layout(ROWS).WS;
  static constexpr size_t BYTES = layout(ROWS).BYTES;
};

// Chunks per tile of a level-0 kernel (one per lane, 64, unless LDS would
// hold the kernel below the occupancy its registers allow).  For 3 x 3
// blocks: the gradient back-substitution and the fused back-substitution +
// reduce hold WPS = 2 waves per SIMD by their registers (8 per CU); the
// back-substitution of a refinement solve and the reduce of dl/dy hold 3
// at chunk 4 in FP64 (12 per CU) and 2 at chunk 8 with float I/O.  With
// one chunk per lane the slices of the gradient pass and the adjoint fused
// pass exceed an eighth of the CU's 160 KB of LDS, and those of the other
// two a twelfth, so LDS admitted 7, 7, 9 and 11 waves.  Each of them takes
// the largest tile whose slice fits 1/(4 WPS) of the LDS (57, 63, 52 and
// 60 chunks at chunk 4 in FP64; lanes beyond it idle), or 64 if that would
// be under 48; measured 3 %, 7 %, 4 % and 3 % faster.  Every other kernel
// takes 64.
constexpr size_t LDS_PER_CU = 160 * 1024;
template <int K, int L, class TIO, int RHS, int OUT, class F, int WPS>
struct TileChunks {
  static constexpr size_t BUDGET = WPS > 0 ? LDS_PER_CU / (4 * WPS) : LDS_PER_CU;
  static constexpr int fit() {
    int ch = WAVE;
    while (ch > 3 * WAVE / 4 && Stage<K, L, TIO, RHS, OUT, F>::layout(ch * L + 2).BYTES > BUDGET) --ch;
    return Stage<K, L, TIO, RHS, OUT, F>::layout(ch * L + 2).BYTES > BUDGET ? WAVE : ch;
  }
  static constexpr int value = WPS > 0 && K == 3 ? fit() : WAVE;
};
template <int L, class TIO>
struct WavesRefine {   // waves per SIMD of the refinement back-substitution and the dl/dy reduce
  static constexpr int value = L == 4 && sizeof(TIO) == 8 ? 3 : 2;
};
template <int K, int L, class TIO, int RHS, int OUT, class F>
using B0Chunks = TileChunks<K, L, TIO, RHS, OUT, F,
                            OUT == OUT_GRAD ? 2 : (RHS == RHS_RESID || RHS == RHS_GRESID ? WavesRefine<L, TIO>::value : 0)>;
template <int K, int L, class TIO, int RHS, class F>
using R0Chunks = TileChunks<K, L, TIO, RHS, OUT_STORE, F, RHS == RHS_G ? WavesRefine<L, TIO>::value : 0>;
template <int K, int L, class TIO, int ROUT, class F>
using BRChunks = TileChunks<K, L, TIO, ROUT, OUT_STORE, F, 2>;

// Wave-cooperative copy of rows [lo, hi) of an array with W elements per row
// into LDS in the swizzled placement of LdsSwz<K, L, T> (4 bytes per lane per
// load; the loads write LDS directly and are all in flight together).  Load
// b / 64 writes LDS dwords [b, b + 64) and its lanes fetch the input dwords
// those positions hold, all within the same 256 bytes.  Every lane of the
// wave calls this with the same arguments; the caller waits for completion
// before reading.
template <class T, int K, int W, int L>
__device__ __forceinline__ void stage_rows(const void* src, int64_t lo, int64_t hi, unsigned char* dst, int lane) {
  constexpr int DPE = static_cast<int>(sizeof(T)) / 4;   // dwords per element
  const int ndw = static_cast<int>((hi - lo) * W * static_cast<int64_t>(sizeof(T)) / 4);
  const uint32_t* gsrc = reinterpret_cast<const uint32_t*>(static_cast<const T*>(src) + lo * W);
  uint32_t* l = reinterpret_cast<uint32_t*>(dst);
  for (int b = 0; b < ndw; b += WAVE) {
    const int e = static_cast<int>(LdsSwz<K, L, T>::template at<W>(b / DPE + lane / DPE));
    const int sdw = e * DPE + lane % DPE;
    if (sdw < ndw) __builtin_amdgcn_global_load_lds(gsrc + sdw, l + b, 4, 0, 0);
  }
}

// Per-row weights: the governing weights (QE per row) and the smoothness
// weight of each step.
template <int K, int L, class TIO, int RHS, int OUT, class F, int CH = WAVE>
__device__ __forceinline__ void stage_weights(const Level0Args& a, int64_t lo, int64_t hi, unsigned char* sl,
                                              int lane) {
  using ST = Stage<K, L, TIO, RHS, OUT, F, CH>;
  if constexpr (F::WROW) {
    stage_rows<TIO, K, F::QE, L>(a.wg, lo, hi, sl + ST::WG, lane);
    stage_rows<TIO, K, 1, L>(a.ws, lo, hi, sl + ST::WS, lane);
  }
}

// Copies rows [lo, hi) of every array the variant reads into the slice.
template <int K, int L, class TIO, int RHS, int OUT, class F, int CH = WAVE>
__device__ __forceinline__ void stage_tile(const Level0Args& a, int64_t lo, int64_t hi, unsigned char* sl,
                                           int lane) {
  using ST = Stage<K, L, TIO, RHS, OUT, F, CH>;
  using RD = Reads<RHS, OUT>;
  stage_rows<TIO, K, F::QE * K, L>(a.c, lo, hi, sl + ST::C, lane);
  stage_rows<TIO, K, 1, L>(a.s, lo, hi, sl + ST::S, lane);
  if (RD::d) stage_rows<TIO, K, F::QE, L>(a.d, lo, hi, sl + ST::D, lane);
  if (RD::g) stage_rows<TIO, K, K, L>(a.g, lo, hi, sl + ST::G, lane);
  if (RD::v) stage_rows<TIO, K, K, L>(a.v, lo, hi, sl + ST::V, lane);
  stage_weights<K, L, TIO, RHS, OUT, F, CH>(a, lo, hi, sl, lane);
}

// Rows of the tile of chunks [g0, g1): from the step before the first chunk
// to the step after the last one, clipped to the arrays.  r0, r1: the rows
// the chunks own (first row of g0, first row of g1).
__device__ __forceinline__ void tile_rows(const LevelDev& l0, int64_t g0, int64_t g1, int64_t S, int64_t& lo,
                                          int64_t& hi, int64_t& r0, int64_t& r1) {
  r0 = l0.chunk_step[g0];
  r1 = l0.chunk_step[g1];
  lo = r0 > 0 ? r0 - 1 : 0;
  hi = r1 + 1 < S ? r1 + 1 : S;
}

// Wave-cooperative copy of rows [r0, r1) (W elements each) from a slot of
// the wave's LDS slice (slice row = global row - lo; rows LS elements apart
// in the slot, 0: W; swizzled as LdsSwz<K, L, T> places them) to global
// memory: every store instruction writes 64 consecutive elements.
template <class T, int K, int W, int L, int LS = 0>
__device__ __forceinline__ void unstage_rows(void* dst, int64_t r0, int64_t r1, int64_t lo,
                                             const unsigned char* slot, int lane) {
  constexpr int RW = LS ? LS : W;
  T* g = static_cast<T*>(dst) + r0 * W;
  const int n = static_cast<int>((r1 - r0) * W);
  const T* l = reinterpret_cast<const T*>(slot);
  const int base = static_cast<int>((r0 - lo) * RW);
  for (int k = lane; k < n; k += WAVE) {
    const int e = base + (RW == W ? k : (k / W) * RW + k % W);
    g[k] = l[LdsSwz<K, L, T>::template at<RW>(e)];
  }
}

template <int K, class TIO>
__device__ __forceinline__ Inst<K> load_inst(const Level0Args& a, int64_t i) {
  const TIO* w = static_cast<const TIO*>(a.w);   // null with per-row weights
  Inst<K> p;
  p.wg = w ? static_cast<double>(w[3 * i]) : 0.0;
  p.wi = w ? static_cast<double>(w[3 * i + 1]) : 0.0;
  p.ws = w ? static_cast<double>(w[3 * i + 2]) : 0.0;
  p.n_init = a.n_init;
  p.t_init = a.t_init;
  return p;
}

// Source reading the wave's LDS slice: node i of the instance at global
// row off is slice row off - lo + i.
template <int K, int L, class TIO, int RHS, int OUT, class F, int LRHS = RHS, int CH = WAVE>
__device__ __forceinline__ Src0<K, TIO, RHS, F, LdsSwz<K, L, TIO>> make_src0_lds(const Level0Args& a, int64_t i, int64_t off,
                                                              int64_t n, int64_t lo, unsigned char* sl) {
  using ST = Stage<K, L, TIO, LRHS, OUT, F, CH>;   // slice layout of the variant LRHS
  Src0<K, TIO, RHS, F, LdsSwz<K, L, TIO>> S;
  S.c = reinterpret_cast<const TIO*>(sl + ST::C);
  S.s = reinterpret_cast<const TIO*>(sl + ST::S);
  S.d = reinterpret_cast<const TIO*>(sl + ST::D);
  S.g = reinterpret_cast<const TIO*>(sl + ST::G);
  S.v = reinterpret_cast<const TIO*>(sl + ST::V);
  S.wg = reinterpret_cast<const TIO*>(sl + ST::WG);
  S.wsm = reinterpret_cast<const TIO*>(sl + ST::WS);
  S.wi = static_cast<const TIO*>(a.wi);
  S.u = static_cast<const TIO*>(a.u0);
  S.uo = static_cast<int>(i) * a.t_init * F::V * a.n_init;
  S.o = off - lo;
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
// record of this lane's left separator, node m (instance-relative) of the
// next level, in that level's interleaved layout (chunk_off0 = the
// instance's first chunk there).  All 64 lanes must call this.
template <int K>
__device__ __forceinline__ void exchange_and_write(const Reduced<K>& red, bool writer, const LevelDev& nx,
                                                   int64_t chunk_off0, int64_t m, int L1, bool write_rec) {
  constexpr int Q = Dim<K>::Q;
  double rA[Q], rf[K];
#pragma unroll
  for (int e = 0; e < Q; ++e) rA[e] = __shfl_up(red.rA[e], 1, WAVE);
#pragma unroll
  for (int e = 0; e < K; ++e) rf[e] = __shfl_up(red.rf[e], 1, WAVE);
  if (writer) combine_separator_t<K>(rA, rf, red, nx.rec, nx.rhs, chunk_off0 + m / L1, m % L1, L1, write_rec);
}

// ------------------------------------------------------------ level 0 reduce
template <int K, int L, class TIO, int RHS, bool WREC, class F>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_reduce0(LevelDev l0, LevelDev l1, Level0Args a) {
  constexpr int CH = R0Chunks<K, L, TIO, RHS, F>::value;   // chunks per tile
  using ST = Stage<K, L, TIO, RHS, OUT_STORE, F, CH>;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* sl = smem + (threadIdx.x / WAVE) * ST::BYTES;
  const int lane = lane_id();
  const int64_t G = l0.chunks;
  const int64_t tiles = G > 1 ? (G - 2) / (CH - 1) + 1 : 1;
  for (int64_t tw = first_tile(a); tw < tiles; tw = next_tile(a, tw)) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const int64_t g0 = tile * (CH - 1);
    const int64_t g1 = g0 + CH < G ? g0 + CH : G;
    // chunk metadata first: its loads then return ahead of the staged tile
    const int64_t g = g0 + lane;
    const bool valid = lane < CH && g < G;
    const int64_t gg = valid ? g : G - 1;
    const int64_t inst = l0.chunk_inst[gg];
    int64_t lo, hi, r0, r1;
    tile_rows(l0, g0, g1, l0.nodes, lo, hi, r0, r1);
    const int64_t j0 = l0.chunk_off[inst];
    const int64_t off = l0.node_off[inst];
    const int64_t n = l0.node_off[inst + 1] - off;
    const int64_t c1 = l1.chunk_off[inst];
    const auto src = make_src0_lds<K, L, TIO, RHS, OUT_STORE, F, RHS, CH>(a, inst, off, n, lo, sl);
    stage_tile<K, L, TIO, RHS, OUT_STORE, F, CH>(a, lo, hi, sl, lane);
    const int64_t j = gg - j0;
    const ChunkGeom geo = chunk_geom(j, n, L);
    Reduced<K> red;
#pragma unroll
    for (int e = 0; e < Dim<K>::Q; ++e) { red.rA[e] = 0.0; red.lA[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < K; ++e) { red.rf[e] = 0.0; red.lf[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < Dim<K>::KK; ++e) red.lB[e] = 0.0;
    red.fail = 0;
    __builtin_amdgcn_s_waitcnt(0);
    if (valid && (geo.has_left || geo.has_right)) {
      reduce_chunk<K, L>(src, geo.a, geo.b, geo.has_left, geo.has_right, red);
      if (red.fail) report_fail(a, inst, 0, geo.a + red.fail - 1);
    }
    const bool writer = valid && lane > 0 && geo.has_left;
    exchange_and_write<K>(red, writer, l1, c1, j - 1, a.L1, WREC);
  }
}

// -------------------------------------------------------- level >= 1 reduce
template <int K, int L, bool WREC>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_reduceN(LevelDev lv, LevelDev nx, Level0Args a, int level) {
  const int lane = lane_id();
  const int64_t G = lv.chunks;
  const int64_t tiles = G > 1 ? (G - 2) / (WAVE - 1) + 1 : 1;
  for (int64_t tw = first_tile(a); tw < tiles; tw = next_tile(a, tw)) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
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
    const int64_t c1 = nx.chunk_off[inst];
    if (valid && (geo.has_left || geo.has_right)) {
      SrcT<K> S;
      S.rec = lv.rec;
      S.rhs = lv.rhs;
      S.C = gg;
      S.a = geo.a;
      S.L = L;
      reduce_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, red);
      if (red.fail) report_fail(a, inst, level, geo.a + red.fail - 1);
    }
    const bool writer = valid && lane > 0 && geo.has_left;
    exchange_and_write<K>(red, writer, nx, c1, j - 1, L, WREC);
  }
}

// --------------------------------------------------- level >= 1 back-subst.
template <int K, int L>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_backsubN(LevelDev lv, LevelDev nx, bool has_next, Level0Args a,
                                                 int level) {
  const int lane = lane_id();
  const int64_t G = lv.chunks;
  const int64_t tiles = (G + WAVE - 1) / WAVE;
  for (int64_t tw = first_tile(a); tw < tiles; tw = next_tile(a, tw)) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const int64_t g = tile * WAVE + lane;
    if (g < G) {   // (no early continue: the tile schedule is claimed by the whole wave)
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
    SrcT<K> S;
    S.rec = lv.rec;
    S.rhs = lv.rhs;
    S.C = g;
    S.a = geo.a;
    S.L = L;
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
}

// ------------------------------------------------------- level 0 back-subst.
// Waves per SIMD the compiler must fit the kernel into.  The gradient pass at
// block size 3 and chunk 8 needs 256 VGPRs plus ~56 AGPRs (one wave per
// SIMD); held to two waves it spills a little and measured 9 % faster.
template <int K, int L, int OUT>
struct Backsub0Waves {
  static constexpr int value = (K == 3 && L == 8 && OUT == OUT_GRAD) ? 2 : SMNN_MIN_WAVES;
};

template <int K, int L, class TIO, int RHS, int OUT, class F>
__global__ void __launch_bounds__(256, (Backsub0Waves<K, L, OUT>::value)) k_backsub0(LevelDev l0, LevelDev l1,
                                                                                     bool has_next, Level0Args a) {
  constexpr bool ADD = (RHS == RHS_RESID || RHS == RHS_GRESID);
  constexpr int QE = F::QE, NI = F::V;   // governing equations per point; variables per initial point
  constexpr int CH = B0Chunks<K, L, TIO, RHS, OUT, F>::value;   // chunks per tile
  using ST = Stage<K, L, TIO, RHS, OUT, F, CH>;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* sl = smem + (threadIdx.x / WAVE) * ST::BYTES;
  const int lane = lane_id();
  const int64_t G = l0.chunks;
  const int64_t tiles = (G + CH - 1) / CH;
  for (int64_t tw = first_tile(a); tw < tiles; tw = next_tile(a, tw)) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const int64_t g0 = tile * CH;
    const int64_t g1 = g0 + CH < G ? g0 + CH : G;
    // chunk metadata first: its loads then return ahead of the staged tile
    const int64_t g = g0 + lane;
    const bool valid = lane < CH && g < G;
    const int64_t gg = valid ? g : G - 1;
    const int64_t inst = l0.chunk_inst[gg];
    int64_t lo, hi, r0, r1;
    tile_rows(l0, g0, g1, l0.nodes, lo, hi, r0, r1);
    const int64_t j0 = l0.chunk_off[inst];
    const int64_t off = l0.node_off[inst];
    const int64_t n = l0.node_off[inst + 1] - off;
    const int64_t up0 = (has_next ? l1.node_off : l0.node_off)[inst];   // unconditional load
    const auto src = make_src0_lds<K, L, TIO, RHS, OUT, F, RHS, CH>(a, inst, off, n, lo, sl);
    stage_tile<K, L, TIO, RHS, OUT, F, CH>(a, lo, hi, sl, lane);
    const int64_t j = gg - j0;
    const int64_t up = has_next ? up0 : 0;
    const ChunkGeom geo = chunk_geom(j, n, L);
    double xl[K], xr[K], xs[L][K];
#pragma unroll
    for (int e = 0; e < K; ++e) {
      xl[e] = valid && geo.has_left ? l1.x[(up + j - 1) * K + e] : 0.0;
      xr[e] = valid && geo.has_right ? l1.x[(up + j) * K + e] : 0.0;
    }
    const TIO* vs = reinterpret_cast<const TIO*>(sl + ST::V);
    // ds rows of the tile: the step before each chunk (when it is in the
    // same instance) through the chunk's last interior step, and an
    // instance's last step in its last chunk
    const int last = static_cast<int>(g1 - g0) - 1;
    const bool first_starts = __shfl(static_cast<int>(j == 0), 0, WAVE) != 0;
    const bool last_ends = __shfl(static_cast<int>(!geo.has_right), last, WAVE) != 0;
    __builtin_amdgcn_s_waitcnt(0);
    // Outputs go into the slice in place of inputs no lane reads afterwards
    // (out / dc over c, dd over d, ds over s, and the per-row weight
    // gradients over their weights; a lane reads another lane's rows only
    // for s, the smoothness weight, v and y of its left separator and v
    // after its right one, before it writes anything), then out to HBM in
    // whole rows.
    if (OUT == OUT_STORE && valid) {
      // the solution goes over c, row for row (c rows hold QE K values)
      StoreSink<TIO, ADD, QE * K, LdsSwz<K, L, TIO>> sink{reinterpret_cast<TIO*>(sl + ST::C), vs, off - lo, off - lo};
      if (geo.has_right) sink.template node<K>(geo.b + 1, xr);   // owned right separator
      const int fail = backsub_chunk<K, L>(src, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, xs, sink);
      if (fail) report_fail(a, inst, 0, geo.a + fail - 1);
    }
    if (OUT == OUT_GRAD) {
      // forward sweep; then y (read only by the gradient formation) is staged
      // over dl/dy, which only the forward sweep reads; then the backward
      // sweep forms the gradients
      double Ls[L][Dim<K>::Q];
      int fail = 0;
      if (valid) fail = backsub_forward<K, L>(src, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, Ls, xs);
      __builtin_amdgcn_wave_barrier();
      stage_rows<TIO, K, K, L>(a.y, lo, hi, sl + ST::Y, lane);
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        GradSink<K, TIO, ADD, F, LdsSwz<K, L, TIO>> sink;
        sink.c = src.c; sink.d = src.d; sink.s = src.s;
        sink.wg = src.wg; sink.wsm = src.wsm; sink.wi = src.wi;
        sink.y = reinterpret_cast<const TIO*>(sl + ST::Y);
        sink.v = vs;
        sink.o = off - lo;
        sink.dc = reinterpret_cast<TIO*>(sl + ST::C);
        sink.dd = reinterpret_cast<TIO*>(sl + ST::D);
        sink.ds = reinterpret_cast<TIO*>(sl + ST::S);
        sink.oo = off - lo;
        sink.du0 = static_cast<TIO*>(a.du0) + inst * a.t_init * NI * a.n_init;
        if constexpr (F::WROW) {
          sink.dwg = reinterpret_cast<TIO*>(sl + ST::WG);
          sink.dws = reinterpret_cast<TIO*>(sl + ST::WS);
          sink.dwi = static_cast<TIO*>(a.dwi) + inst * a.t_init * NI * a.n_init;
        }
        sink.u = src.u;
        sink.uo = src.uo;
        sink.p = src.p;
        if (geo.has_right) sink.start(geo.b + 1, xr);
        backsub_backward<K, L>(src, geo.a, geo.b, Ls, xs, sink);
        if (geo.has_left) sink.left(geo.a - 1, xl);
        if (!geo.has_right) {
          sink.last_point(n);   // the last point's step slot enters no row
          sink.zero_past_end(n);
        }
        if constexpr (!F::WROW) {
#pragma unroll
          for (int e = 0; e < 3; ++e) a.dw_part[g * 3 + e] = sink.dw[e];
        }
        if (fail) report_fail(a, inst, 0, geo.a + fail - 1);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (OUT == OUT_STORE) {
      unstage_rows<TIO, K, K, L, QE * K>(a.out, r0, r1, lo, sl + ST::C, lane);
    } else {
      const int64_t s0 = r0 - (first_starts ? 0 : 1), s1 = r1 - (last_ends ? 0 : 1);
      unstage_rows<TIO, K, QE * K, L>(a.dc, r0, r1, lo, sl + ST::C, lane);
      unstage_rows<TIO, K, QE, L>(a.dd, r0, r1, lo, sl + ST::D, lane);
      unstage_rows<TIO, K, 1, L>(a.ds, s0, s1, lo, sl + ST::S, lane);
      if constexpr (F::WROW) {
        unstage_rows<TIO, K, QE, L>(a.dwg, r0, r1, lo, sl + ST::WG, lane);
        unstage_rows<TIO, K, 1, L>(a.dws, s0, s1, lo, sl + ST::WS, lane);
      }
    }
  }
}

// ------------------------------- level 0: back-substitution + next reduce
// The level-0 back-substitution of one solve fused with the level-0 reduce
// of the refinement solve that follows it (RIN = beta, ROUT = residual; or
// RIN = dl/dy, ROUT = adjoint residual).  The new iterate stays in the LDS
// slice, where the residual reduce reads it, so that reduce re-reads no
// input from HBM.  A tile owns CH - 2 chunks (62 with one chunk per lane);
// lane 0 back-substitutes and reduces the previous tile's last owned chunk
// (each separator is combined from the chunks on both of its sides) and
// lane CH - 1 back-substitutes the next tile's first chunk (the residual at
// a chunk's right separator needs the iterate one step past it).
template <int K, int L, class TIO, int RIN, int ROUT, class F>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_backsub_reduce0(LevelDev l0, LevelDev l1, Level0Args a) {
  constexpr int CH = BRChunks<K, L, TIO, ROUT, F>::value;   // chunks per tile
  using ST = Stage<K, L, TIO, ROUT, OUT_STORE, F, CH>;   // c, h, (b | dl/dy) staged; the iterate in the v slot
  constexpr int OWN = CH - 2;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* sl = smem + (threadIdx.x / WAVE) * ST::BYTES;
  TIO* it = reinterpret_cast<TIO*>(sl + ST::V);
  const int lane = lane_id();
  const int64_t G = l0.chunks;
  const int64_t tiles = (G + OWN - 1) / OWN;
  for (int64_t tw = first_tile(a); tw < tiles; tw = next_tile(a, tw)) {
    const int64_t tile = a.rev ? tiles - 1 - tw : tw;
    const int64_t t0 = tile * OWN;                   // owned chunks [t0, t1)
    const int64_t t1 = t0 + OWN < G ? t0 + OWN : G;
    const int64_t gb = t0 > 0 ? t0 - 1 : 0;          // tile chunks [gb, ge)
    const int64_t ge = t1 < G ? t1 + 1 : G;
    const int64_t g = t0 - 1 + lane;
    const bool valid = g >= gb && g < ge;
    const bool owned = g >= t0 && g < t1;
    const int64_t gg = valid ? g : (g < gb ? gb : ge - 1);
    const int64_t inst = l0.chunk_inst[gg];
    int64_t lo, hi, r0, r1;
    tile_rows(l0, gb, ge, l0.nodes, lo, hi, r0, r1);
    const int64_t o0 = l0.chunk_step[t0], o1 = l0.chunk_step[t1];   // owned rows
    const int64_t j0 = l0.chunk_off[inst];
    const int64_t off = l0.node_off[inst];
    const int64_t n = l0.node_off[inst + 1] - off;
    const int64_t up0 = (l1.node_off ? l1.node_off : l0.node_off)[inst];
    const int64_t c1 = (l1.chunk_off ? l1.chunk_off : l0.chunk_off)[inst];
    const auto src = make_src0_lds<K, L, TIO, RIN, OUT_STORE, F, ROUT, CH>(a, inst, off, n, lo, sl);
    stage_rows<TIO, K, F::QE * K, L>(a.c, lo, hi, sl + ST::C, lane);
    stage_rows<TIO, K, 1, L>(a.s, lo, hi, sl + ST::S, lane);
    if (RIN == RHS_BETA) stage_rows<TIO, K, F::QE, L>(a.d, lo, hi, sl + ST::D, lane);
    if (RIN == RHS_G) stage_rows<TIO, K, K, L>(a.g, lo, hi, sl + ST::G, lane);
    stage_weights<K, L, TIO, ROUT, OUT_STORE, F, CH>(a, lo, hi, sl, lane);
    const int64_t j = gg - j0;
    const ChunkGeom geo = chunk_geom(j, n, L);
    double xl[K], xr[K], xs[L][K];
#pragma unroll
    for (int e = 0; e < K; ++e) {
      xl[e] = valid && geo.has_left ? l1.x[(up0 + j - 1) * K + e] : 0.0;
      xr[e] = valid && geo.has_right ? l1.x[(up0 + j) * K + e] : 0.0;
    }
    __builtin_amdgcn_s_waitcnt(0);
    // 1. back-substitution: the iterate of every tile chunk into the slice
    //    (lane 0 also stores its left separator's value, the step before the
    //    tile, which its residual reads).  Where registers allow (KEEP), the
    //    chunk's factor Ls is kept for the reduce below, which eliminates the
    //    same nodes of the same matrix; otherwise the reduce refactors.
    constexpr bool KEEP = K <= 3 && K * L <= 16;   // still 2 waves per SIMD
    double Ls[KEEP ? L : 1][Dim<K>::Q];
    if (valid) {
      StoreSink<TIO, false, 0, LdsSwz<K, L, TIO>> sink{it, nullptr, src.o, src.o};
      if (geo.has_right) sink.template node<K>(geo.b + 1, xr);
      if (lane == 0 && geo.has_left) sink.template node<K>(geo.a - 1, xl);
      int fail;
      if constexpr (KEEP) {
        fail = backsub_forward<K, L>(src, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, Ls, xs);
        backsub_backward<K, L>(src, geo.a, geo.b, Ls, xs, sink);
      } else {
        fail = backsub_chunk<K, L>(src, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, xs, sink);
      }
      if (fail) report_fail(a, inst, 0, geo.a + fail - 1);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // 2. reduce with the residual of that iterate as right-hand side
    Src0<K, TIO, ROUT, F, LdsSwz<K, L, TIO>> rs;
    rs.c = src.c; rs.d = src.d; rs.s = src.s; rs.g = src.g; rs.v = it;
    rs.wg = src.wg; rs.wsm = src.wsm; rs.wi = src.wi;
    rs.n = src.n; rs.o = src.o; rs.p = src.p; rs.u = src.u; rs.uo = src.uo;
    Reduced<K> red;
#pragma unroll
    for (int e = 0; e < Dim<K>::Q; ++e) { red.rA[e] = 0.0; red.lA[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < K; ++e) { red.rf[e] = 0.0; red.lf[e] = 0.0; }
#pragma unroll
    for (int e = 0; e < Dim<K>::KK; ++e) red.lB[e] = 0.0;
    red.fail = 0;
    if (valid && g < t1 && (geo.has_left || geo.has_right)) {
      if constexpr (KEEP) {
        reduce_chunk_rhs<K, L>(rs, geo.a, geo.b, geo.has_left, geo.has_right, Ls, red);   // pivots reported above
      } else {
        reduce_chunk<K, L>(rs, geo.a, geo.b, geo.has_left, geo.has_right, red);
        if (red.fail) report_fail(a, inst, 0, geo.a + red.fail - 1);
      }
    }
    exchange_and_write<K>(red, owned && geo.has_left, l1, c1, j - 1, a.L1, false);
    // 3. the owned chunks' iterate out to HBM in whole rows
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    unstage_rows<TIO, K, K, L>(a.out, o0, o1, lo, sl + ST::V, lane);
  }
}

// ------------------------------ levels >= lt: SW lanes per instance
// Used when every instance has at most SW chunks at level lt.  A group of SW
// lanes takes one instance (a wave takes 64 / SW of them): each lane reduces
// one level-lt chunk from HBM, the separator systems of the levels above (at
// most 63, 15, 3 nodes for SW = 64 and L = 4) are kept in the group's part of
// the LDS in the natural layout and reduced there while they have more than
// one chunk, the group's first lane solves the top one, and the
// back-substitutions come down to level lt, whose solution goes to HBM.  One
// launch replaces the reduce and back-substitution launches of levels lt and
// above; the upper levels' records are rebuilt in LDS by every solve rather
// than stored.  SW = 64 (one instance per wave) for blocks of up to 3
// unknowns; 16 for larger blocks, whose kernel holds a whole SIMD: with one
// instance per wave a batch of a few thousand instances would take several
// rounds of waves.
template <int L, int SW = WAVE>
struct TopCaps {   // separator nodes one instance can have at LDS levels 1..3
  static constexpr int c1 = SW - 1;
  static constexpr int c2 = c1 > L ? (c1 + L - 1) / L - 1 : 0;
  static constexpr int c3 = c2 > L ? (c2 + L - 1) / L - 1 : 0;
  static_assert(c3 <= L, "the top is reached within three LDS levels");
  static constexpr int nodes = c1 + c2 + c3;
};

template <int K>
struct TopLevel {
  double* rec;   // [cap][Q + KK]
  double* rhs;   // [cap][K]
  double* x;     // [cap][K]
};

template <int K, int L, int SW>
__device__ __forceinline__ TopLevel<K> top_level(double* base, int d) {
  using C = TopCaps<L, SW>;
  constexpr int REC = Dim<K>::Q + Dim<K>::KK;
  const int off = d == 1 ? 0 : (d == 2 ? C::c1 : C::c1 + C::c2);
  const int cap = d == 1 ? C::c1 : (d == 2 ? C::c2 : C::c3);
  double* p = base + off * (REC + 2 * K);
  return {p, p + cap * REC, p + cap * (REC + K)};
}

// Nodes of LDS level d of an instance with G chunks at level lt.
template <int L>
__device__ __forceinline__ int64_t top_nodes(int G, int d) {
  int64_t n = G - 1;
  for (int k = 1; k < d; ++k) n = (n + L - 1) / L - 1;
  return n;
}

// Separator m of the level just reduced = node m of LDS level `to`: lane
// m + 1 of the group combines the right pieces of lane m with its own left
// pieces.  Every lane of the group must call this (a group's first lane
// reads the lane before it, in another group or none, and does not write).
template <int K>
__device__ __forceinline__ void top_combine(const Reduced<K>& red, bool writer, const TopLevel<K>& to, int m) {
  constexpr int Q = Dim<K>::Q, KK = Dim<K>::KK;
  double rA[Q], rf[K];
#pragma unroll
  for (int e = 0; e < Q; ++e) rA[e] = __shfl_up(red.rA[e], 1, WAVE);
#pragma unroll
  for (int e = 0; e < K; ++e) rf[e] = __shfl_up(red.rf[e], 1, WAVE);
  if (writer) combine_separator<K>(rA, rf, red, to.rec + m * (Q + KK), to.rhs + m * K, true);
}

template <int K>
__device__ __forceinline__ void zero_reduced(Reduced<K>& red) {
#pragma unroll
  for (int e = 0; e < Dim<K>::Q; ++e) { red.rA[e] = 0.0; red.lA[e] = 0.0; }
#pragma unroll
  for (int e = 0; e < K; ++e) { red.rf[e] = 0.0; red.lf[e] = 0.0; }
#pragma unroll
  for (int e = 0; e < Dim<K>::KK; ++e) red.lB[e] = 0.0;
  red.fail = 0;
}

template <int K, int L, int SW>
__global__ void __launch_bounds__(256, SMNN_MIN_WAVES) k_top(LevelDev lv, Level0Args a, int level) {
  constexpr int PER = Dim<K>::Q + Dim<K>::KK + 2 * K;
  constexpr int IPW = WAVE / SW;   // instances per wave
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id() % SW;   // lane within the instance's group
  const int sub = lane_id() / SW;    // the group within the wave
  double* base = reinterpret_cast<double*>(smem) + ((threadIdx.x / WAVE) * IPW + sub) * (TopCaps<L, SW>::nodes * PER);
  const int64_t groups = (a.N + IPW - 1) / IPW;
  for (int64_t tw = first_tile(a); tw < groups; tw = next_tile(a, tw)) {
    // ragged batches: instances longest first (the plan's order), so the
    // longest chains start first; equal lengths: alternate the direction
    const int64_t slot = tw * IPW + sub;
    const bool live = slot < a.N;
    const int64_t si = live ? slot : a.N - 1;
    const int64_t inst = a.order ? a.order[si] : (a.rev ? a.N - 1 - si : si);
    const int64_t off = lv.node_off[inst];
    const int64_t n = lv.node_off[inst + 1] - off;
    const int64_t c0 = lv.chunk_off[inst];
    const int G = static_cast<int>(lv.chunk_off[inst + 1] - c0);   // <= SW (checked on the host)
    if (live && n > 0) {   // (no early continue: the groups of a wave share its loop)
    double xl[K], xr[K], xs[L][K];
    if (G > 1) {
      // 1. level lt: lane j reduces chunk j; separators into LDS level 1
      {
        const ChunkGeom geo = chunk_geom(lane, n, L);
        Reduced<K> red;
        zero_reduced<K>(red);
        if (lane < G) {
          SrcT<K> S;
          S.rec = lv.rec;
          S.rhs = lv.rhs;
          S.C = c0 + lane;
          S.a = geo.a;
          S.L = L;
          reduce_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, red);
          if (red.fail) report_fail(a, inst, level, geo.a + red.fail - 1);
        }
        top_combine<K>(red, lane > 0 && lane < G, top_level<K, L, SW>(base, 1), lane - 1);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      // 2. reduce the LDS levels until one is a single chunk
      int d = 1;
      int64_t nl = G - 1;
      while (nl > L) {
        const int Gd = static_cast<int>((nl + L - 1) / L);
        const TopLevel<K> cur = top_level<K, L, SW>(base, d);
        const ChunkGeom geo = chunk_geom(lane, nl, L);
        Reduced<K> red;
        zero_reduced<K>(red);
        if (lane < Gd) {
          SrcN<K> S{cur.rec, cur.rhs};
          reduce_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, red);
          if (red.fail) report_fail(a, inst, level + d, geo.a + red.fail - 1);
        }
        top_combine<K>(red, lane > 0 && lane < Gd, top_level<K, L, SW>(base, d + 1), lane - 1);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        nl = Gd - 1;
        ++d;
      }
      // 3. the top level: a single chunk, solved by lane 0
      {
        const TopLevel<K> top = top_level<K, L, SW>(base, d);
        if (lane == 0) {
#pragma unroll
          for (int e = 0; e < K; ++e) { xl[e] = 0.0; xr[e] = 0.0; }
          SrcN<K> S{top.rec, top.rhs};
          const int fail = backsub_chunk<K, L>(S, 0, nl - 1, false, false, xl, xr, xs);
          if (fail) report_fail(a, inst, level + d, fail - 1);
#pragma unroll
          for (int u = 0; u < L; ++u)
            if (u < nl) {
#pragma unroll
              for (int e = 0; e < K; ++e) top.x[u * K + e] = xs[u][e];
            }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      // 4. back-substitute the LDS levels below the top
      for (int dd = d - 1; dd >= 1; --dd) {
        const TopLevel<K> cur = top_level<K, L, SW>(base, dd), up = top_level<K, L, SW>(base, dd + 1);
        const int64_t nd = top_nodes<L>(G, dd);
        const int Gd = static_cast<int>((nd + L - 1) / L);
        if (lane < Gd) {
          const ChunkGeom geo = chunk_geom(lane, nd, L);
#pragma unroll
          for (int e = 0; e < K; ++e) {
            xl[e] = geo.has_left ? up.x[(lane - 1) * K + e] : 0.0;
            xr[e] = geo.has_right ? up.x[lane * K + e] : 0.0;
          }
          SrcN<K> S{cur.rec, cur.rhs};
          const int fail = backsub_chunk<K, L>(S, geo.a, geo.b, geo.has_left, geo.has_right, xl, xr, xs);
          if (fail) report_fail(a, inst, level + dd, geo.a + fail - 1);
#pragma unroll
          for (int u = 0; u < L; ++u) {
            const int64_t t = geo.a + u;
            if (t > geo.b) break;
#pragma unroll
            for (int e = 0; e < K; ++e) cur.x[t * K + e] = xs[u][e];
          }
          if (geo.has_right) {
#pragma unroll
            for (int e = 0; e < K; ++e) cur.x[(geo.b + 1) * K + e] = xr[e];
          }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
      }
    }
    // 5. level lt: back-substitute every chunk into HBM
    if (lane < G) {
      const ChunkGeom geo = chunk_geom(lane, n, L);
      const TopLevel<K> up = top_level<K, L, SW>(base, 1);
#pragma unroll
      for (int e = 0; e < K; ++e) {
        xl[e] = geo.has_left ? up.x[(lane - 1) * K + e] : 0.0;
        xr[e] = geo.has_right ? up.x[lane * K + e] : 0.0;
      }
      SrcT<K> S;
      S.rec = lv.rec;
      S.rhs = lv.rhs;
      S.C = c0 + lane;
      S.a = geo.a;
      S.L = L;
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
    // the next instance reuses the LDS slice
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
}

int64_t grid_for(int64_t tiles, const Launch& cfg) {
  const int64_t waves_per_block = cfg.block / WAVE;
  int64_t blocks = (tiles + waves_per_block - 1) / waves_per_block;
  if (cfg.max_blocks > 0 && blocks > cfg.max_blocks) blocks = cfg.max_blocks;
  return blocks < 1 ? 1 : blocks;
}

// Grid, workgroup and dynamic LDS of a level-0 launch: as many waves per
// workgroup as cfg.block asks for and the per-workgroup LDS limit allows.
template <int K, int L, class TIO, int RHS, int OUT, class F, int CH = WAVE>
bool level0_grid(int64_t tiles, const Launch& cfg, dim3& grid, dim3& block, size_t& lds) {
  constexpr size_t wb = Stage<K, L, TIO, RHS, OUT, F, CH>::BYTES;
  const int64_t fit = static_cast<int64_t>(cfg.lds_max) / static_cast<int64_t>(wb);
  if (fit < 1) return false;
  int wpb = cfg.block / WAVE;
  if (wpb > fit) wpb = static_cast<int>(fit);
  if (wpb < 1) wpb = 1;
  Launch c = cfg;
  c.block = wpb * WAVE;
  grid = dim3(static_cast<unsigned>(grid_for(tiles, c)));
  block = dim3(c.block);
  lds = wb * wpb;
  return true;
}

template <int K, int L, class TIO, int RHS, bool WREC, class F>
hipError_t launch_r0(const LevelDev& l0, const LevelDev& l1, const Level0Args& a, const Launch& cfg,
                     hipStream_t st) {
  constexpr int CH = R0Chunks<K, L, TIO, RHS, F>::value;
  const int64_t tiles = l0.chunks > 1 ? (l0.chunks - 2) / (CH - 1) + 1 : 1;
  dim3 grid, block;
  size_t lds;
  if (!level0_grid<K, L, TIO, RHS, OUT_STORE, F, CH>(tiles, cfg, grid, block, lds)) return hipErrorInvalidConfiguration;
  Level0Args b = a;
  b.wpb = static_cast<int>(block.x) / WAVE;
  b.nwaves = static_cast<int64_t>(grid.x) * b.wpb;
  hipLaunchKernelGGL((k_reduce0<K, L, TIO, RHS, WREC, F>), grid, block, lds, st, l0, l1, b);
  return hipGetLastError();
}

template <int K, int L, class TIO, int RHS, int OUT, class F>
hipError_t launch_b0(const LevelDev& l0, const LevelDev* l1, const Level0Args& a, const Launch& cfg,
                     hipStream_t st) {
  constexpr int CH = B0Chunks<K, L, TIO, RHS, OUT, F>::value;
  const int64_t tiles = (l0.chunks + CH - 1) / CH;
  dim3 grid, block;
  size_t lds;
  if (!level0_grid<K, L, TIO, RHS, OUT, F, CH>(tiles, cfg, grid, block, lds)) return hipErrorInvalidConfiguration;
  const LevelDev nx = l1 ? *l1 : LevelDev{};
  Level0Args b = a;
  b.wpb = static_cast<int>(block.x) / WAVE;
  b.nwaves = static_cast<int64_t>(grid.x) * b.wpb;
  hipLaunchKernelGGL((k_backsub0<K, L, TIO, RHS, OUT, F>), grid, block, lds, st, l0, nx, l1 != nullptr, b);
  return hipGetLastError();
}

template <int K, int L, class TIO, int RIN, int ROUT, class F>
hipError_t launch_br0(const LevelDev& l0, const LevelDev& l1, const Level0Args& a, const Launch& cfg,
                      hipStream_t st) {
  constexpr int CH = BRChunks<K, L, TIO, ROUT, F>::value;
  const int64_t tiles = (l0.chunks + CH - 3) / (CH - 2);
  dim3 grid, block;
  size_t lds;
  if (!level0_grid<K, L, TIO, ROUT, OUT_STORE, F, CH>(tiles, cfg, grid, block, lds)) return hipErrorInvalidConfiguration;
  Level0Args b = a;
  b.wpb = static_cast<int>(block.x) / WAVE;
  b.nwaves = static_cast<int64_t>(grid.x) * b.wpb;
  hipLaunchKernelGGL((k_backsub_reduce0<K, L, TIO, RIN, ROUT, F>), grid, block, lds, st, l0, l1, b);
  return hipGetLastError();
}

// ------------------------------------------------------------- dispatchers
template <int K, int L, class TIO, class F>
hipError_t reduce0_t(int rhs, bool wrec, const LevelDev& l0, const LevelDev& l1, const Level0Args& a,
                     const Launch& cfg, hipStream_t st) {
  switch (rhs) {
    case RHS_BETA:
      return wrec ? launch_r0<K, L, TIO, RHS_BETA, true, F>(l0, l1, a, cfg, st)
                  : launch_r0<K, L, TIO, RHS_BETA, false, F>(l0, l1, a, cfg, st);
    case RHS_RESID: return launch_r0<K, L, TIO, RHS_RESID, false, F>(l0, l1, a, cfg, st);
    case RHS_G:
      return wrec ? launch_r0<K, L, TIO, RHS_G, true, F>(l0, l1, a, cfg, st)
                  : launch_r0<K, L, TIO, RHS_G, false, F>(l0, l1, a, cfg, st);
    case RHS_GRESID: return launch_r0<K, L, TIO, RHS_GRESID, false, F>(l0, l1, a, cfg, st);
    default: return hipErrorInvalidValue;
  }
}

template <int K, int L, class TIO, class F>
hipError_t backsub0_t(int rhs, int out, const LevelDev& l0, const LevelDev* l1, const Level0Args& a,
                      const Launch& cfg, hipStream_t st) {
  if (out == OUT_STORE) {
    switch (rhs) {
      case RHS_BETA: return launch_b0<K, L, TIO, RHS_BETA, OUT_STORE, F>(l0, l1, a, cfg, st);
      case RHS_RESID: return launch_b0<K, L, TIO, RHS_RESID, OUT_STORE, F>(l0, l1, a, cfg, st);
      case RHS_G: return launch_b0<K, L, TIO, RHS_G, OUT_STORE, F>(l0, l1, a, cfg, st);
      case RHS_GRESID: return launch_b0<K, L, TIO, RHS_GRESID, OUT_STORE, F>(l0, l1, a, cfg, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (rhs) {
    case RHS_G: return launch_b0<K, L, TIO, RHS_G, OUT_GRAD, F>(l0, l1, a, cfg, st);
    case RHS_GRESID: return launch_b0<K, L, TIO, RHS_GRESID, OUT_GRAD, F>(l0, l1, a, cfg, st);
    default: return hipErrorInvalidValue;
  }
}

template <int K, int L, class TIO, class F>
hipError_t backsub_reduce0_t(int rhs_in, const LevelDev& l0, const LevelDev& l1, const Level0Args& a,
                             const Launch& cfg, hipStream_t st) {
  switch (rhs_in) {
    case RHS_BETA: return launch_br0<K, L, TIO, RHS_BETA, RHS_RESID, F>(l0, l1, a, cfg, st);
    case RHS_G: return launch_br0<K, L, TIO, RHS_G, RHS_GRESID, F>(l0, l1, a, cfg, st);
    default: return hipErrorInvalidValue;
  }
}

template <int K, int L, class TIO, class F>
size_t lds_bytes_t(int rhs, int out) {
  if (out == OUT_GRAD)
    return rhs == RHS_GRESID
               ? Stage<K, L, TIO, RHS_GRESID, OUT_GRAD, F, B0Chunks<K, L, TIO, RHS_GRESID, OUT_GRAD, F>::value>::BYTES
               : Stage<K, L, TIO, RHS_G, OUT_GRAD, F, B0Chunks<K, L, TIO, RHS_G, OUT_GRAD, F>::value>::BYTES;
  switch (rhs) {
    case RHS_BETA: return Stage<K, L, TIO, RHS_BETA, OUT_STORE, F>::BYTES;
    case RHS_RESID: return Stage<K, L, TIO, RHS_RESID, OUT_STORE, F>::BYTES;
    case RHS_G: return Stage<K, L, TIO, RHS_G, OUT_STORE, F>::BYTES;
    default: return Stage<K, L, TIO, RHS_GRESID, OUT_STORE, F>::BYTES;
  }
}

#if SMNN_TU_FORMS == 0
template <int K, int L>
hipError_t reduceN_t(bool wrec, int level, const LevelDev& l, const LevelDev& nx, const Level0Args& a,
                     const Launch& cfg, hipStream_t st) {
  const int64_t tiles = l.chunks > 1 ? (l.chunks - 2) / (WAVE - 1) + 1 : 1;
  const dim3 grid(static_cast<unsigned>(grid_for(tiles, cfg))), block(cfg.block);
  Level0Args b = a;
  b.wpb = cfg.block / WAVE;
  b.nwaves = static_cast<int64_t>(grid.x) * b.wpb;
  if (wrec) hipLaunchKernelGGL((k_reduceN<K, L, true>), grid, block, 0, st, l, nx, b, level);
  else hipLaunchKernelGGL((k_reduceN<K, L, false>), grid, block, 0, st, l, nx, b, level);
  return hipGetLastError();
}

template <int K, int L>
hipError_t backsubN_t(int level, const LevelDev& l, const LevelDev* nx, const Level0Args& a, const Launch& cfg,
                      hipStream_t st) {
  const int64_t tiles = (l.chunks + WAVE - 1) / WAVE;
  const dim3 grid(static_cast<unsigned>(grid_for(tiles, cfg))), block(cfg.block);
  const LevelDev n2 = nx ? *nx : LevelDev{};
  Level0Args b = a;
  b.wpb = cfg.block / WAVE;
  b.nwaves = static_cast<int64_t>(grid.x) * b.wpb;
  hipLaunchKernelGGL((k_backsubN<K, L>), grid, block, 0, st, l, n2, nx != nullptr, b, level);
  return hipGetLastError();
}

template <int K>
constexpr int top_width() { return top_lanes(K); }

template <int K, int L>
size_t top_lds_bytes_t() {   // per wave
  constexpr int SW = top_width<K>();
  return sizeof(double) * (WAVE / SW) * TopCaps<L, SW>::nodes * (Dim<K>::Q + Dim<K>::KK + 2 * K);
}

template <int K, int L>
hipError_t top_t(int level, const LevelDev& l, const Level0Args& a, const Launch& cfg, hipStream_t st) {
  constexpr int SW = top_width<K>();
  const size_t wb = top_lds_bytes_t<K, L>();
  int wpb = cfg.block / WAVE;
  while (wpb > 1 && wb * static_cast<size_t>(wpb) > static_cast<size_t>(cfg.lds_max)) --wpb;
  if (wb > static_cast<size_t>(cfg.lds_max)) return hipErrorInvalidConfiguration;
  Launch c = cfg;
  c.block = wpb * WAVE;
  const int64_t groups = (a.N + WAVE / SW - 1) / (WAVE / SW);   // one wave per 64 / SW instances
  const dim3 grid(static_cast<unsigned>(grid_for(groups, c))), block(c.block);
  Level0Args b = a;
  b.wpb = wpb;
  b.nwaves = static_cast<int64_t>(grid.x) * wpb;
  hipLaunchKernelGGL((k_top<K, L, SW>), grid, block, wb * wpb, st, l, b, level);
  return hipGetLastError();
}
#endif

}  // namespace

// What this translation unit compiles in.
//   SMNN_FOR_EACH_KL(X):    (K, L) pairs of the separator levels (X(K, L)),
//                           SMNN_TU_FORMS == 0 only;
//   SMNN_FOR_EACH_KLF(X):   level-0 (K, L, instance form, form id) tuples,
//                           form ids as in smnn_internal.h (SMNN_FORM_*).
// SMNN_TU_FORMS == 0 holds the scalar form (one variable, one governing
// equation, three scalar weights) and the separator levels; 1 the scalar
// shape with per-row weights; 2 two coupled variables (block size 4).
#if SMNN_TU_FORMS == 0
#if SMNN_TU_K == 2
#define SMNN_FOR_EACH_KL(X) X(2, 8) X(2, 16)
#elif SMNN_TU_K == 3
#define SMNN_FOR_EACH_KL(X) X(3, 4) X(3, 8) X(3, 16)
#elif SMNN_TU_K == 4
#define SMNN_FOR_EACH_KL(X) X(4, 4) X(4, 8)
#elif SMNN_TU_K == 5
#define SMNN_FOR_EACH_KL(X) X(5, 4)
#endif
#define SMNN_X_SCALAR(KV, LV) X(KV, LV, FormScalar, SMNN_FORM_SCALAR)
#define SMNN_FOR_EACH_KLF(X) SMNN_FOR_EACH_KL(SMNN_X_SCALAR)
#elif SMNN_TU_FORMS == 1
using FormRows = Form<1, 1, true>;
#if SMNN_TU_K == 2
#define SMNN_FOR_EACH_KLF(X) X(2, 8, FormRows, SMNN_FORM_ROWS)
#elif SMNN_TU_K == 3
#define SMNN_FOR_EACH_KLF(X) X(3, 4, FormRows, SMNN_FORM_ROWS) X(3, 8, FormRows, SMNN_FORM_ROWS)
#elif SMNN_TU_K == 4
#define SMNN_FOR_EACH_KLF(X) X(4, 4, FormRows, SMNN_FORM_ROWS) X(4, 8, FormRows, SMNN_FORM_ROWS)
#elif SMNN_TU_K == 5
#define SMNN_FOR_EACH_KLF(X) X(5, 4, FormRows, SMNN_FORM_ROWS)
#endif
#elif SMNN_TU_FORMS == 2
#if SMNN_TU_K != 4
#error "two coupled variables of order 1 have block size 4"
#endif
using FormV2 = Form<2, 2, false>;
using FormV2Rows = Form<2, 2, true>;
using FormV2Q1 = Form<2, 1, false>;
#define SMNN_FOR_EACH_KLF(X)                                                                 \
  X(4, 4, FormV2, SMNN_FORM_V2) X(4, 8, FormV2, SMNN_FORM_V2)                                \
  X(4, 4, FormV2Rows, SMNN_FORM_V2_ROWS) X(4, 8, FormV2Rows, SMNN_FORM_V2_ROWS)              \
  X(4, 4, FormV2Q1, SMNN_FORM_V2_Q1) X(4, 8, FormV2Q1, SMNN_FORM_V2_Q1)
#endif

bool SMNN_KFN(supported0)(int K, int L, int form) {
#define X(KV, LV, FT, FID) if (K == KV && L == LV && form == FID) return true;
  SMNN_FOR_EACH_KLF(X)
#undef X
  return false;
}

size_t SMNN_KFN(level0_lds_bytes)(int K, int L, int form, bool f32, int rhs_mode, int out_mode) {
#define X(KV, LV, FT, FID)                                                                                   \
  if (K == KV && L == LV && form == FID)                                                                     \
    return f32 ? lds_bytes_t<KV, LV, float, FT>(rhs_mode, out_mode) : lds_bytes_t<KV, LV, double, FT>(rhs_mode, out_mode);
  SMNN_FOR_EACH_KLF(X)
#undef X
  return 0;
}

hipError_t SMNN_KFN(launch_reduce0)(int K, int L, int form, bool f32, int rhs_mode, bool write_rec, const LevelDev& l0,
                                    const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV, FT, FID)                                                                           \
  if (K == KV && L == LV && form == FID)                                                             \
    return f32 ? reduce0_t<KV, LV, float, FT>(rhs_mode, write_rec, l0, l1, a, cfg, st)              \
               : reduce0_t<KV, LV, double, FT>(rhs_mode, write_rec, l0, l1, a, cfg, st);
  SMNN_FOR_EACH_KLF(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_KFN(launch_backsub0)(int K, int L, int form, bool f32, int rhs_mode, int out_mode, const LevelDev& l0,
                                     const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
#define X(KV, LV, FT, FID)                                                                           \
  if (K == KV && L == LV && form == FID)                                                             \
    return f32 ? backsub0_t<KV, LV, float, FT>(rhs_mode, out_mode, l0, l1, a, cfg, st)              \
               : backsub0_t<KV, LV, double, FT>(rhs_mode, out_mode, l0, l1, a, cfg, st);
  SMNN_FOR_EACH_KLF(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t SMNN_KFN(launch_backsub_reduce0)(int K, int L, int form, bool f32, int rhs_in, const LevelDev& l0,
                                            const LevelDev& l1, const Level0Args& a, const Launch& cfg,
                                            hipStream_t st) {
#define X(KV, LV, FT, FID)                                                                           \
  if (K == KV && L == LV && form == FID)                                                             \
    return f32 ? backsub_reduce0_t<KV, LV, float, FT>(rhs_in, l0, l1, a, cfg, st)                   \
               : backsub_reduce0_t<KV, LV, double, FT>(rhs_in, l0, l1, a, cfg, st);
  SMNN_FOR_EACH_KLF(X)
#undef X
  return hipErrorInvalidValue;
}

#if SMNN_TU_FORMS == 0
bool SMNN_KFN(supported)(int K, int L) {
#define X(KV, LV) if (K == KV && L == LV) return true;
  SMNN_FOR_EACH_KL(X)
#undef X
  return false;
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

size_t SMNN_KFN(top_lds_bytes)(int K, int L) {
#define X(KV, LV) \
  if (K == KV && L == LV) return top_lds_bytes_t<KV, LV>();
  SMNN_FOR_EACH_KL(X)
#undef X
  return 0;
}

hipError_t SMNN_KFN(launch_top)(int K, int L, int level, const LevelDev& l, const Level0Args& a, const Launch& cfg,
                                hipStream_t st) {
#define X(KV, LV) \
  if (K == KV && L == LV) return top_t<KV, LV>(level, l, a, cfg, st);
  SMNN_FOR_EACH_KL(X)
#undef X
  return hipErrorInvalidValue;
}
#endif

}  // namespace smnn
