// C-ABI of libsmnn (include/smnn.h): plan creation, buffer layout and the
// launch sequence of the forward and backward passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/smnn.h"
#include "smnn_core.h"
#include "smnn_internal.h"
#include "smnn_levels.h"

using namespace smnn;

struct smnn_plan {
  int R = 0, K = 0, n_init = 0, mode = 0, refine = 0, L0 = 8, L1 = 8;
  int V = 1, QE = 1;          // variables and governing equations per point (K = V (R+1))
  bool rows = false;          // per-row weights
  bool wide = false;          // K > 5: one 16-lane group per chunk (smnn_wide.hip)
  int form = 0;               // FormId of the level-0 kernels
  int t_init = 1;   // time points carrying initial values
  int top = 0;      // > 0: levels >= top are solved by one launch per solve (launch_top)
  int64_t N = 0, S = 0;
  int device = 0;
  bool f32 = false;
  Launch cfg;
  std::vector<LevelDev> lev;     // device views; rec/rhs/x hold byte offsets until bound
  std::vector<size_t> rec_off, rhs_off, x_off;
  size_t factor_bytes = 0, workspace_bytes = 0;
  size_t buf_off[2] = {0, 0}, dwp_off = 0, dwq_off = 0, info_off = 0, queue_off = 0;
  int dw_split = 1;               // workgroups per instance of the weight-gradient sum
  void* meta = nullptr;          // device metadata (chunk_inst, chunk_off, node_off of every level)
  const int32_t* order = nullptr;  // in meta: instances by decreasing T (ragged batches only)
  // launch tracing (smnn_trace_enable); mutable: recorded during const calls
  mutable std::vector<hipEvent_t> ev;
  mutable std::vector<smnn_trace_record> rec;
  mutable size_t used = 0;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Default chunk lengths (level 0, levels >= 1) per block size K, measured
// fastest on MI355X for 1536 x 10,000-step batches (block size 2: 8 / 8 took
// 2.47 ms per fp64r step against 4.23 ms at 16 / 16).  Level 0 with float I/O
// stages half the bytes per step, so a lane can own twice the steps in the
// same LDS, which halves the separator system.
int default_chunk(int K, bool upper, bool f32) {
  switch (K) {
    case 2: return 8;
    case 3:
    case 4: return upper || f32 ? 8 : 4;
    default: return 4;
  }
}

// Float I/O takes level-0 chunks of 8 from this many time steps on.  Below it
// chunks of 8 leave too few tiles to fill the chip more than about twice and
// the last round of waves idles most CUs: on 1536 x 1,000 steps chunk 4 was
// faster (0.352 against 0.385 ms per fp32r step), while from 5e6 steps on
// chunk 8 was 15-18 % faster.
constexpr int64_t kFloatChunk8Steps = int64_t(1) << 22;

// First level >= 1 from which one launch per solve can take the upper levels
// (0: none): every instance has at most `lanes` chunks there, the level holds
// at most 2^19 nodes, and it is not the last level (so that it replaces at
// least two).  Level l has the chunk length L0 at l = 0 and L1 above.
int top_start(const std::vector<int64_t>& T, int L0, int L1, int lanes) {
  std::vector<int64_t> n = T;
  for (int l = 0;; ++l) {
    const int L = l == 0 ? L0 : L1;
    int64_t gmax = 0, nodes = 0;
    bool any_next = false;
    for (auto& ni : n) {
      const int64_t g = ni > 0 ? ceil_div(ni, L) : 0;
      gmax = std::max(gmax, g);
      nodes += ni;
      ni = ni > L ? g - 1 : 0;
      any_next = any_next || ni > 0;
    }
    if (l >= 1 && any_next && gmax <= lanes && nodes <= (int64_t(1) << 19)) return l;
    if (!any_next) return 0;
  }
}

struct Bound {
  std::vector<LevelDev> lev;
  void* buf[2];
  double* dwp;
  double* dwq;
  uint32_t* info;
  uint32_t* queue;
};

// Tile counters of the persistent launches of one call (device work queue).
constexpr int kQueueSlots = 512;

Bound bind(const smnn_plan* p, void* factor, void* workspace) {
  Bound b;
  b.lev = p->lev;
  char* f = static_cast<char*>(factor);
  char* ws = static_cast<char*>(workspace);
  for (size_t l = 1; l < b.lev.size(); ++l) {
    b.lev[l].rec = reinterpret_cast<double*>(f + p->rec_off[l]);
    b.lev[l].rhs = reinterpret_cast<double*>(ws + p->rhs_off[l]);
    b.lev[l].x = reinterpret_cast<double*>(ws + p->x_off[l]);
  }
  b.buf[0] = ws + p->buf_off[0];
  b.buf[1] = ws + p->buf_off[1];
  b.dwp = reinterpret_cast<double*>(ws + p->dwp_off);
  b.dwq = reinterpret_cast<double*>(ws + p->dwq_off);
  b.info = reinterpret_cast<uint32_t*>(ws + p->info_off);
  b.queue = reinterpret_cast<uint32_t*>(ws + p->queue_off);
  return b;
}

#define SMNN_HIP(call)                          \
  do {                                          \
    if ((call) != hipSuccess) return SMNN_ERR_HIP; \
  } while (0)

// Launch tracing: an event pair around every launch while enabled.
struct Tracer {
  const smnn_plan* p;
  hipStream_t st;
  bool on(int kernel, int level, int rhs, int out) const {
    if (p->used >= p->rec.size()) return false;
    smnn_trace_record& r = p->rec[p->used];
    r.kernel = kernel; r.level = level; r.rhs = rhs; r.out = out; r.ms = 0.f;
    return hipEventRecord(p->ev[2 * p->used], st) == hipSuccess;
  }
  void off() const {
    (void)hipEventRecord(p->ev[2 * p->used + 1], st);
    ++p->used;
  }
};

// Every launch takes its tiles in the direction opposite to the launch
// before it (Level0Args::rev), so that it starts on the data the previous
// launch touched last.
// Persistent launches each claim their tiles from a counter of their own.
#define SMNN_LAUNCH(TR, A, KIND, LEVEL, RHS, OUT, CALL)     \
  do {                                                      \
    (A).rev ^= 1;                                           \
    (A).queue = (A).queue_next < (A).queue_slots ? (A).queue_base + (A).queue_next++ : nullptr; \
    const bool traced_ = (TR).on(KIND, LEVEL, RHS, OUT);    \
    const hipError_t e_ = (CALL);                           \
    if (traced_) (TR).off();                                \
    if (e_ != hipSuccess) return SMNN_ERR_HIP;              \
  } while (0)

// The part of a solve of M x = f above the level-0 back-substitution: the
// level-0 reduce (unless skip_reduce0: a fused kernel already wrote the
// level-1 right-hand sides), the reduces of levels >= 1 up and their
// back-substitutions down.
smnn_status solve_upper(const smnn_plan* p, const Bound& b, int rhs, bool write_rec, const Level0Args& a,
                        hipStream_t st, bool skip_reduce0 = false) {
  const int nl = static_cast<int>(b.lev.size());
  const int lt = p->top > 0 ? p->top : nl;   // levels >= lt in one launch
  const Tracer tr{p, st};
  if (p->wide) {   // every level by its own launches, no one-launch upper levels
    if (nl > 1)
      SMNN_LAUNCH(tr, a, SMNN_K_REDUCE0, 0, rhs, 0,
                  launch_wreduce0(p->K, p->L0, p->form, p->f32, rhs, write_rec, b.lev[0], b.lev[1], a, p->cfg, st));
    for (int l = 1; l + 1 < nl; ++l)
      SMNN_LAUNCH(tr, a, SMNN_K_REDUCEN, l, rhs, 0,
                  launch_wreduceN(p->K, p->L1, write_rec, l, b.lev[l], b.lev[l + 1], a, p->cfg, st));
    for (int l = nl - 1; l >= 1; --l)
      SMNN_LAUNCH(tr, a, SMNN_K_BACKSUBN, l, rhs, 0,
                  launch_wbacksubN(p->K, p->L1, l, b.lev[l], l + 1 < nl ? &b.lev[l + 1] : nullptr, a, p->cfg, st));
    return SMNN_OK;
  }
  if (nl > 1 && !skip_reduce0)
    SMNN_LAUNCH(tr, a, SMNN_K_REDUCE0, 0, rhs, 0,
                launch_reduce0(p->K, p->L0, p->form, p->f32, rhs, write_rec, b.lev[0], b.lev[1], a, p->cfg, st));
  for (int l = 1; l + 1 < nl && l < lt; ++l)
    SMNN_LAUNCH(tr, a, SMNN_K_REDUCEN, l, rhs, 0,
                launch_reduceN(p->K, p->L1, write_rec, l, b.lev[l], b.lev[l + 1], a, p->cfg, st));
  if (lt < nl)
    SMNN_LAUNCH(tr, a, SMNN_K_TOP, lt, rhs, 0, launch_top(p->K, p->L1, lt, b.lev[lt], a, p->cfg, st));
  for (int l = (lt < nl ? lt : nl) - 1; l >= 1; --l)
    SMNN_LAUNCH(tr, a, SMNN_K_BACKSUBN, l, rhs, 0,
                launch_backsubN(p->K, p->L1, l, b.lev[l], l + 1 < nl ? &b.lev[l + 1] : nullptr, a, p->cfg, st));
  return SMNN_OK;
}

smnn_status backsub0(const smnn_plan* p, const Bound& b, int rhs, int out_mode, const Level0Args& a,
                     hipStream_t st) {
  const int nl = static_cast<int>(b.lev.size());
  const Tracer tr{p, st};
  if (p->wide) {
    SMNN_LAUNCH(tr, a, SMNN_K_BACKSUB0, 0, rhs, out_mode,
                launch_wbacksub0(p->K, p->L0, p->form, p->f32, rhs, out_mode, b.lev[0], nl > 1 ? &b.lev[1] : nullptr,
                                 a, p->cfg, st));
    return SMNN_OK;
  }
  SMNN_LAUNCH(tr, a, SMNN_K_BACKSUB0, 0, rhs, out_mode,
              launch_backsub0(p->K, p->L0, p->form, p->f32, rhs, out_mode, b.lev[0], nl > 1 ? &b.lev[1] : nullptr,
                              a, p->cfg, st));
  return SMNN_OK;
}

// One solve of M x = f through every level.  rhs selects f; the level-0
// back-substitution writes `a.out` (OUT_STORE) or the gradients (OUT_GRAD).
smnn_status solve(const smnn_plan* p, const Bound& b, int rhs, bool write_rec, int out_mode,
                  const Level0Args& a, hipStream_t st) {
  const smnn_status s = solve_upper(p, b, rhs, write_rec, a, st);
  if (s != SMNN_OK) return s;
  return backsub0(p, b, rhs, out_mode, a, st);
}

// A solve with right-hand side rhs (beta or dl/dy) storing its iterate to
// a.out, whose level-0 back-substitution also does the level-0 reduce of
// the first refinement solve (needs a level 1).
smnn_status solve_then_reduce(const smnn_plan* p, const Bound& b, int rhs, bool write_rec, const Level0Args& a,
                              hipStream_t st) {
  const smnn_status s = solve_upper(p, b, rhs, write_rec, a, st);
  if (s != SMNN_OK) return s;
  const Tracer tr{p, st};
  SMNN_LAUNCH(tr, a, SMNN_K_BACKSUB_REDUCE0, 0, rhs, 0,
              launch_backsub_reduce0(p->K, p->L0, p->form, p->f32, rhs, b.lev[0], b.lev[1], a, p->cfg, st));
  return SMNN_OK;
}

// Per-row weights: the weight buffer (and its gradient) holds the governing
// weights [S][QE], then the initial weights [N][T_init][V][n_init], then the
// smoothness weights [S].
void bind_row_weights(const smnn_plan* p, const void* w, void* dw, Level0Args& a) {
  if (!p->rows) return;
  a.w = nullptr;   // no scalar weights
  const size_t io = p->f32 ? sizeof(float) : sizeof(double);
  const size_t ng = static_cast<size_t>(p->S) * p->QE;
  const size_t ni = static_cast<size_t>(p->N) * p->t_init * p->V * p->n_init;
  a.wg = w;
  a.wi = static_cast<const char*>(w) + io * ng;
  a.ws = static_cast<const char*>(w) + io * (ng + ni);
  if (dw) {
    a.dwg = dw;
    a.dwi = static_cast<char*>(dw) + io * ng;
    a.dws = static_cast<char*>(dw) + io * (ng + ni);
  }
}

smnn_status check_device(const smnn_plan* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SMNN_ERR_HIP;
  return dev == p->device ? SMNN_OK : SMNN_ERR_DEVICE;
}

}  // namespace

extern "C" {

smnn_status smnn_plan_create(const smnn_plan_desc* d, smnn_plan** out) {
  if (!out) return SMNN_ERR_INVALID_ARG;
  *out = nullptr;
  if (!d) return SMNN_ERR_INVALID_ARG;
  if (d->order < 1 || d->order > 4) return SMNN_ERR_INVALID_ARG;
  if (d->n_init < 0 || d->n_init > d->order + 1) return SMNN_ERR_INVALID_ARG;
  if (d->init_points < 0 || d->init_points > (1 << 30)) return SMNN_ERR_INVALID_ARG;
  if (d->n_inst < 1 || d->n_inst > INT32_MAX) return SMNN_ERR_INVALID_ARG;
  if (d->variables < 0 || d->equations < 0 || (d->row_weights != 0 && d->row_weights != 1))
    return SMNN_ERR_INVALID_ARG;
  const int V = d->variables ? d->variables : 1;
  const int QE = d->equations ? d->equations : V;
  // the kernels index the initial values with 32-bit offsets
  if (d->n_inst * V * d->n_init > INT32_MAX / std::max(1, d->init_points)) return SMNN_ERR_INVALID_ARG;
  if (d->mode < SMNN_MODE_FP64 || d->mode > SMNN_MODE_FP32_REFINED) return SMNN_ERR_INVALID_ARG;
  if (d->refine_steps < -1 || d->refine_steps > 4) return SMNN_ERR_INVALID_ARG;
  if (d->block < 0 || d->block > 256 || d->block % 64 != 0) return SMNN_ERR_INVALID_ARG;
  if (d->max_blocks < 0) return SMNN_ERR_INVALID_ARG;
  if (V > 5 || QE > 5) return SMNN_ERR_UNSUPPORTED;
  const int K = V * (d->order + 1);
  const int form = form_id(V, QE, d->row_weights != 0);
  const bool wide = K > 5;
  if (form < 0) return SMNN_ERR_UNSUPPORTED;
  const bool f32 = d->mode == SMNN_MODE_FP32_REFINED;
  if (d->chunk < 0 || d->chunk_upper < 0) return SMNN_ERR_INVALID_ARG;
  std::vector<int64_t> T(static_cast<size_t>(d->n_inst));
  int64_t steps = 0;
  for (int64_t i = 0; i < d->n_inst; ++i) {
    T[i] = d->steps ? d->steps[i] : d->steps_uniform;
    if (T[i] < 1 || T[i] > (int64_t(1) << 40)) return SMNN_ERR_INVALID_ARG;
    steps += T[i];
  }
  const int L0 = d->chunk ? d->chunk : (wide ? 4 : default_chunk(K, false, f32 && steps >= kFloatChunk8Steps));
  int L1 = d->chunk_upper ? d->chunk_upper : (wide ? 4 : default_chunk(K, true, f32));
  // 3 x 3 blocks: separator chunks of 4 where the one-launch upper levels
  // start at the same level as with 8.  That launch's first and last sweeps
  // then take 4 dependent steps per lane instead of 8 (1536 x 1,000 steps:
  // 43 -> 31 us per solve, fp64r 0.456 -> 0.411 ms per step).  Where chunks
  // of 4 would add a level below it (1536 x 10,000 steps), 8 stays faster.
  if (!d->chunk_upper && !wide && K == 3 && L1 == 8) {
    const int t8 = top_start(T, L0, 8, top_lanes(K)), t4 = top_start(T, L0, 4, top_lanes(K));
    if (t4 > 0 && t8 > 0 && t4 <= t8) L1 = 4;
  }
  if (wide ? !(wide_supported(K, L0, form) && wide_supported(K, L1, form))
           : !(supported0(K, L0, form) && supported(K, L1)))
    return SMNN_ERR_UNSUPPORTED;

  smnn_plan* p = new (std::nothrow) smnn_plan;
  if (!p) return SMNN_ERR_HIP;
  p->R = d->order;
  p->K = K;
  p->V = V;
  p->QE = QE;
  p->rows = d->row_weights != 0;
  p->wide = wide;
  p->form = form;
  p->n_init = d->n_init;
  p->t_init = d->init_points > 0 ? d->init_points : 1;
  p->mode = d->mode;
  // Default refinement: each step contracts the error by about cond(M) 2^-53.
  // Order >= 3 meets cond(M) ~ 1e13 at h ~ 0.01, where one step leaves ~1e-8
  // in FP64 I/O, so the double modes take two there.
  p->refine = d->mode == SMNN_MODE_FP64 ? 0
              : d->refine_steps >= 0 ? d->refine_steps
              : (d->order >= 3 && d->mode == SMNN_MODE_FP64_REFINED) ? 2 : 1;
  p->L0 = L0;
  p->L1 = L1;
  p->N = d->n_inst;
  p->f32 = d->mode == SMNN_MODE_FP32_REFINED;
  p->cfg.block = d->block ? d->block : 64;
  p->cfg.max_blocks = d->max_blocks;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return SMNN_ERR_HIP; }
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess ||
      lds_max <= 0) {
    delete p;
    return SMNN_ERR_HIP;
  }
  p->cfg.lds_max = lds_max;
  // every level-0 kernel variant must fit one wave's tile into LDS
  {
    const int combos[6][2] = {{RHS_BETA, OUT_STORE}, {RHS_RESID, OUT_STORE}, {RHS_G, OUT_STORE},
                              {RHS_GRESID, OUT_STORE}, {RHS_G, OUT_GRAD}, {RHS_GRESID, OUT_GRAD}};
    for (const auto& cb : combos)
      if (!wide && level0_lds_bytes(K, L0, form, p->f32, cb[0], cb[1]) > static_cast<size_t>(lds_max)) {
        delete p;
        return SMNN_ERR_UNSUPPORTED;
      }
  }

  std::vector<Level> lv = build_levels(T, L0, L1);
  p->S = lv[0].nodes;
  // The upper levels of a solve are short dependent chains: from the first
  // level >= 1 at which every instance has at most top_lanes(K) chunks and
  // the level holds at most 2^19 nodes, they are solved by one launch per
  // solve (top_lanes(K) lanes per instance), when that replaces at least two
  // levels.  Blocks of up to 3 unknowns take it where that kernel keeps its
  // state in VGPRs (K * L1 <= 24): measured faster on the 1536 x 1,000 and
  // 1536 x 10,000 batches, slower when it starts at a level of millions of
  // nodes.  Larger blocks hold a whole SIMD per wave, so they take four
  // instances per wave (at most 16 chunks each).
  const bool top_fits = K <= 3 ? K * L1 <= 24 : true;
  if (!wide && top_fits && top_lds_bytes(K, L1) > 0 && top_lds_bytes(K, L1) <= static_cast<size_t>(lds_max))
    p->top = top_start(T, L0, L1, top_lanes(K));
  const int Q = K * (K + 1) / 2;
  // separator records: packed A and the coupling block; wide blocks keep
  // full K x K halves of A and the coupling block (3 K^2), and two halves of
  // the right-hand side
  const int REC = wide ? 3 * K * K : Q + K * K, RHSW = wide ? 2 * K : K;
  const size_t io = p->f32 ? sizeof(float) : sizeof(double);

  // factor: level >= 1 node records
  size_t fb = 0;
  p->rec_off.assign(lv.size(), 0);
  // separator levels use the interleaved layout: TILE_W chunks x L1 slots
  // per group (wide blocks: the natural layout, one slot per node)
  auto slots = [&](size_t l) {
    if (wide) return static_cast<size_t>(lv[l].nodes);
    return static_cast<size_t>((lv[l].chunks + TILE_W - 1) / TILE_W) * TILE_W * L1;
  };
  for (size_t l = 1; l < lv.size(); ++l) {
    p->rec_off[l] = fb;
    fb = align_up(fb + sizeof(double) * REC * slots(l));
  }
  // workspace: level >= 1 rhs and solution, two iterate buffers, chunk partials, info
  size_t wb = 0;
  p->rhs_off.assign(lv.size(), 0);
  p->x_off.assign(lv.size(), 0);
  for (size_t l = 1; l < lv.size(); ++l) {
    p->rhs_off[l] = wb;
    wb = align_up(wb + sizeof(double) * RHSW * slots(l));
    p->x_off[l] = wb;
    wb = align_up(wb + sizeof(double) * K * lv[l].nodes);
  }
  const int nbuf = std::min(p->refine, 2);
  for (int q = 0; q < 2; ++q) {
    p->buf_off[q] = wb;
    if (q < nbuf) wb = align_up(wb + io * K * p->S);
  }
  p->dwp_off = wb;
  wb = align_up(wb + sizeof(double) * 3 * lv[0].chunks);
  // The per-instance sums of those partials: batches of fewer than 512
  // instances split each instance's chunks over several workgroups (each
  // slice at least 1024 chunks), whose sums go through [N][split][3].
  {
    int64_t cmax = 0;
    for (int64_t i = 0; i < p->N; ++i) cmax = std::max(cmax, lv[0].chunk_off[i + 1] - lv[0].chunk_off[i]);
    const int64_t want = p->N >= 512 ? 1 : (512 + p->N - 1) / p->N;
    p->dw_split = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, cmax / 1024)));
  }
  p->dwq_off = wb;
  if (p->dw_split > 1) wb = align_up(wb + sizeof(double) * 3 * p->N * p->dw_split);
  p->info_off = wb;
  wb = align_up(wb + sizeof(uint32_t) * p->N);
  p->queue_off = wb;
  wb = align_up(wb + sizeof(uint32_t) * kQueueSlots);
  p->factor_bytes = std::max<size_t>(fb, kAlign);
  p->workspace_bytes = wb;

  // device metadata
  size_t mb = 0;
  std::vector<size_t> ci(lv.size()), co(lv.size()), no(lv.size());
  for (size_t l = 0; l < lv.size(); ++l) {
    co[l] = mb; mb = align_up(mb + sizeof(int64_t) * (p->N + 1));
    no[l] = mb; mb = align_up(mb + sizeof(int64_t) * (p->N + 1));
    ci[l] = mb; mb = align_up(mb + sizeof(int32_t) * std::max<int64_t>(lv[l].chunks, 1));
  }
  const size_t cs = mb;   // level-0 chunk_step
  mb = align_up(mb + sizeof(int64_t) * (lv[0].chunks + 1));
  const size_t od = mb;   // instances by decreasing T
  mb = align_up(mb + sizeof(int32_t) * p->N);
  std::vector<char> host(mb, 0);
  {
    int32_t* ord = reinterpret_cast<int32_t*>(host.data() + od);
    for (int64_t i = 0; i < p->N; ++i) ord[i] = static_cast<int32_t>(i);
    std::stable_sort(ord, ord + p->N, [&](int32_t x, int32_t y) { return T[x] > T[y]; });
  }
  for (size_t l = 0; l < lv.size(); ++l) {
    std::copy(lv[l].chunk_off.begin(), lv[l].chunk_off.end(), reinterpret_cast<int64_t*>(host.data() + co[l]));
    std::copy(lv[l].node_off.begin(), lv[l].node_off.end(), reinterpret_cast<int64_t*>(host.data() + no[l]));
    std::copy(lv[l].chunk_inst.begin(), lv[l].chunk_inst.end(), reinterpret_cast<int32_t*>(host.data() + ci[l]));
  }
  {
    int64_t* step = reinterpret_cast<int64_t*>(host.data() + cs);
    for (int64_t g = 0; g < lv[0].chunks; ++g) {
      const int32_t i = lv[0].chunk_inst[g];
      step[g] = lv[0].node_off[i] + (g - lv[0].chunk_off[i]) * L0;
    }
    step[lv[0].chunks] = lv[0].nodes;
  }
  if (hipMalloc(&p->meta, mb) != hipSuccess) { delete p; return SMNN_ERR_HIP; }
  if (hipMemcpy(p->meta, host.data(), mb, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->meta);
    delete p;
    return SMNN_ERR_HIP;
  }
  char* m = static_cast<char*>(p->meta);
  p->lev.resize(lv.size());
  for (size_t l = 0; l < lv.size(); ++l) {
    p->lev[l].chunk_inst = reinterpret_cast<const int32_t*>(m + ci[l]);
    p->lev[l].chunk_off = reinterpret_cast<const int64_t*>(m + co[l]);
    p->lev[l].node_off = reinterpret_cast<const int64_t*>(m + no[l]);
    p->lev[l].chunks = lv[l].chunks;
    p->lev[l].nodes = lv[l].nodes;
  }
  p->lev[0].chunk_step = reinterpret_cast<const int64_t*>(m + cs);
  // (no order for equal lengths: those launches alternate their direction)
  const bool ragged = std::any_of(T.begin(), T.end(), [&](int64_t t) { return t != T[0]; });
  p->order = ragged ? reinterpret_cast<const int32_t*>(m + od) : nullptr;
  *out = p;
  return SMNN_OK;
}

smnn_status smnn_trace_enable(smnn_plan* p, int32_t capacity) {
  if (!p || capacity < 0) return SMNN_ERR_INVALID_ARG;
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->rec.clear();
  p->used = 0;
  if (capacity == 0) return SMNN_OK;
  p->ev.resize(2 * static_cast<size_t>(capacity), nullptr);
  for (auto& e : p->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      smnn_trace_enable(p, 0);
      return SMNN_ERR_HIP;
    }
  p->rec.resize(capacity);
  return SMNN_OK;
}

int32_t smnn_trace_read(smnn_plan* p, smnn_trace_record* out, int32_t cap) {
  if (!p || (!out && cap > 0)) return -1;
  int32_t n = 0;
  for (size_t i = 0; i < p->used && n < cap; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess) return -1;
    out[n] = p->rec[i];
    out[n].ms = ms;
    ++n;
  }
  p->used = 0;
  return n;
}

smnn_status smnn_plan_destroy(smnn_plan* p) {
  if (!p) return SMNN_ERR_INVALID_ARG;
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  if (p->meta) (void)hipFree(p->meta);
  delete p;
  return SMNN_OK;
}

smnn_status smnn_plan_sizes(const smnn_plan* p, size_t* factor_bytes, size_t* workspace_bytes,
                            int64_t* total_steps) {
  if (!p) return SMNN_ERR_INVALID_ARG;
  if (factor_bytes) *factor_bytes = p->factor_bytes;
  if (workspace_bytes) *workspace_bytes = p->workspace_bytes;
  if (total_steps) *total_steps = p->S;
  return SMNN_OK;
}

int64_t smnn_plan_query(const smnn_plan* p, int32_t key) {
  if (!p) return -1;
  if (key == SMNN_Q_LEVELS) return static_cast<int64_t>(p->lev.size());
  if (key == SMNN_Q_CHUNK) return p->L0;
  if (key == SMNN_Q_CHUNK_UPPER) return p->L1;
  if (key == SMNN_Q_REFINE) return p->refine;
  if (key == SMNN_Q_MODE) return p->mode;
  if (key == SMNN_Q_INIT_POINTS) return p->t_init;
  if (key == SMNN_Q_TOP_LEVEL) return p->top;
  if (key >= 1000 && key < 1000 + static_cast<int32_t>(p->lev.size())) return p->lev[key - 1000].nodes;
  if (key >= 2000 && key < 2000 + static_cast<int32_t>(p->lev.size())) return p->lev[key - 2000].chunks;
  return -1;
}

smnn_status smnn_forward(const smnn_plan* p, const void* c, const void* b, const void* h, const void* u0,
                         const void* w, void* y, void* factor, size_t factor_bytes, void* workspace,
                         size_t workspace_bytes, int32_t* info, void* stream) {
  if (!p || !c || !b || !h || !w || !y || !factor || !workspace) return SMNN_ERR_INVALID_ARG;
  if (factor_bytes < p->factor_bytes || workspace_bytes < p->workspace_bytes) return SMNN_ERR_WORKSPACE;
  if (p->n_init > 0 && !u0) return SMNN_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(factor) | reinterpret_cast<uintptr_t>(workspace)) % kAlign)
    return SMNN_ERR_INVALID_ARG;
  const smnn_status ds = check_device(p);
  if (ds != SMNN_OK) return ds;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Bound bd = bind(p, factor, workspace);
  Level0Args a;
  a.c = c; a.d = b; a.s = h; a.u0 = u0; a.w = w;
  bind_row_weights(p, w, nullptr, a);
  a.n_init = p->n_init;
  a.t_init = p->t_init;
  a.L0 = p->L0;
  a.L1 = p->L1;
  a.N = p->N;
  a.info = info ? bd.info : nullptr;
  a.order = p->order;
  if (p->cfg.max_blocks > 0) {   // persistent launches: a device work queue per launch
    a.queue_base = bd.queue;
    a.queue_slots = kQueueSlots;
    SMNN_HIP(launch_fill_u32(bd.queue, kQueueSlots, 0u, st));
  }
  SMNN_HIP(launch_info_init(a, st));
  const bool fused = !p->wide && p->refine > 0 && bd.lev.size() > 1;
  a.out = p->refine == 0 ? y : bd.buf[0];
  smnn_status s = fused ? solve_then_reduce(p, bd, RHS_BETA, true, a, st)
                        : solve(p, bd, RHS_BETA, true, OUT_STORE, a, st);
  if (s != SMNN_OK) return s;
  for (int m = 1; m <= p->refine; ++m) {
    a.v = a.out;
    a.out = (m == p->refine) ? y : bd.buf[m % 2];
    if (m == 1 && fused) {
      s = solve_upper(p, bd, RHS_RESID, false, a, st, true);
      if (s == SMNN_OK) s = backsub0(p, bd, RHS_RESID, OUT_STORE, a, st);
    } else {
      s = solve(p, bd, RHS_RESID, false, OUT_STORE, a, st);
    }
    if (s != SMNN_OK) return s;
  }
  SMNN_HIP(launch_info_finalize(a, info, st));
  return SMNN_OK;
}

smnn_status smnn_backward(const smnn_plan* p, const void* c, const void* b, const void* h, const void* u0,
                          const void* w, const void* y, const void* factor, size_t factor_bytes, const void* gy,
                          void* dc, void* db, void* dh, void* du0, void* dw, void* workspace,
                          size_t workspace_bytes, int32_t* info, void* stream) {
  if (!p || !c || !b || !h || !w || !y || !factor || !gy || !dc || !db || !dh || !dw || !workspace)
    return SMNN_ERR_INVALID_ARG;
  if (factor_bytes < p->factor_bytes || workspace_bytes < p->workspace_bytes) return SMNN_ERR_WORKSPACE;
  if (p->n_init > 0 && (!u0 || !du0)) return SMNN_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(factor) | reinterpret_cast<uintptr_t>(workspace)) % kAlign)
    return SMNN_ERR_INVALID_ARG;
  const smnn_status ds = check_device(p);
  if (ds != SMNN_OK) return ds;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Bound bd = bind(p, const_cast<void*>(factor), workspace);
  Level0Args a;
  a.c = c; a.d = b; a.s = h; a.u0 = u0; a.w = w; a.g = gy; a.y = y;
  a.dc = dc; a.dd = db; a.ds = dh; a.du0 = du0; a.dw = dw; a.dw_part = bd.dwp;
  bind_row_weights(p, w, dw, a);
  a.n_init = p->n_init;
  a.t_init = p->t_init;
  a.L0 = p->L0;
  a.L1 = p->L1;
  a.N = p->N;
  a.info = info ? bd.info : nullptr;
  a.order = p->order;
  if (p->cfg.max_blocks > 0) {   // persistent launches: a device work queue per launch
    a.queue_base = bd.queue;
    a.queue_slots = kQueueSlots;
    SMNN_HIP(launch_fill_u32(bd.queue, kQueueSlots, 0u, st));
  }
  SMNN_HIP(launch_info_init(a, st));
  smnn_status s;
  if (p->refine == 0) {
    s = solve(p, bd, RHS_G, false, OUT_GRAD, a, st);
    if (s != SMNN_OK) return s;
  } else {
    const bool fused = !p->wide && bd.lev.size() > 1;
    a.out = bd.buf[0];
    s = fused ? solve_then_reduce(p, bd, RHS_G, false, a, st)
              : solve(p, bd, RHS_G, false, OUT_STORE, a, st);
    if (s != SMNN_OK) return s;
    for (int m = 1; m <= p->refine; ++m) {
      a.v = a.out;
      const bool lastm = m == p->refine;
      a.out = lastm ? nullptr : bd.buf[m % 2];
      if (m == 1 && fused) {
        s = solve_upper(p, bd, RHS_GRESID, false, a, st, true);
        if (s == SMNN_OK) s = backsub0(p, bd, RHS_GRESID, lastm ? OUT_GRAD : OUT_STORE, a, st);
      } else {
        s = solve(p, bd, RHS_GRESID, false, lastm ? OUT_GRAD : OUT_STORE, a, st);
      }
      if (s != SMNN_OK) return s;
    }
  }
  const Tracer tr{p, st};
  if (!p->rows)
    SMNN_LAUNCH(tr, a, SMNN_K_DW, 0, 0, 0, launch_dw_reduce(p->f32, bd.lev[0], a, p->dw_split, bd.dwq, st));
  SMNN_HIP(launch_info_finalize(a, info, st));
  return SMNN_OK;
}

namespace {

// Time one candidate: mean ms of forward + backward over `iters` calls.
smnn_status time_candidate(const smnn_plan_desc& d, const void* c, const void* b, const void* h, const void* u0,
                           const void* w, const void* gy, int iters, hipStream_t st, float* ms) {
  smnn_plan* p = nullptr;
  smnn_status s = smnn_plan_create(&d, &p);
  if (s != SMNN_OK) return s;
  const size_t io = p->f32 ? sizeof(float) : sizeof(double);
  const size_t S = static_cast<size_t>(p->S), K = static_cast<size_t>(p->K), N = static_cast<size_t>(p->N);
  void *y = nullptr, *fac = nullptr, *ws = nullptr, *dc = nullptr, *db = nullptr, *dh = nullptr, *du0 = nullptr,
       *dw = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    for (void* q : {y, fac, ws, dc, db, dh, du0, dw})
      if (q) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    smnn_plan_destroy(p);
  };
  const size_t QE = static_cast<size_t>(p->QE);
  const size_t ni = N * p->t_init * p->V * p->n_init;
  const size_t nw = p->rows ? S * QE + ni + S : N * 3;
  if (hipMalloc(&y, io * S * K) != hipSuccess || hipMalloc(&fac, p->factor_bytes) != hipSuccess ||
      hipMalloc(&ws, p->workspace_bytes) != hipSuccess || hipMalloc(&dc, io * S * QE * K) != hipSuccess ||
      hipMalloc(&db, io * S * QE) != hipSuccess || hipMalloc(&dh, io * S) != hipSuccess ||
      hipMalloc(&du0, io * (ni + 1)) != hipSuccess || hipMalloc(&dw, io * nw) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return SMNN_ERR_HIP;
  }
  auto step = [&]() -> smnn_status {
    smnn_status r = smnn_forward(p, c, b, h, u0, w, y, fac, p->factor_bytes, ws, p->workspace_bytes, nullptr, st);
    if (r != SMNN_OK) return r;
    return smnn_backward(p, c, b, h, u0, w, y, fac, p->factor_bytes, gy, dc, db, dh, du0, dw, ws,
                         p->workspace_bytes, nullptr, st);
  };
  s = step();  // warm-up
  if (s == SMNN_OK && hipEventRecord(e0, st) != hipSuccess) s = SMNN_ERR_HIP;
  for (int it = 0; it < iters && s == SMNN_OK; ++it) s = step();
  if (s == SMNN_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    s = SMNN_ERR_HIP;
  if (s == SMNN_OK) *ms /= static_cast<float>(iters);
  cleanup();
  return s;
}

}  // namespace

smnn_status smnn_autotune(const smnn_plan_desc* desc, const void* c, const void* b, const void* h,
                          const void* u0, const void* w, const void* gy, int32_t iters, void* stream,
                          smnn_tune_result* best, smnn_tune_result* all, int32_t cap, int32_t* n_all) {
  if (!desc || !c || !b || !h || !w || !gy || !best || iters < 1 || cap < 0) return SMNN_ERR_INVALID_ARG;
  if (desc->n_init > 0 && !u0) return SMNN_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int V = desc->variables > 0 ? desc->variables : 1;
  const int K = V * (desc->order + 1);
  const int form = form_id(V, desc->equations > 0 ? desc->equations : V, desc->row_weights != 0);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SMNN_ERR_HIP;
  int n = 0;
  smnn_tune_result cur{};
  cur.ms = -1.f;
  auto visit = [&](smnn_plan_desc d) -> smnn_status {
    if (!supported0(K, d.chunk, form) || !supported(K, d.chunk_upper)) return SMNN_OK;
    float ms = 0.f;
    const smnn_status s = time_candidate(d, c, b, h, u0, w, gy, iters, st, &ms);
    if (s == SMNN_ERR_UNSUPPORTED) return SMNN_OK;
    if (s != SMNN_OK) return s;
    smnn_tune_result r{d.chunk, d.chunk_upper, d.block, d.max_blocks, ms};
    if (all && n < cap) all[n] = r;
    ++n;
    if (cur.ms < 0.f || ms < cur.ms) cur = r;
    return SMNN_OK;
  };
  smnn_plan_desc d = *desc;
  d.block = d.block ? d.block : 64;
  const int chunks[] = {4, 8, 16};
  // 1. chunk lengths (level 0 x separator levels), default launch shape
  for (int l0 : chunks)
    for (int l1 : chunks) {
      d.chunk = l0;
      d.chunk_upper = l1;
      d.max_blocks = 0;
      const smnn_status s = visit(d);
      if (s != SMNN_OK) return s;
    }
  if (cur.ms < 0.f) return SMNN_ERR_UNSUPPORTED;
  // 2. workgroup size and persistent grid for the best chunk lengths
  d.chunk = cur.chunk;
  d.chunk_upper = cur.chunk_upper;
  const int blocks[] = {64, 128, 256};
  const int grids[] = {0, 2, 4, 8};
  for (int bl : blocks)
    for (int g : grids) {
      if (bl == cur.block && g == 0) continue;
      d.block = bl;
      d.max_blocks = g ? g * cus * (256 / bl) : 0;
      const smnn_status s = visit(d);
      if (s != SMNN_OK) return s;
    }
  *best = cur;
  if (n_all) *n_all = n;
  return SMNN_OK;
}

const char* smnn_status_string(smnn_status s) {
  switch (s) {
    case SMNN_OK: return "ok";
    case SMNN_ERR_INVALID_ARG: return "invalid argument";
    case SMNN_ERR_UNSUPPORTED: return "unsupported order or chunk length";
    case SMNN_ERR_WORKSPACE: return "workspace or factor too small";
    case SMNN_ERR_HIP: return "HIP runtime error";
    case SMNN_ERR_DEVICE: return "current device differs from the plan's device";
  }
  return "unknown status";
}

}  // extern "C"
