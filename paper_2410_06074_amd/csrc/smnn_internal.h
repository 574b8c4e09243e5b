// Interface between the C-ABI host code (smnn_api.cpp) and the kernels
// (smnn_kernels.hip).  Internal; not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smnn {

// Device view of one level of the partition.
struct LevelDev {
  const int32_t* chunk_inst = nullptr;  // [chunks]
  const int64_t* chunk_off = nullptr;   // [N+1]
  const int64_t* node_off = nullptr;    // [N+1]
  const int64_t* chunk_step = nullptr;  // level 0: [chunks+1] global row of each chunk's first node
  int64_t chunks = 0, nodes = 0;
  double* rec = nullptr;                // level >= 1: [nodes][Q+KK] (in the factor buffer)
  double* rhs = nullptr;                // level >= 1: [nodes][K]    (workspace)
  double* x = nullptr;                  // level >= 1: [nodes][K]    (workspace)
};

// Level-0 (per time step) arrays of one call.  Element type is double or
// float (fp32 I/O form) for every pointer typed void.
struct Level0Args {
  const void* c = nullptr;   // [S][QE][K]
  const void* d = nullptr;   // [S][QE]
  const void* s = nullptr;   // [S]
  const void* u0 = nullptr;  // [N][t_init][V][n_init]
  const void* w = nullptr;   // [N][3]
  const void* g = nullptr;   // [S][K]  dl/dy
  const void* v = nullptr;   // [S][K]  previous iterate (refinement passes)
  void* out = nullptr;       // [S][K]  result (x, or v + x)
  const void* y = nullptr;   // [S][K]  forward solution (gradient pass)
  void* dc = nullptr;        // [S][QE][K]
  void* dd = nullptr;        // [S][QE]
  void* ds = nullptr;        // [S]
  void* du0 = nullptr;       // [N][t_init][V][n_init]
  double* dw_part = nullptr; // [chunks0][3] per-chunk partial sums
  void* dw = nullptr;        // [N][3]
  uint32_t* info = nullptr;  // [N] smallest failing step + 1 (UINT32_MAX = none)
  const void* wg = nullptr;  // per-row weights: [S][QE] governing,
  const void* wi = nullptr;  //   [N][t_init][V][n_init] initial,
  const void* ws = nullptr;  //   [S] smoothness (of the rows between points t and t+1)
  void* dwg = nullptr;       // their gradients, same layouts
  void* dwi = nullptr;
  void* dws = nullptr;
  int n_init = 0;
  int t_init = 1;            // points carrying initial values
  int L0 = 8, L1 = 8;        // chunk lengths of level 0 and of levels >= 1
  int64_t N = 0;
  mutable uint32_t* queue = nullptr;  // persistent launches: this launch's tile counter, one of
  uint32_t* queue_base = nullptr;     //   queue_slots counters zeroed at the start of the call,
  int queue_slots = 0;                //   handed out in launch order (queue_next)
  mutable int queue_next = 0;
  const int32_t* order = nullptr;  // [N] instances by decreasing T (one-wave-per-instance launches
                                   // of ragged batches; null: equal lengths)
  mutable int rev = 0;       // 1: take the tiles (instances) in decreasing order; the
                             // host flips it before every launch of a call
  int wpb = 1;               // waves per workgroup of the launch (set by the launcher)
  int64_t nwaves = 0;        // waves in the grid of the launch (set by the launcher)
};

struct Launch {
  int block = 256;      // threads per workgroup (multiple of 64)
  int max_blocks = 0;   // 0: one wave per tile; >0: persistent grid-stride cap
  int lds_max = 65536;  // LDS bytes a workgroup may allocate on the device
};

enum OutMode : int { OUT_STORE = 0, OUT_GRAD = 1 };

// Instance forms of the level-0 kernels (smnn_core.h Form): variables V,
// governing equations QE per point, per-row weights.
enum FormId : int {
  SMNN_FORM_SCALAR = 0,     // V = QE = 1, three scalar weights per instance
  SMNN_FORM_ROWS = 1,       // V = QE = 1, per-row weights
  SMNN_FORM_V2 = 2,         // V = QE = 2, scalar weights
  SMNN_FORM_V2_ROWS = 3,    // V = QE = 2, per-row weights
  SMNN_FORM_V2_Q1 = 4,      // V = 2, QE = 1, scalar weights
  SMNN_FORM_V3 = 5,         // V = QE = 3, scalar weights
  SMNN_FORM_V3_ROWS = 6     // V = QE = 3, per-row weights
};
// Form id of (V, QE, per-row weights), -1 if none is built.
inline int form_id(int V, int QE, bool rows) {
  if (V == 1 && QE == 1) return rows ? SMNN_FORM_ROWS : SMNN_FORM_SCALAR;
  if (V == 2 && QE == 2) return rows ? SMNN_FORM_V2_ROWS : SMNN_FORM_V2;
  if (V == 2 && QE == 1 && !rows) return SMNN_FORM_V2_Q1;
  if (V == 3 && QE == 3) return rows ? SMNN_FORM_V3_ROWS : SMNN_FORM_V3;
  return -1;
}

// Wide blocks (K > 5, smnn_wide.hip): one 16-lane group per chunk; separator
// records are full K x K blocks in the natural layout (WRec in smnn_wide.h:
// 3 K^2 doubles per node; right-hand sides 2 K).
bool wide_supported(int K, int L, int form);
hipError_t launch_wreduce0(int K, int L, int form, bool f32, int rhs_mode, bool write_rec, const LevelDev& l0,
                           const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st);
hipError_t launch_wbacksub0(int K, int L, int form, bool f32, int rhs_mode, int out_mode, const LevelDev& l0,
                            const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st);
hipError_t launch_wreduceN(int K, int L, bool write_rec, int level, const LevelDev& l, const LevelDev& lnext,
                           const Level0Args& a, const Launch& cfg, hipStream_t st);
hipError_t launch_wbacksubN(int K, int L, int level, const LevelDev& l, const LevelDev* lnext,
                            const Level0Args& a, const Launch& cfg, hipStream_t st);

// All return hipSuccess or the launch error.  K = V (R+1), L = chunk length,
// form = FormId of the level-0 kernels, f32 selects the float I/O form.
hipError_t launch_reduce0(int K, int L, int form, bool f32, int rhs_mode, bool write_rec, const LevelDev& l0,
                          const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st);
hipError_t launch_reduceN(int K, int L, bool write_rec, int level, const LevelDev& l, const LevelDev& lnext,
                          const Level0Args& a, const Launch& cfg, hipStream_t st);
hipError_t launch_backsubN(int K, int L, int level, const LevelDev& l, const LevelDev* lnext,
                           const Level0Args& a, const Launch& cfg, hipStream_t st);
hipError_t launch_backsub0(int K, int L, int form, bool f32, int rhs_mode, int out_mode, const LevelDev& l0,
                           const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st);
// Level-0 back-substitution of a solve with right-hand side rhs_in (beta or
// dl/dy), storing the iterate to a.out, fused with the level-0 reduce of the
// refinement solve that follows (residual or adjoint residual of that
// iterate; writes the level-1 right-hand sides only).
hipError_t launch_backsub_reduce0(int K, int L, int form, bool f32, int rhs_in, const LevelDev& l0,
                                  const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st);
// Levels >= level of a solve in one launch, one wave per instance (every
// instance must have at most 64 chunks at that level); writes that level's x.
// Lanes per instance of the one-launch upper levels (k_top): one wave per
// instance for blocks of up to 3 unknowns, 16 lanes (four instances per wave)
// for larger blocks.
constexpr int top_lanes(int K) { return K <= 3 ? 64 : 16; }
hipError_t launch_top(int K, int L, int level, const LevelDev& l, const Level0Args& a, const Launch& cfg,
                      hipStream_t st);
size_t top_lds_bytes(int K, int L);   // per wave
// Per-instance weight gradients from the per-chunk partials: `split`
// workgroups per instance (partial sums in `part`, [N][split][3], when > 1).
hipError_t launch_dw_reduce(bool f32, const LevelDev& l0, const Level0Args& a, int split, double* part,
                            hipStream_t st);
hipError_t launch_info_init(const Level0Args& a, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t st);

// LDS bytes one wave of a level-0 kernel stages its tile in (0 if (K, L) is
// not compiled in).  The largest variant of a mode is the gradient pass.
size_t level0_lds_bytes(int K, int L, int form, bool f32, int rhs_mode, int out_mode);
hipError_t launch_info_finalize(const Level0Args& a, int32_t* info, hipStream_t st);

bool supported(int K, int L);            // separator levels (and the scalar form at level 0)
bool supported0(int K, int L, int form);  // level-0 kernels of the form

// Name of a per-block-size launcher (smnn_kernels.hip is built once per K
// and group of instance forms).
#define SMNN_WFN_CAT2(a, b) a##_w##b
#define SMNN_WFN_CAT(a, b) SMNN_WFN_CAT2(a, b)
#define SMNN_WFN(name) SMNN_WFN_CAT(name, SMNN_TU_K)
#ifndef SMNN_TU_FORMS
#define SMNN_TU_FORMS 0
#endif
#if SMNN_TU_FORMS == 0
#define SMNN_KFN_CAT2(a, b) a##_k##b
#define SMNN_KFN_CAT(a, b) SMNN_KFN_CAT2(a, b)
#define SMNN_KFN(name) SMNN_KFN_CAT(name, SMNN_TU_K)
#else
#define SMNN_KFN_CAT2(a, b, g) a##_k##b##f##g
#define SMNN_KFN_CAT(a, b, g) SMNN_KFN_CAT2(a, b, g)
#define SMNN_KFN(name) SMNN_KFN_CAT(name, SMNN_TU_K, SMNN_TU_FORMS)
#endif

}  // namespace smnn
