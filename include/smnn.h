/*
 * smnn.h -- C-ABI of libsmnn: the batched linear-ODE least-squares solve of
 * Scalable Mechanistic Neural Networks (S-MNN), on AMD Instinct MI355X (gfx950).
 *
 * What is solved (Sec. 3.1, Eqs. 4-9; App. A.1-A.2).  An instance has T
 * time points, V variables (commonly one: a (batch element, variable) pair)
 * and unknowns y_{t,v,r}, r = 0..R (the r-th derivative of variable v at
 * point t).  Its weighted constraints are
 *   governing (Eq. 4):   sum_{v,r} c_{t,q,v,r} y_{t,v,r} = b_{t,q},
 *                        q = 1..Q equations per point       weight w_gov
 *   initial   (Eq. 5):   y_{t,v,r} = u0_{t,v,r}, t < T_init, r < n_init
 *                                                             weight w_init
 *                        (T_init = init_points; points past an instance's
 *                        last one carry no row)
 *   smoothness (Eqs. 6-7): forward and backward Taylor expansions of every
 *                        variable between points t and t+1 with step h_t,
 *                        every order r = 0..R, each row weighted by
 *                        w_smooth * h_t^r
 * (the weights are three scalars per instance, or one per row), and the
 * solution is the weighted least-squares minimiser (Eq. 9),
 *   y = (A^T W A)^{-1} A^T W b.
 * The normal matrix is block tridiagonal with V(R+1) x V(R+1) blocks (Eq. 10)
 * and is factored and solved in O(T) by block Cholesky with forward and back
 * substitution (Eqs. 11-13, Alg. 1, 3, 4).  The backward pass solves the
 * adjoint system of Eq. 14, lam = M^{-1} dl/dy, and forms the gradients with
 * respect to every input (Alg. 2 chained through App. A.2).
 *
 * Element types.  In SMNN_MODE_FP64 and SMNN_MODE_FP64_REFINED every array
 * argument is double.  In SMNN_MODE_FP32_REFINED every array argument is
 * float; the factorisation, substitutions and residuals still run in double
 * precision in registers, only memory traffic is single precision.
 *
 * Modes.
 *   SMNN_MODE_FP64          the paper's method: one block-Cholesky solve of
 *                           the normal equations (error ~ cond(M) * 2^-53).
 *   SMNN_MODE_FP64_REFINED  plus `refine_steps` steps of iterative refinement
 *                           whose residual A^T W (b - A y) is evaluated row by
 *                           row from the constraints (never as beta - M y), so
 *                           the result converges to the least-squares solution
 *                           at the accuracy of the constraint rows
 *                           (~cond(A) * 2^-53).  Same for the adjoint.
 *   SMNN_MODE_FP32_REFINED  FP32 inputs/outputs and intermediates in memory,
 *                           FP64 recurrence, refinement as above.
 *
 * Memory layout (all array pointers are DEVICE pointers).  Per-step arrays
 * are instance-major and time-contiguous: instance i owns rows
 * off[i] .. off[i]+T[i]-1, off = exclusive prefix sum of T, S = sum(T).
 * An instance has V variables (default 1) and Q governing equations per
 * point (default V); K = V (R+1) unknowns per point, variable-major:
 * unknown v (R+1) + r is derivative r of variable v (App. A.1's y_t).
 *   c   [S][Q][K]  governing coefficients c_{t,q,v,r}
 *   b   [S][Q]     governing right-hand sides d_{t,q}
 *   h   [S]        h[off[i]+t] = step between points t and t+1; the last slot
 *                  of each instance is read by nothing
 *   u0  [N][T_init][V][n_init]  initial values (point-major per instance)
 *   w   scalar weights (row_weights = 0): [N][3] (w_gov, w_init, w_smooth),
 *       unsquared, > 0, each applied to every row of its kind;
 *       per-row weights (row_weights = 1), unsquared, > 0, one buffer of
 *       S Q + N T_init V n_init + S elements: [S][Q] the weight of each
 *       governing row, then [N][T_init][V][n_init] the weight of each
 *       initial row, then [S] the weight of the smoothness rows between
 *       points t and t+1 (every variable and order; the row of order r is
 *       weighted by that weight times h_t^r), last slot of each instance
 *       unused (App. A.1's W = diag(w))
 *   y   [S][K]     solution; gy shares this shape, dc c's, db b's, dh h's;
 *                  du0 shares u0's (entries for points past an instance's
 *                  end are written as 0); dw shares w's (per-row weights:
 *                  the gradient of every row's weight, the unused slots 0).
 * For a uniform one-variable batch these are contiguous (N, T, R+1),
 * (N, T), ... arrays.  This natural layout is the only one: there is no
 * lane-tiled layout (instances interleaved across lanes) and so no pack,
 * unpack or layout-query calls.  The kernels give each wave a contiguous
 * range of steps, which they copy into LDS with coalesced loads before any
 * arithmetic, so the natural layout streams at the same rate a tiled one
 * would and the caller's tensors are used as they are.
 *
 * Ownership.  The caller allocates and owns every buffer.  `factor`
 * (smnn_plan_sizes) is written by smnn_forward and read by smnn_backward of
 * the same inputs; it must not change in between.  `workspace` is scratch
 * for one call at a time; calls that overlap in time need distinct
 * workspaces.  The library allocates device memory only in
 * smnn_plan_create (plan metadata) and frees it in smnn_plan_destroy.
 * smnn_forward / smnn_backward allocate nothing, synchronise nothing and
 * read nothing back, so they can always be captured into a hipGraph (the
 * counters some launches use are cleared by kernels, not memset nodes);
 * there is therefore no "not capturable" status.  smnn_autotune, which
 * times launches and synchronises, is a separate call made before capture.
 *
 * Errors.  Every call returns an smnn_status.  Argument errors are detected
 * on the host before anything is enqueued.  Numerical breakdown is reported
 * per instance through `info` (optional, device int32 [N]): 0 if every pivot
 * of that instance was > 0, else 1 + the time step (0-based) of a pivot that
 * was not (the smallest such step among those met), saturated at INT32_MAX
 * for steps beyond it; that instance's outputs are then NaN or Inf while the
 * other instances are unaffected.  Read `info` after synchronising the stream.
 */
#ifndef SMNN_H_
#define SMNN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SMNN_OK = 0,
  SMNN_ERR_INVALID_ARG = 1, /* bad size, mode, pointer or plan */
  SMNN_ERR_UNSUPPORTED = 2, /* order, chunk length or instance shape not compiled in */
  SMNN_ERR_WORKSPACE = 3,   /* workspace or factor smaller than required */
  SMNN_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
  SMNN_ERR_DEVICE = 5       /* called with another device current than at plan creation */
} smnn_status;

typedef enum {
  SMNN_MODE_FP64 = 0,
  SMNN_MODE_FP64_REFINED = 1,
  SMNN_MODE_FP32_REFINED = 2
} smnn_mode;

typedef struct smnn_plan smnn_plan; /* opaque; immutable after creation */

typedef struct {
  int32_t order;          /* R, 1..4.  Instance shapes built (else SMNN_ERR_UNSUPPORTED):
                             one variable, Q = 1, R = 1..4, scalar or per-row weights;
                             two variables, R = 1 with Q = 1 or 2 (scalar weights) or
                             Q = 2 (per-row weights), R = 2 with Q = 2; three
                             variables with Q = 3, R = 1 or 2 (per-row weights at R = 2).
                             Blocks of more than 5 unknowns (V (R+1) = 6, 9) run on
                             16-lane groups, chunk length 4 at every level */
  int32_t n_init;         /* initial orders fixed at each initial point, 0..R+1 */
  int64_t n_inst;         /* N >= 1 */
  const int64_t* steps;   /* HOST array [N] of T_i >= 1, or NULL: all T_i = steps_uniform */
  int64_t steps_uniform;
  int32_t mode;           /* smnn_mode */
  int32_t refine_steps;   /* refinement steps in the refined modes, 0..4; -1: default
                             (2 for SMNN_MODE_FP64_REFINED at order >= 3, else 1) */
  int32_t chunk;          /* nodes per lane at level 0 (time steps; 4, 8 or 16); 0: default for the order and
                             mode (float I/O at 3 x 3 and 4 x 4 blocks: 8 from 2^22 steps per batch on, else 4) */
  int32_t chunk_upper;    /* nodes per lane at the separator levels >= 1; 0: default for the order (3 x 3
                             blocks: 4 where the single upper-level launch then starts at the same level
                             as with 8, else 8); SMNN_Q_CHUNK / SMNN_Q_CHUNK_UPPER report the choice */
  int32_t block;          /* threads per workgroup (64..256, multiple of 64); 0: 64 */
  int32_t max_blocks;     /* >0: persistent launches of at most this many workgroups per
                             kernel, whose waves claim tiles from a device work queue
                             until none is left; 0: one wavefront per tile */
  int32_t init_points;    /* T_init: leading time points with initial values (Eq. 5); 0: 1.
                             N * T_init * V * n_init must not exceed INT32_MAX */
  int32_t variables;      /* V, coupled variables per instance (Sec. 3.1); 0: 1 */
  int32_t equations;      /* Q, governing equations per time point over all V (R+1)
                             unknowns (Eq. 4, App. A.2's C_t is Q x V(R+1)); 0: V */
  int32_t row_weights;    /* 0: w holds three scalar weights per instance;
                             1: w holds one weight per row (layout below) */
} smnn_plan_desc;

/* Create a plan on the current HIP device: validates the description,
 * builds the per-level partition of every instance and uploads its metadata.
 * *out receives the plan (NULL on error). */
smnn_status smnn_plan_create(const smnn_plan_desc* desc, smnn_plan** out);

/* Release the plan and its device metadata.  No call using it may be in flight. */
smnn_status smnn_plan_destroy(smnn_plan* plan);

/* Bytes of the factor and workspace buffers one forward/backward needs
 * (device memory, 256-byte aligned base required), and S = sum T_i. */
smnn_status smnn_plan_sizes(const smnn_plan* plan, size_t* factor_bytes, size_t* workspace_bytes,
                            int64_t* total_steps);

/* Introspection: SMNN_Q_LEVELS, SMNN_Q_CHUNK, SMNN_Q_CHUNK_UPPER, SMNN_Q_NODES(l),
 * SMNN_Q_CHUNKS(l), SMNN_Q_REFINE, SMNN_Q_MODE, SMNN_Q_INIT_POINTS, SMNN_Q_TOP_LEVEL.
 * Returns -1 for an unknown key. */
#define SMNN_Q_LEVELS 1
#define SMNN_Q_CHUNK 2
#define SMNN_Q_REFINE 3
#define SMNN_Q_MODE 4
#define SMNN_Q_CHUNK_UPPER 5
#define SMNN_Q_INIT_POINTS 6
#define SMNN_Q_TOP_LEVEL 7    /* first level solved by the one-wave-per-instance launch (0: none) */
#define SMNN_Q_NODES(l) (1000 + (l))
#define SMNN_Q_CHUNKS(l) (2000 + (l))
int64_t smnn_plan_query(const smnn_plan* plan, int32_t key);

/* Forward solve (Eq. 9; Alg. 1 with the factorisation of Alg. 3 and the
 * substitutions of Alg. 4).  Reads c, b, h, u0, w; writes y and factor;
 * uses workspace; optional info.  factor_bytes / workspace_bytes are the
 * sizes of the buffers passed; SMNN_ERR_WORKSPACE if either is below
 * smnn_plan_sizes, SMNN_ERR_INVALID_ARG if either base is not 256-byte aligned.  Enqueued on `stream` (a hipStream_t;
 * NULL = the null stream).  Asynchronous. */
smnn_status smnn_forward(const smnn_plan* plan, const void* c, const void* b, const void* h, const void* u0,
                         const void* w, void* y, void* factor, size_t factor_bytes, void* workspace,
                         size_t workspace_bytes, int32_t* info, void* stream);

/* Backward pass (Eq. 14, Alg. 2): given dl/dy = gy and the y and factor of
 * smnn_forward on the same inputs, solve lam = M^{-1} gy (with the same
 * refinement as the forward) and write dl/dc, dl/db, dl/dh (dh of each
 * instance's last slot is 0), dl/du0 and dl/dw.  Asynchronous. */
smnn_status smnn_backward(const smnn_plan* plan, const void* c, const void* b, const void* h, const void* u0,
                          const void* w, const void* y, const void* factor, size_t factor_bytes, const void* gy,
                          void* dc, void* db, void* dh, void* du0, void* dw, void* workspace,
                          size_t workspace_bytes, int32_t* info, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): smnn_forward
 * with its workspace taken from a static device array of the library
 * (SMNN_NOALLOC_WORKSPACE_MAX bytes, held on every device the library runs
 * on until the process ends) instead of a caller buffer.  Same kernels,
 * arguments and results as smnn_forward.  Returns SMNN_ERR_WORKSPACE when
 * the plan's workspace (smnn_plan_sizes) exceeds SMNN_NOALLOC_WORKSPACE_MAX,
 * SMNN_ERR_HIP if the array's device address cannot be obtained.  The call
 * itself allocates nothing (the address lookup happens once per device, at
 * the first call there).  Every call on a device shares that device's array:
 * calls that overlap in time on one device race and give undefined results;
 * serialise them (one stream, or events).  Nothing in the array needs to be
 * cleared between calls: every word a call reads it has written first. */
#define SMNN_NOALLOC_WORKSPACE_MAX (128u << 20)
smnn_status smnn_forward_noalloc(const smnn_plan* plan, const void* c, const void* b, const void* h,
                                 const void* u0, const void* w, void* y, void* factor, size_t factor_bytes,
                                 int32_t* info, void* stream);

/* Per-launch timing (profiling aid; not for concurrent or captured calls).
 * smnn_trace_enable(plan, n) makes the following smnn_forward/smnn_backward
 * calls on this plan record a hipEvent before and after each kernel launch,
 * for up to n launches (n = 0 turns tracing off and releases the events).
 * smnn_trace_read, after the stream has been synchronised, copies up to
 * `cap` records of the launches traced so far into `out`, returns how many
 * were written and clears the trace (-1 on error). */
typedef struct {
  int32_t kernel;  /* SMNN_K_* */
  int32_t level;   /* partition level the launch worked on */
  int32_t rhs;     /* right-hand side form: 0 beta, 1 residual, 2 dl/dy, 3 adjoint residual */
  int32_t out;     /* level-0 back-substitution: 0 stores a solution, 1 forms gradients */
  float ms;        /* elapsed time between the two events */
} smnn_trace_record;
#define SMNN_K_REDUCE0 1
#define SMNN_K_REDUCEN 2
#define SMNN_K_BACKSUBN 3
#define SMNN_K_BACKSUB0 4
#define SMNN_K_DW 5
#define SMNN_K_INFO 6
#define SMNN_K_BACKSUB_REDUCE0 7   /* level-0 back-substitution fused with the next solve's level-0 reduce */
#define SMNN_K_TOP 8               /* every separator level from `level` up, one wave per instance */
smnn_status smnn_trace_enable(smnn_plan* plan, int32_t capacity);
int32_t smnn_trace_read(smnn_plan* plan, smnn_trace_record* out, int32_t cap);

/* Autotuner.  Times smnn_forward + smnn_backward on the caller's inputs for
 * candidate launch mappings of `desc` -- chunk lengths (level 0 and the
 * separator levels), workgroup size and persistent grid size -- by a
 * coordinate search, and returns the fastest in *best (fields chunk,
 * chunk_upper, block, max_blocks; ms = mean time of one forward+backward).
 * Every candidate visited is written to all[0 .. *n_all-1] (up to cap).
 * Inputs are device arrays in desc's layout and element type; gy is dl/dy.
 * Unlike the solve calls this one allocates (temporary device buffers) and
 * synchronises `stream`; run it once, before capture, and create the plan
 * with the returned fields. */
typedef struct {
  int32_t chunk, chunk_upper, block, max_blocks;
  float ms;
} smnn_tune_result;
smnn_status smnn_autotune(const smnn_plan_desc* desc, const void* c, const void* b, const void* h,
                          const void* u0, const void* w, const void* gy, int32_t iters, void* stream,
                          smnn_tune_result* best, smnn_tune_result* all, int32_t cap, int32_t* n_all);

/* Static description of a status code. */
const char* smnn_status_string(smnn_status status);

#ifdef __cplusplus
}
#endif

#endif /* SMNN_H_ */
