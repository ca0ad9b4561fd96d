/*
 * ttx -- out-of-place N-dimensional tensor transposition with scaling and
 * update on AMD Instinct MI355X (gfx950).
 *
 * Every entry point computes, for all multi-indices i of A,
 *
 *     B_{Pi(i0,...,iN-1)} <- alpha * A_{i0,...,iN-1} + beta * B_{Pi(i0,...,iN-1)}
 *
 * (Springer, Sankaran, Bientinesi, "TTC: A Tensor Transposition Compiler for
 * Multiple Architectures", Sec. 1, Eqn. 1).  Conventions shared by all calls:
 *
 *  - Layout: column-major (Fortran) storage, index 0 has stride 1 (Sec. 1,
 *    footnote 2).
 *  - perm[0..n-1] is a permutation of 0..n-1 in the gather reading of the
 *    paper's index notation: B's index k is A's index perm[k], so the
 *    extent of B's index k is size[perm[k]].  The merge example of Sec. 2.1,
 *    Pi(i0,i1,i2) = (i1,i2,i0), is perm = {1,2,0}.
 *  - size[m] >= 0 is the extent of A's index m.  Any zero extent makes the
 *    call a no-op that returns TTX_OK.
 *  - outer_a[m] / outer_b[k] are the per-index leading dimensions of Sec. 2.1
 *    (Table 1, Fig. 2): A and B may be sub-tensors of larger column-major
 *    tensors whose extents are outer_a (indexed by A position) and outer_b
 *    (indexed by B position).  Strides are strideA[m] = prod_{j<m} outer_a[j]
 *    and strideB[k] = prod_{j<k} outer_b[j].  NULL means the tensor is stored
 *    contiguously (outer = size).  outer < size is TTX_EINVAL.  Elements of
 *    the outer tensor of B outside the sub-tensor are never touched.
 *  - dtype selects FP32 or FP64 for both A and B (Sec. 2.1, Table 1 "s", "d").
 *  - alpha and beta are rounded once to the element type (round to nearest).
 *    When the rounded beta is zero (+0 or -0) B is written without being
 *    read (Sec. 1: with beta = 0 the output is overwritten), so NaN or Inf
 *    in B do not propagate.  Otherwise each element is computed as
 *    fl(fl(alpha*a) + fl(beta*b)): two rounded products and a rounded sum,
 *    never a fused multiply-add.
 *  - A and B (device pointers) must be aligned to the element size and the
 *    byte ranges they address must not overlap (the operation is
 *    out-of-place, Sec. 1): overlap is TTX_EOVERLAP.
 *  - 1 <= n <= TTX_MAX_DIMS.  Index arithmetic is 64-bit.
 *
 * Ownership: the caller owns A and B; the per-call and plan paths never
 * allocate device memory.  Calls that take a hipStream_t are asynchronous on
 * that stream; argument errors are reported synchronously before anything
 * is enqueued.  A failed launch is TTX_EHIP.  ttx_last_error() gives a
 * human-readable detail for the last failure on the calling thread.  All
 * entry points are thread-safe.
 */
#ifndef TTX_H
#define TTX_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTX_MAX_DIMS 16

typedef enum ttx_dtype { TTX_F32 = 0, TTX_F64 = 1 } ttx_dtype;

typedef enum ttx_status {
    TTX_OK = 0,
    TTX_EINVAL = 1,        /* bad argument: dtype, n, size, outer sizes, NULL pointer, option */
    TTX_EPERM = 2,         /* perm is not a permutation of 0..n-1 */
    TTX_EOVERLAP = 3,      /* the byte ranges addressed in A and B overlap */
    TTX_EUNSUPPORTED = 4,  /* valid request outside what the library implements */
    TTX_ENOMEM = 5,        /* a host or device allocation failed (tuner, batch, server only) */
    TTX_EHIP = 6,          /* a HIP runtime call or kernel launch failed */
    TTX_EBUSY = 7,         /* server: request refused by admission control */
    TTX_ENOTFOUND = 8      /* unknown ticket or table key */
} ttx_status;

/* Kernel families chosen by the planner (Sec. 2.2 and Sec. 3.2). */
typedef enum ttx_family {
    TTX_FAMILY_EMPTY = 0,      /* some extent is zero: nothing to do */
    TTX_FAMILY_FLAT = 1,       /* everything merged into one index: a strided axpby */
    TTX_FAMILY_PRESERVED = 2,  /* A's stride-1 index stays B's stride-1 index (Sec. 3.2) */
    TTX_FAMILY_MOVED = 3       /* the stride-1 index moves: LDS-staged 2D tiles (Sec. 2.2) */
} ttx_family;

/* Config flags. */
#define TTX_CFG_XCD_SWIZZLE 1  /* map consecutive tile ids onto one XCD */
#define TTX_CFG_NT_STORE 2     /* non-temporal (streaming) stores to B */

/* One implementation candidate (Sec. 2.2: blocking and loop order).
 *   tile_a  : tile extent along A's stride-1 index (merged index 0);
 *   tile_b  : MOVED: tile extent along B's stride-1 index;
 *             PRESERVED: rows per tile along B's second index;
 *             FLAT: elements per workgroup iteration (informational);
 *   threads : threads per workgroup;
 *   order   : the merged indices in the order tile ids enumerate them,
 *             fastest first (the "loop order" of Sec. 2.2); n_order entries;
 *   flags   : TTX_CFG_* bits. */
typedef struct ttx_config {
    int family;
    int tile_a;
    int tile_b;
    int threads;
    int n_order;
    int order[TTX_MAX_DIMS];
    int flags;
} ttx_config;

/* What the planner made of a problem (Sec. 2.1 stage 1 and the family split
 * of Sec. 3.2).  Dimensions are the merged ones, in A order. */
typedef struct ttx_plan_info {
    int dtype;
    int family;
    int n;                              /* merged rank (0 when EMPTY) */
    int perm[TTX_MAX_DIMS];             /* merged gather permutation */
    int64_t size[TTX_MAX_DIMS];         /* merged extents, A order */
    int64_t stride_a[TTX_MAX_DIMS];     /* A stride of merged index m */
    int64_t stride_b[TTX_MAX_DIMS];     /* B stride of merged index m (A order) */
    int64_t elements;                   /* prod(size) */
    int64_t extent_a_bytes;             /* bytes from A's first to one past its last element */
    int64_t extent_b_bytes;
    ttx_config config[2];               /* [0]: beta != 0, [1]: beta == 0 */
    int config_from_table[2];           /* 1 when the config came from the tune table */
} ttx_plan_info;

/* -- errors --------------------------------------------------------------- */
const char *ttx_status_string(ttx_status status);
/* Detail of the last failure on the calling thread ("" if none). */
const char *ttx_last_error(void);
const char *ttx_version(void);

/* -- per call (Eqn. 1) ------------------------------------------------------
 * B_{Pi(i)} <- alpha*A_i + beta*B_{Pi(i)} on `stream` (see the conventions
 * above).  Plans (index merging, family and config choice) are cached per
 * problem, so repeated calls with the same shape only launch. */
ttx_status ttx_transpose(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                         const int64_t *outer_a, const int64_t *outer_b,
                         double alpha, const void *A, double beta, void *B,
                         hipStream_t stream);

/* -- plans ------------------------------------------------------------------
 * A plan fixes dtype, perm, size and outer sizes (host work only: no HIP
 * call is made, so plans can be built and inspected without a GPU).  The
 * plan owns only host memory; destroy it with ttx_plan_destroy. */
typedef struct ttx_plan ttx_plan;

ttx_status ttx_plan_create(ttx_plan **plan, ttx_dtype dtype, int n, const int *perm,
                           const int64_t *size, const int64_t *outer_a, const int64_t *outer_b);
/* Runs the plan on A and B (Eqn. 1); B is read only when the rounded beta is non-zero. */
ttx_status ttx_plan_execute(const ttx_plan *plan, double alpha, const void *A, double beta,
                            void *B, hipStream_t stream);
/* Same, reading beta*B from B_in and writing the result to B_out (B_in may
 * equal B_out).  The arithmetic is identical to ttx_plan_execute. */
ttx_status ttx_plan_execute_split(const ttx_plan *plan, double alpha, const void *A, double beta,
                                  const void *B_in, void *B_out, hipStream_t stream);
ttx_status ttx_plan_describe(const ttx_plan *plan, ttx_plan_info *info);
/* Overrides the config used for beta == 0 (beta_is_zero = 1) or beta != 0.
 * The config must be one the planner accepts for this problem (its family,
 * a tile shape from the kernel menu, a permutation of the merged indices):
 * otherwise TTX_EINVAL.  Every accepted config computes the same bits. */
ttx_status ttx_plan_set_config(ttx_plan *plan, int beta_is_zero, const ttx_config *config);
ttx_status ttx_plan_destroy(ttx_plan *plan);
/* Name of the kernel ttx_plan_execute would launch for these pointers (the
 * vector variant depends on their alignment), e.g.
 * "k_moved<float, false, 64, 64, 4, 4>", as profilers print it; written
 * NUL-terminated into buf (len bytes).  Host only. */
ttx_status ttx_plan_kernel_name(const ttx_plan *plan, double beta, const void *A, const void *B,
                                char *buf, int len);

/* -- autotuner (Sec. 2.1 stages 2-6, Sec. 2.3) --------------------------------
 * Enumerates every candidate (tile shape from the kernel menu x loop order
 * x flags), ranks them with the blocking and loop-order heuristics, keeps
 * the best `max_candidates` (200 by default when 0 is passed; -1 keeps all,
 * as --maxImplementations=-1), times each on scratch buffers the tuner
 * allocates (minimum of `reps` runs, caches flushed before each run) and
 * stores the fastest in the in-process tune table, which later plans for
 * the same merged problem use.  *best receives the winner; *n_timed (may be
 * NULL) the number of candidates timed.  Needs a GPU; blocks the caller. */
ttx_status ttx_tune(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                    const int64_t *outer_a, const int64_t *outer_b, int beta_is_zero,
                    int max_candidates, int reps, ttx_config *best, int *n_timed);
/* The ranked candidate list (host only, no GPU): up to `cap` configs in
 * increasing estimated cost, with their estimated costs in cost[] (may be
 * NULL).  *count receives how many were written. */
ttx_status ttx_tune_candidates(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                               const int64_t *outer_a, const int64_t *outer_b,
                               int max_candidates, ttx_config *out, double *cost, int cap,
                               int *count);
/* Tune table persistence (one text line per entry) and reset. */
ttx_status ttx_tune_table_save(const char *path);
ttx_status ttx_tune_table_load(const char *path);
ttx_status ttx_tune_table_clear(void);
int ttx_tune_table_size(void);

/* -- measurement kernels --------------------------------------------------------
 * Bandwidth ceilings the transposition is compared with (Sec. 3: the peak is
 * the bandwidth of an optimised SAXPY).  Both are plain streaming kernels. */
/* dst[0..bytes) <- src[0..bytes); both 16-byte aligned, bytes % 16 == 0. */
ttx_status ttx_copy_kernel(const void *src, void *dst, int64_t bytes, hipStream_t stream);
/* y <- alpha*x + beta*y over n contiguous elements (unfused), 16-byte aligned. */
ttx_status ttx_axpby_kernel(ttx_dtype dtype, int64_t n, double alpha, const void *x,
                            double beta, void *y, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* TTX_H */
