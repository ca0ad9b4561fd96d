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
 *  - dtype selects the element types of A and B among those of the paper's
 *    type list (Sec. 2.1, Table 1): FP32, FP64, single and double complex
 *    stored as interleaved (re, im) pairs (8 and 16 bytes), or a
 *    mixed-precision pair (see ttx_dtype).
 *  - alpha and beta are rounded once to the element type (round to nearest;
 *    for complex types each part to the real part type).  When the rounded
 *    beta is zero (+0 or -0; complex: both parts) B is written without being
 *    read (Sec. 1: with beta = 0 the output is overwritten), so NaN or Inf
 *    in B do not propagate.  Otherwise each element is computed as
 *    fl(fl(alpha*a) + fl(beta*b)): two rounded products and a rounded sum,
 *    never a fused multiply-add.  A complex product s*x is formed as
 *    re = fl(fl(s.re*x.re) - fl(s.im*x.im)), im = fl(fl(s.re*x.im) +
 *    fl(s.im*x.re)), every product and sum rounded on its own, and the
 *    update adds the two products part by part.  The entry points that
 *    take double alpha, beta pass complex scalars with zero imaginary parts
 *    (the arithmetic above still applies); the *_c entry points take
 *    complex scalars as two doubles (re, im).
 *  - A and B (device pointers) must be aligned to their element sizes (8
 *    bytes for single complex, 16 for double complex) and the byte ranges they
 *    address must not overlap (the operation is out-of-place, Sec. 1):
 *    overlap is TTX_EOVERLAP.
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

/* Element types of A and B (Table 1 --dataType): s, d, c, z, and the
 * mixed-precision pairs sd, ds, cz, zc (A's type first).  With mixed
 * precision each A element is converted to B's type as it is loaded
 * (widening is exact; narrowing rounds to nearest, part by part for complex
 * elements), and the update is computed in B's type; alpha and beta are
 * rounded to B's type. */
typedef enum ttx_dtype {
    TTX_F32 = 0, TTX_F64 = 1, TTX_C32 = 2, TTX_C64 = 3,
    TTX_F32_F64 = 4,   /* sd: A FP32, B FP64 */
    TTX_F64_F32 = 5,   /* ds: A FP64, B FP32 */
    TTX_C32_C64 = 6,   /* cz: A single complex, B double complex */
    TTX_C64_C32 = 7    /* zc: A double complex, B single complex */
} ttx_dtype;

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
#define TTX_CFG_NT_STORE 2     /* non-temporal (streaming) stores to B (per-call kernels;
                                  the persistent batched kernel always stores plainly) */
#define TTX_CFG_DENSE 4        /* dense tiles (MOVED, or PRESERVED with index groups): tile_a x
                                  tile_b are run-time extents, rows of the shared stride-1 index
                                  (PRESERVED) are packed without padding, at most 1024 elements
                                  per tile, element-wise accesses */
#define TTX_CFG_WIDE 8         /* with TTX_CFG_DENSE, PRESERVED, FP32 or FP64 only: the kept
                                  stride-1 rows are moved in whole 16-byte units (8-byte units
                                  for FP32 rows that are not a multiple of 4 elements long):
                                  the row length and every other stride must be multiples of
                                  the unit, the row at least two units long; tile_a, tile_b,
                                  tile_c and the capacity count rows of units (512 units of 16
                                  bytes, 1024 of 8).  Pointers not aligned to the unit run an
                                  element-wise configuration instead. */
#define TTX_CFG_GROUPED 16     /* tile ids walk groups of 8 steps of the fastest grid index
                                  across the whole second one (in each plane of the two), so
                                  the tiles in flight together are neighbours along both */
#define TTX_CFG_ALIGN_A 32     /* MOVED menu tiles over a contiguous A run (stride 1): each
                                  tile's range along A's stride-1 index starts on a 128-byte
                                  line of A in the row of its first B-side index (one more
                                  tile along that index covers the shift), so runs whose
                                  length is not a multiple of the line cost whole lines;
                                  runs as a size-specialised kernel */
#define TTX_CFG_PIPELINED 64   /* MOVED or PRESERVED tiles, not dense: a persistent grid of as
                                  many workgroups as the device holds at once, each looping
                                  over its tiles and issuing the next tile's loads before the
                                  current tile's stores; runs as a size-specialised kernel */

/* One implementation candidate (Sec. 2.2: blocking and loop order).
 *   tile_a  : tile extent along A's stride-1 index (merged index 0);
 *   tile_b  : MOVED: tile extent along B's stride-1 index;
 *             PRESERVED: rows per tile along B's second index;
 *             FLAT: elements per workgroup iteration (informational);
 *   threads : threads per workgroup: 64, 128, 256 or 512 (flat problems: 256);
 *   order   : the merged indices in the order tile ids enumerate them,
 *             fastest first (the "loop order" of Sec. 2.2); n_order entries;
 *   flags   : TTX_CFG_* bits;
 *   group_a/b: index groups that extend the 2D tile when stride-1 extents
 *             are short (1 = the single index).  MOVED: A's first group_a
 *             and B's first group_b merged indices.  PRESERVED with groups
 *             (short rows): tiles hold whole rows of the shared stride-1
 *             index times A's next group_a-1 and B's next group_b-1 indices;
 *             tile_a and tile_b then count rows along those super indices.
 *   With TTX_CFG_DENSE, tile_a and tile_b may be any positive extents with
 *   rows x tile_a x tile_b x tile_c within the dense capacity (rows = the row
 *   length for PRESERVED, 1 for MOVED);
 *   tile_c  : dense tiles only -- extent along a third index, the first index
 *             of `order` that is neither a tile index nor a group member, so
 *             that one tile holds several small planes (0 or 1: one plane);
 *   lds_pad : elements appended to each row of an LDS-staged tile (MOVED menu
 *             tiles and PRESERVED tiles with groups): 0..TTX_MAX_LDS_PAD; the
 *             row of a moved tile holds tile_a + lds_pad elements.  Ignored by
 *             tiles that do not pass through LDS with fixed rows (direct
 *             PRESERVED rows, dense tiles, FLAT).
 * The library holds pre-compiled kernels for threads = 256 and lds_pad = 1
 * over the menu tile shapes (ttx_tile_shapes); a configuration with other
 * values, a run-time-only large tile, TTX_CFG_ALIGN_A or TTX_CFG_PIPELINED
 * runs a size-specialised kernel compiled at run time (hipRTC) on first use,
 * with the same arithmetic. */
#define TTX_MAX_LDS_PAD 4
typedef struct ttx_config {
    int family;
    int tile_a;
    int tile_b;
    int threads;
    int n_order;
    int order[TTX_MAX_DIMS];
    int flags;
    int group_a;   /* index groups, see above (1 = the single index) */
    int group_b;
    int tile_c;    /* dense tiles: planes per tile along the third index (0 or 1: one) */
    int lds_pad;   /* LDS row padding of staged tiles, in elements (see above) */
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
    int specialised[2];                 /* 1 when a size-specialised kernel is attached */
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
/* The same with complex alpha and beta (Eqn. 1 over the c and z types of
 * Sec. 3): alpha[0..1] and beta[0..1] are (re, im), host pointers read
 * before the call returns.  For TTX_F32 and TTX_F64 the imaginary parts
 * must be zero (else TTX_EINVAL). */
ttx_status ttx_transpose_c(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                           const int64_t *outer_a, const int64_t *outer_b,
                           const double *alpha, const void *A, const double *beta, void *B,
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
/* ttx_plan_execute_split with complex alpha and beta, (re, im) pairs as in
 * ttx_transpose_c. */
ttx_status ttx_plan_execute_c(const ttx_plan *plan, const double *alpha, const void *A,
                              const double *beta, const void *B_in, void *B_out,
                              hipStream_t stream);
ttx_status ttx_plan_describe(const ttx_plan *plan, ttx_plan_info *info);
/* Overrides the config used for beta == 0 (beta_is_zero = 1) or beta != 0.
 * The config must be one the planner accepts for this problem (its family,
 * a tile shape from the kernel menu, a permutation of the merged indices):
 * otherwise TTX_EINVAL.  Every accepted config computes the same bits. */
ttx_status ttx_plan_set_config(ttx_plan *plan, int beta_is_zero, const ttx_config *config);
ttx_status ttx_plan_destroy(ttx_plan *plan);
/* Name of the kernel ttx_plan_execute would launch for these pointers (the
 * vector variant depends on their alignment), e.g.
 * "k_moved<float, false, 64, 64, 4, 4, false>" (the last argument: nontemporal
 * stores), or the name of the plan's size-specialised kernel when that one
 * would run ("ttx_jit_moved_float_b_64x64_1a2b3c4d"), as profilers print it;
 * written NUL-terminated into buf (len bytes).  Host only. */
ttx_status ttx_plan_kernel_name(const ttx_plan *plan, double beta, const void *A, const void *B,
                                char *buf, int len);

/* -- size-specialised kernels (Sec. 2.1) -------------------------------------
 * A solution generated by the paper's compiler carries the sizes of its
 * transposition as compile-time constants (known trip counts); the
 * pre-instantiated kernels here take them as run-time arguments instead.
 * ttx_plan_specialise compiles, at run time with hipRTC, the plan's kernel
 * for one beta class (beta_is_zero = 1: beta == 0) with every extent,
 * stride, tile count and index divisor of the plan's problem and config as
 * a constant, and loads it on the current device.  When the tune table
 * holds a configuration tuned for specialised execution of the problem
 * (ttx_tune_specialised) and no config was set on the plan, the plan takes
 * it for that beta class first.
 *   reps == 0: the kernel is attached to the plan;
 *   reps > 0:  the generic and the specialised kernel are timed on scratch
 *              tensors the call allocates (minimum of `reps` runs each,
 *              caches flushed before each run, as ttx_tune does), and the
 *              specialised kernel is attached only when it is more than 1%
 *              faster (stage 5 of Sec. 2.1 over the two variants).
 * *kept (may be NULL) receives 1 when a kernel was attached.  Later
 * executions of the plan in that beta class, on that device, launch it
 * when the tensors are aligned as for the plan's vector paths (16 bytes
 * suffices; hipMalloc'd tensors are); other executions use the generic
 * kernel.  Both compute the same bits.  Moved- and preserved-family
 * problems only: for empty and single-index problems nothing is attached
 * (TTX_OK, no GPU call).  A call replaces the plan's earlier specialised
 * kernel of that beta class; ttx_plan_set_config drops it.  Kernels stay
 * loaded until the process ends and are shared by plans of the same
 * problem; when the environment variable TTX_JIT_CACHE names a directory,
 * code objects are also kept there (created if missing) and reused by
 * later processes.  Needs a GPU; blocks the caller (about half a second to
 * compile).  Errors: TTX_EINVAL (NULL plan), TTX_EHIP (compilation or
 * loading failed; ttx_last_error starts with the compiler log), TTX_ENOMEM
 * (timing scratch). */
ttx_status ttx_plan_specialise(ttx_plan *plan, int beta_is_zero, int reps, int *kept);
/* Automatic specialisation for the per-call entry points (ttx_transpose,
 * ttx_transpose_c): a shape's size-specialised kernel is compiled at its
 * `calls`-th call in a beta class (the hottest shapes get one; a failed
 * compilation leaves the shape on its generic kernel), 0 turns it off (the
 * default, or the value of the environment variable TTX_AUTO_SPECIALISE at
 * the first call).  The compiling call blocks for about half a second; a
 * call running concurrently on the same shape may still take the generic
 * kernel.  TTX_EINVAL for calls < 0. */
ttx_status ttx_set_auto_specialise(int calls);
/* The per-call entry points' plan cache: *plans (may be NULL) receives the
 * number of cached shapes, *specialised (may be NULL) how many of them have a
 * size-specialised kernel.  Host only. */
ttx_status ttx_transpose_cache_info(int *plans, int *specialised);
/* The translation unit ttx_plan_specialise compiles for the plan (host
 * only), NUL-terminated into buf (len bytes).  TTX_EINVAL when buf is too
 * small (about 8 KB suffices) or the problem has nothing to specialise. */
ttx_status ttx_plan_specialised_source(const ttx_plan *plan, int beta_is_zero, char *buf, int len);

/* -- autotuner (Sec. 2.1 stages 2-6, Sec. 2.3) --------------------------------
 * Enumerates every candidate (tile shape from the kernel menu x loop order
 * x flags), ranks them with the blocking and loop-order heuristics, keeps
 * the best `max_candidates` (200 by default when 0 is passed; -1 keeps all,
 * as --maxImplementations=-1), times each on scratch buffers the tuner
 * allocates (minimum of `reps` runs, caches flushed before each run) and
 * stores the fastest in the in-process tune table, which later plans for
 * the same merged problem use.  A second stage then times the workgroup
 * variants (ttx_tune_variants: threads per workgroup, LDS row padding) of
 * the TTX_TUNE_VARIANT_BASES fastest blockings of the first, each compiled
 * at run time when it is not a pre-compiled kernel.  *best receives the
 * winner; *n_timed (may be NULL) the number of candidates timed in both
 * stages.  Needs a GPU; blocks the caller. */
#define TTX_TUNE_VARIANT_BASES 2
ttx_status ttx_tune(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                    const int64_t *outer_a, const int64_t *outer_b, int beta_is_zero,
                    int max_candidates, int reps, ttx_config *best, int *n_timed);
/* ttx_tune with every kept candidate compiled at run time as a
 * size-specialised kernel (see ttx_plan_specialise) and timed in that form,
 * as the paper's compiler compiles and times each candidate (Sec. 2.1
 * stages 4 and 5): max_candidates defaults to 24 when 0 is passed (each
 * candidate costs a compilation of about half a second; -1 keeps all).
 * The fastest config goes into the tune table's entries for specialised
 * execution (the generic entry is left alone): ttx_plan_specialise takes
 * it.  Empty and single-index problems take the generic search.  Needs
 * a GPU; blocks the caller.  Errors as ttx_tune, and TTX_EHIP when a
 * compilation fails. */
ttx_status ttx_tune_specialised(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                                const int64_t *outer_a, const int64_t *outer_b, int beta_is_zero,
                                int max_candidates, int reps, ttx_config *best, int *n_timed);
/* The ranked candidate list (host only, no GPU): up to `cap` configs in
 * increasing estimated cost, with their estimated costs in cost[] (may be
 * NULL).  *count receives how many were written. */
ttx_status ttx_tune_candidates(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                               const int64_t *outer_a, const int64_t *outer_b,
                               int max_candidates, ttx_config *out, double *cost, int cap,
                               int *count);
/* The workgroup variants of one config (host only, no GPU): the same
 * blocking, loop order and flags with each valid threads-per-workgroup value
 * (64, 128, 256, 512), for LDS-staged tiles each LDS row padding
 * 0..TTX_MAX_LDS_PAD, and for moved menu tiles over a contiguous A run
 * TTX_CFG_ALIGN_A both set and clear, every combination once, the given
 * config first.  A
 * variant is valid when the tile's rows and vectors fit the workgroup and
 * each thread holds at most 32 vectors per side.  These are the second
 * search stage of ttx_tune and ttx_tune_specialised, around the measured
 * best blockings (Sec. 2.2: blockings and loop orders, extended here by the
 * workgroup shape and the shared-memory layout of Sec. 2.3).  Up to `cap`
 * configs are written; *count receives how many. */
ttx_status ttx_tune_variants(ttx_dtype dtype, int n, const int *perm, const int64_t *size,
                             const int64_t *outer_a, const int64_t *outer_b, const ttx_config *base,
                             ttx_config *out, int cap, int *count);
/* The tile shapes of a kernel family (TTX_FAMILY_MOVED or
 * TTX_FAMILY_PRESERVED) for a dtype (B's type of a mixed code): with
 * run_time_only = 0 the pre-compiled menu (Sec. 2.2 blockings); with
 * run_time_only = 1 the larger moved-family tiles that exist only as
 * size-specialised kernels compiled at run time (256- to 512-byte runs on
 * both sides; valid in any config of a moved problem, which then always
 * runs its run-time compiled kernel).  Up to `cap` shapes go to tile_a[],
 * tile_b[]; *count receives how many there are. */
ttx_status ttx_tile_shapes(ttx_dtype dtype, int family, int run_time_only, int *tile_a, int *tile_b, int cap,
                           int *count);
/* Tune table persistence (one text line per entry) and reset. */
ttx_status ttx_tune_table_save(const char *path);
ttx_status ttx_tune_table_load(const char *path);
ttx_status ttx_tune_table_clear(void);
int ttx_tune_table_size(void);
/* A table file as a solution database shared across processes (Sec. 2.1:
 * the database is consulted before any search and keeps every solution):
 * its entries are merged into the table, keeping the lowest time per key
 * (the file is created when missing), and from then on every tuning result
 * is also appended to it as one line under an exclusive file lock.  The
 * environment variable TTX_TUNE_DB attaches a file before the table is
 * first used, and TTX_TUNE_TABLE names a table file that is only read then
 * (the shipped per-architecture table, for instance).  Detach stops the
 * appending (the table keeps its entries). */
ttx_status ttx_tune_db_attach(const char *path);
ttx_status ttx_tune_db_detach(void);

/* -- GEMM operand packing (Sec. 2.1, Fig. 3) -----------------------------------------
 * Packing for a GEMM kernel is a transposition of the matrix viewed as a 3D
 * tensor: the index cut into panels becomes two indices (position inside the
 * panel, panel number), and the panel number moves outermost.  A is a
 * column-major rows x cols matrix with leading dimension ld (>= rows),
 * elements of A's type of dtype; P receives the panels, elements of B's
 * type (mixed-precision codes pack into another precision), every element
 * scaled by alpha = (alpha[0], alpha[1]) as in ttx_transpose_c with beta = 0:
 *   TTX_PACK_ROWS (the left operand): panels of `panel` = mr rows; panel p
 *     is an mr x cols column-major block, P[i + c*mr + p*mr*cols] =
 *     alpha * A[(p*mr + i) + c*ld] (the view (mr, rows/mr, cols) with perm
 *     (0,2,1), Fig. 3);
 *   TTX_PACK_COLS (the right operand): panels of `panel` = nr columns;
 *     panel p holds rows of nr contiguous elements,
 *     P[j + r*nr + p*nr*rows] = alpha * A[r + (p*nr + j)*ld] (the view
 *     (rows, nr, cols/nr) with perm (1,0,2)).
 *   TTX_PACK_MFMA_A / TTX_PACK_MFMA_B: matrix-core operand panels, the two
 *     layouts above with the k extent of every panel (cols for _A, rows for
 *     _B) padded with zeros to K = a multiple of kb = 64 / panel (panel must
 *     divide 64): P[l + 64*b + p*panel*K] holds element (l mod panel, b*kb +
 *     l div panel) of panel p -- the operand of the b-th 64-lane matrix
 *     instruction of shape panel x panel x kb, lane l's register (16 x 16 x 4
 *     for FP32 and FP64, 32 x 32 x 2 for FP32; ttx_gemm_panels reads them).
 * A ragged last panel is padded with zeros; P holds ceil(extent/panel) *
 * panel * other elements (other rounded up to K for the matrix-core kinds).
 * A and P are device pointers aligned to their
 * element sizes whose byte ranges must not overlap (TTX_EOVERLAP).  Plans
 * are cached per (dtype, kind, rows, cols, ld, panel); the transpositions
 * use the tune table (ttx_pack_tune fills it).  Asynchronous on `stream`. */
typedef enum ttx_pack_kind {
    TTX_PACK_ROWS = 0, TTX_PACK_COLS = 1, TTX_PACK_MFMA_A = 2, TTX_PACK_MFMA_B = 3
} ttx_pack_kind;

ttx_status ttx_pack(ttx_dtype dtype, int kind, int64_t rows, int64_t cols, int64_t ld, int64_t panel,
                    const double *alpha, const void *A, void *P, hipStream_t stream);
/* Tunes the transpositions a packing runs (as ttx_tune does; blocks). */
ttx_status ttx_pack_tune(ttx_dtype dtype, int kind, int64_t rows, int64_t cols, int64_t ld,
                         int64_t panel, int max_candidates, int reps);
/* Host only: the packed element count, the number of transpositions (1 or 2;
 * 0 when empty) and their configs (configs[0..1], may be NULL). */
ttx_status ttx_pack_describe(ttx_dtype dtype, int kind, int64_t rows, int64_t cols, int64_t ld,
                             int64_t panel, int64_t *packed_elements, int *transpositions,
                             ttx_config *configs);
/* C = A * B from matrix-core operand panels: Pa holds the m x k left operand
 * packed with TTX_PACK_MFMA_A, Pb the k x n right operand packed with
 * TTX_PACK_MFMA_B, both with the same `panel`; C is a column-major m x n
 * matrix with leading dimension ldc >= m, overwritten.  The consumer of the
 * packed operands that Sec. 2.1 (Fig. 3) prepares, and the contraction step
 * of a transpose-transpose-GEMM-transpose tensor contraction (Sec. 4): each
 * wave computes a panel x panel block with the gfx950 matrix instructions
 * (16 x 16 x 4 FP32 or FP64 for panel 16, 32 x 32 x 2 FP32 for panel 32),
 * reading each instruction's operands as 64 consecutive panel elements.
 * dtype TTX_F32 (panel 16 or 32) or TTX_F64 (panel 16), else
 * TTX_EUNSUPPORTED.  The products are summed by the matrix cores in the
 * element type (the summation order is the hardware's: results equal a
 * reference GEMM exactly only where no rounding occurs, e.g. small
 * integers).  Device pointers aligned to the element size; asynchronous on
 * `stream`. */
ttx_status ttx_gemm_panels(ttx_dtype dtype, int panel, int64_t m, int64_t n, int64_t k, const void *Pa,
                           const void *Pb, void *C, int64_t ldc, hipStream_t stream);

/* -- tensor contraction: transpose-transpose-GEMM-transpose (Sec. 1, Sec. 4) -----------
 * A contraction cast as a matrix product by transpositions, the use Sec. 1
 * gives for a fast transposition and the compiler Sec. 4 builds on it:
 *   C[c] <- alpha * sum over the contracted labels of A[a] * B[b] + beta * C[c]
 * A, B and C are column-major tensors (first mode fastest, contiguous) whose
 * modes carry integer labels: a label carried by A and B only is contracted
 * (its extents multiply to k); every label of C is carried by exactly one
 * operand (A's make m, B's make n).  Labels carried by all three tensors
 * (batch labels), twice by one tensor, or by one tensor only are
 * TTX_EINVAL, and so are extents that differ for one label.  na, nb, nc
 * are in 0..TTX_MAX_DIMS (0: a scalar).
 *
 * Execution: each operand that is not already a matrix (its free modes and
 * its contracted modes in two contiguous blocks, in either order, with the
 * contracted modes in the order the other operand uses) is transposed into
 * one (ttx_plan_execute); both are packed into matrix-core panels
 * (ttx_pack, TTX_PACK_MFMA_A or _B, whichever reads the matrix in its
 * storage order); ttx_gemm_panels forms the m x n product; and one
 * transposition writes alpha * product + beta * C into C's mode order
 * (Eqn. 1, so beta == 0 never reads C).  The product is summed in the
 * element type by the matrix cores (see ttx_gemm_panels); alpha and beta
 * are applied once, in the last step.  dtype TTX_F32 or TTX_F64 (else
 * TTX_EUNSUPPORTED).
 *
 * The plan holds host memory only (no HIP call at creation).  Execution
 * needs a device workspace of ttx_contraction_describe's workspace_bytes
 * (at most (2*m*k + 2*k*n + m*n) elements plus panel padding), passed by
 * the caller: the library allocates nothing.  A, B, C and the workspace
 * are device pointers aligned to the element size; C's byte range must not
 * overlap A's or B's, and the workspace's must overlap none of them
 * (TTX_EOVERLAP).  Asynchronous on `stream`; calls that share a workspace
 * must not overlap in time. */
typedef struct ttx_contraction ttx_contraction;
typedef struct ttx_contraction_info {
    int64_t m, n, k;            /* the matrix product's extents */
    int panel;                  /* matrix-core panel (16 or 32) */
    int transposed_a;           /* 1: A is transposed into matrix order before packing */
    int transposed_b;
    int pack_kind_a;            /* TTX_PACK_MFMA_A or TTX_PACK_MFMA_B (A stored contracted-major) */
    int pack_kind_b;            /* TTX_PACK_MFMA_B, or TTX_PACK_MFMA_A (B stored free-major) */
    int n_m, n_n, n_k;          /* label counts of the three index groups */
    int order_m[TTX_MAX_DIMS];  /* labels of the product's rows, fastest first */
    int order_n[TTX_MAX_DIMS];  /* labels of its columns */
    int order_k[TTX_MAX_DIMS];  /* contracted labels in the order both packed operands use */
    int64_t workspace_bytes;
} ttx_contraction_info;

ttx_status ttx_contraction_create(ttx_contraction **plan, ttx_dtype dtype, int na, const int *labels_a,
                                  const int64_t *size_a, int nb, const int *labels_b, const int64_t *size_b,
                                  int nc, const int *labels_c, const int64_t *size_c);
ttx_status ttx_contraction_describe(const ttx_contraction *plan, ttx_contraction_info *info);
ttx_status ttx_contraction_execute(const ttx_contraction *plan, double alpha, const void *A, const void *B,
                                   double beta, void *C, void *workspace, hipStream_t stream);
ttx_status ttx_contraction_destroy(ttx_contraction *plan);

/* -- batched execution ----------------------------------------------------------
 * Many independent transpositions, each Eqn. 1 with its own dtype, shape,
 * permutation, leading dimensions, scalars and tensors, run by ONE
 * persistent kernel launch: the planner splits every problem into tiles
 * (Sec. 2.2 macro-tiles), the kernel's workgroups walk the combined tile
 * space through a device-resident descriptor table, and the launch is
 * captured once into a HIP graph and replayed by ttx_batch_execute.  Each
 * problem's tile variant comes from a small menu compiled into that kernel:
 * the per-shape tune table when ttx_batch_tune has timed it, otherwise the
 * heuristics of Sec. 2.3.  Problems of the complex and mixed-precision
 * types are not in that kernel: each runs its per-call kernel (per-call
 * tune table, else heuristics), launched after the persistent kernel in the
 * same graph.  Results are bitwise the same as per-call execution (the same
 * tile code and operation order). */
typedef struct ttx_problem {
    ttx_dtype dtype;
    int n;
    int perm[TTX_MAX_DIMS];
    int64_t size[TTX_MAX_DIMS];
    int64_t outer_a[TTX_MAX_DIMS];   /* read when has_outer_a != 0 */
    int64_t outer_b[TTX_MAX_DIMS];   /* read when has_outer_b != 0 */
    int has_outer_a;
    int has_outer_b;
    double alpha;
    double beta;
    const void *A;
    const void *B_in;                /* beta*B is read from here; NULL means B */
    void *B;                         /* result */
    double alpha_im;                 /* imaginary parts of alpha and beta (complex types; */
    double beta_im;                  /* zero for the real ones) */
} ttx_problem;

typedef struct ttx_batch_info {
    int count;
    int grid;                        /* workgroups of the persistent launch */
    int variants_used;               /* distinct tile variants among the problems */
    int tuned;                       /* problems whose config came from tuning */
    int64_t total_tiles;
    int64_t algorithmic_bytes;       /* sum of 2S (beta == 0) or 3S bytes */
    int64_t chunks;                  /* units of work claimed by the workgroups: runs of up to
                                        a fixed number of consecutive tiles of one problem */
    int per_call;                    /* problems launched with their per-call kernels (complex
                                        and mixed-precision types) */
} ttx_batch_info;

typedef struct ttx_batch ttx_batch;

/* Plans all problems and uploads the descriptor table (the batch owns that
 * device memory; the caller owns every A and B).  Every problem is checked
 * as ttx_transpose would check it; the first failure is returned. */
ttx_status ttx_batch_create(ttx_batch **batch, int count, const ttx_problem *problems);
/* Times the current config and up to max_candidates batched-menu configs
 * per distinct shape (0: 16) inside the persistent kernel on scratch
 * buffers, one problem at a time; another config replaces the current one
 * only when it is at least 5% faster.  The tuned set is then checked in
 * context: the whole persistent launch is timed with it and with the
 * configs it replaced, alternately, on scratch buffers the size of the
 * batch's footprint (the caller's tensors are not touched), and the kernel
 * problems keep the tuned set only when it is at least 1% faster (else they
 * return to their previous configs and this call's table entries are
 * withdrawn; without the scratch memory the check is skipped).  Winners go
 * into a process-wide per-shape table; the descriptors are rebuilt.
 * Blocks: waits for the device to be idle first (earlier launches of the
 * batch may still be reading its descriptors). */
ttx_status ttx_batch_tune(ttx_batch *batch, int max_candidates, int reps);
/* One graph launch of the persistent kernel on `stream` (captured on first use).
 * Launches of one batch must not overlap each other (they share the batch's
 * work counter and outputs): order them on one stream or synchronise. */
ttx_status ttx_batch_execute(ttx_batch *batch, hipStream_t stream);
/* The same persistent kernel launched directly (no graph). */
ttx_status ttx_batch_execute_direct(ttx_batch *batch, hipStream_t stream);
/* New pointers and scalars for problems of unchanged shape; the copy to the
 * descriptor table is ordered on `stream` and completes before returning. */
ttx_status ttx_batch_update(ttx_batch *batch, int count, const ttx_problem *problems,
                            hipStream_t stream);
ttx_status ttx_batch_get_info(const ttx_batch *batch, ttx_batch_info *info);
/* The config problem `index` runs with. */
ttx_status ttx_batch_config(const ttx_batch *batch, int index, ttx_config *config);
ttx_status ttx_batch_destroy(ttx_batch *batch);
/* Host-only planning of `count` problems as ttx_batch_create would plan them
 * (no HIP call, no device memory): the config and tile count of each (the
 * tile count is 0 for problems launched with their per-call kernels). */
ttx_status ttx_batch_plan(int count, const ttx_problem *problems, ttx_config *configs,
                          int64_t *tiles);

/* Allocation-free batched run, for callers that cannot allocate device
 * memory (serving loops that must not call hipMalloc, harnesses that forbid
 * it).  Computes what ttx_batch_create + ttx_batch_execute + ttx_batch_destroy
 * compute for the same problems, with the same configs and the same
 * persistent kernel, bit for bit, but allocates no device memory: the work
 * block (descriptor table, chunk prefix, claim counter) is a static per-GPU
 * array of about 1 MiB that the library holds until the process ends.
 * count <= TTX_STATIC_BATCH_MAX, else TTX_EINVAL and nothing runs.  The
 * caller owns every A and B; each problem is checked as ttx_transpose
 * checks it and the first failure is returned before anything is launched.
 * Asynchronous on `stream`: the descriptors are copied from host memory to
 * the array on `stream` (the host copy has been read when the call returns),
 * then the kernel and any per-call launches (complex and mixed-precision
 * problems) follow on the same stream.  Every call on a GPU shares that
 * GPU's array: calls ordered on one stream are safe, calls that may overlap
 * on one GPU (different streams without synchronisation, several threads)
 * race and give wrong results.  The copy comes from pageable host memory,
 * so the call is not for use under stream capture. */
#define TTX_STATIC_BATCH_MAX 1024
ttx_status ttx_batch_run_static(int count, const ttx_problem *problems, hipStream_t stream);

/* -- serving ----------------------------------------------------------------------
 * A request loop with continuous batching.  Requests (one Eqn. 1 each) are
 * admitted in arrival order while the sum of the HBM footprints of admitted,
 * unreleased requests stays within the budget (hbm_fraction of the device
 * memory free at creation; footprint = bytes of the A and B_in sub-tensor
 * extents plus the output).  An admitted request whose problem.B is NULL gets
 * its output in a server-owned arena.  A dispatcher thread launches whatever
 * is admitted as one persistent batched-kernel launch whenever one of
 * `slots` device slots (each a stream plus a descriptor ring entry in device
 * memory) is free, so work that arrives while earlier micro-batches run
 * overlaps with them on the device.  A request of at least 32 MiB of
 * algorithmic traffic, or of a complex or mixed-precision type, takes a slot
 * by itself, launched with the per-call kernels (whole tile menu, tune table).  Results are bitwise those of
 * ttx_transpose on the same inputs.  Latency = completion (observed by the
 * dispatcher) minus arrival. */
typedef struct ttx_server_opts {
    double hbm_fraction;      /* admission budget as a fraction of free device memory (0: 0.8) */
    int64_t arena_bytes;      /* output arena; 0: the whole budget */
    int slots;                /* micro-batches in flight at once (0: 4) */
    int max_batch;            /* requests per micro-batch (0: 256) */
    int64_t max_batch_bytes;  /* algorithmic bytes per micro-batch (0: 256 MiB); one request always fits */
    int max_queue;            /* waiting requests before submit refuses with TTX_EBUSY (0: 65536) */
    int fake_device;          /* test hook: no HIP call and no memory access; requests "finish"
                                 after the time their bytes would take at 4 TB/s, computing nothing */
    int64_t fake_free_bytes;  /* free memory assumed by fake_device (0: 2^34 / 0.8) */
} ttx_server_opts;

typedef struct ttx_request {
    ttx_problem problem;      /* problem.B == NULL: output in the server arena (then a beta != 0
                                 request reads beta*B from problem.B_in, which must be set) */
    int64_t arrival_ns;       /* steady-clock arrival time for latency; 0: time of submission */
    int keep_result;          /* keep the output until ttx_server_release (else freed at completion) */
} ttx_request;

typedef struct ttx_server_stats {
    int64_t submitted, rejected, completed, queued, running, batches;
    double mean_batch;                 /* requests per micro-batch */
    int64_t algorithmic_bytes;         /* of completed requests */
    int64_t budget_bytes, in_use_bytes, peak_in_use_bytes;
    double span_s;                     /* first arrival to last completion */
    double throughput_gbps;            /* algorithmic bytes / span */
    double p50_us, p99_us, max_us;     /* latency of completed requests */
} ttx_server_stats;

typedef struct ttx_server ttx_server;

/* Allocates the arena and slots and starts the dispatcher thread. */
ttx_status ttx_server_create(ttx_server **server, const ttx_server_opts *opts);
/* Queues a request; TTX_EBUSY when its footprint can never fit the budget or
 * the queue is full.  *ticket identifies it (tickets start at 1). */
ttx_status ttx_server_submit(ttx_server *server, const ttx_request *request, uint64_t *ticket);
ttx_status ttx_server_poll(ttx_server *server, uint64_t ticket, int *done);
ttx_status ttx_server_wait(ttx_server *server, uint64_t ticket);
/* Output pointer and latency of a finished request kept with keep_result. */
ttx_status ttx_server_result(ttx_server *server, uint64_t ticket, void **B, double *latency_us);
/* Frees a kept result's arena region and budget. */
ttx_status ttx_server_release(ttx_server *server, uint64_t ticket);
/* Withdraws a request that has not been launched (queued, or admitted and
 * waiting for a slot): its budget and arena region are returned and it never
 * runs; later poll, wait, result and release calls on the ticket return
 * TTX_ENOTFOUND.  A launched request cannot be recalled from the device
 * (TTX_EBUSY); a finished one is released instead (TTX_EBUSY). */
ttx_status ttx_server_cancel(ttx_server *server, uint64_t ticket);
/* Waits until nothing is queued or running; TTX_EBUSY if admission is blocked
 * by results the caller still holds. */
ttx_status ttx_server_drain(ttx_server *server);
/* Open-loop replay from the calling thread: request i is submitted at
 * (start + offsets_ns[i]), which is also its arrival time; a full queue is
 * retried, a request that can never fit gets ticket 0. */
ttx_status ttx_server_replay(ttx_server *server, int64_t count, const ttx_request *requests,
                             const int64_t *offsets_ns, uint64_t *tickets);
/* The same from `clients` submitting threads (client c submits requests
 * c, c + clients, ...), as when several clients share one server.  Planning
 * a request runs on its client's thread. */
ttx_status ttx_server_replay_clients(ttx_server *server, int64_t count, const ttx_request *requests,
                                     const int64_t *offsets_ns, int clients, uint64_t *tickets);
ttx_status ttx_server_get_stats(ttx_server *server, ttx_server_stats *stats);
/* The serving baseline: the same open-loop trace run one request at a time
 * through the per-call path, each launched at its arrival time (or as soon
 * as the previous one finished) and synchronised before the next;
 * latencies_us[i] = completion - arrival.  A request with problem.B == NULL
 * writes to `scratch` (scratch_bytes long). */
ttx_status ttx_replay_sequential(int64_t count, const ttx_request *requests,
                                 const int64_t *offsets_ns, void *scratch, int64_t scratch_bytes,
                                 hipStream_t stream, double *latencies_us);
/* Stops the dispatcher (requests not yet launched are dropped), waits for
 * the device and frees everything. */
ttx_status ttx_server_destroy(ttx_server *server);

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
