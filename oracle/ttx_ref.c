/*
 * CPU oracle for out-of-place tensor transposition with scaling and update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline timing leg of the benchmark load it; the library never
 * links, calls or includes it, and it includes nothing from the library.
 *
 * What it computes (Sec. 1, Eqn. 1), for every multi-index i of A:
 *
 *     B_{Pi(i)} <- alpha * A_i + beta * B_{Pi(i)}
 *
 * Layout and arguments, as read from the paper:
 *   - column-major storage: index 0 has stride 1 (Sec. 1, footnote 2);
 *   - perm uses the gather reading of the permutation notation of Sec. 2.1:
 *     position k of B holds A's index perm[k], so sizeB[k] = size[perm[k]]
 *     (the merge example of Sec. 2.1 is perm = (1,2,0));
 *   - outer_a / outer_b are the per-index leading dimensions of Table 1 and
 *     Fig. 2 (a sub-tensor inside a larger tensor).  outer_a is indexed by A
 *     position, outer_b by B position; NULL means "stored contiguously",
 *     i.e. outer == size (Sec. 2.1, text around Fig. 2);
 *   - strideA[m] = prod_{j<m} outer_a[j],  strideB[k] = prod_{j<k} outer_b[j];
 *   - alpha and beta are first rounded to the element type; when the
 *     rounded beta is zero, B is only written, never read (Sec. 1: beta = 0
 *     overwrites B);
 *   - each product and the sum are rounded separately in the element type
 *     (no fused multiply-add).  Build with -ffp-contract=off.
 *
 * The loop nest walks B linearly (B index 0 fastest), the loop order of the
 * reference implementation of Sec. 3.2, with the outermost B index shared
 * among OpenMP threads.  Threading does not change any result: every B
 * element is written once, by one thread, from one A element.
 *
 * Status codes (returned, never printed):
 *   0 ok, 1 invalid argument, 2 perm is not a permutation of 0..n-1,
 *   3 the byte ranges of A and B overlap, 4 unsupported.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

enum { REF_OK = 0, REF_EINVAL = 1, REF_EPERM = 2, REF_EOVERLAP = 3, REF_EUNSUPPORTED = 4 };
enum { REF_F32 = 0, REF_F64 = 1 };
#define REF_MAX_DIMS 16

/* Checks the arguments and fills in sizeB and the two stride vectors.
 * Returns REF_OK with *empty set when some extent is zero. */
static int ref_prepare(int dtype, int n, const int *perm, const int64_t *size,
                       const int64_t *outer_a, const int64_t *outer_b,
                       int64_t *size_b, int64_t *stride_a, int64_t *stride_b,
                       int *empty)
{
    int seen[REF_MAX_DIMS] = {0};
    int64_t prod;

    if (dtype != REF_F32 && dtype != REF_F64)
        return REF_EINVAL;
    if (n < 1 || n > REF_MAX_DIMS || perm == NULL || size == NULL)
        return REF_EINVAL;
    for (int k = 0; k < n; ++k) {
        if (perm[k] < 0 || perm[k] >= n || seen[perm[k]])
            return REF_EPERM;
        seen[perm[k]] = 1;
    }
    for (int m = 0; m < n; ++m)
        if (size[m] < 0)
            return REF_EINVAL;
    for (int k = 0; k < n; ++k)
        size_b[k] = size[perm[k]];

    prod = 1;
    for (int m = 0; m < n; ++m) {
        int64_t o = outer_a ? outer_a[m] : size[m];
        if (o < size[m])
            return REF_EINVAL;
        stride_a[m] = prod;
        if (__builtin_mul_overflow(prod, o, &prod))
            return REF_EINVAL;
    }
    prod = 1;
    for (int k = 0; k < n; ++k) {
        int64_t o = outer_b ? outer_b[k] : size_b[k];
        if (o < size_b[k])
            return REF_EINVAL;
        stride_b[k] = prod;
        if (__builtin_mul_overflow(prod, o, &prod))
            return REF_EINVAL;
    }
    *empty = 0;
    for (int m = 0; m < n; ++m)
        if (size[m] == 0)
            *empty = 1;
    return REF_OK;
}

/* Number of bytes from the first to one past the last addressed element. */
static int64_t ref_extent_bytes(int n, const int64_t *extent, const int64_t *stride, int64_t elem)
{
    int64_t last = 0;
    for (int d = 0; d < n; ++d)
        last += (extent[d] - 1) * stride[d];
    return (last + 1) * elem;
}

static void ref_update_f32(const float *A, float *B, int64_t off_a, int64_t off_b,
                           float alpha, float beta)
{
    if (beta == 0.0f) {
        B[off_b] = alpha * A[off_a];
    } else {
        float scaled_a = alpha * A[off_a];
        float scaled_b = beta * B[off_b];
        B[off_b] = scaled_a + scaled_b;
    }
}

static void ref_update_f64(const double *A, double *B, int64_t off_a, int64_t off_b,
                           double alpha, double beta)
{
    if (beta == 0.0) {
        B[off_b] = alpha * A[off_a];
    } else {
        double scaled_a = alpha * A[off_a];
        double scaled_b = beta * B[off_b];
        B[off_b] = scaled_a + scaled_b;
    }
}

/* Validation only: the status ttx_ref_transpose would return, without
 * touching A or B (A and B are compared as addresses only). */
int ttx_ref_check(int dtype, int n, const int *perm, const int64_t *size,
                  const int64_t *outer_a, const int64_t *outer_b,
                  const void *A, const void *B)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int empty, st;
    int64_t elem, a_lo, a_hi, b_lo, b_hi;

    st = ref_prepare(dtype, n, perm, size, outer_a, outer_b, size_b, stride_a, stride_b, &empty);
    if (st != REF_OK || empty)
        return st;
    if (A == NULL || B == NULL)
        return REF_EINVAL;
    elem = dtype == REF_F32 ? 4 : 8;
    a_lo = (int64_t)(uintptr_t)A;
    a_hi = a_lo + ref_extent_bytes(n, size, stride_a, elem);
    b_lo = (int64_t)(uintptr_t)B;
    b_hi = b_lo + ref_extent_bytes(n, size_b, stride_b, elem);
    if (a_lo < b_hi && b_lo < a_hi)
        return REF_EOVERLAP;
    return REF_OK;
}

/* B_{Pi(i)} <- alpha*A_i + beta*B_{Pi(i)} over host arrays (Eqn. 1). */
int ttx_ref_transpose(int dtype, int n, const int *perm, const int64_t *size,
                      const int64_t *outer_a, const int64_t *outer_b,
                      double alpha, const void *A, double beta, void *B)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int64_t a_stride_in_b_order[REF_MAX_DIMS];
    int empty, st;
    const float alpha_f = (float)alpha, beta_f = (float)beta;

    st = ttx_ref_check(dtype, n, perm, size, outer_a, outer_b, A, B);
    if (st != REF_OK)
        return st;
    st = ref_prepare(dtype, n, perm, size, outer_a, outer_b, size_b, stride_a, stride_b, &empty);
    if (st != REF_OK || empty)
        return st;

    /* Moving one step along B index k moves one step along A index perm[k]. */
    for (int k = 0; k < n; ++k)
        a_stride_in_b_order[k] = stride_a[perm[k]];

    /* Outermost B index split among threads; an odometer walks the rest,
     * B index 0 fastest. */
    #pragma omp parallel for schedule(static)
    for (int64_t top = 0; top < size_b[n - 1]; ++top) {
        int64_t j[REF_MAX_DIMS] = {0};
        int64_t inner_count = 1;
        for (int k = 0; k < n - 1; ++k)
            inner_count *= size_b[k];
        for (int64_t step = 0; step < inner_count; ++step) {
            int64_t off_a = top * a_stride_in_b_order[n - 1];
            int64_t off_b = top * stride_b[n - 1];
            for (int k = 0; k < n - 1; ++k) {
                off_a += j[k] * a_stride_in_b_order[k];
                off_b += j[k] * stride_b[k];
            }
            if (dtype == REF_F32)
                ref_update_f32((const float *)A, (float *)B, off_a, off_b, alpha_f, beta_f);
            else
                ref_update_f64((const double *)A, (double *)B, off_a, off_b, alpha, beta);
            for (int k = 0; k < n - 1; ++k) {   /* advance the odometer */
                if (++j[k] < size_b[k])
                    break;
                j[k] = 0;
            }
        }
    }
    return REF_OK;
}

/* Eqn. 1 at chosen elements only: for each q < count, B_index[q] is the
 * position of an element of B's sub-tensor in B-linear order (B index 0
 * fastest); out[q] receives alpha*A + beta*B_in at that position, where A is
 * the element the permutation sends there.  B_in is read only when the
 * rounded beta is non-zero.  Lets large problems be checked on samples. */
int ttx_ref_sample(int dtype, int n, const int *perm, const int64_t *size,
                   const int64_t *outer_a, const int64_t *outer_b,
                   double alpha, const void *A, double beta, const void *B_in,
                   int64_t count, const int64_t *B_index, void *out)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int empty, st;
    const float alpha_f = (float)alpha, beta_f = (float)beta;

    st = ref_prepare(dtype, n, perm, size, outer_a, outer_b, size_b, stride_a, stride_b, &empty);
    if (st != REF_OK)
        return st;
    if (empty)
        return count == 0 ? REF_OK : REF_EINVAL;
    for (int64_t q = 0; q < count; ++q) {
        int64_t rest = B_index[q], off_a = 0, off_b = 0;
        for (int k = 0; k < n; ++k) {
            int64_t j = rest % size_b[k];
            rest /= size_b[k];
            off_a += j * stride_a[perm[k]];
            off_b += j * stride_b[k];
        }
        if (B_index[q] < 0 || rest != 0)
            return REF_EINVAL;
        if (dtype == REF_F32) {
            float b = beta_f == 0.0f ? 0.0f : ((const float *)B_in)[off_b];
            float r = alpha_f * ((const float *)A)[off_a];
            if (beta_f != 0.0f) {
                float scaled_b = beta_f * b;
                r = r + scaled_b;
            }
            ((float *)out)[q] = r;
        } else {
            double b = beta == 0.0 ? 0.0 : ((const double *)B_in)[off_b];
            double r = alpha * ((const double *)A)[off_a];
            if (beta != 0.0) {
                double scaled_b = beta * b;
                r = r + scaled_b;
            }
            ((double *)out)[q] = r;
        }
    }
    return REF_OK;
}

/* Offset (in elements) of each B-linear sub-tensor position inside B's outer
 * tensor, so that samples can be compared against a full B buffer. */
int ttx_ref_b_offsets(int n, const int *perm, const int64_t *size, const int64_t *outer_b,
                      int64_t count, const int64_t *B_index, int64_t *off)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int empty;
    int st = ref_prepare(REF_F32, n, perm, size, NULL, outer_b, size_b, stride_a, stride_b, &empty);
    if (st != REF_OK)
        return st;
    for (int64_t q = 0; q < count; ++q) {
        int64_t rest = B_index[q], o = 0;
        for (int k = 0; k < n; ++k) {
            o += (rest % size_b[k]) * stride_b[k];
            rest /= size_b[k];
        }
        off[q] = o;
    }
    return REF_OK;
}

/* Threads the parallel loop of ttx_ref_transpose uses. */
int ttx_ref_threads(void)
{
    return omp_get_max_threads();
}
