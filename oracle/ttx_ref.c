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
 *     (no fused multiply-add).  Build with -ffp-contract=off;
 *   - data types (the four of the paper's type list, Sec. 3): 0 = float,
 *     1 = double, 2 = single complex, 3 = double complex.  Complex elements
 *     are interleaved (re, im) pairs and alpha, beta may be complex (the
 *     _c entry points); the order of the complex arithmetic is stated at
 *     ref_update_c32 below.  The _x entry points take A and B in different
 *     precisions of one kind (mixed precision, Table 1), see
 *     ttx_ref_transpose_x.
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
enum { REF_F32 = 0, REF_F64 = 1, REF_C32 = 2, REF_C64 = 3 };
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

    if (dtype != REF_F32 && dtype != REF_F64 && dtype != REF_C32 && dtype != REF_C64)
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

/* Complex elements (the c and z data types of the paper's type list) are
 * interleaved (re, im) pairs.  The product of scalar s = (sr, si) and
 * element x = (xr, xi) is written out as
 *     re = fl( fl(sr*xr) - fl(si*xi) ),   im = fl( fl(sr*xi) + fl(si*xr) ),
 * every product and sum rounded separately in the element type (the paper
 * fixes no order for complex arithmetic; this one is the textbook formula,
 * evaluated left to right).  The update adds the two products part by part:
 * B = fl(alpha*a + beta*b) componentwise, and B is not read when both parts
 * of the rounded beta are zero. */
static void ref_update_c32(const float *A, float *B, int64_t off_a, int64_t off_b,
                           float ar, float ai, float br, float bi)
{
    const float xr = A[2 * off_a], xi = A[2 * off_a + 1];
    float t1 = ar * xr, t2 = ai * xi, t3 = ar * xi, t4 = ai * xr;
    float pr = t1 - t2, pi = t3 + t4;
    if (br == 0.0f && bi == 0.0f) {
        B[2 * off_b] = pr;
        B[2 * off_b + 1] = pi;
    } else {
        const float yr = B[2 * off_b], yi = B[2 * off_b + 1];
        float u1 = br * yr, u2 = bi * yi, u3 = br * yi, u4 = bi * yr;
        float qr = u1 - u2, qi = u3 + u4;
        B[2 * off_b] = pr + qr;
        B[2 * off_b + 1] = pi + qi;
    }
}

static void ref_update_c64(const double *A, double *B, int64_t off_a, int64_t off_b,
                           double ar, double ai, double br, double bi)
{
    const double xr = A[2 * off_a], xi = A[2 * off_a + 1];
    double t1 = ar * xr, t2 = ai * xi, t3 = ar * xi, t4 = ai * xr;
    double pr = t1 - t2, pi = t3 + t4;
    if (br == 0.0 && bi == 0.0) {
        B[2 * off_b] = pr;
        B[2 * off_b + 1] = pi;
    } else {
        const double yr = B[2 * off_b], yi = B[2 * off_b + 1];
        double u1 = br * yr, u2 = bi * yi, u3 = br * yi, u4 = bi * yr;
        double qr = u1 - u2, qi = u3 + u4;
        B[2 * off_b] = pr + qr;
        B[2 * off_b + 1] = pi + qi;
    }
}

/* Validation only: the status ttx_ref_transpose would return, without
 * touching A or B (A and B are compared as addresses only). */
static int64_t ref_elem_bytes(int dtype)
{
    return dtype == REF_F32 ? 4 : dtype == REF_C64 ? 16 : 8;
}

/* The pairs of data types a transposition may take (Table 1): A and B of
 * one type, or mixed precision with A and B of the same kind (real or
 * complex) in different precisions: sd, ds, cz, zc. */
static int ref_pair_valid(int dtype_a, int dtype_b)
{
    if (dtype_a == dtype_b)
        return 1;
    return (dtype_a == REF_F32 && dtype_b == REF_F64) || (dtype_a == REF_F64 && dtype_b == REF_F32) ||
           (dtype_a == REF_C32 && dtype_b == REF_C64) || (dtype_a == REF_C64 && dtype_b == REF_C32);
}

/* ttx_ref_check with A of type dtype_a and B of type dtype_b. */
int ttx_ref_check_x(int dtype_a, int dtype_b, int n, const int *perm, const int64_t *size,
                    const int64_t *outer_a, const int64_t *outer_b,
                    const void *A, const void *B)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int empty, st;
    int64_t a_lo, a_hi, b_lo, b_hi;

    st = ref_prepare(dtype_b, n, perm, size, outer_a, outer_b, size_b, stride_a, stride_b, &empty);
    if (st != REF_OK)
        return st;
    if (!ref_pair_valid(dtype_a, dtype_b))
        return REF_EINVAL;
    if (empty)
        return REF_OK;
    if (A == NULL || B == NULL)
        return REF_EINVAL;
    a_lo = (int64_t)(uintptr_t)A;
    a_hi = a_lo + ref_extent_bytes(n, size, stride_a, ref_elem_bytes(dtype_a));
    b_lo = (int64_t)(uintptr_t)B;
    b_hi = b_lo + ref_extent_bytes(n, size_b, stride_b, ref_elem_bytes(dtype_b));
    if (a_lo < b_hi && b_lo < a_hi)
        return REF_EOVERLAP;
    return REF_OK;
}

int ttx_ref_check(int dtype, int n, const int *perm, const int64_t *size,
                  const int64_t *outer_a, const int64_t *outer_b,
                  const void *A, const void *B)
{
    return ttx_ref_check_x(dtype, dtype, n, perm, size, outer_a, outer_b, A, B);
}

/* B_{Pi(i)} <- alpha*A_i + beta*B_{Pi(i)} over host arrays (Eqn. 1), with
 * complex scalars alpha = (alpha[0], alpha[1]) and beta likewise; for the
 * real data types the imaginary parts must be zero.  A holds elements of
 * type dtype_a and B of type dtype (mixed precision, Table 1 "sd", "ds",
 * "cz", "zc"): each A element is first converted to B's type (widening is
 * exact; narrowing rounds to nearest, part by part for complex), and the
 * update is then computed in B's type exactly as when both types agree. */
int ttx_ref_transpose_x(int dtype_a, int dtype, int n, const int *perm, const int64_t *size,
                        const int64_t *outer_a, const int64_t *outer_b,
                        const double *alpha, const void *A, const double *beta, void *B)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int64_t a_stride_in_b_order[REF_MAX_DIMS];
    int empty, st;
    const float alpha_f = (float)alpha[0], beta_f = (float)beta[0];
    const float alpha_fi = (float)alpha[1], beta_fi = (float)beta[1];

    if ((dtype == REF_F32 || dtype == REF_F64) && (alpha[1] != 0.0 || beta[1] != 0.0))
        return REF_EINVAL;

    st = ttx_ref_check_x(dtype_a, dtype, n, perm, size, outer_a, outer_b, A, B);
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
            if (dtype_a != dtype) {
                /* mixed precision: convert the A element to B's type first */
                if (dtype == REF_F64) {
                    const double a = (double)((const float *)A)[off_a];
                    ref_update_f64(&a, (double *)B, 0, off_b, alpha[0], beta[0]);
                } else if (dtype == REF_F32) {
                    const float a = (float)((const double *)A)[off_a];
                    ref_update_f32(&a, (float *)B, 0, off_b, alpha_f, beta_f);
                } else if (dtype == REF_C64) {
                    const float *x = (const float *)A + 2 * off_a;
                    const double a[2] = {(double)x[0], (double)x[1]};
                    ref_update_c64(a, (double *)B, 0, off_b, alpha[0], alpha[1], beta[0], beta[1]);
                } else {
                    const double *x = (const double *)A + 2 * off_a;
                    const float a[2] = {(float)x[0], (float)x[1]};
                    ref_update_c32(a, (float *)B, 0, off_b, alpha_f, alpha_fi, beta_f, beta_fi);
                }
            } else if (dtype == REF_F32)
                ref_update_f32((const float *)A, (float *)B, off_a, off_b, alpha_f, beta_f);
            else if (dtype == REF_F64)
                ref_update_f64((const double *)A, (double *)B, off_a, off_b, alpha[0], beta[0]);
            else if (dtype == REF_C32)
                ref_update_c32((const float *)A, (float *)B, off_a, off_b, alpha_f, alpha_fi, beta_f, beta_fi);
            else
                ref_update_c64((const double *)A, (double *)B, off_a, off_b, alpha[0], alpha[1], beta[0],
                               beta[1]);
            for (int k = 0; k < n - 1; ++k) {   /* advance the odometer */
                if (++j[k] < size_b[k])
                    break;
                j[k] = 0;
            }
        }
    }
    return REF_OK;
}

/* A and B of one type. */
int ttx_ref_transpose_c(int dtype, int n, const int *perm, const int64_t *size,
                        const int64_t *outer_a, const int64_t *outer_b,
                        const double *alpha, const void *A, const double *beta, void *B)
{
    return ttx_ref_transpose_x(dtype, dtype, n, perm, size, outer_a, outer_b, alpha, A, beta, B);
}

/* The real-scalar form of ttx_ref_transpose_c (any data type). */
int ttx_ref_transpose(int dtype, int n, const int *perm, const int64_t *size,
                      const int64_t *outer_a, const int64_t *outer_b,
                      double alpha, const void *A, double beta, void *B)
{
    const double a2[2] = {alpha, 0.0}, b2[2] = {beta, 0.0};
    return ttx_ref_transpose_c(dtype, n, perm, size, outer_a, outer_b, a2, A, b2, B);
}

/* Eqn. 1 at chosen elements only: for each q < count, B_index[q] is the
 * B-linear position inside the sub-tensor (first B index fastest); out[q]
 * receives the value the transposition leaves there, given B's prior
 * contents B_in (not read when beta rounds to zero).  Complex scalars as in
 * ttx_ref_transpose_c; each element takes the same operations, in the same
 * order, as in the full loop nest. */
int ttx_ref_sample_c(int dtype, int n, const int *perm, const int64_t *size,
                     const int64_t *outer_a, const int64_t *outer_b,
                     const double *alpha, const void *A, const double *beta, const void *B_in,
                     int64_t count, const int64_t *B_index, void *out)
{
    int64_t size_b[REF_MAX_DIMS], stride_a[REF_MAX_DIMS], stride_b[REF_MAX_DIMS];
    int empty, st;
    const float alpha_f = (float)alpha[0], beta_f = (float)beta[0];
    const float alpha_fi = (float)alpha[1], beta_fi = (float)beta[1];
    int reads_b;

    if ((dtype == REF_F32 || dtype == REF_F64) && (alpha[1] != 0.0 || beta[1] != 0.0))
        return REF_EINVAL;
    st = ref_prepare(dtype, n, perm, size, outer_a, outer_b, size_b, stride_a, stride_b, &empty);
    if (st != REF_OK)
        return st;
    if (empty)
        return count == 0 ? REF_OK : REF_EINVAL;
    if (dtype == REF_F32 || dtype == REF_C32)
        reads_b = beta_f != 0.0f || beta_fi != 0.0f;
    else
        reads_b = beta[0] != 0.0 || beta[1] != 0.0;
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
        /* out[q] stands in for B's element: load B's prior value, update. */
        switch (dtype) {
        case REF_F32:
            ((float *)out)[q] = reads_b ? ((const float *)B_in)[off_b] : 0.0f;
            ref_update_f32((const float *)A, (float *)out, off_a, q, alpha_f, beta_f);
            break;
        case REF_F64:
            ((double *)out)[q] = reads_b ? ((const double *)B_in)[off_b] : 0.0;
            ref_update_f64((const double *)A, (double *)out, off_a, q, alpha[0], beta[0]);
            break;
        case REF_C32:
            ((float *)out)[2 * q] = reads_b ? ((const float *)B_in)[2 * off_b] : 0.0f;
            ((float *)out)[2 * q + 1] = reads_b ? ((const float *)B_in)[2 * off_b + 1] : 0.0f;
            ref_update_c32((const float *)A, (float *)out, off_a, q, alpha_f, alpha_fi, beta_f, beta_fi);
            break;
        default:
            ((double *)out)[2 * q] = reads_b ? ((const double *)B_in)[2 * off_b] : 0.0;
            ((double *)out)[2 * q + 1] = reads_b ? ((const double *)B_in)[2 * off_b + 1] : 0.0;
            ref_update_c64((const double *)A, (double *)out, off_a, q, alpha[0], alpha[1], beta[0],
                           beta[1]);
            break;
        }
    }
    return REF_OK;
}

/* The real-scalar form of ttx_ref_sample_c. */
int ttx_ref_sample(int dtype, int n, const int *perm, const int64_t *size,
                   const int64_t *outer_a, const int64_t *outer_b,
                   double alpha, const void *A, double beta, const void *B_in,
                   int64_t count, const int64_t *B_index, void *out)
{
    const double a2[2] = {alpha, 0.0}, b2[2] = {beta, 0.0};
    return ttx_ref_sample_c(dtype, n, perm, size, outer_a, outer_b, a2, A, b2, B_in, count, B_index,
                            out);
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

/* Sets the number of threads later calls use (n >= 1); results do not
 * depend on it.  Returns the number now in effect. */
int ttx_ref_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
}
