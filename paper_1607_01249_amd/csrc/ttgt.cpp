// Tensor contraction as transpose-transpose-GEMM-transpose (Sec. 1: a
// contraction cast as a matrix product through transpositions; Sec. 4: the
// transposition as the building block of a contraction compiler).
//
// Planning (host only) splits the labels into the product's rows (A's free
// labels), columns (B's free labels) and the contracted labels, and picks
// the orders that let the most operands go to the packing step as they are
// stored: an operand whose free and contracted labels form two contiguous
// blocks is already a matrix (packed with the left- or right-operand panel
// kind, whichever reads it in storage order, since both kinds produce the
// same panel layout), provided both operands use one contracted order.
// Execution chains the library's own steps on one stream: transpositions
// into matrix order where needed, packing into matrix-core panels, the
// panel GEMM, and the transposition of the product into C with alpha and
// beta (Eqn. 1).
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "ttx_internal.h"

struct ttx_contraction {
    int dtype = TTX_F32, panel = 16;
    int64_t m = 1, n = 1, k = 1;
    int64_t bytes_a = 0, bytes_b = 0, bytes_c = 0;     // byte extents of A, B, C
    bool trans_a = false, trans_b = false;
    int kind_a = TTX_PACK_MFMA_A, kind_b = TTX_PACK_MFMA_B;
    int64_t rows_a = 1, cols_a = 1, rows_b = 1, cols_b = 1;   // the packed matrices (ld = rows)
    ttx_plan* to_mat_a = nullptr;      // A into matrix order (trans_a)
    ttx_plan* to_mat_b = nullptr;
    ttx_plan* to_c = nullptr;          // the m x n product into C's mode order
    int64_t off_a = 0, off_b = 0, off_pa = 0, off_pb = 0, off_prod = 0, ws = 0;   // workspace bytes
    std::vector<int> ord_m, ord_n, ord_k;

    ~ttx_contraction() {
        if (to_mat_a) ttx_plan_destroy(to_mat_a);
        if (to_mat_b) ttx_plan_destroy(to_mat_b);
        if (to_c) ttx_plan_destroy(to_c);
    }
};

namespace ttx {
namespace {

// 1: `labels` is block X then block Y; 2: block Y then block X; 0: neither.
// X and Y hold the tensor's labels of each group in its own order.
int block_layout(const std::vector<int>& labels, const std::vector<int>& X, const std::vector<int>& Y) {
    std::vector<int> xy(X), yx(Y);
    xy.insert(xy.end(), Y.begin(), Y.end());
    yx.insert(yx.end(), X.begin(), X.end());
    if (labels == xy) return 1;
    if (labels == yx) return 2;
    return 0;
}

// Product of the labels' extents; -1 when it does not fit in int64_t.
int64_t product(const std::vector<int>& labels, const std::vector<std::pair<int, int64_t>>& ext) {
    int64_t p = 1;
    for (int l : labels)
        for (const auto& e : ext)
            if (e.first == l && __builtin_mul_overflow(p, e.second, &p)) return -1;
    return p;
}

int64_t extent_of(int l, const std::vector<std::pair<int, int64_t>>& ext) {
    for (const auto& e : ext)
        if (e.first == l) return e.second;
    return 1;
}

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// A plan transposing a tensor with modes `from` (extents via ext) into the
// mode order `to` (a permutation of `from`); a scalar becomes one element.
ttx_status order_plan(int dtype, const std::vector<int>& from, const std::vector<int>& to,
                      const std::vector<std::pair<int, int64_t>>& ext, ttx_plan** out) {
    std::vector<int> perm;
    std::vector<int64_t> size;
    for (int l : from) size.push_back(extent_of(l, ext));
    for (int l : to) perm.push_back(int(std::find(from.begin(), from.end(), l) - from.begin()));
    if (from.empty()) {
        perm.push_back(0);
        size.push_back(1);
    }
    return ttx_plan_create(out, ttx_dtype(dtype), int(perm.size()), perm.data(), size.data(), nullptr, nullptr);
}

bool overlaps(const void* p, int64_t pn, const void* q, int64_t qn) {
    if (pn <= 0 || qn <= 0) return false;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p), b = reinterpret_cast<uintptr_t>(q);
    return a < b + uint64_t(qn) && b < a + uint64_t(pn);
}

}  // namespace
}  // namespace ttx

using namespace ttx;

extern "C" {

ttx_status ttx_contraction_create(ttx_contraction** plan, ttx_dtype dtype, int na, const int* labels_a,
                                  const int64_t* size_a, int nb, const int* labels_b, const int64_t* size_b,
                                  int nc, const int* labels_c, const int64_t* size_c) {
    if (!plan) return fail(TTX_EINVAL, "plan must not be NULL");
    *plan = nullptr;
    if (!dtype_valid(dtype)) return fail(TTX_EINVAL, "unknown dtype");
    if (dtype != TTX_F32 && dtype != TTX_F64)
        return fail(TTX_EUNSUPPORTED, "contraction: TTX_F32 or TTX_F64 (the matrix-core GEMM's types)");
    const int cnt[3] = {na, nb, nc};
    const int* lab[3] = {labels_a, labels_b, labels_c};
    const int64_t* siz[3] = {size_a, size_b, size_c};
    std::vector<int> L[3];
    std::vector<std::pair<int, int64_t>> ext;
    for (int t = 0; t < 3; ++t) {
        if (cnt[t] < 0 || cnt[t] > TTX_MAX_DIMS) return fail(TTX_EINVAL, "mode count outside 0..TTX_MAX_DIMS");
        if (cnt[t] > 0 && (!lab[t] || !siz[t])) return fail(TTX_EINVAL, "NULL labels or extents");
        for (int d = 0; d < cnt[t]; ++d) {
            const int l = lab[t][d];
            const int64_t s = siz[t][d];
            if (s < 0) return fail(TTX_EINVAL, "negative extent");
            if (std::find(L[t].begin(), L[t].end(), l) != L[t].end())
                return fail(TTX_EINVAL, "a tensor carries a label twice");
            L[t].push_back(l);
            bool seen = false;
            for (const auto& e : ext)
                if (e.first == l) {
                    seen = true;
                    if (e.second != s) return fail(TTX_EINVAL, "a label has two extents");
                }
            if (!seen) ext.push_back({l, s});
        }
    }
    auto has = [&](int t, int l) { return std::find(L[t].begin(), L[t].end(), l) != L[t].end(); };
    for (const auto& e : ext) {
        const int c = has(0, e.first) + has(1, e.first) + has(2, e.first);
        if (c == 3) return fail(TTX_EINVAL, "batch label (carried by A, B and C)");
        if (c != 2) return fail(TTX_EINVAL, "a label is carried by one tensor only");
    }
    for (int t = 0; t < 3; ++t)
        if (product(L[t], ext) < 0 || product(L[t], ext) > (int64_t(1) << 56))
            return fail(TTX_EINVAL, "tensor too large");
    std::unique_ptr<ttx_contraction> p(new ttx_contraction);
    p->dtype = dtype;
    // groups, each in its own tensor's order
    std::vector<int> Ma, Ka, Kb, Nb;
    for (int l : L[0]) (has(2, l) ? Ma : Ka).push_back(l);
    for (int l : L[1]) (has(2, l) ? Nb : Kb).push_back(l);
    const int lay_a = block_layout(L[0], Ma, Ka);   // 1: (M, K), 2: (K, M)
    const int lay_b = block_layout(L[1], Kb, Nb);   // 1: (K, N), 2: (N, K)
    std::vector<int> K;
    if (lay_a && lay_b && Ka == Kb) {
        K = Ka;
    } else if (lay_a && lay_b) {   // both matrices, contracted orders differ: transpose the smaller
        const bool a_smaller = product(L[0], ext) <= product(L[1], ext);
        K = a_smaller ? Kb : Ka;
        (a_smaller ? p->trans_a : p->trans_b) = true;
    } else if (lay_a) {
        K = Ka;
        p->trans_b = true;
    } else if (lay_b) {
        K = Kb;
        p->trans_a = true;
    } else {
        K = Ka;
        p->trans_a = p->trans_b = true;
    }
    if (!p->trans_b && Kb != K) p->trans_b = true;
    if (!p->trans_a && Ka != K) p->trans_a = true;
    p->ord_m = Ma;
    p->ord_n = Nb;
    p->ord_k = K;
    p->m = product(Ma, ext);
    p->n = product(Nb, ext);
    p->k = product(K, ext);
    const int64_t es = elem_bytes(dtype);
    p->bytes_a = product(L[0], ext) * es;
    p->bytes_b = product(L[1], ext) * es;
    p->bytes_c = product(L[2], ext) * es;
    p->panel = (dtype == TTX_F32 && p->m >= 32 && p->n >= 32) ? 32 : 16;
    // how each operand is read by the packing step
    std::vector<int> mat_a(Ma), mat_b(K);
    mat_a.insert(mat_a.end(), K.begin(), K.end());
    mat_b.insert(mat_b.end(), Nb.begin(), Nb.end());
    if (p->trans_a || lay_a == 1) {
        p->kind_a = TTX_PACK_MFMA_A;
        p->rows_a = p->m;
        p->cols_a = p->k;
    } else {   // stored (K, M): the right-operand kind reads it as a k x m matrix
        p->kind_a = TTX_PACK_MFMA_B;
        p->rows_a = p->k;
        p->cols_a = p->m;
    }
    if (p->trans_b || lay_b == 1) {
        p->kind_b = TTX_PACK_MFMA_B;
        p->rows_b = p->k;
        p->cols_b = p->n;
    } else {   // stored (N, K)
        p->kind_b = TTX_PACK_MFMA_A;
        p->rows_b = p->n;
        p->cols_b = p->k;
    }
    ttx_status st;
    if (p->trans_a && (st = order_plan(dtype, L[0], mat_a, ext, &p->to_mat_a)) != TTX_OK) return st;
    if (p->trans_b && (st = order_plan(dtype, L[1], mat_b, ext, &p->to_mat_b)) != TTX_OK) return st;
    std::vector<int> prod(Ma);
    prod.insert(prod.end(), Nb.begin(), Nb.end());
    if ((st = order_plan(dtype, prod, L[2], ext, &p->to_c)) != TTX_OK) return st;
    // workspace: operand matrices (when transposed), panels, product
    const int64_t kb = 64 / p->panel, Kp = (p->k + kb - 1) / kb * kb;
    const int64_t mp = (p->m + p->panel - 1) / p->panel, nq = (p->n + p->panel - 1) / p->panel;
    int64_t off = 0;
    auto take = [&](int64_t elems) {
        const int64_t at = off;
        off += align256(elems * es);
        return at;
    };
    p->off_a = p->trans_a ? take(p->m * p->k) : 0;
    p->off_b = p->trans_b ? take(p->k * p->n) : 0;
    p->off_pa = take(mp * p->panel * Kp);
    p->off_pb = take(nq * p->panel * Kp);
    p->off_prod = take(p->m * p->n);
    p->ws = (p->m == 0 || p->n == 0) ? 0 : off;
    *plan = p.release();
    return TTX_OK;
}

ttx_status ttx_contraction_describe(const ttx_contraction* plan, ttx_contraction_info* info) {
    if (!plan || !info) return fail(TTX_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->m = plan->m;
    info->n = plan->n;
    info->k = plan->k;
    info->panel = plan->panel;
    info->transposed_a = plan->trans_a;
    info->transposed_b = plan->trans_b;
    info->pack_kind_a = plan->kind_a;
    info->pack_kind_b = plan->kind_b;
    info->n_m = int(plan->ord_m.size());
    info->n_n = int(plan->ord_n.size());
    info->n_k = int(plan->ord_k.size());
    std::copy(plan->ord_m.begin(), plan->ord_m.end(), info->order_m);
    std::copy(plan->ord_n.begin(), plan->ord_n.end(), info->order_n);
    std::copy(plan->ord_k.begin(), plan->ord_k.end(), info->order_k);
    info->workspace_bytes = plan->ws;
    return TTX_OK;
}

ttx_status ttx_contraction_execute(const ttx_contraction* plan, double alpha, const void* A, const void* B,
                                   double beta, void* C, void* workspace, hipStream_t stream) {
    if (!plan) return fail(TTX_EINVAL, "plan must not be NULL");
    if (plan->m == 0 || plan->n == 0) return TTX_OK;   // C is empty
    if ((plan->bytes_a && !A) || (plan->bytes_b && !B) || !C || !workspace)
        return fail(TTX_EINVAL, "NULL tensor or workspace pointer");
    const uintptr_t es = uintptr_t(elem_bytes(plan->dtype));
    if (reinterpret_cast<uintptr_t>(A) % es || reinterpret_cast<uintptr_t>(B) % es ||
        reinterpret_cast<uintptr_t>(C) % es || reinterpret_cast<uintptr_t>(workspace) % es)
        return fail(TTX_EINVAL, "pointer not aligned to the element size");
    if (overlaps(C, plan->bytes_c, A, plan->bytes_a) || overlaps(C, plan->bytes_c, B, plan->bytes_b))
        return fail(TTX_EOVERLAP, "C overlaps an operand");
    if (overlaps(workspace, plan->ws, A, plan->bytes_a) || overlaps(workspace, plan->ws, B, plan->bytes_b) ||
        overlaps(workspace, plan->ws, C, plan->bytes_c))
        return fail(TTX_EOVERLAP, "the workspace overlaps a tensor");
    char* ws = static_cast<char*>(workspace);
    ttx_status st;
    const void* mat_a = A;
    const void* mat_b = B;
    if (plan->k > 0 && plan->trans_a) {
        if ((st = ttx_plan_execute(plan->to_mat_a, 1.0, A, 0.0, ws + plan->off_a, stream)) != TTX_OK) return st;
        mat_a = ws + plan->off_a;
    }
    if (plan->k > 0 && plan->trans_b) {   // k == 0: nothing to read; the product is zero
        if ((st = ttx_plan_execute(plan->to_mat_b, 1.0, B, 0.0, ws + plan->off_b, stream)) != TTX_OK) return st;
        mat_b = ws + plan->off_b;
    }
    const double one[2] = {1.0, 0.0};
    if ((st = ttx_pack(ttx_dtype(plan->dtype), plan->kind_a, plan->rows_a, plan->cols_a,
                       std::max<int64_t>(plan->rows_a, 1), plan->panel, one, mat_a, ws + plan->off_pa, stream)) !=
        TTX_OK)
        return st;
    if ((st = ttx_pack(ttx_dtype(plan->dtype), plan->kind_b, plan->rows_b, plan->cols_b,
                       std::max<int64_t>(plan->rows_b, 1), plan->panel, one, mat_b, ws + plan->off_pb, stream)) !=
        TTX_OK)
        return st;
    if ((st = ttx_gemm_panels(ttx_dtype(plan->dtype), plan->panel, plan->m, plan->n, plan->k, ws + plan->off_pa,
                              ws + plan->off_pb, ws + plan->off_prod, plan->m, stream)) != TTX_OK)
        return st;
    return ttx_plan_execute(plan->to_c, alpha, ws + plan->off_prod, beta, C, stream);
}

ttx_status ttx_contraction_destroy(ttx_contraction* plan) {
    delete plan;
    return TTX_OK;
}

}  // extern "C"
