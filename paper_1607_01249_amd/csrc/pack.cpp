// GEMM operand packing (Sec. 2.1, Fig. 3): a column-major matrix is viewed
// as a 3D tensor whose first index is split into panels, and the packed
// panels are that tensor transposed, so packing is a transposition of the
// view plus zero rows (or columns) that fill the last panel.
//
//   rows packing (the A operand, panels of mr rows): A is m x k; the view
//   A(i, p, kk) = A[i + p*mr + kk*ld] (i < mr, p < m/mr) is written as
//   P(i, kk, p) = P[i + kk*mr + p*mr*k], perm (0, 2, 1): each panel is an
//   mr x k column-major block with its mr rows contiguous.
//
//   columns packing (the B operand, panels of nr columns): A is k x n; the
//   view A(kk, j, p) = A[kk + (j + p*nr)*ld] is written as
//   P(j, kk, p) = P[j + kk*nr + p*nr*k], perm (1, 0, 2): each panel is
//   k rows of nr contiguous elements.
//
// The whole panels are one transposition; a ragged last panel is a second,
// two-index one, and the rest of that panel is set to zero.
//
// Matrix-core operand panels (TTX_PACK_MFMA_A / _B) are the same two
// layouts with the k extent of every panel padded with zeros to a multiple
// of kb = 64 / panel: a 64-lane matrix instruction with M (or N) = panel
// takes kb values of k per instruction, lane l holding element
// (l mod panel, l div panel) of the block, so with the panel stride
// panel*K (K = k rounded up to kb) each instruction's operand is 64
// consecutive elements in lane order.  The k padding is one more zero
// region: the last (K - k) * panel elements of every panel.
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>

#include "ttx_internal.h"

namespace ttx {

struct PackPlan {
    int parts = 0;
    Problem prob[2];              // whole panels, ragged last panel
    ttx_config cfg[2];
    int64_t a_off[2] = {0, 0};    // element offsets into A and P
    int64_t p_off[2] = {0, 0};
    int64_t pad_off = 0;          // zero region of the last panel (elements of P)
    int64_t pad_width = 0, pad_height = 0, pad_pitch = 0;
    int64_t kpad_off = 0;         // matrix-core panels: the k padding of every panel
    int64_t kpad_width = 0, kpad_height = 0, kpad_pitch = 0;
    int64_t a_extent = 0, p_extent = 0;   // bytes
    int elem_p = 0;
    uint64_t table_gen = 0;
};

static ttx_status make_pack_plan(int dtype, int kind, int64_t rows, int64_t cols, int64_t ld, int64_t panel,
                                 PackPlan* pl) {
    if (!dtype_valid(dtype)) return fail(TTX_EINVAL, "unknown dtype");
    if (kind != TTX_PACK_ROWS && kind != TTX_PACK_COLS && kind != TTX_PACK_MFMA_A && kind != TTX_PACK_MFMA_B)
        return fail(TTX_EINVAL, "unknown packing kind");
    if (rows < 0 || cols < 0 || panel < 1) return fail(TTX_EINVAL, "negative extent or panel < 1");
    if (ld < rows || ld < 1) return fail(TTX_EINVAL, "ld smaller than the row count");
    const bool mfma = kind == TTX_PACK_MFMA_A || kind == TTX_PACK_MFMA_B;
    if (mfma && (panel > 64 || 64 % panel)) return fail(TTX_EINVAL, "matrix-core panels must divide 64");
    if (kind == TTX_PACK_MFMA_A) kind = TTX_PACK_ROWS;   // the same layouts, k padded below
    if (kind == TTX_PACK_MFMA_B) kind = TTX_PACK_COLS;
    *pl = PackPlan();
    pl->elem_p = elem_bytes(dtype_b_of(dtype));
    const int64_t ea = elem_bytes(dtype_a_of(dtype));
    const int64_t split = kind == TTX_PACK_ROWS ? rows : cols;   // the extent cut into panels
    const int64_t other = kind == TTX_PACK_ROWS ? cols : rows;   // k
    if (split == 0 || other == 0) return TTX_OK;
    const int64_t np = (split + panel - 1) / panel, full = split / panel, tail = split % panel;
    const int64_t kb = mfma ? 64 / panel : 1;
    const int64_t K = (other + kb - 1) / kb * kb;   // k of a stored panel
    int64_t tmp;
    if (__builtin_mul_overflow(np * panel, K, &tmp) || __builtin_mul_overflow(ld, cols, &tmp))
        return fail(TTX_EINVAL, "sizes overflow");
    pl->a_extent = ((cols - 1) * ld + rows) * ea;
    pl->p_extent = np * panel * K * pl->elem_p;
    if (K > other) {   // the k padding of every panel: its last (K - k) * panel elements
        pl->kpad_off = other * panel;
        pl->kpad_width = (K - other) * panel;
        pl->kpad_height = np;
        pl->kpad_pitch = panel * K;
    }
    auto add = [&](int n, const int* perm, const int64_t* size, const int64_t* sa, const int64_t* sb,
                   int64_t a_off, int64_t p_off) -> ttx_status {
        Problem& p = pl->prob[pl->parts];
        ttx_status st = make_problem_strided(dtype, n, perm, size, sa, sb, &p);
        if (st != TTX_OK) return st;
        pl->a_off[pl->parts] = a_off;
        pl->p_off[pl->parts] = p_off;
        ++pl->parts;
        return TTX_OK;
    };
    if (kind == TTX_PACK_ROWS) {
        const int64_t k = cols, mr = panel;
        if (full > 0) {
            const int perm[3] = {0, 2, 1};
            const int64_t size[3] = {mr, full, k}, sa[3] = {1, mr, ld}, sb[3] = {1, mr * K, mr};
            ttx_status st = add(3, perm, size, sa, sb, 0, 0);
            if (st != TTX_OK) return st;
        }
        if (tail > 0) {
            const int perm[2] = {0, 1};
            const int64_t size[2] = {tail, k}, sa[2] = {1, ld}, sb[2] = {1, mr};
            ttx_status st = add(2, perm, size, sa, sb, full * mr, full * mr * K);
            if (st != TTX_OK) return st;
            pl->pad_off = full * mr * K + tail;
            pl->pad_width = mr - tail;
            pl->pad_height = k;
            pl->pad_pitch = mr;
        }
    } else {
        const int64_t k = rows, nr = panel;
        if (full > 0) {
            const int perm[3] = {1, 0, 2};
            const int64_t size[3] = {k, nr, full}, sa[3] = {1, ld, ld * nr}, sb[3] = {nr, 1, nr * K};
            ttx_status st = add(3, perm, size, sa, sb, 0, 0);
            if (st != TTX_OK) return st;
        }
        if (tail > 0) {
            const int perm[2] = {1, 0};
            const int64_t size[2] = {k, tail}, sa[2] = {1, ld}, sb[2] = {nr, 1};
            ttx_status st = add(2, perm, size, sa, sb, full * nr * ld, full * nr * K);
            if (st != TTX_OK) return st;
            pl->pad_off = full * nr * K + tail;
            pl->pad_width = nr - tail;
            pl->pad_height = k;
            pl->pad_pitch = nr;
        }
    }
    pl->table_gen = table_generation();
    for (int i = 0; i < pl->parts; ++i)
        if (!table_lookup(pl->prob[i], true, &pl->cfg[i])) pl->cfg[i] = default_config(pl->prob[i]);
    return TTX_OK;
}

static std::mutex g_pack_mu;
static std::unordered_map<std::string, std::shared_ptr<PackPlan>> g_pack_cache;

static std::shared_ptr<PackPlan> cached_pack_plan(int dtype, int kind, int64_t rows, int64_t cols, int64_t ld,
                                                  int64_t panel, ttx_status* st) {
    const int64_t key_v[6] = {dtype, kind, rows, cols, ld, panel};
    const std::string key(reinterpret_cast<const char*>(key_v), sizeof(key_v));
    {
        std::lock_guard<std::mutex> lock(g_pack_mu);
        auto it = g_pack_cache.find(key);
        if (it != g_pack_cache.end() && it->second->table_gen == table_generation()) {
            *st = TTX_OK;
            return it->second;
        }
    }
    auto pl = std::make_shared<PackPlan>();
    *st = make_pack_plan(dtype, kind, rows, cols, ld, panel, pl.get());
    if (*st != TTX_OK) return nullptr;
    std::lock_guard<std::mutex> lock(g_pack_mu);
    if (g_pack_cache.size() >= 1024) g_pack_cache.clear();
    g_pack_cache[key] = pl;
    return pl;
}

}  // namespace ttx

using namespace ttx;

extern "C" {

ttx_status ttx_pack(ttx_dtype dtype, int kind, int64_t rows, int64_t cols, int64_t ld, int64_t panel,
                    const double* alpha, const void* A, void* P, hipStream_t stream) {
    if (!alpha) return fail(TTX_EINVAL, "alpha must not be NULL");
    ttx_status st;
    auto pl = cached_pack_plan(dtype, kind, rows, cols, ld, panel, &st);
    if (!pl) return st;
    const Scalar a(alpha[0], alpha[1]);
    if (!dtype_complex(dtype_b_of(dtype)) && a.im != 0.0)
        return fail(TTX_EINVAL, "complex alpha for a real element type");
    if (pl->p_extent == 0) return TTX_OK;
    if (!A || !P) return fail(TTX_EINVAL, "NULL matrix pointer");
    const uintptr_t ua = reinterpret_cast<uintptr_t>(A), up = reinterpret_cast<uintptr_t>(P);
    if (ua % elem_bytes(dtype_a_of(dtype)) || up % pl->elem_p)
        return fail(TTX_EINVAL, "pointer not aligned to the element size");
    if (ua < up + uint64_t(pl->p_extent) && up < ua + uint64_t(pl->a_extent))
        return fail(TTX_EOVERLAP, "A and the packed panels overlap");
    const int ea = elem_bytes(dtype_a_of(dtype));
    for (int i = 0; i < pl->parts; ++i) {
        const char* Ai = static_cast<const char*>(A) + pl->a_off[i] * ea;
        char* Pi = static_cast<char*>(P) + pl->p_off[i] * pl->elem_p;
        hipError_t e = launch_tiles(pl->prob[i], pl->cfg[i], true, Ai, nullptr, Pi, a, Scalar(0.0), stream);
        if (e != hipSuccess) return fail(TTX_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    if (pl->pad_width > 0) {
        hipError_t e = launch_fill_zero(static_cast<char*>(P) + pl->pad_off * pl->elem_p,
                                        pl->pad_width * pl->elem_p, pl->pad_height,
                                        pl->pad_pitch * pl->elem_p, stream);
        if (e != hipSuccess) return fail(TTX_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    if (pl->kpad_width > 0) {
        hipError_t e = launch_fill_zero(static_cast<char*>(P) + pl->kpad_off * pl->elem_p,
                                        pl->kpad_width * pl->elem_p, pl->kpad_height,
                                        pl->kpad_pitch * pl->elem_p, stream);
        if (e != hipSuccess) return fail(TTX_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return TTX_OK;
}

ttx_status ttx_pack_tune(ttx_dtype dtype, int kind, int64_t rows, int64_t cols, int64_t ld, int64_t panel,
                         int max_candidates, int reps) {
    PackPlan pl;
    ttx_status st = make_pack_plan(dtype, kind, rows, cols, ld, panel, &pl);
    if (st != TTX_OK) return st;
    for (int i = 0; i < pl.parts; ++i) {
        ttx_config best;
        st = tune_problem(pl.prob[i], true, max_candidates, reps, &best, nullptr);
        if (st != TTX_OK) return st;
    }
    return TTX_OK;
}

ttx_status ttx_pack_describe(ttx_dtype dtype, int kind, int64_t rows, int64_t cols, int64_t ld, int64_t panel,
                             int64_t* packed_elements, int* transpositions, ttx_config* configs) {
    PackPlan pl;
    ttx_status st = make_pack_plan(dtype, kind, rows, cols, ld, panel, &pl);
    if (st != TTX_OK) return st;
    if (packed_elements) *packed_elements = pl.p_extent / (pl.elem_p ? pl.elem_p : 1);
    if (transpositions) *transpositions = pl.parts;
    if (configs)
        for (int i = 0; i < pl.parts; ++i) configs[i] = pl.cfg[i];
    return TTX_OK;
}

}  // extern "C"
