// Host planner: argument validation, stride form, size-1 removal, index
// merging (Sec. 2.1 stage 1), family choice (Sec. 2.2, Sec. 3.2), the
// blocking and loop-order heuristics of Sec. 2.3 and candidate ranking
// (Sec. 2.1 stages 2-3).  No HIP call is made here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <vector>

#include "menu.h"
#include "ttx_internal.h"

namespace ttx {

// ---------------------------------------------------------------------------------------
// Menus
#define TTX_SHAPE(a, b) {a, b},
static const TileShape kMovedF32[] = {TTX_MOVED_MENU_F32(TTX_SHAPE)};
static const TileShape kMovedF64[] = {TTX_MOVED_MENU_F64(TTX_SHAPE)};
static const TileShape kMovedC64[] = {TTX_MOVED_MENU_C64(TTX_SHAPE)};
static const TileShape kPresF32[] = {TTX_PRESERVED_MENU_F32(TTX_SHAPE)};
static const TileShape kPresF64[] = {TTX_PRESERVED_MENU_F64(TTX_SHAPE)};
static const TileShape kPresC64[] = {TTX_PRESERVED_MENU_C64(TTX_SHAPE)};
#undef TTX_SHAPE

#define TTX_COUNT(arr) int(sizeof(arr) / sizeof(arr[0]))

// Single complex elements have the byte size of FP64 ones and use the FP64 menus.
int tile_menu(int dtype, int family, const TileShape** shapes) {
    if (family == TTX_FAMILY_MOVED) {
        if (dtype == TTX_F32) return *shapes = kMovedF32, TTX_COUNT(kMovedF32);
        if (dtype == TTX_C64) return *shapes = kMovedC64, TTX_COUNT(kMovedC64);
        return *shapes = kMovedF64, TTX_COUNT(kMovedF64);
    }
    if (family == TTX_FAMILY_PRESERVED) {
        if (dtype == TTX_F32) return *shapes = kPresF32, TTX_COUNT(kPresF32);
        if (dtype == TTX_C64) return *shapes = kPresC64, TTX_COUNT(kPresC64);
        return *shapes = kPresF64, TTX_COUNT(kPresF64);
    }
    *shapes = nullptr;
    return 0;
}

#define TTX_STAGED(n0, tx, ty) {n0, tx, ty},
struct StagedShape { int n0, tx, ty; };
static const StagedShape kStagedF32[] = {TTX_STAGED_MENU_F32(TTX_STAGED)};
static const StagedShape kStagedF64[] = {TTX_STAGED_MENU_F64(TTX_STAGED)};
static const StagedShape kStagedC64[] = {TTX_STAGED_MENU_C64(TTX_STAGED)};
#undef TTX_STAGED

int staged_lanes(int64_t n0) {
    if (n0 <= 16) return 16;
    if (n0 <= 32) return 32;
    if (n0 <= 64) return 64;
    return 0;
}

static int staged_menu(int dtype, const StagedShape** out) {
    if (dtype == TTX_F32) return *out = kStagedF32, TTX_COUNT(kStagedF32);
    if (dtype == TTX_C64) return *out = kStagedC64, TTX_COUNT(kStagedC64);
    return *out = kStagedF64, TTX_COUNT(kStagedF64);
}

bool staged_in_menu(int dtype, int n0_max, int tx, int ty) {
    const StagedShape* m;
    const int n = staged_menu(dtype, &m);
    for (int i = 0; i < n; ++i)
        if (m[i].n0 == n0_max && m[i].tx == tx && m[i].ty == ty) return true;
    return false;
}

bool tile_in_menu(int dtype, int family, int ta, int tb) {
    const TileShape* s;
    int n = tile_menu(dtype, family, &s);
    for (int i = 0; i < n; ++i)
        if (s[i].ta == ta && s[i].tb == tb) return true;
    return false;
}

#define TTX_SHAPE(a, b) {a, b},
static const TileShape kLargeF32[] = {TTX_MOVED_LARGE_F32(TTX_SHAPE)};
static const TileShape kLargeF64[] = {TTX_MOVED_LARGE_F64(TTX_SHAPE)};
static const TileShape kLargeC64[] = {TTX_MOVED_LARGE_C64(TTX_SHAPE)};
#undef TTX_SHAPE

int large_tile_menu(int dtype, const TileShape** shapes) {
    if (dtype == TTX_F32) return *shapes = kLargeF32, TTX_COUNT(kLargeF32);
    if (dtype == TTX_C64) return *shapes = kLargeC64, TTX_COUNT(kLargeC64);
    return *shapes = kLargeF64, TTX_COUNT(kLargeF64);
}

bool tile_in_large_menu(int dtype, int ta, int tb) {
    const TileShape* s;
    const int n = large_tile_menu(dtype, &s);
    for (int i = 0; i < n; ++i)
        if (s[i].ta == ta && s[i].tb == tb) return true;
    return false;
}

// ---------------------------------------------------------------------------------------
// Problem construction
ttx_status make_problem(int dtype, int n, const int* perm, const int64_t* size,
                        const int64_t* outer_a, const int64_t* outer_b, Problem* out) {
    if (!dtype_valid(dtype)) return fail(TTX_EINVAL, "unknown dtype");
    if (n < 1 || n > kMaxDims) return fail(TTX_EINVAL, "n must be in 1..16");
    if (!perm || !size) return fail(TTX_EINVAL, "perm and size must not be NULL");
    bool seen[kMaxDims] = {};
    for (int k = 0; k < n; ++k) {
        if (perm[k] < 0 || perm[k] >= n || seen[perm[k]])
            return fail(TTX_EPERM, "perm is not a permutation of 0..n-1");
        seen[perm[k]] = true;
    }
    for (int m = 0; m < n; ++m)
        if (size[m] < 0) return fail(TTX_EINVAL, "negative extent");

    // Stride form: A strides by A position, B strides by B position.
    int64_t sa[kMaxDims], sbpos[kMaxDims], sb[kMaxDims];
    int64_t prod = 1;
    for (int m = 0; m < n; ++m) {
        int64_t o = outer_a ? outer_a[m] : size[m];
        if (o < size[m]) return fail(TTX_EINVAL, "outer_a smaller than size");
        sa[m] = prod;
        if (__builtin_mul_overflow(prod, o, &prod)) return fail(TTX_EINVAL, "outer_a overflows");
    }
    prod = 1;
    for (int k = 0; k < n; ++k) {
        int64_t sz = size[perm[k]];
        int64_t o = outer_b ? outer_b[k] : sz;
        if (o < sz) return fail(TTX_EINVAL, "outer_b smaller than the B extent");
        sbpos[k] = prod;
        if (__builtin_mul_overflow(prod, o, &prod)) return fail(TTX_EINVAL, "outer_b overflows");
    }
    for (int k = 0; k < n; ++k) sb[perm[k]] = sbpos[k];
    return make_problem_strided(dtype, n, perm, size, sa, sb, out);
}

ttx_status make_problem_strided(int dtype, int n, const int* perm, const int64_t* size,
                                const int64_t* sa, const int64_t* sb, Problem* out) {
    Problem p;
    p.code = dtype;
    p.dtype = dtype_b_of(dtype);
    p.dtype_a = dtype_a_of(dtype);
    p.n_orig = n;
    const int ea = elem_bytes(p.dtype_a), eb = elem_bytes(p.dtype);
    bool empty = false;
    int64_t last_a = 0, last_b = 0, elems = 1;
    for (int m = 0; m < n; ++m) {
        if (size[m] == 0) empty = true;
        last_a += (size[m] - 1) * sa[m];
        last_b += (size[m] - 1) * sb[m];
        elems *= size[m] ? size[m] : 1;
    }
    if (empty) {
        p.family = TTX_FAMILY_EMPTY;
        p.n = 0;
        p.elements = 0;
        *out = p;
        return TTX_OK;
    }
    p.elements = elems;
    p.extent_a = (last_a + 1) * ea;
    p.extent_b = (last_b + 1) * eb;

    // Drop extent-1 indices; their leading dimensions already sit in the
    // strides of the later indices.
    int keep_id[kMaxDims];
    int nk = 0;
    for (int m = 0; m < n; ++m) {
        keep_id[m] = -1;
        if (size[m] != 1) {
            keep_id[m] = nk;
            p.dim[nk] = Dim{size[m], sa[m], sb[m]};
            ++nk;
        }
    }
    int kp = 0;
    for (int k = 0; k < n; ++k)
        if (keep_id[perm[k]] >= 0) p.perm[kp++] = keep_id[perm[k]];
    if (nk == 0) {  // a single element
        p.n = 1;
        p.dim[0] = Dim{1, 1, 1};
        p.perm[0] = 0;
        p.family = TTX_FAMILY_FLAT;
        *out = p;
        return TTX_OK;
    }
    p.n = nk;

    // Merge (Sec. 2.1 stage 1): A indices m and m+1 fuse into one super index
    // when they are neighbours in the same order in B and contiguous in both
    // tensors (no leading-dimension gap between them in A or in B).
    bool merged = true;
    while (merged) {
        merged = false;
        for (int k = 0; k + 1 < p.n; ++k) {
            int m = p.perm[k];
            if (p.perm[k + 1] != m + 1) continue;
            const Dim& lo = p.dim[m];
            const Dim& hi = p.dim[m + 1];
            if (hi.sa != lo.sa * lo.size || hi.sb != lo.sb * lo.size) continue;
            p.dim[m].size = lo.size * hi.size;
            for (int d = m + 1; d + 1 < p.n; ++d) p.dim[d] = p.dim[d + 1];
            for (int q = k + 1; q + 1 < p.n; ++q) p.perm[q] = p.perm[q + 1];
            --p.n;
            for (int q = 0; q < p.n; ++q)
                if (p.perm[q] > m) --p.perm[q];
            merged = true;
            break;
        }
    }

    if (p.n == 1)
        p.family = TTX_FAMILY_FLAT;
    else if (p.perm[0] == 0)
        p.family = TTX_FAMILY_PRESERVED;
    else
        p.family = TTX_FAMILY_MOVED;
    *out = p;
    return TTX_OK;
}

// ---------------------------------------------------------------------------------------
// Tile layout.  A moved-family tile spans two "super indices": the A side is
// the first ga merged indices (consecutive in A and contiguous there, so the
// tile reads runs of TA elements across all of them), the B side the first
// gb indices in B's order (contiguous in B).  With ga = gb = 1 this is the
// 2D macro-tile of Sec. 2.2; larger groups keep tiles full when the stride-1
// extents are short (e.g. 24 x 17 for a 6D reversal).  The preserved family
// tiles A's stride-1 index against B's second index; flat has one index.
struct Layout {
    int a = 0, b = 0;                 // leaders (merged index numbers)
    int ga = 1, gb = 1;
    bool staged = false;              // preserved family with short rows: staged tiles
    // group members: moved layouts list all ga (gb) indices; staged layouts
    // list the ga - 1 (gb - 1) indices after the shared row index
    int memA[kMaxGroup] = {}, memB[kMaxGroup] = {};
    int64_t SA = 1, SB = 1;           // super extents
    bool member[kMaxDims] = {};       // non-leader group members: not grid indices
};

static bool make_layout(const Problem& p, int ga, int gb, Layout* L) {
    L->ga = ga < 1 ? 1 : ga;
    L->gb = gb < 1 ? 1 : gb;
    L->a = 0;
    if (p.family == TTX_FAMILY_FLAT) {
        L->b = 0;
        L->SA = L->SB = p.dim[0].size;
        return L->ga == 1 && L->gb == 1;
    }
    if (p.family == TTX_FAMILY_PRESERVED && L->ga == 1 && L->gb == 1) {
        L->b = p.perm[1];
        L->SA = p.dim[0].size;
        L->SB = p.dim[L->b].size;
        return true;
    }
    if (p.family == TTX_FAMILY_PRESERVED) {
        // staged: A's indices 1..ga-1 (contiguous with each other in A) and
        // B's indices perm[1..gb-1] (contiguous with each other in B) span the
        // tile; the row index 0 lies wholly inside every tile
        if (L->ga < 2 || L->gb < 2 || L->ga > kMaxGroup + 1 || L->gb > kMaxGroup + 1) return false;
        if (L->ga > p.n || L->gb > p.n || staged_lanes(p.dim[0].size) == 0) return false;
        bool inA[kMaxDims] = {};
        L->SA = 1;
        for (int k = 1; k < L->ga; ++k) {
            if (k > 1 && p.dim[k].sa != p.dim[k - 1].sa * p.dim[k - 1].size) return false;
            L->memA[k - 1] = k;
            inA[k] = true;
            L->SA *= p.dim[k].size;
        }
        L->SB = 1;
        for (int k = 1; k < L->gb; ++k) {
            const int d = p.perm[k], prev = p.perm[k - 1];
            if (inA[d] || (k > 1 && p.dim[d].sb != p.dim[prev].sb * p.dim[prev].size)) return false;
            L->memB[k - 1] = d;
            L->SB *= p.dim[d].size;
        }
        if (L->SA >= (int64_t(1) << 31) || L->SB >= (int64_t(1) << 31)) return false;
        L->staged = true;
        L->a = 1;
        L->b = p.perm[1];
        L->member[0] = true;
        for (int k = 1; k < L->ga - 1; ++k) L->member[L->memA[k]] = true;
        for (int k = 1; k < L->gb - 1; ++k) L->member[L->memB[k]] = true;
        return true;
    }
    if (L->ga > kMaxGroup || L->gb > kMaxGroup || L->ga > p.n || L->gb > p.n) return false;
    bool inA[kMaxDims] = {};
    L->SA = 1;
    for (int k = 0; k < L->ga; ++k) {
        const int d = k;   // A's first ga indices
        if (k > 0 && p.dim[d].sa != p.dim[d - 1].sa * p.dim[d - 1].size) return false;
        L->memA[k] = d;
        inA[d] = true;
        L->SA *= p.dim[d].size;
    }
    L->SB = 1;
    for (int k = 0; k < L->gb; ++k) {
        const int d = p.perm[k];   // B's first gb indices
        if (inA[d]) return false;
        if (k > 0) {
            const int prev = p.perm[k - 1];
            if (p.dim[d].sb != p.dim[prev].sb * p.dim[prev].size) return false;
        }
        L->memB[k] = d;
        L->SB *= p.dim[d].size;
    }
    // digits are extracted with 32-bit divisions when a group has several members
    if ((L->ga > 1 && L->SA >= (int64_t(1) << 31)) || (L->gb > 1 && L->SB >= (int64_t(1) << 31)))
        return false;
    L->b = p.perm[0];
    for (int k = 1; k < L->ga; ++k) L->member[L->memA[k]] = true;
    for (int k = 1; k < L->gb; ++k) L->member[L->memB[k]] = true;
    return true;
}

// Group sizes worth considering: a group grows only while its super extent
// is still short of a full tile edge (< 64 elements).
static std::vector<std::pair<int, int>> group_options(const Problem& p) {
    std::vector<std::pair<int, int>> out;
    if (p.family == TTX_FAMILY_PRESERVED) {
        out.push_back({1, 1});
        // staged tiles for rows shorter than a 256-byte run; each side grows
        // while its run (row length times the rows fused so far) is short
        const int64_t n0 = p.dim[0].size;
        if (n0 * elem_bytes(p.dtype) >= 256 || staged_lanes(n0) == 0) return out;
        for (int ga = 2; ga <= kMaxGroup + 1; ++ga)
            for (int gb = 2; gb <= kMaxGroup + 1; ++gb) {
                Layout L;
                if (!make_layout(p, ga, gb, &L)) continue;
                if (ga > 2 && n0 * (L.SA / p.dim[L.memA[ga - 2]].size) >= 256) continue;
                if (gb > 2 && n0 * (L.SB / p.dim[L.memB[gb - 2]].size) >= 256) continue;
                out.push_back({ga, gb});
            }
        return out;
    }
    if (p.family != TTX_FAMILY_MOVED) {
        out.push_back({1, 1});
        return out;
    }
    for (int ga = 1; ga <= kMaxGroup; ++ga)
        for (int gb = 1; gb <= kMaxGroup; ++gb) {
            Layout L;
            if (!make_layout(p, ga, gb, &L)) continue;
            if (ga > 1 && L.SA / p.dim[L.memA[ga - 1]].size >= 64) continue;
            if (gb > 1 && L.SB / p.dim[L.memB[gb - 1]].size >= 64) continue;
            out.push_back({ga, gb});
        }
    return out;
}

static Group make_group(const Problem& p, const int* members, int ng, bool strides_of_a) {
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.ng = ng;
    for (int k = 0; k < ng; ++k) {
        if (k + 1 < ng) g.div[k].init(uint32_t(p.dim[members[k]].size));
        g.stride[k] = strides_of_a ? p.dim[members[k]].sa : p.dim[members[k]].sb;
    }
    return g;
}

// The third index of a dense tile: the first index of the loop order that is
// neither a tile index nor a group member (-1 if there is none).
static int dense_z(const Problem& p, const Layout& L, const int* order, int n) {
    for (int k = 0; k < n; ++k) {
        const int d = order[k];
        if (d != L.a && d != L.b && !L.member[d]) return d;
    }
    return -1;
}

// ---------------------------------------------------------------------------------------
// Config validation and the kernel-side grid
bool widen(const Problem& p, Problem* w) {
    if (p.family != TTX_FAMILY_PRESERVED || p.dtype != p.dtype_a) return false;
    if (p.dtype != TTX_F32 && p.dtype != TTX_F64) return false;
    if (p.dim[0].sa != 1 || p.dim[0].sb != 1) return false;
    auto fits = [&](int64_t k) {
        if (p.dim[0].size % k || p.dim[0].size / k < 2) return false;
        for (int d = 1; d < p.n; ++d)
            if (p.dim[d].sa % k || p.dim[d].sb % k) return false;
        return true;
    };
    int k = 0, code = 0;
    if (p.dtype == TTX_F32) {
        if (fits(4)) k = 4, code = kWideF32x4;
        else if (fits(2)) k = 2, code = kWideF32x2;
    } else if (fits(2)) {
        k = 2, code = kWideF64x2;
    }
    if (!k) return false;
    *w = p;
    w->dtype = w->dtype_a = w->code = code;
    w->dim[0].size /= k;
    for (int d = 1; d < p.n; ++d) {
        w->dim[d].sa /= k;
        w->dim[d].sb /= k;
    }
    w->elements /= k;
    return true;
}

// Whether a tile of config c (shape already validated) can run with
// c.threads threads and c.lds_pad padding: the tile's rows (in vectors)
// must fit the workgroup, each thread may hold at most kMaxVectors vectors
// per side (register budget), staged and dense tiles must split into whole
// passes, and the LDS tile must fit a workgroup's 64 KiB.  The vector widths
// are the ones the launch will use (kernel_flags: they depend on strides
// and the tile shape only).  The pre-compiled configurations (256 threads,
// padding 1) all pass.
static constexpr int kMaxVectors = 32;

static int per_thread(int run, int rows, int nt) {   // vectors per thread: runs of `run` over `rows`
    int lanes = 1;
    while (lanes < run) lanes <<= 1;
    if (lanes > nt) return -1;
    const int per_pass = nt / lanes;
    return (rows + per_pass - 1) / per_pass;
}

static bool workgroup_fits(const Problem& p, const Layout& L, const ttx_config& c, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    const int nt = c.threads;
    const int es = elem_bytes(p.dtype);
    if (config_is_dense(c)) {
        const int cap = dense_cap(p.dtype);
        if (cap % nt || cap / nt > 16) return bad("dense tile slots do not split over this many threads");
        return true;
    }
    if (L.staged) {
        const int n0 = staged_lanes(p.dim[0].size);
        const int slots = n0 * c.tile_a * c.tile_b;
        if (slots % nt || slots / nt > kMaxVectors) return bad("staged tile does not split over this many threads");
        if (int64_t(c.tile_b) * (int64_t(c.tile_a) * n0 + c.lds_pad) * es > 65536)
            return bad("staged LDS tile larger than 64 KiB");
        return true;
    }
    const int VAe = 16 / elem_bytes(p.dtype_a), VBe = 16 / es;
    if (p.family == TTX_FAMILY_PRESERVED) {
        const int V = VAe < VBe ? VAe : VBe;
        const int v = (p.dim[0].sa == 1 && p.dim[0].sb == 1 && c.tile_a % V == 0) ? V : 1;
        const int k = per_thread(c.tile_a / v, c.tile_b, nt);
        if (k < 0 || k > kMaxVectors) return bad("preserved tile rows do not fit this many threads");
        return true;
    }
    const int va = (p.dim[L.a].sa == 1 && c.tile_a % VAe == 0) ? VAe : 1;
    const int vb = (p.dim[L.b].sb == 1 && c.tile_b % VBe == 0) ? VBe : 1;
    const int ka = per_thread(c.tile_a / va, c.tile_b, nt), kb = per_thread(c.tile_b / vb, c.tile_a, nt);
    if (ka < 0 || kb < 0 || ka > kMaxVectors || kb > kMaxVectors)
        return bad("moved tile runs do not fit this many threads");
    if (int64_t(c.tile_b) * (c.tile_a + c.lds_pad) * es > 65536) return bad("LDS tile larger than 64 KiB");
    return true;
}

bool config_valid(const Problem& p, const ttx_config& c, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (c.family != p.family) return bad("config family does not match the problem");
    if (c.threads != 64 && c.threads != 128 && c.threads != 256 && c.threads != 512)
        return bad("threads must be 64, 128, 256 or 512");
    if (c.lds_pad < 0 || c.lds_pad > TTX_MAX_LDS_PAD) return bad("lds_pad out of range");
    if (c.flags & ~(TTX_CFG_XCD_SWIZZLE | TTX_CFG_NT_STORE | TTX_CFG_DENSE | TTX_CFG_WIDE | TTX_CFG_GROUPED |
                    TTX_CFG_ALIGN_A | TTX_CFG_PIPELINED))
        return bad("unknown flag");
    if (config_is_wide(c)) {
        if (!config_is_dense(c)) return bad("whole-unit rows are for dense tiles only");
        Problem w;
        if (!widen(p, &w)) return bad("the rows cannot be moved in whole units");
        ttx_config cw = c;
        cw.flags &= ~TTX_CFG_WIDE;
        return config_valid(w, cw, why);
    }
    if (p.family == TTX_FAMILY_EMPTY) return true;
    if (c.n_order != p.n) return bad("order must list every merged index");
    bool seen[kMaxDims] = {};
    for (int i = 0; i < c.n_order; ++i) {
        if (c.order[i] < 0 || c.order[i] >= p.n || seen[c.order[i]])
            return bad("order is not a permutation of the merged indices");
        seen[c.order[i]] = true;
    }
    Layout L;
    if (!make_layout(p, c.group_a, c.group_b, &L)) return bad("invalid index groups for this problem");
    if ((c.flags & TTX_CFG_PIPELINED) && (p.family == TTX_FAMILY_FLAT || config_is_dense(c)))
        return bad("pipelined grids are for moved and preserved tiles (dense tiles always pipeline)");
    if (p.family == TTX_FAMILY_FLAT) {
        if (config_is_dense(c)) return bad("dense tiles need a moved or preserved problem");
        if (c.threads != kThreads) return bad("flat problems run 256 threads per workgroup");
        return true;
    }
    const int64_t tc = c.tile_c > 1 ? c.tile_c : 1;
    int z = -1;
    if (config_is_dense(c)) {
        if (p.family == TTX_FAMILY_PRESERVED && !L.staged)
            return bad("dense preserved tiles need index groups (short rows)");
        const int64_t rows = L.staged ? p.dim[0].size : 1;
        if (c.tile_a < 1 || c.tile_b < 1 || c.tile_a > dense_cap(p.dtype) || c.tile_b > dense_cap(p.dtype) ||
            tc > dense_cap(p.dtype) || rows * c.tile_a * c.tile_b * tc > dense_cap(p.dtype))
            return bad("dense tile larger than the dense capacity");
        if (tc > 1) {
            z = dense_z(p, L, c.order, c.n_order);
            if (z < 0) return bad("tile_c needs a third index outside the tile");
        }
        // offsets within a dense tile are 32-bit
        if (p.extent_a / elem_bytes(p.dtype_a) >= (int64_t(1) << 31) ||
            p.extent_b / elem_bytes(p.dtype) >= (int64_t(1) << 31))
            return bad("dense tiles need tensors below 2^31 elements");
    } else if (tc > 1) {
        return bad("tile_c is for dense tiles only");
    } else if (L.staged) {
        if (!staged_in_menu(p.dtype, staged_lanes(p.dim[0].size), c.tile_a, c.tile_b))
            return bad("staged tile shape not in menu");
    } else if (!tile_in_menu(p.dtype, p.family, c.tile_a, c.tile_b) &&
               !(p.family == TTX_FAMILY_MOVED && tile_in_large_menu(p.dtype, c.tile_a, c.tile_b))) {
        return bad("tile shape not in menu");
    }
    const int aln = config_align_elems(c, elem_bytes(p.dtype_a));
    if (aln && (p.family != TTX_FAMILY_MOVED || config_is_dense(c) || L.staged || p.dim[L.a].sa != 1 ||
                128 % elem_bytes(p.dtype_a)))
        return bad("line-aligned A runs need a moved menu tile over a contiguous A run");
    // the tile id space must fit 32 bits (line-aligned runs add one tile along A's run)
    uint64_t tiles = uint64_t((L.SA + (aln ? aln - 1 : 0) + c.tile_a - 1) / c.tile_a) *
                     uint64_t((L.SB + c.tile_b - 1) / c.tile_b);
    for (int d = 0; d < p.n; ++d) {
        if (d == L.a || d == L.b || L.member[d]) continue;
        tiles *= d == z ? uint64_t((p.dim[d].size + tc - 1) / tc) : uint64_t(p.dim[d].size);
        if (tiles >= (uint64_t(1) << 32)) return bad("too many tiles for this tile shape");
    }
    if (tiles >= (uint64_t(1) << 32)) return bad("too many tiles for this tile shape");
    return workgroup_fits(p, L, c, why);
}

void build_grid(const Problem& p, const ttx_config& c, TileArgsHost* h) {
    if (config_is_wide(c)) {   // the grid of the problem over whole units
        Problem w;
        widen(p, &w);
        ttx_config cw = c;
        cw.flags &= ~TTX_CFG_WIDE;
        build_grid(w, cw, h);
        return;
    }
    Layout L;
    make_layout(p, c.group_a, c.group_b, &L);
    TileGrid* g = &h->g;
    std::memset(g, 0, sizeof(*g));
    g->pa = g->pb = g->pz = -1;
    const bool moved = p.family == TTX_FAMILY_MOVED || L.staged;
    const int tc = config_is_dense(c) && c.tile_c > 1 ? c.tile_c : 1;
    const int z = tc > 1 ? dense_z(p, L, c.order, c.n_order) : -1;
    uint64_t tiles = 1;
    int q = 0;
    for (int i = 0; i < p.n; ++i) {
        const int d = c.order[i];
        if (L.member[d]) continue;
        int64_t ext = 1, extent = p.dim[d].size;
        int64_t stepA, stepB;
        if (d == L.a) {
            ext = c.tile_a;
            // line-aligned A runs shift each tile down by up to a line less
            // one element: one more tile covers the end of the run
            const int aln = config_align_elems(c, elem_bytes(p.dtype_a));
            extent = L.SA + (aln ? aln - 1 : 0);
        } else if (d == L.b) {
            ext = c.tile_b;
            extent = L.SB;
        } else if (d == z) {
            ext = tc;
        }
        stepA = ext * p.dim[d].sa;
        stepB = ext * p.dim[d].sb;
        // moved tiles add the group offsets of their absolute coordinates in
        // the body, so the cross terms are left out of the origin here
        if (moved && d == L.a) stepB = 0;
        if (moved && d == L.b) stepA = 0;
        const uint32_t cnt = uint32_t((extent + ext - 1) / ext);
        g->count[q] = cnt;
        g->div[q].init(cnt);
        g->stepA[q] = stepA;
        g->stepB[q] = stepB;
        if (d == L.a) g->pa = q;
        if (d == L.b) g->pb = q;
        if (d == z) g->pz = q;
        tiles *= cnt;
        ++q;
    }
    g->nd = q;
    g->ntiles = uint32_t(tiles);
    g->gk = 0;
    if ((c.flags & TTX_CFG_GROUPED) && q >= 2 && g->count[0] > 1 && g->count[1] > 1 &&
        uint64_t(kGroupedSteps) * g->count[1] < (uint64_t(1) << 31) &&
        uint64_t(g->count[0]) * g->count[1] < (uint64_t(1) << 31)) {
        g->gk = kGroupedSteps;
        g->dvg.init(kGroupedSteps * g->count[1]);
        g->dvp.init(g->count[0] * g->count[1]);
    }
    g->ext_a = L.SA;
    g->ext_b = L.SB;
    h->sAa = p.dim[L.a].sa;
    h->sAb = p.dim[L.b].sa;
    h->sBa = p.dim[L.a].sb;
    h->sBb = p.dim[L.b].sb;
    h->gA = make_group(p, L.memA, L.staged ? L.ga - 1 : (moved ? L.ga : 1), false);   // B offsets of the A side
    h->gB = make_group(p, L.memB, L.staged ? L.gb - 1 : (moved ? L.gb : 1), true);    // A offsets of the B side
    if (!moved) {
        h->gA.stride[0] = p.dim[L.a].sb;
        h->gB.stride[0] = p.dim[L.b].sa;
    }
    h->s0A = p.dim[0].sa;
    h->s0B = p.dim[0].sb;
    h->n0 = int(p.dim[0].size);
    // dense tiles (harmless values for the other kinds)
    h->dn0 = L.staged ? int(p.dim[0].size) : 1;
    h->tx = c.tile_a > 0 ? c.tile_a : 1;
    h->ty = c.tile_b > 0 ? c.tile_b : 1;
    h->runA = uint32_t(h->dn0) * uint32_t(h->tx);
    h->runB = uint32_t(h->dn0) * uint32_t(h->ty);
    h->ldr = int(h->runA % 2 == 0 ? h->runA + 1 : h->runA);   // odd rows spread the banks
    h->dv0.init(uint32_t(h->dn0));
    h->dvA.init(h->runA);
    h->dvB.init(h->runB);
    g->ext_z = z >= 0 ? p.dim[z].size : 1;
    h->tz = tc;
    h->sAz = z >= 0 ? p.dim[z].sa : 0;
    h->sBz = z >= 0 ? p.dim[z].sb : 0;
    h->planeA = h->runA * uint32_t(h->ty);
    h->planeB = h->runB * uint32_t(h->tx);
    h->dvPA.init(h->planeA);
    h->dvPB.init(h->planeB);
}

static bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; }

int kernel_flags(const Problem& p, const ttx_config& c, const void* A, const void* Bsrc,
                 const void* Bdst) {
    int f = 0;
    if (c.flags & TTX_CFG_NT_STORE) f |= KF_NT_STORE;
    if (c.flags & TTX_CFG_XCD_SWIZZLE) f |= KF_SWIZZLE;
    // elements per 16-byte vector of A and of B; kept-row tiles (and flat)
    // use one width for both sides
    const int VA = 16 / elem_bytes(p.dtype_a), VB = 16 / elem_bytes(p.dtype);
    const int V = VA < VB ? VA : VB;
    const bool bptrs = aligned16(Bdst) && (Bsrc == nullptr || aligned16(Bsrc));
    if (p.family == TTX_FAMILY_FLAT) {
        if (p.dim[0].sa == 1 && p.dim[0].sb == 1 && aligned16(A) && bptrs) f |= KF_VEC_A;
        return f;
    }
    if (config_is_dense(c)) return f;   // dense tiles move single elements
    Layout L;
    if (!make_layout(p, c.group_a, c.group_b, &L)) return f;
    if (L.staged) return f;   // staged tiles move single elements
    // Menu tiles take 16-byte vectors wherever the tile's run is contiguous:
    // the vectors need only element alignment (runs may start anywhere) and
    // a run's last, partial vector is moved element by element.
    if (p.family == TTX_FAMILY_PRESERVED) {
        if (p.dim[0].sa == 1 && p.dim[0].sb == 1 && c.tile_a % V == 0) f |= KF_VEC_A | KF_VEC_B;
        return f;
    }
    if (p.dim[L.a].sa == 1 && c.tile_a % VA == 0) f |= KF_VEC_A;
    if (p.dim[L.b].sb == 1 && c.tile_b % VB == 0) f |= KF_VEC_B;
    return f;
}

// ---------------------------------------------------------------------------------------
// Heuristics (Sec. 2.3).
//
// Blocking: the cost of a tile shape is the estimated HBM traffic per useful
// byte.  Memory moves in 128-byte lines, so a contiguous run is charged its
// line-rounded size (the cache-line preference of Sec. 2.3); edge tiles of
// indices not divisible by the tile edge are charged separately (the
// remainder S mod b of Sec. 2.3), and every tile pays a fixed overhead for
// its decode and barrier, which favours larger tiles.  Idle lanes in edge
// tiles add an instruction-issue term (a quarter of the idle fraction).
//
// Loop order: Sec. 2.3 prefers loop orders whose innermost loops have small
// strides in A and B.  On the GPU the "innermost loops" are the tile
// indices that vary fastest with the workgroup id; about 2048 tiles are
// resident at once (256 CUs x 8 workgroups), so an order is charged the
// address span those resident tiles cover in A and B, relative to the bytes
// they move: compact spans keep DRAM pages and TLB entries hot.
static constexpr double kLine = 128.0;
static constexpr double kTileOverhead = 1536.0;  // bytes-equivalent per tile
static constexpr double kResident = 2048.0;

// Element-wise accesses (dense and staged tiles, and menu tiles whose runs
// cannot take 16-byte vectors) are charged a fixed 15% over vector tiles,
// except for 16-byte elements (double complex), which are whole vectors.
static constexpr double kScalarPenalty = 1.15;
static double scalar_penalty(const Problem& p) { return elem_bytes(p.dtype) >= 16 ? 1.0 : kScalarPenalty; }
// Dense tiles also decode every element's coordinates at run time; over
// whole units of kept rows (8 or 16 bytes each) that work is shared by
// several elements.
static constexpr double kDensePenalty = 1.3;
static constexpr double kWideDensePenalty = 1.1;

static double lines(double bytes) { return std::ceil(bytes / kLine) * kLine; }

// Staged tiles: A runs of n0*x rows, B runs of n0*y rows, n0_max lanes per row.
static double staged_cost(const Problem& p, const Layout& L, int tx, int ty) {
    const double e = elem_bytes(p.dtype);
    const double n0 = double(p.dim[0].size), lanes_row = staged_lanes(p.dim[0].size);
    double traffic = 0, useful = 0, lanes = 0, work = 0;
    for (int ix = 0; ix < 2; ++ix)
        for (int iy = 0; iy < 2; ++iy) {
            const double cx = ix ? (L.SA % tx ? 1 : 0) : double(L.SA / tx);
            const double cy = iy ? (L.SB % ty ? 1 : 0) : double(L.SB / ty);
            const double ex = ix ? double(L.SA % tx) : tx, ey = iy ? double(L.SB % ty) : ty;
            const double cnt = cx * cy;
            if (cnt == 0) continue;
            traffic += cnt * (ey * lines(n0 * ex * e) + ex * lines(n0 * ey * e) + kTileOverhead);
            useful += cnt * 2.0 * n0 * ex * ey * e;
            lanes += cnt * lanes_row * tx * ty;
            work += cnt * n0 * ex * ey;
        }
    if (useful == 0) return 1e30;
    return scalar_penalty(p) * traffic / useful * (1.0 + 0.25 * (lanes / work - 1.0));
}

// Whether a menu tile of this layout can use 16-byte accesses on both sides,
// judged from extents and strides alone (pointer alignment aside).
static bool vector_shape(const Problem& p, const Layout& L, int ta, int tb) {
    const int VA = 16 / elem_bytes(p.dtype_a), VB = 16 / elem_bytes(p.dtype);
    const int V = VA < VB ? VA : VB;
    if (L.staged) return false;
    if (p.family == TTX_FAMILY_PRESERVED) return p.dim[0].sa == 1 && p.dim[0].sb == 1 && ta % V == 0;
    return p.dim[L.a].sa == 1 && ta % VA == 0 && p.dim[L.b].sb == 1 && tb % VB == 0;
}

// Dense tiles: rows of n0, tx x ty rows per plane, tz planes (along index z,
// -1 for none), CAP slots per tile (idle slots cost issue time, as idle
// lanes do).  A is read in runs along (row, x), which continue across y and
// then z where those are adjacent in A and the tile spans the whole extent
// before them; B likewise along (row, y), then x, then z.
static double dense_cost(const Problem& p, const Layout& L, int tx, int ty, int tz, int z) {
    const double e = elem_bytes(p.dtype);
    const int64_t n0 = L.staged ? p.dim[0].size : 1;
    const double cap = dense_cap(p.dtype);
    const int64_t zs = z >= 0 ? p.dim[z].size : 1;
    // element strides of the tile's coordinates in A and B
    const int64_t rowA = L.staged ? p.dim[0].size * p.dim[0].sa : 1;      // contiguous (row, x) runs
    const bool xa_lin = L.staged ? p.dim[L.a].sa == rowA : true;
    const int64_t rowB = L.staged ? p.dim[0].size * p.dim[0].sb : 1;
    const bool yb_lin = L.staged ? p.dim[L.b].sb == rowB : true;
    const bool y_single = L.staged ? L.gb == 2 : L.gb == 1;
    const bool x_single = L.staged ? L.ga == 2 : L.ga == 1;
    double traffic = 0, useful = 0, slots = 0, work = 0;
    for (int ix = 0; ix < 2; ++ix)
        for (int iy = 0; iy < 2; ++iy)
            for (int iz = 0; iz < 2; ++iz) {
                const double cx = ix ? (L.SA % tx ? 1 : 0) : double(L.SA / tx);
                const double cy = iy ? (L.SB % ty ? 1 : 0) : double(L.SB / ty);
                const double cz = iz ? (zs % tz ? 1 : 0) : double(zs / tz);
                const int64_t ex = ix ? L.SA % tx : tx, ey = iy ? L.SB % ty : ty, ez = iz ? zs % tz : tz;
                const double cnt = cx * cy * cz;
                if (cnt == 0) continue;
                const double elems = double(n0 * ex * ey * ez);
                // A runs
                double ra = xa_lin ? double(n0 * ex) : double(n0);
                if (xa_lin && ex == L.SA && y_single && p.dim[L.b].sa == L.SA * rowA) {
                    ra *= double(ey);
                    if (ey == L.SB && z >= 0 && p.dim[z].sa == L.SB * L.SA * rowA) ra *= double(ez);
                }
                // B runs
                double rb = yb_lin ? double(n0 * ey) : double(n0);
                if (yb_lin && ey == L.SB && x_single && p.dim[L.a].sb == L.SB * rowB) {
                    rb *= double(ex);
                    if (ex == L.SA && z >= 0 && p.dim[z].sb == L.SA * L.SB * rowB) rb *= double(ez);
                }
                traffic += cnt * (elems / ra * lines(ra * e) + elems / rb * lines(rb * e) + kTileOverhead);
                useful += cnt * 2.0 * elems * e;
                slots += cnt * cap;
                work += cnt * elems;
            }
    if (useful == 0) return 1e30;
    const double pen = p.dtype >= kWideF32x4 ? kWideDensePenalty : kDensePenalty;
    return pen * traffic / useful * (1.0 + 0.25 * (slots / work - 1.0));
}

// Planes per dense tile worth trying along index z (1 = one plane).
static std::vector<int> dense_planes(const Problem& p, const Layout& L, int tx, int ty, int z) {
    std::vector<int> out = {1};
    if (z < 0) return out;
    const int64_t n0 = L.staged ? p.dim[0].size : 1;
    const int64_t most = std::min<int64_t>(dense_cap(p.dtype) / (n0 * tx * ty), p.dim[z].size);
    if (most < 2) return out;
    const int64_t pieces = (p.dim[z].size + most - 1) / most;
    out.push_back(int(most));
    const int64_t even = (p.dim[z].size + pieces - 1) / pieces;
    if (even != most && even > 1) out.push_back(int(even));
    return out;
}

// Dense tile extents worth trying: tx from powers of two, the whole extent
// and near-even splits of it; ty as large as the capacity allows, or an
// even split of B's extent.
static std::vector<TileShape> dense_shapes(const Problem& p, const Layout& L) {
    std::vector<TileShape> out;
    const int64_t n0 = L.staged ? p.dim[0].size : 1, cap = dense_cap(p.dtype);
    const int64_t maxa = cap / n0;
    if (maxa < 1) return out;
    std::vector<int64_t> txs;
    for (int64_t v = 1; v <= maxa; v *= 2) txs.push_back(std::min<int64_t>(v, L.SA));
    for (int64_t k = 1; k <= 8; ++k) {
        const int64_t v = (L.SA + k - 1) / k;
        if (v <= maxa) txs.push_back(v);
    }
    std::sort(txs.begin(), txs.end());
    txs.erase(std::unique(txs.begin(), txs.end()), txs.end());
    for (int64_t tx : txs) {
        const int64_t tymax = std::min<int64_t>(cap / (n0 * tx), L.SB);
        if (tymax < 1) continue;
        const int64_t even = (L.SB + ((L.SB + tymax - 1) / tymax) - 1) / ((L.SB + tymax - 1) / tymax);
        for (int64_t ty : {tymax, even}) {
            bool dup = false;
            for (const auto& t : out) dup |= t.ta == tx && t.tb == ty;
            if (!dup) out.push_back(TileShape{int(tx), int(ty)});
        }
    }
    return out;
}

// Whether a layout can take dense tiles.
static bool dense_layout(const Problem& p, const Layout& L) {
    return p.family == TTX_FAMILY_MOVED || (p.family == TTX_FAMILY_PRESERVED && L.staged);
}

static double blocking_cost(const Problem& p, const Layout& L, int ta, int tb) {
    if (L.staged) return staged_cost(p, L, ta, tb);
    const double e = elem_bytes(p.dtype);
    const int64_t Sa = L.SA, Sb = L.SB;
    struct Edge { double ext, count; };
    auto edges = [](int64_t S, int t, Edge out[2]) {
        int64_t full = S / t, rem = S % t;
        out[0] = {double(t), double(full)};
        out[1] = {double(rem), rem ? 1.0 : 0.0};
    };
    Edge ea[2], eb[2];
    edges(Sa, ta, ea);
    edges(Sb, tb, eb);
    // other indices multiply every tile count equally; they cancel in the ratio
    const bool moved = p.family == TTX_FAMILY_MOVED;
    const bool a_cols_adjacent = p.dim[L.b].sa == Sa * p.dim[L.a].sa;   // A columns back to back
    const bool b_rows_adjacent = moved ? p.dim[L.a].sb == Sb * p.dim[L.b].sb
                                       : p.dim[L.b].sb == Sa * p.dim[L.a].sb;
    double traffic = 0, useful = 0, lanes = 0, work = 0;
    for (const Edge& x : ea)
        for (const Edge& y : eb) {
            double cnt = x.count * y.count;
            if (cnt == 0) continue;
            double ax = x.ext, by = y.ext;
            double bytes_a = (ax == Sa && a_cols_adjacent) ? lines(ax * by * e) : by * lines(ax * e);
            double bytes_b;
            if (moved)
                bytes_b = (by == Sb && b_rows_adjacent) ? lines(ax * by * e) : ax * lines(by * e);
            else
                bytes_b = (ax == Sa && b_rows_adjacent) ? lines(ax * by * e) : by * lines(ax * e);
            traffic += cnt * (bytes_a + bytes_b + kTileOverhead);
            useful += cnt * 2.0 * ax * by * e;
            lanes += cnt * double(ta) * tb;
            work += cnt * ax * by;
        }
    if (useful == 0) return 1e30;
    const double scalar = vector_shape(p, L, ta, tb) ? 1.0 : scalar_penalty(p);
    return scalar * traffic / useful * (1.0 + 0.25 * (lanes / work - 1.0));
}

// Grid indices of a layout (leaders and the indices outside both groups).
static std::vector<int> grid_indices(const Problem& p, const Layout& L) {
    std::vector<int> g;
    for (int d = 0; d < p.n; ++d)
        if (!L.member[d]) g.push_back(d);
    return g;
}

static void grid_step(const Problem& p, const Layout& L, int d, int ta, int tb, double* cnt,
                      double* sA, double* sB) {
    double ext = 1, extent = double(p.dim[d].size);
    if (d == L.a) {
        ext = ta;
        extent = double(L.SA);
    } else if (d == L.b) {
        ext = tb;
        extent = double(L.SB);
    }
    *cnt = std::ceil(extent / ext);
    *sA = ext * double(p.dim[d].sa);
    *sB = ext * double(p.dim[d].sb);
}

static double order_cost(const Problem& p, const Layout& L, int ta, int tb, const int* order, int n) {
    const double e = elem_bytes(p.dtype);
    double resident = 1, spanA = 0, spanB = 0;
    for (int q = 0; q < n && resident < kResident; ++q) {
        const int d = order[q];
        if (L.member[d]) continue;
        double cnt, sA, sB;
        grid_step(p, L, d, ta, tb, &cnt, &sA, &sB);
        double take = std::min(cnt, std::ceil(kResident / resident));
        spanA += (take - 1) * sA;
        spanB += (take - 1) * sB;
        resident *= cnt;
    }
    double tiles = std::min(resident, kResident);
    double moved_bytes = tiles * double(ta) * tb * e;
    double ratio = (spanA + spanB) * e / (2.0 * moved_bytes);
    return 0.02 * std::log2(1.0 + ratio);
}

static double flag_cost(int flags) {
    // no measured preference: order plain before swizzled before streaming
    return 0.001 * ((flags & TTX_CFG_XCD_SWIZZLE) ? 1 : 0) + 0.002 * ((flags & TTX_CFG_NT_STORE) ? 1 : 0);
}

// Full orders (every merged index) from orders of the grid indices: group
// members, which the grid skips, are appended in index order.
static std::vector<std::vector<int>> loop_orders(const Problem& p, const Layout& L) {
    std::vector<std::vector<int>> out;
    std::vector<int> g = grid_indices(p, L), tail;
    for (int d = 0; d < p.n; ++d)
        if (L.member[d]) tail.push_back(d);
    auto full = [&](std::vector<int> o) {
        o.insert(o.end(), tail.begin(), tail.end());
        return o;
    };
    if (g.size() <= 6) {
        std::vector<int> o = g;
        do out.push_back(full(o));
        while (std::next_permutation(o.begin(), o.end()));
        return out;
    }
    std::vector<int> border;
    for (int k = 0; k < p.n; ++k)
        if (!L.member[p.perm[k]]) border.push_back(p.perm[k]);
    out.push_back(full(g));
    out.push_back(full(border));
    for (const auto& base : {g, border}) {
        std::vector<int> t = {L.a};
        if (L.b != L.a) t.push_back(L.b);
        for (int d : base)
            if (d != L.a && d != L.b) t.push_back(d);
        out.push_back(full(t));
    }
    return out;
}

static ttx_config make_config(const Problem& p, int ta, int tb, const std::vector<int>& order,
                              int flags, int ga = 1, int gb = 1) {
    ttx_config c;
    std::memset(&c, 0, sizeof(c));
    c.family = p.family;
    c.tile_a = ta;
    c.tile_b = tb;
    c.threads = kThreads;
    c.lds_pad = 1;
    c.n_order = int(order.size());
    for (size_t i = 0; i < order.size(); ++i) c.order[i] = order[i];
    c.flags = flags;
    c.group_a = ga;
    c.group_b = gb;
    return c;
}

// The staged menu's (tile_x, tile_y) shapes for this problem's row length.
static std::vector<TileShape> staged_shape_list(const Problem& p) {
    std::vector<TileShape> out;
    const StagedShape* m;
    const int n = staged_menu(p.dtype, &m);
    const int lanes = staged_lanes(p.dim[0].size);
    for (int i = 0; i < n; ++i)
        if (m[i].n0 == lanes) out.push_back(TileShape{m[i].tx, m[i].ty});
    return out;
}

int rank_candidates(const Problem& p, int max_candidates, ttx_config* out, double* cost,
                    int cap) {
    if (max_candidates == 0) max_candidates = 200;
    if (p.family == TTX_FAMILY_EMPTY) return 0;
    struct Cand {
        double cost;
        int index;   // enumeration index: the final tie-break
        ttx_config cfg;
    };
    auto worse = [](const Cand& x, const Cand& y) {
        return x.cost < y.cost || (x.cost == y.cost && x.index < y.index);
    };
    // Bounded list (Sec. 2.1 stage 3): a max-heap on cost; a candidate enters
    // while the list has room, or replaces the worst when it is cheaper.  One
    // list per kernel kind (menu, staged, dense tiles): the estimates compare
    // shapes of one kind better than they compare kinds, so each kind keeps a
    // quarter of the final list when it has that many candidates.
    using Heap = std::priority_queue<Cand, std::vector<Cand>, decltype(worse)>;
    Heap heaps[3] = {Heap(worse), Heap(worse), Heap(worse)};
    int index = 0;
    auto offer = [&](double c, const ttx_config& cfg) {
        Cand cand{c, index++, cfg};
        Heap& heap = heaps[config_is_dense(cfg) ? 2 : config_is_staged(cfg) ? 1 : 0];
        if (max_candidates < 0 || int(heap.size()) < max_candidates) {
            heap.push(cand);
        } else if (worse(cand, heap.top())) {
            heap.pop();
            heap.push(cand);
        }
    };
    const int flag_sets[4] = {0, TTX_CFG_XCD_SWIZZLE, TTX_CFG_NT_STORE,
                              TTX_CFG_XCD_SWIZZLE | TTX_CFG_NT_STORE};
    if (p.family == TTX_FAMILY_FLAT) {
        for (int f : {0, TTX_CFG_NT_STORE}) offer(1.0 + flag_cost(f), make_config(p, 0, 0, {0}, f));
    } else {
        const TileShape* menu;
        const int nmenu = tile_menu(p.dtype, p.family, &menu);
        for (auto [ga, gb] : group_options(p)) {
            Layout L;
            make_layout(p, ga, gb, &L);
            std::vector<TileShape> staged_shapes;
            const TileShape* shapes = menu;
            int ns = nmenu;
            if (L.staged) {
                staged_shapes = staged_shape_list(p);
                shapes = staged_shapes.data();
                ns = int(staged_shapes.size());
            }
            auto orders = loop_orders(p, L);
            for (int s = 0; s < ns; ++s) {
                ttx_config probe = make_config(p, shapes[s].ta, shapes[s].tb, orders[0], 0, ga, gb);
                if (!config_valid(p, probe, nullptr)) continue;
                double bc = blocking_cost(p, L, shapes[s].ta, shapes[s].tb);
                for (const auto& o : orders) {
                    double oc = order_cost(p, L, shapes[s].ta, shapes[s].tb, o.data(), p.n);
                    for (int f : flag_sets)
                        offer(bc * (1.0 + oc) + flag_cost(f),
                              make_config(p, shapes[s].ta, shapes[s].tb, o, f, ga, gb));
                }
            }
        }
        // dense tiles, over elements and (when the rows allow it) over whole units of the rows
        Problem w;
        const bool wide = widen(p, &w);
        for (int pass = 0; pass < (wide ? 2 : 1); ++pass) {
            const Problem& q = pass ? w : p;
            const int extra = pass ? TTX_CFG_WIDE : 0;
            for (auto [ga, gb] : group_options(q)) {
                Layout L;
                make_layout(q, ga, gb, &L);
                if (!dense_layout(q, L)) continue;
                auto orders = loop_orders(q, L);
                for (const TileShape& d : dense_shapes(q, L)) {
                    ttx_config probe = make_config(q, d.ta, d.tb, orders[0], TTX_CFG_DENSE, ga, gb);
                    if (!config_valid(q, probe, nullptr)) continue;
                    for (const auto& o : orders) {
                        const int z = dense_z(q, L, o.data(), q.n);
                        double oc = order_cost(q, L, d.ta, d.tb, o.data(), q.n);
                        for (int tz : dense_planes(q, L, d.ta, d.tb, z)) {
                            const double bc = dense_cost(q, L, d.ta, d.tb, tz, z);
                            for (int f : flag_sets) {
                                ttx_config c = make_config(q, d.ta, d.tb, o, f | TTX_CFG_DENSE | extra, ga, gb);
                                c.tile_c = tz;
                                offer(bc * (1.0 + oc) + flag_cost(f), c);
                            }
                        }
                    }
                }
            }
        }
    }
    std::vector<Cand> kinds[3], all;
    for (int k = 0; k < 3; ++k) {
        while (!heaps[k].empty()) {
            kinds[k].push_back(heaps[k].top());
            heaps[k].pop();
        }
        std::sort(kinds[k].begin(), kinds[k].end(), [&](const Cand& x, const Cand& y) { return worse(x, y); });
    }
    if (max_candidates < 0) {
        for (auto& v : kinds) all.insert(all.end(), v.begin(), v.end());
    } else {
        // each kind's quota first, then the cheapest of the rest
        const size_t quota = size_t(max_candidates) / 4;
        std::vector<Cand> rest;
        for (auto& v : kinds) {
            const size_t q = std::min(quota, v.size());
            all.insert(all.end(), v.begin(), v.begin() + q);
            rest.insert(rest.end(), v.begin() + q, v.end());
        }
        std::sort(rest.begin(), rest.end(), [&](const Cand& x, const Cand& y) { return worse(x, y); });
        for (const Cand& c : rest) {
            if (all.size() >= size_t(max_candidates)) break;
            all.push_back(c);
        }
    }
    std::sort(all.begin(), all.end(), [&](const Cand& x, const Cand& y) { return worse(x, y); });
    int n = std::min<int>(int(all.size()), cap);
    for (int i = 0; i < n; ++i) {
        out[i] = all[i].cfg;
        if (cost) cost[i] = all[i].cost;
    }
    return n;
}

int workgroup_variants(const Problem& p, const ttx_config& base, ttx_config* out, int cap) {
    int n = 0;
    if (cap <= 0) return 0;
    out[n++] = base;
    if (p.family != TTX_FAMILY_MOVED && p.family != TTX_FAMILY_PRESERVED) return n;
    static const int kThreadMenu[] = {64, 128, 256, 512};
    const bool padded = config_uses_pad(base);
    // line-aligned A runs, both ways, where the tile allows them
    ttx_config toggled = base;
    toggled.flags ^= TTX_CFG_ALIGN_A;
    const bool align_dim = config_valid(p, toggled, nullptr);
    for (int al = 0; al < (align_dim ? 2 : 1); ++al)
        for (int t : kThreadMenu)
            for (int pad = 0; pad <= (padded ? TTX_MAX_LDS_PAD : 0); ++pad) {
                ttx_config c = al ? toggled : base;
                c.threads = t;
                if (padded) c.lds_pad = pad;
                if (c.threads == base.threads && config_pad(c) == config_pad(base) && c.flags == base.flags)
                    continue;   // the base itself
                if (!config_valid(p, c, nullptr)) continue;
                if (n < cap) out[n++] = c;
            }
    return n;
}

ttx_config default_config_from(const Problem& p, const TileShape* shapes, int ns,
                               const TileShape* staged, int nstaged, bool dense, bool wide) {
    ttx_config best;
    std::memset(&best, 0, sizeof(best));
    best.family = p.family;
    best.threads = kThreads;
    best.lds_pad = 1;
    best.group_a = best.group_b = 1;
    if (p.family == TTX_FAMILY_EMPTY) return best;
    if (p.family == TTX_FAMILY_FLAT) {
        best.n_order = 1;
        best.order[0] = 0;
        return best;
    }
    // Greedy use of both heuristics: the cheapest groups and tile shape, then
    // the grid indices sorted by the span one step covers (smallest first).
    // A shape whose blocking cost alone is not below the best so far is
    // skipped (the loop-order factor is at least 1).
    double bestc = 1e300;
    for (auto [ga, gb] : group_options(p)) {
        Layout L;
        make_layout(p, ga, gb, &L);
        int gi[kMaxDims], ng = 0, tail[kMaxDims], nt = 0;
        double span[kMaxDims] = {};
        for (int d = 0; d < p.n; ++d) {
            if (L.member[d]) {
                tail[nt++] = d;
                continue;
            }
            gi[ng++] = d;
            double cnt, sA, sB;
            grid_step(p, L, d, 1, 1, &cnt, &sA, &sB);
            span[d] = sA + sB;
        }
        // the order for tile extents (ta, tb): the tile indices' steps scale
        auto make_order = [&](int ta, int tb, std::vector<int>& o) {
            double sp[kMaxDims];
            for (int k = 0; k < ng; ++k) {
                const int d = gi[k];
                sp[d] = span[d] * (d == L.a ? ta : d == L.b ? tb : 1);
            }
            o.assign(gi, gi + ng);
            std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return sp[x] < sp[y]; });
            o.insert(o.end(), tail, tail + nt);
        };
        std::vector<int> o;
        std::vector<TileShape> own;
        const TileShape* sh = shapes;
        int nsh = ns;
        if (L.staged) {
            if (nstaged < 0) {
                own = staged_shape_list(p);
            } else {
                const int lanes = staged_lanes(p.dim[0].size);
                for (int i = 0; i < nstaged; ++i)   // (lanes, tx, ty) packed as {lanes*65536 + tx, ty}
                    if (staged[i].ta >> 16 == lanes) own.push_back(TileShape{staged[i].ta & 0xffff, staged[i].tb});
            }
            sh = own.data();
            nsh = int(own.size());
        }
        for (int s = 0; s < nsh; ++s) {
            const int ta = sh[s].ta, tb = sh[s].tb;
            const double bc = blocking_cost(p, L, ta, tb);
            if (bc >= bestc) continue;
            make_order(ta, tb, o);
            ttx_config c = make_config(p, ta, tb, o, 0, ga, gb);
            // shapes outside the per-call menu (batched-kernel variants) are checked by their caller
            if ((L.staged || tile_in_menu(p.dtype, p.family, ta, tb)) && !config_valid(p, c, nullptr)) continue;
            const double cost = bc * (1.0 + order_cost(p, L, ta, tb, o.data(), p.n));
            if (cost < bestc) {
                bestc = cost;
                best = c;
            }
        }
        if (!dense || !dense_layout(p, L)) continue;
        for (const TileShape& d : dense_shapes(p, L)) {
            make_order(d.ta, d.tb, o);
            const int z = dense_z(p, L, o.data(), p.n);
            for (int tz : dense_planes(p, L, d.ta, d.tb, z)) {
                const double dc = dense_cost(p, L, d.ta, d.tb, tz, z);
                if (dc >= bestc) continue;
                ttx_config c = make_config(p, d.ta, d.tb, o, TTX_CFG_DENSE, ga, gb);
                c.tile_c = tz;
                if (!config_valid(p, c, nullptr)) continue;
                const double cost = dc * (1.0 + order_cost(p, L, d.ta, d.tb, o.data(), p.n));
                if (cost < bestc) {
                    bestc = cost;
                    best = c;
                }
            }
        }
    }
    // dense tiles over whole units of the rows
    Problem w;
    if (dense && wide && widen(p, &w)) {
        for (auto [ga, gb] : group_options(w)) {
            Layout L;
            make_layout(w, ga, gb, &L);
            if (!dense_layout(w, L)) continue;
            int gi[kMaxDims], ng = 0, tail[kMaxDims], nt = 0;
            double span[kMaxDims] = {};
            for (int d = 0; d < w.n; ++d) {
                if (L.member[d]) {
                    tail[nt++] = d;
                    continue;
                }
                gi[ng++] = d;
                double cnt, sA, sB;
                grid_step(w, L, d, 1, 1, &cnt, &sA, &sB);
                span[d] = sA + sB;
            }
            std::vector<int> o;
            for (const TileShape& d : dense_shapes(w, L)) {
                double sp[kMaxDims];
                for (int k = 0; k < ng; ++k) sp[gi[k]] = span[gi[k]] * (gi[k] == L.a ? d.ta : gi[k] == L.b ? d.tb : 1);
                o.assign(gi, gi + ng);
                std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return sp[x] < sp[y]; });
                o.insert(o.end(), tail, tail + nt);
                const int z = dense_z(w, L, o.data(), w.n);
                for (int tz : dense_planes(w, L, d.ta, d.tb, z)) {
                    const double dc = dense_cost(w, L, d.ta, d.tb, tz, z);
                    if (dc >= bestc) continue;
                    ttx_config c = make_config(w, d.ta, d.tb, o, TTX_CFG_DENSE | TTX_CFG_WIDE, ga, gb);
                    c.tile_c = tz;
                    if (!config_valid(p, c, nullptr)) continue;
                    const double cost = dc * (1.0 + order_cost(w, L, d.ta, d.tb, o.data(), w.n));
                    if (cost < bestc) {
                        bestc = cost;
                        best = c;
                    }
                }
            }
        }
    }
    return best;
}

ttx_config default_config(const Problem& p) {
    const TileShape* shapes;
    int ns = tile_menu(p.dtype, p.family, &shapes);
    return default_config_from(p, shapes, ns, nullptr, -1, true, true);
}

ttx_config default_config_elementwise(const Problem& p) {
    const TileShape* shapes;
    int ns = tile_menu(p.dtype, p.family, &shapes);
    return default_config_from(p, shapes, ns, nullptr, -1, true, false);
}

}  // namespace ttx
