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

static int elem_bytes(int dtype) { return dtype == TTX_F32 ? 4 : 8; }

// ---------------------------------------------------------------------------------------
// Menus
#define TTX_SHAPE(a, b) {a, b},
static const TileShape kMovedF32[] = {TTX_MOVED_MENU_F32(TTX_SHAPE)};
static const TileShape kMovedF64[] = {TTX_MOVED_MENU_F64(TTX_SHAPE)};
static const TileShape kPresF32[] = {TTX_PRESERVED_MENU_F32(TTX_SHAPE)};
static const TileShape kPresF64[] = {TTX_PRESERVED_MENU_F64(TTX_SHAPE)};
#undef TTX_SHAPE

int tile_menu(int dtype, int family, const TileShape** shapes) {
    if (family == TTX_FAMILY_MOVED) {
        *shapes = dtype == TTX_F32 ? kMovedF32 : kMovedF64;
        return dtype == TTX_F32 ? int(sizeof(kMovedF32) / sizeof(TileShape))
                                : int(sizeof(kMovedF64) / sizeof(TileShape));
    }
    if (family == TTX_FAMILY_PRESERVED) {
        *shapes = dtype == TTX_F32 ? kPresF32 : kPresF64;
        return dtype == TTX_F32 ? int(sizeof(kPresF32) / sizeof(TileShape))
                                : int(sizeof(kPresF64) / sizeof(TileShape));
    }
    *shapes = nullptr;
    return 0;
}

bool tile_in_menu(int dtype, int family, int ta, int tb) {
    const TileShape* s;
    int n = tile_menu(dtype, family, &s);
    for (int i = 0; i < n; ++i)
        if (s[i].ta == ta && s[i].tb == tb) return true;
    return false;
}

// ---------------------------------------------------------------------------------------
// Problem construction
ttx_status make_problem(int dtype, int n, const int* perm, const int64_t* size,
                        const int64_t* outer_a, const int64_t* outer_b, Problem* out) {
    if (dtype != TTX_F32 && dtype != TTX_F64) return fail(TTX_EINVAL, "unknown dtype");
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

    Problem p;
    p.dtype = dtype;
    p.n_orig = n;
    const int eb = elem_bytes(dtype);
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
    p.extent_a = (last_a + 1) * eb;
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

// The two merged indices that span a tile: A's stride-1 index and, for the
// moved family, B's stride-1 index; for the preserved family, B's second index.
static void tile_dims(const Problem& p, int* a, int* b) {
    *a = 0;
    *b = p.family == TTX_FAMILY_MOVED ? p.perm[0] : (p.n > 1 ? p.perm[1] : 0);
}

// ---------------------------------------------------------------------------------------
// Config validation and the kernel-side grid
bool config_valid(const Problem& p, const ttx_config& c, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (c.family != p.family) return bad("config family does not match the problem");
    if (c.threads != kThreads) return bad("threads must be 256");
    if (c.flags & ~(TTX_CFG_XCD_SWIZZLE | TTX_CFG_NT_STORE)) return bad("unknown flag");
    if (p.family == TTX_FAMILY_EMPTY) return true;
    if (c.n_order != p.n) return bad("order must list every merged index");
    bool seen[kMaxDims] = {};
    for (int i = 0; i < c.n_order; ++i) {
        if (c.order[i] < 0 || c.order[i] >= p.n || seen[c.order[i]])
            return bad("order is not a permutation of the merged indices");
        seen[c.order[i]] = true;
    }
    if (p.family == TTX_FAMILY_FLAT) return true;
    if (!tile_in_menu(p.dtype, p.family, c.tile_a, c.tile_b)) return bad("tile shape not in menu");
    // the tile id space must fit 32 bits
    int a, b;
    tile_dims(p, &a, &b);
    uint64_t tiles = 1;
    for (int d = 0; d < p.n; ++d) {
        int64_t ext = d == a ? c.tile_a : d == b ? c.tile_b : 1;
        tiles *= uint64_t((p.dim[d].size + ext - 1) / ext);
        if (tiles >= (uint64_t(1) << 32)) return bad("too many tiles for this tile shape");
    }
    return true;
}

void build_grid(const Problem& p, const ttx_config& c, TileGrid* g, int64_t s[4]) {
    int a, b;
    tile_dims(p, &a, &b);
    std::memset(g, 0, sizeof(*g));
    g->nd = p.n;
    g->pa = g->pb = -1;
    uint64_t tiles = 1;
    for (int q = 0; q < p.n; ++q) {
        int d = c.order[q];
        int64_t ext = d == a ? c.tile_a : d == b ? c.tile_b : 1;
        uint32_t cnt = uint32_t((p.dim[d].size + ext - 1) / ext);
        g->count[q] = cnt;
        g->div[q].init(cnt);
        g->stepA[q] = ext * p.dim[d].sa;
        g->stepB[q] = ext * p.dim[d].sb;
        if (d == a) g->pa = q;
        if (d == b) g->pb = q;
        tiles *= cnt;
    }
    g->ntiles = uint32_t(tiles);
    g->ext_a = p.dim[a].size;
    g->ext_b = p.dim[b].size;
    s[0] = p.dim[a].sa;
    s[1] = p.dim[b].sa;
    s[2] = p.dim[a].sb;
    s[3] = p.dim[b].sb;
}

static bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; }

int kernel_flags(const Problem& p, const ttx_config& c, const void* A, const void* Bsrc,
                 const void* Bdst) {
    int f = 0;
    if (c.flags & TTX_CFG_NT_STORE) f |= KF_NT_STORE;
    if (c.flags & TTX_CFG_XCD_SWIZZLE) f |= KF_SWIZZLE;
    const int V = 16 / elem_bytes(p.dtype);
    const bool bptrs = aligned16(Bdst) && (Bsrc == nullptr || aligned16(Bsrc));
    if (p.family == TTX_FAMILY_FLAT) {
        if (p.dim[0].sa == 1 && p.dim[0].sb == 1 && aligned16(A) && bptrs) f |= KF_VEC_A;
        return f;
    }
    int a, b;
    tile_dims(p, &a, &b);
    auto multiples = [&](bool use_a, int skip) {
        for (int d = 0; d < p.n; ++d) {
            if (d == skip) continue;
            int64_t s = use_a ? p.dim[d].sa : p.dim[d].sb;
            if (s % V) return false;
        }
        return true;
    };
    if (p.family == TTX_FAMILY_MOVED) {
        if (p.dim[a].sa == 1 && c.tile_a % V == 0 && p.dim[a].size % V == 0 && aligned16(A) &&
            multiples(true, a))
            f |= KF_VEC_A;
        if (p.dim[b].sb == 1 && c.tile_b % V == 0 && p.dim[b].size % V == 0 && bptrs &&
            multiples(false, b))
            f |= KF_VEC_B;
    } else {  // preserved: rows contiguous in both tensors
        if (p.dim[a].sa == 1 && p.dim[a].sb == 1 && c.tile_a % V == 0 && p.dim[a].size % V == 0 &&
            aligned16(A) && bptrs && multiples(true, a) && multiples(false, a))
            f |= KF_VEC_A | KF_VEC_B;
    }
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

static double lines(double bytes) { return std::ceil(bytes / kLine) * kLine; }

static double blocking_cost(const Problem& p, int ta, int tb) {
    int a, b;
    tile_dims(p, &a, &b);
    const double e = elem_bytes(p.dtype);
    const int64_t Sa = p.dim[a].size, Sb = p.dim[b].size;
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
    const bool a_cols_adjacent = p.dim[b].sa == Sa * p.dim[a].sa;   // A columns back to back
    const bool b_rows_adjacent = moved ? p.dim[a].sb == Sb * p.dim[b].sb
                                       : p.dim[b].sb == Sa * p.dim[a].sb;
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
    return traffic / useful * (1.0 + 0.25 * (lanes / work - 1.0));
}

static double order_cost(const Problem& p, int ta, int tb, const int* order) {
    int a, b;
    tile_dims(p, &a, &b);
    const double e = elem_bytes(p.dtype);
    double resident = 1, spanA = 0, spanB = 0;
    for (int q = 0; q < p.n && resident < kResident; ++q) {
        int d = order[q];
        int64_t ext = d == a ? ta : d == b ? tb : 1;
        double cnt = double((p.dim[d].size + ext - 1) / ext);
        double take = std::min(cnt, std::ceil(kResident / resident));
        spanA += (take - 1) * double(ext) * double(p.dim[d].sa);
        spanB += (take - 1) * double(ext) * double(p.dim[d].sb);
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

// Loop orders considered for a problem of merged rank n: all n! when n <= 6
// (as Sec. 2.2 explores all d! orders), otherwise a few structured ones.
static std::vector<std::vector<int>> loop_orders(const Problem& p) {
    std::vector<std::vector<int>> out;
    std::vector<int> o(p.n);
    std::iota(o.begin(), o.end(), 0);
    if (p.n <= 6) {
        do out.push_back(o);
        while (std::next_permutation(o.begin(), o.end()));
        return out;
    }
    int a, b;
    tile_dims(p, &a, &b);
    std::vector<int> border(p.perm, p.perm + p.n);
    out.push_back(o);        // A order
    out.push_back(border);   // B order
    for (const auto& base : {o, border}) {
        std::vector<int> t = {a};
        if (b != a) t.push_back(b);
        for (int d : base)
            if (d != a && d != b) t.push_back(d);
        out.push_back(t);
    }
    return out;
}

static ttx_config make_config(const Problem& p, int ta, int tb, const std::vector<int>& order,
                              int flags) {
    ttx_config c;
    std::memset(&c, 0, sizeof(c));
    c.family = p.family;
    c.tile_a = ta;
    c.tile_b = tb;
    c.threads = kThreads;
    c.n_order = int(order.size());
    for (size_t i = 0; i < order.size(); ++i) c.order[i] = order[i];
    c.flags = flags;
    return c;
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
    // while the list has room, or replaces the worst when it is cheaper.
    std::priority_queue<Cand, std::vector<Cand>, decltype(worse)> heap(worse);
    int index = 0;
    auto offer = [&](double c, const ttx_config& cfg) {
        Cand cand{c, index++, cfg};
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
        const TileShape* shapes;
        int ns = tile_menu(p.dtype, p.family, &shapes);
        auto orders = loop_orders(p);
        for (int s = 0; s < ns; ++s) {
            ttx_config probe = make_config(p, shapes[s].ta, shapes[s].tb, orders[0], 0);
            if (!config_valid(p, probe, nullptr)) continue;
            double bc = blocking_cost(p, shapes[s].ta, shapes[s].tb);
            for (const auto& o : orders) {
                double oc = order_cost(p, shapes[s].ta, shapes[s].tb, o.data());
                for (int f : flag_sets)
                    offer(bc * (1.0 + oc) + flag_cost(f), make_config(p, shapes[s].ta, shapes[s].tb, o, f));
            }
        }
    }
    std::vector<Cand> all;
    while (!heap.empty()) {
        all.push_back(heap.top());
        heap.pop();
    }
    std::sort(all.begin(), all.end(), [&](const Cand& x, const Cand& y) { return worse(x, y); });
    int n = std::min<int>(int(all.size()), cap);
    for (int i = 0; i < n; ++i) {
        out[i] = all[i].cfg;
        if (cost) cost[i] = all[i].cost;
    }
    return n;
}

ttx_config default_config_from(const Problem& p, const TileShape* shapes, int ns) {
    ttx_config best;
    std::memset(&best, 0, sizeof(best));
    best.family = p.family;
    best.threads = kThreads;
    if (p.family == TTX_FAMILY_EMPTY) return best;
    if (p.family == TTX_FAMILY_FLAT) {
        best.n_order = 1;
        best.order[0] = 0;
        return best;
    }
    // Greedy use of both heuristics: the cheapest tile shape, then the
    // indices sorted by the span one step covers (smallest first).
    int a, b;
    tile_dims(p, &a, &b);
    double bestc = 1e300;
    for (int s = 0; s < ns; ++s) {
        std::vector<int> o(p.n);
        std::iota(o.begin(), o.end(), 0);
        const int ta = shapes[s].ta, tb = shapes[s].tb;
        auto span = [&](int d) {
            int64_t ext = d == a ? ta : d == b ? tb : 1;
            return double(ext) * double(p.dim[d].sa + p.dim[d].sb);
        };
        std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return span(x) < span(y); });
        ttx_config c = make_config(p, ta, tb, o, 0);
        // shapes outside the per-call menu (batched-kernel variants) are checked by their caller
        if (tile_in_menu(p.dtype, p.family, ta, tb) && !config_valid(p, c, nullptr)) continue;
        double cost = blocking_cost(p, ta, tb) * (1.0 + order_cost(p, ta, tb, o.data()));
        if (cost < bestc) {
            bestc = cost;
            best = c;
        }
    }
    return best;
}

ttx_config default_config(const Problem& p) {
    const TileShape* shapes;
    int ns = tile_menu(p.dtype, p.family, &shapes);
    return default_config_from(p, shapes, ns);
}

}  // namespace ttx
