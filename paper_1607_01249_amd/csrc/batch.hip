// Batched execution: many independent transpositions, each Eqn. 1 with its
// own shape, permutation, scalars and tensors, run by ONE persistent kernel.
//
// The host plans every problem, picks a tile variant from the small batched
// menu (tuned per shape or chosen by the heuristics of Sec. 2.3), and writes
// a descriptor table plus the prefix sums of the per-problem tile counts to
// device memory.  The kernel is launched with about one wave of resident
// workgroups; workgroup w takes tiles w, w + G, w + 2G, ... of the combined
// tile space, finds the owning problem by advancing a cursor over the prefix
// sums (tile ids only grow, so the cursor only moves forward), and runs that
// problem's tile body -- the same device code as the per-call kernels.  The
// launch is captured once into a HIP graph and replayed.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "menu.h"
#include "tile_kernels.h"

struct ttx_batch {
    std::vector<ttx::Problem> prob;
    std::vector<ttx_problem> src;
    std::vector<ttx_config> cfg;
    std::vector<int> forced;
    std::vector<ttx::BatchDesc> desc;
    std::vector<uint32_t> prefix;
    ttx::BatchDesc* d_desc = nullptr;
    uint32_t* d_prefix = nullptr;
    uint32_t total = 0;
    int grid = 0;
    int64_t bytes = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
};

namespace ttx {

struct BatchEntry {
    int index, kind, p1, p2, p3;
};
#define TTX_BATCH_ENTRY(i, kind, p1, p2, p3) {i, kind, p1, p2, p3},
static const BatchEntry kBatchF32[] = {TTX_BATCH_MENU_F32(TTX_BATCH_ENTRY)};
static const BatchEntry kBatchF64[] = {TTX_BATCH_MENU_F64(TTX_BATCH_ENTRY)};
#undef TTX_BATCH_ENTRY

static const BatchEntry* batch_menu(int dtype) { return dtype == TTX_F32 ? kBatchF32 : kBatchF64; }

static int batch_index(int dtype, int family, int ta, int tb, int vec) {
    const BatchEntry* m = batch_menu(dtype);
    for (int i = 0; i < TTX_BATCH_MENU_SIZE; ++i)
        if (m[i].kind == family && m[i].p1 == ta && m[i].p2 == tb && m[i].p3 == vec) return i;
    return -1;
}

static int staged_index(int dtype, int lanes, int tx, int ty) {
    const BatchEntry* m = batch_menu(dtype);
    for (int i = 0; i < TTX_BATCH_MENU_SIZE; ++i)
        if (m[i].kind == TTX_BATCH_STAGED && m[i].p1 == lanes && m[i].p2 == tx && m[i].p3 == ty) return i;
    return -1;
}

// LDS of the largest LDS-staged variant of either dtype.
constexpr int lds_need(int kind, int p1, int p2, int p3, int esize) {
    return kind == TTX_FAMILY_MOVED ? p2 * (p1 + 1) * esize
                                    : kind == TTX_BATCH_STAGED ? p3 * (p2 * p1 + 1) * esize : 0;
}
#define TTX_LDS_F32(i, kind, p1, p2, p3) lds_need(kind, p1, p2, p3, 4),
#define TTX_LDS_F64(i, kind, p1, p2, p3) lds_need(kind, p1, p2, p3, 8),
constexpr int batch_lds_bytes() {
    constexpr int list[] = {TTX_BATCH_MENU_F32(TTX_LDS_F32) TTX_BATCH_MENU_F64(TTX_LDS_F64) 0};
    int m = 0;
    for (int v : list) m = v > m ? v : m;
    return m;
}
#undef TTX_LDS_F32
#undef TTX_LDS_F64
constexpr int kBatchLds = batch_lds_bytes();

template <typename T, bool B0, int KIND, int P1, int P2, int P3>
__device__ __noinline__ void batch_body(unsigned char* lds, const TileArgs<T>& a, uint32_t local) {
    if constexpr (KIND == TTX_BATCH_STAGED) {
        const TileCoord c = decode_tile(a.g, local, P2, P3);
        staged_tile<T, B0, P1, P2, P3>(reinterpret_cast<T*>(lds), a, c);
    } else {
        constexpr int V = P3 ? kVec<T> : 1;
        const TileCoord c = decode_tile(a.g, local, P1, P2);
        if constexpr (KIND == TTX_FAMILY_MOVED)
            moved_tile<T, B0, P1, P2, V, V>(reinterpret_cast<T*>(lds), a, c);
        else
            preserved_tile<T, B0, P1, P2, V>(a, c);
    }
}

template <bool B0>
__device__ __forceinline__ void batch_dispatch_f32(int idx, unsigned char* lds, const BatchDesc& d,
                                                   uint32_t local) {
    const TileArgs<float>& a = *reinterpret_cast<const TileArgs<float>*>(d.args);
    switch (idx) {
#define TTX_CASE(i, kind, p1, p2, p3) \
    case i: batch_body<float, B0, kind, p1, p2, p3>(lds, a, local); break;
        TTX_BATCH_MENU_F32(TTX_CASE)
#undef TTX_CASE
        default: break;
    }
}

template <bool B0>
__device__ __forceinline__ void batch_dispatch_f64(int idx, unsigned char* lds, const BatchDesc& d,
                                                   uint32_t local) {
    const TileArgs<double>& a = *reinterpret_cast<const TileArgs<double>*>(d.args);
    switch (idx) {
#define TTX_CASE(i, kind, p1, p2, p3) \
    case i: batch_body<double, B0, kind, p1, p2, p3>(lds, a, local); break;
        TTX_BATCH_MENU_F64(TTX_CASE)
#undef TTX_CASE
        default: break;
    }
}

// prefix[0] = 0 and prefix[count] = total; problems without tiles have
// equal consecutive prefix entries and are skipped by the cursor.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_batch(const BatchDesc* __restrict__ desc,
                                                    const uint32_t* __restrict__ prefix, int count,
                                                    uint32_t total) {
    __shared__ __align__(16) unsigned char lds[kBatchLds];
    int p = 0;
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        while (p + 1 < count && t >= prefix[p + 1]) ++p;
        // p is the same in every lane: say so, so that the descriptor is read
        // through the scalar cache into scalar registers
        p = __builtin_amdgcn_readfirstlane(p);
        const BatchDesc& d = desc[p];
        const int v = d.variant;
        if (v < 0) continue;
        const uint32_t local = t - prefix[p];
        const int idx = v % TTX_BATCH_MENU_SIZE;
        switch (v / TTX_BATCH_MENU_SIZE) {
            case 0: batch_dispatch_f32<false>(idx, lds, d, local); break;
            case 1: batch_dispatch_f32<true>(idx, lds, d, local); break;
            case 2: batch_dispatch_f64<false>(idx, lds, d, local); break;
            case 3: batch_dispatch_f64<true>(idx, lds, d, local); break;
            default: break;
        }
    }
}

int batch_grid(uint32_t total) {
    static std::mutex mu;
    static int per_cu[64] = {};
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!per_cu[dev]) {
            int nb = 0, c = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, kThreads, 0) != hipSuccess || nb <= 0)
                nb = 4;
            if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
                c = 256;
            per_cu[dev] = nb;
            cus[dev] = c;
        }
    }
    const uint64_t g = uint64_t(per_cu[dev]) * uint64_t(cus[dev]);
    return int(total < g ? total : g);
}

hipError_t launch_batch(const BatchDesc* d_desc, const uint32_t* d_prefix, int count,
                        uint32_t total, int grid, hipStream_t stream) {
    if (total == 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kThreads), 0, stream, d_desc, d_prefix, count, total);
    return hipGetLastError();
}

// -- host side --------------------------------------------------------------------------
static int elem_size(int dtype) { return dtype == TTX_F32 ? 4 : 8; }

// Whether 16-byte accesses are possible on both sides for this problem and
// these pointers (the batched tile shapes are all multiples of the vector
// width, so the answer does not depend on the shape).
static bool vector_ok(const Problem& p, const void* A, const void* Bsrc, const void* Bdst) {
    if (p.family == TTX_FAMILY_FLAT) {
        ttx_config c;
        std::memset(&c, 0, sizeof(c));
        c.family = p.family;
        const int V = 16 / elem_size(p.dtype);
        return (kernel_flags(p, c, A, Bsrc, Bdst) & KF_VEC_A) && p.dim[0].size % V == 0;
    }
    ttx_config c;
    std::memset(&c, 0, sizeof(c));
    c.family = p.family;
    c.tile_a = c.tile_b = 32;
    return (kernel_flags(p, c, A, Bsrc, Bdst) & (KF_VEC_A | KF_VEC_B)) == (KF_VEC_A | KF_VEC_B);
}

static ttx_config batch_default(const Problem& p, bool vec) {
    if (p.family == TTX_FAMILY_FLAT) {
        ttx_config c = default_config(p);
        return c;
    }
    std::vector<TileShape> shapes, staged;
    const BatchEntry* m = batch_menu(p.dtype);
    for (int i = 0; i < TTX_BATCH_MENU_SIZE; ++i) {
        if (m[i].kind == TTX_BATCH_STAGED) {
            if (p.family == TTX_FAMILY_PRESERVED) staged.push_back(TileShape{m[i].p1 * 65536 + m[i].p2, m[i].p3});
            continue;
        }
        if (m[i].kind != p.family || (m[i].p3 && !vec)) continue;
        bool dup = false;
        for (const auto& s : shapes) dup |= s.ta == m[i].p1 && s.tb == m[i].p2;
        if (!dup) shapes.push_back(TileShape{m[i].p1, m[i].p2});
    }
    return default_config_from(p, shapes.data(), int(shapes.size()), staged.data(), int(staged.size()));
}

ttx_status batch_describe(const Problem& p, const ttx_config* forced, bool beta0, const void* A,
                          const void* Bsrc, void* Bdst, double alpha, double beta, BatchDesc* d,
                          ttx_config* used) {
    std::memset(d, 0, sizeof(*d));
    d->dtype = p.dtype;
    d->variant = -1;
    if (p.family == TTX_FAMILY_EMPTY) {
        if (used) *used = default_config(p);
        return TTX_OK;
    }
    const bool vec = vector_ok(p, A, beta0 ? nullptr : Bsrc, Bdst);
    ttx_config c = forced ? *forced : batch_default(p, vec);
    if (c.family != p.family) return fail(TTX_EINVAL, "config family does not match the problem");
    c.flags &= ~TTX_CFG_XCD_SWIZZLE;  // tile ids are global in the persistent launch
    int idx;
    bool use_vec = vec;
    if (p.family == TTX_FAMILY_FLAT) {
        c.tile_a = use_vec ? (p.dtype == TTX_F32 ? 1024 : 512) : 256;
        c.tile_b = 1;
        idx = batch_index(p.dtype, p.family, c.tile_a, 1, use_vec ? 1 : 0);
    } else if (config_is_staged(c)) {
        idx = staged_index(p.dtype, staged_lanes(p.dim[0].size), c.tile_a, c.tile_b);
        if (idx < 0 && forced) {
            c = batch_default(p, false);
            idx = config_is_staged(c) ? staged_index(p.dtype, staged_lanes(p.dim[0].size), c.tile_a, c.tile_b)
                                      : batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 0);
        }
    } else {
        if (c.n_order != p.n) return fail(TTX_EINVAL, "order must list every merged index");
        idx = use_vec ? batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 1) : -1;
        if (idx < 0) {
            use_vec = false;
            idx = batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 0);
        }
        if (idx < 0 && forced) {
            // a tuned shape that only exists as a vector variant, now with
            // pointers that rule vectors out: fall back to the heuristic choice
            c = batch_default(p, false);
            idx = batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 0);
        }
    }
    if (idx < 0) return fail(TTX_EINVAL, "tile shape not in the batched menu");
    const int vclass = (p.dtype == TTX_F32 ? 0 : 2) + (beta0 ? 1 : 0);
    if (p.dtype == TTX_F32) {
        TileArgs<float> a;
        build_grid(p, c, &a);
        a.A = static_cast<const float*>(A);
        a.Bsrc = static_cast<const float*>(beta0 ? nullptr : Bsrc);
        a.Bdst = static_cast<float*>(Bdst);
        a.alpha = float(alpha);
        a.beta = float(beta);
        a.flags = (c.flags & TTX_CFG_NT_STORE) ? KF_NT_STORE : 0;
        d->tiles = a.g.ntiles;
        std::memcpy(d->args, &a, sizeof(a));
    } else {
        TileArgs<double> a;
        build_grid(p, c, &a);
        a.A = static_cast<const double*>(A);
        a.Bsrc = static_cast<const double*>(beta0 ? nullptr : Bsrc);
        a.Bdst = static_cast<double*>(Bdst);
        a.alpha = alpha;
        a.beta = beta;
        a.flags = (c.flags & TTX_CFG_NT_STORE) ? KF_NT_STORE : 0;
        d->tiles = a.g.ntiles;
        std::memcpy(d->args, &a, sizeof(a));
    }
    d->variant = vclass * TTX_BATCH_MENU_SIZE + idx;
    if (used) *used = c;
    return TTX_OK;
}

int batch_candidates(const Problem& p, int max_candidates, ttx_config* out, int cap) {
    if (p.family == TTX_FAMILY_EMPTY) return 0;
    int n = 0;
    if (max_candidates == 0) max_candidates = 200;
    const int limit = max_candidates < 0 ? cap : (max_candidates < cap ? max_candidates : cap);
    if (p.family == TTX_FAMILY_FLAT) {
        for (int f : {0, TTX_CFG_NT_STORE}) {
            if (n >= limit) break;
            out[n] = default_config(p);
            out[n].flags = f;
            ++n;
        }
        return n;
    }
    std::vector<ttx_config> all(1 << 17);
    int na = rank_candidates(p, -1, all.data(), nullptr, int(all.size()));
    for (int i = 0; i < na && n < limit; ++i) {
        const ttx_config& c = all[i];
        if (c.flags & TTX_CFG_XCD_SWIZZLE) continue;
        if (config_is_staged(c)) {
            if (staged_index(p.dtype, staged_lanes(p.dim[0].size), c.tile_a, c.tile_b) < 0) continue;
        } else if (batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 0) < 0 &&
                   batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 1) < 0) {
            continue;
        }
        out[n++] = c;
    }
    return n;
}

static std::string batch_key(const Problem& p, bool beta0, int vec) {
    std::string k = "B|v" + std::to_string(vec) + "|d" + std::to_string(p.dtype) + "|b" +
                    std::to_string(beta0 ? 1 : 0) + "|";
    for (int i = 0; i < p.n; ++i)
        k += std::to_string(p.dim[i].size) + "," + std::to_string(p.perm[i]) + "," +
             std::to_string(p.dim[i].sa) + "," + std::to_string(p.dim[i].sb) + ";";
    return k;
}

static std::mutex g_btab_mu;
static std::map<std::string, ttx_config> g_btab;

}  // namespace ttx

using namespace ttx;

static ttx_status problem_from(const ttx_problem& q, Problem* p) {
    return make_problem(q.dtype, q.n, q.perm, q.size, q.has_outer_a ? q.outer_a : nullptr,
                        q.has_outer_b ? q.outer_b : nullptr, p);
}

static ttx_status describe_all(ttx_batch* b) {
    const int count = int(b->prob.size());
    b->desc.assign(count, BatchDesc());
    b->prefix.assign(count + 1, 0);
    uint64_t total = 0;
    b->bytes = 0;
    for (int i = 0; i < count; ++i) {
        const ttx_problem& q = b->src[i];
        const Problem& p = b->prob[i];
        const bool beta0 = beta_is_zero(p.dtype, q.beta);
        const void* Bin = q.B_in ? q.B_in : q.B;
        ttx_config used;
        ttx_status st = batch_describe(p, b->forced[i] ? &b->cfg[i] : nullptr, beta0, q.A, Bin, q.B,
                                       q.alpha, q.beta, &b->desc[i], &used);
        if (st != TTX_OK) return st;
        b->cfg[i] = used;
        b->prefix[i] = uint32_t(total);
        total += b->desc[i].tiles;
        if (total >= (uint64_t(1) << 32)) return fail(TTX_EUNSUPPORTED, "batch has too many tiles");
        b->bytes += p.elements * (p.dtype == TTX_F32 ? 4 : 8) * (beta0 ? 2 : 3);
    }
    b->prefix[count] = uint32_t(total);
    b->total = uint32_t(total);
    b->grid = batch_grid(b->total);
    return TTX_OK;
}

static ttx_status upload(ttx_batch* b, hipStream_t stream) {
    const size_t nd = b->desc.size() * sizeof(BatchDesc);
    const size_t np = b->prefix.size() * sizeof(uint32_t);
    if (!b->d_desc) {
        if (hipMalloc(reinterpret_cast<void**>(&b->d_desc), nd ? nd : sizeof(BatchDesc)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&b->d_prefix), np) != hipSuccess)
            return fail(TTX_ENOMEM, "batch descriptor allocation failed");
    }
    if ((nd && hipMemcpyAsync(b->d_desc, b->desc.data(), nd, hipMemcpyHostToDevice, stream) != hipSuccess) ||
        hipMemcpyAsync(b->d_prefix, b->prefix.data(), np, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(TTX_EHIP, "batch descriptor upload failed");
    return TTX_OK;
}

static void drop_graph(ttx_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured = false;
}

extern "C" {

ttx_status ttx_batch_create(ttx_batch** out, int count, const ttx_problem* problems) {
    if (!out || count < 0 || (count > 0 && !problems)) return fail(TTX_EINVAL, "bad batch arguments");
    ttx_batch* b = new (std::nothrow) ttx_batch;
    if (!b) return fail(TTX_ENOMEM, "out of host memory");
    b->prob.resize(count);
    b->src.assign(problems, problems + count);
    b->cfg.resize(count);
    b->forced.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        ttx_status st = problem_from(problems[i], &b->prob[i]);
        if (st == TTX_OK) {
            const bool beta0 = beta_is_zero(problems[i].dtype, problems[i].beta);
            const void* Bin = problems[i].B_in ? problems[i].B_in : problems[i].B;
            st = check_pointers(b->prob[i], problems[i].A, Bin, problems[i].B, beta0);
            if (st == TTX_OK && b->prob[i].family != TTX_FAMILY_EMPTY) {
                std::lock_guard<std::mutex> lock(g_btab_mu);
                auto it = g_btab.find(batch_key(b->prob[i], beta0,
                                                vector_ok(b->prob[i], problems[i].A, beta0 ? nullptr : Bin,
                                                          problems[i].B)));
                if (it != g_btab.end()) {
                    b->cfg[i] = it->second;
                    b->forced[i] = 1;
                }
            }
        }
        if (st != TTX_OK) {
            delete b;
            return fail(st, "problem " + std::to_string(i) + ": " + ttx_last_error());
        }
    }
    ttx_status st = describe_all(b);
    if (st == TTX_OK) st = upload(b, nullptr);
    if (st != TTX_OK) {
        ttx_batch_destroy(b);
        return st;
    }
    *out = b;
    return TTX_OK;
}

ttx_status ttx_batch_update(ttx_batch* b, int count, const ttx_problem* problems, hipStream_t stream) {
    if (!b || !problems || count != int(b->prob.size())) return fail(TTX_EINVAL, "count must match the batch");
    for (int i = 0; i < count; ++i) {
        Problem p;
        ttx_status st = problem_from(problems[i], &p);
        if (st != TTX_OK) return st;
        const Problem& o = b->prob[i];
        bool same = p.dtype == o.dtype && p.n == o.n && p.family == o.family && p.elements == o.elements;
        for (int d = 0; same && d < p.n; ++d)
            same = p.perm[d] == o.perm[d] && p.dim[d].size == o.dim[d].size &&
                   p.dim[d].sa == o.dim[d].sa && p.dim[d].sb == o.dim[d].sb;
        if (!same) return fail(TTX_EINVAL, "problem " + std::to_string(i) + " changed shape");
        const bool beta0 = beta_is_zero(p.dtype, problems[i].beta);
        const void* Bin = problems[i].B_in ? problems[i].B_in : problems[i].B;
        st = check_pointers(p, problems[i].A, Bin, problems[i].B, beta0);
        if (st != TTX_OK) return st;
    }
    const uint32_t old_total = b->total;
    b->src.assign(problems, problems + count);
    for (int i = 0; i < count; ++i) b->forced[i] = b->prob[i].family != TTX_FAMILY_EMPTY;
    ttx_status st = describe_all(b);
    if (st != TTX_OK) return st;
    if (b->total != old_total) drop_graph(b);
    return upload(b, stream);
}

ttx_status ttx_batch_tune(ttx_batch* b, int max_candidates, int reps) {
    if (!b) return fail(TTX_EINVAL, "NULL batch");
    if (max_candidates == 0) max_candidates = 16;
    BatchDesc* d_one = nullptr;
    uint32_t* d_pre = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&d_one), sizeof(BatchDesc)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d_pre), 2 * sizeof(uint32_t)) != hipSuccess) {
        if (d_one) (void)hipFree(d_one);
        return fail(TTX_ENOMEM, "tuner descriptor allocation failed");
    }
    ttx_status result = TTX_OK;
    std::vector<ttx_config> cands(4096);
    for (size_t i = 0; i < b->prob.size() && result == TTX_OK; ++i) {
        const Problem& p = b->prob[i];
        if (p.family == TTX_FAMILY_EMPTY) continue;
        const ttx_problem& q = b->src[i];
        const bool beta0 = beta_is_zero(p.dtype, q.beta);
        const void* Bin = q.B_in ? q.B_in : q.B;
        const int vec = vector_ok(p, q.A, beta0 ? nullptr : Bin, q.B);
        const std::string key = batch_key(p, beta0, vec);
        {
            std::lock_guard<std::mutex> lock(g_btab_mu);
            auto it = g_btab.find(key);
            if (it != g_btab.end()) {
                b->cfg[i] = it->second;
                b->forced[i] = 1;
                continue;
            }
        }
        int nc = batch_candidates(p, max_candidates, cands.data(), int(cands.size()));
        if (nc <= 0) continue;
        // scratch pointers keep the real pointers' offsets modulo 16 bytes, so
        // that each candidate runs the same vector variant it will run for real
        const uintptr_t offa = reinterpret_cast<uintptr_t>(q.A) & 15;
        const uintptr_t offb = reinterpret_cast<uintptr_t>(q.B) & 15;
        int best_i = -1;
        double best_us = 0;
        result = time_candidates(p, beta0, nc, reps,
            [&](int c, const void* A, void* B, hipStream_t s) -> hipError_t {
                BatchDesc one;
                const void* a = static_cast<const char*>(A) + offa;
                void* bb = static_cast<char*>(B) + offb;
                if (batch_describe(p, &cands[c], beta0, a, bb, bb, 1.0, beta0 ? 0.0 : 1.0, &one, nullptr) != TTX_OK)
                    return hipErrorInvalidValue;
                const uint32_t pre[2] = {0, one.tiles};
                hipError_t e = hipMemcpyAsync(d_one, &one, sizeof(one), hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipMemcpyAsync(d_pre, pre, sizeof(pre), hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return e;
                return launch_batch(d_one, d_pre, 1, one.tiles, batch_grid(one.tiles), s);
            },
            &best_i, &best_us);
        if (result == TTX_OK && best_i >= 0) {
            b->cfg[i] = cands[best_i];
            b->forced[i] = 1;
            std::lock_guard<std::mutex> lock(g_btab_mu);
            g_btab[key] = cands[best_i];
        }
    }
    (void)hipFree(d_one);
    (void)hipFree(d_pre);
    if (result != TTX_OK) return result;
    const uint32_t old_total = b->total;
    ttx_status st = describe_all(b);
    if (st != TTX_OK) return st;
    if (b->total != old_total) drop_graph(b);
    return upload(b, nullptr);
}

ttx_status ttx_batch_execute_direct(ttx_batch* b, hipStream_t stream) {
    if (!b) return fail(TTX_EINVAL, "NULL batch");
    hipError_t e = launch_batch(b->d_desc, b->d_prefix, int(b->prob.size()), b->total, b->grid, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
}

ttx_status ttx_batch_execute(ttx_batch* b, hipStream_t stream) {
    if (!b) return fail(TTX_EINVAL, "NULL batch");
    if (b->total == 0) return TTX_OK;
    if (!b->captured) {
        drop_graph(b);
        if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(TTX_EHIP, "capture stream creation failed");
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(TTX_EHIP, "stream capture failed to start");
        hipError_t e = launch_batch(b->d_desc, b->d_prefix, int(b->prob.size()), b->total, b->grid,
                                    b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return fail(TTX_EHIP, "batch capture failed");
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            return fail(TTX_EHIP, "graph instantiation failed");
        }
        b->captured = true;
    }
    hipError_t e = hipGraphLaunch(b->exec, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
}

ttx_status ttx_batch_get_info(const ttx_batch* b, ttx_batch_info* info) {
    if (!b || !info) return fail(TTX_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->count = int(b->prob.size());
    info->total_tiles = b->total;
    info->grid = b->grid;
    info->algorithmic_bytes = b->bytes;
    bool seen[4 * TTX_BATCH_MENU_SIZE] = {};
    for (const auto& d : b->desc)
        if (d.variant >= 0 && !seen[d.variant]) {
            seen[d.variant] = true;
            ++info->variants_used;
        }
    int tuned = 0;
    for (int f : b->forced) tuned += f;
    info->tuned = tuned;
    return TTX_OK;
}

ttx_status ttx_batch_config(const ttx_batch* b, int index, ttx_config* config) {
    if (!b || !config || index < 0 || index >= int(b->prob.size())) return fail(TTX_EINVAL, "bad index");
    *config = b->cfg[index];
    return TTX_OK;
}

ttx_status ttx_batch_plan(int count, const ttx_problem* problems, ttx_config* configs, int64_t* tiles) {
    if (count < 0 || (count > 0 && (!problems || !configs || !tiles))) return fail(TTX_EINVAL, "bad arguments");
    for (int i = 0; i < count; ++i) {
        Problem p;
        ttx_status st = problem_from(problems[i], &p);
        if (st != TTX_OK) return st;
        const bool beta0 = beta_is_zero(p.dtype, problems[i].beta);
        const void* Bin = problems[i].B_in ? problems[i].B_in : problems[i].B;
        st = check_pointers(p, problems[i].A, Bin, problems[i].B, beta0);
        if (st != TTX_OK) return st;
        BatchDesc d;
        ttx_config used;
        st = batch_describe(p, nullptr, beta0, problems[i].A, Bin, problems[i].B, problems[i].alpha,
                            problems[i].beta, &d, &used);
        if (st != TTX_OK) return st;
        configs[i] = used;
        tiles[i] = d.tiles;
    }
    return TTX_OK;
}

ttx_status ttx_batch_destroy(ttx_batch* b) {
    if (!b) return TTX_OK;
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_prefix) (void)hipFree(b->d_prefix);
    delete b;
    return TTX_OK;
}

}  // extern "C"
