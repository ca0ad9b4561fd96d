// Batched execution: many independent transpositions, each Eqn. 1 with its
// own shape, permutation, scalars and tensors, run by ONE persistent kernel.
//
// The host plans every problem, picks a tile variant from the small batched
// menu (tuned per shape or chosen by the heuristics of Sec. 2.3), splits its
// tiles into chunks of consecutive tiles, and writes the descriptor table and
// the prefix sums of the per-problem chunk counts to device memory.  The
// kernel is launched with about one wave of resident workgroups; each claims
// chunks from a counter, finds the owning problem by binary search over the
// prefix sums, and runs that problem's tile body over the chunk -- the same
// tile code as the per-call kernels, pipelined across the chunk's tiles.  The
// launch is captured once into a HIP graph and replayed.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "menu.h"
#include "tile_kernels.h"
#include "ttx_internal.h"

struct ttx_batch {
    std::vector<ttx::Problem> prob;
    std::vector<ttx_problem> src;
    std::vector<ttx_config> cfg;
    std::vector<int> forced;
    std::vector<int> per_call;           // problems launched with their per-call kernels
    std::vector<ttx::BatchDesc> desc;    // kernel problems, in work order
    std::vector<uint32_t> chunk_prefix;  // over the work order
    std::vector<int> order;              // work position -> problem index
    int nk = 0;                          // problems in the persistent kernel
    unsigned char* d_work = nullptr;     // descriptors, chunk prefix, claim counter
    size_t work_bytes = 0;
    uint64_t total = 0;                  // tiles
    uint32_t chunks = 0;
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

static int dense_index(int dtype) {
    const BatchEntry* m = batch_menu(dtype);
    for (int i = 0; i < TTX_BATCH_MENU_SIZE; ++i)
        if (m[i].kind == TTX_BATCH_DENSE) return i;
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
    return kind == TTX_FAMILY_MOVED    ? p2 * (p1 + 1) * esize
           : kind == TTX_BATCH_STAGED ? p3 * (p2 * p1 + 1) * esize
           : kind == TTX_BATCH_DENSE  ? dense_lds_elems(p1) * esize
                                      : 0;
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

// Tiles [t0, t1) of one problem with the variant's tile body, pipelined
// across the tiles, with plain (not nontemporal) stores: a second store kind
// would double every variant's code in the persistent kernel, so its
// candidates do not offer TTX_CFG_NT_STORE.  Thread 0 also claims the workgroup's next chunk: the
// claim is issued first, so that its round trip overlaps the chunk, and its
// result is left in *next (LDS) for the caller's barrier to publish.
//
// The body is a separate function so that each variant gets its own register
// allocation (inlined into one kernel, the variants together need far more
// registers than any one of them).  A callee cannot see that its arguments
// are the same in every lane, so the descriptor address and the tile range
// are made wave-uniform explicitly and the descriptor is read through the
// constant address space: its fields then live in scalar registers, as the
// kernel arguments of the per-call kernels do.
template <typename T, bool B0, int KIND, int P1, int P2, int P3>
__device__ __noinline__ void batch_body(unsigned char* lds, const TileArgs<T>& args, uint32_t t0, uint32_t t1,
                                        uint32_t* counter, uint32_t* next) {
    typedef __attribute__((address_space(4))) const TileArgs<T> ConstArgs;
    const uint64_t bits = reinterpret_cast<uint64_t>(&args);
    // (readfirstlane returns a signed int: widen through uint32_t so that the
    // low word is not sign-extended into the high one)
    const uint64_t ubits = uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(bits >> 32)))) << 32 |
                           uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(bits))));
    const TileArgs<T>& a = *(const TileArgs<T>*)((ConstArgs*)ubits);
    t0 = uint32_t(__builtin_amdgcn_readfirstlane(t0));
    t1 = uint32_t(__builtin_amdgcn_readfirstlane(t1));
    uint32_t claim = 0;
    if (threadIdx.x == 0) claim = atomicAdd(counter, 1u);
    T* l = reinterpret_cast<T*>(lds);
    if constexpr (KIND == TTX_BATCH_STAGED) {
        tile_loop<StagedTile<T, B0, P1, P2, P3, T, 0>, true>(l, a, t0, t1, 1);
    } else if constexpr (KIND == TTX_BATCH_DENSE) {
        tile_loop<DenseTile<T, B0, P1, T, 0>, false>(l, a, t0, t1, 1);
    } else if constexpr (KIND == TTX_FAMILY_FLAT) {
        constexpr int V = P3 ? kVec<T> : 1;
        tile_loop<FlatTile<T, B0, V, P1 / (kThreads * V), 0>, true>(l, a, t0, t1, 1);
    } else {
        constexpr int V = P3 ? kVec<T> : 1;
        if constexpr (KIND == TTX_FAMILY_MOVED)
            tile_loop<MovedTile<T, B0, P1, P2, V, V, T, 0>, true>(l, a, t0, t1, 1);
        else
            tile_loop<PreservedTile<T, B0, P1, P2, V, T, 0>, true>(l, a, t0, t1, 1);
    }
    if (threadIdx.x == 0) *next = claim;
}

template <bool B0>
__device__ __forceinline__ bool batch_dispatch_f32(int idx, unsigned char* lds, const BatchDesc& d, uint32_t t0,
                                                   uint32_t t1, uint32_t* counter, uint32_t* next) {
    const TileArgs<float>& a = *reinterpret_cast<const TileArgs<float>*>(d.args);
    switch (idx) {
#define TTX_CASE(i, kind, p1, p2, p3) \
    case i: batch_body<float, B0, kind, p1, p2, p3>(lds, a, t0, t1, counter, next); return true;
        TTX_BATCH_MENU_F32(TTX_CASE)
#undef TTX_CASE
        default: return false;
    }
}

template <bool B0>
__device__ __forceinline__ bool batch_dispatch_f64(int idx, unsigned char* lds, const BatchDesc& d, uint32_t t0,
                                                   uint32_t t1, uint32_t* counter, uint32_t* next) {
    const TileArgs<double>& a = *reinterpret_cast<const TileArgs<double>*>(d.args);
    switch (idx) {
#define TTX_CASE(i, kind, p1, p2, p3) \
    case i: batch_body<double, B0, kind, p1, p2, p3>(lds, a, t0, t1, counter, next); return true;
        TTX_BATCH_MENU_F64(TTX_CASE)
#undef TTX_CASE
        default: return false;
    }
}

// Persistent kernel: each workgroup claims chunks (runs of up to
// desc.chunk consecutive tiles of one problem) from counter[0] until the
// chunks run out.  The claimed chunk's problem is found by binary search
// over chunk_prefix.  The last workgroup to finish (counted in counter[1])
// resets both words, so the launch can be replayed from a graph without a
// reset node.  Chunk ids are handed out in descriptor order, and the host
// orders descriptors by decreasing size, so the last chunks are short.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_batch(const BatchDesc* __restrict__ desc, const uint32_t* __restrict__ chunk_prefix, int count,
             uint32_t chunks, uint32_t* counter) {
    __shared__ __align__(16) unsigned char lds[kBatchLds];
    __shared__ uint32_t claim[2];
    if (threadIdx.x == 0) claim[0] = atomicAdd(&counter[0], 1u);
    __syncthreads();
    uint32_t c = claim[0];
    int slot = 0;
    while (c < chunks) {
        // largest p with chunk_prefix[p] <= c (chunk_prefix[0] == 0)
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (chunk_prefix[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        const int p = __builtin_amdgcn_readfirstlane(lo);
        const BatchDesc& d = desc[p];
        const int v = d.variant;
        uint32_t* next = &claim[slot ^ 1];
        bool ran = false;
        if (v >= 0) {
            const uint32_t t0 = (c - chunk_prefix[p]) * d.chunk;
            const uint32_t t1 = min(t0 + d.chunk, d.tiles);
            const int idx = v % TTX_BATCH_MENU_SIZE;
            switch (v / TTX_BATCH_MENU_SIZE) {
                case 0: ran = batch_dispatch_f32<false>(idx, lds, d, t0, t1, counter, next); break;
                case 1: ran = batch_dispatch_f32<true>(idx, lds, d, t0, t1, counter, next); break;
                case 2: ran = batch_dispatch_f64<false>(idx, lds, d, t0, t1, counter, next); break;
                case 3: ran = batch_dispatch_f64<true>(idx, lds, d, t0, t1, counter, next); break;
                default: break;
            }
        }
        // a body claims the next chunk itself; without one, claim here
        if (!ran && threadIdx.x == 0) *next = atomicAdd(counter, 1u);
        // publishes *next; every thread read claim[slot] before this barrier
        __syncthreads();
        c = claim[slot ^ 1];
        slot ^= 1;
    }
    if (threadIdx.x == 0) {
        const uint32_t done = atomicAdd(&counter[1], 1u);
        if (done == gridDim.x - 1) {
            // every other workgroup has made its last claim
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

int batch_grid(uint32_t chunks) {
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
    return int(chunks < g ? chunks : g);
}

uint32_t batch_layout(BatchDesc* desc, int count, uint32_t* chunk_prefix, int* grid) {
    uint64_t tiles = 0;
    for (int i = 0; i < count; ++i) tiles += desc[i].tiles;
    // about 8 chunks per workgroup of a full launch, at most 32 tiles each
    const uint64_t g = uint64_t(batch_grid(0xffffffffu));
    uint64_t k = tiles / (8 * g);
    k = k < 1 ? 1 : (k > 32 ? 32 : k);
    uint64_t chunks = 0;
    for (int i = 0; i < count; ++i) {
        chunk_prefix[i] = uint32_t(chunks);
        desc[i].chunk = uint32_t(k);
        chunks += (desc[i].tiles + k - 1) / k;
    }
    chunk_prefix[count] = uint32_t(chunks);
    *grid = batch_grid(uint32_t(chunks));
    return uint32_t(chunks);
}

hipError_t launch_batch(const BatchDesc* d_desc, const uint32_t* d_chunk_prefix, int count, uint32_t chunks,
                        int grid, uint32_t* counter, hipStream_t stream) {
    if (chunks == 0 || grid <= 0 || count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kThreads), 0, stream, d_desc, d_chunk_prefix, count, chunks,
                       counter);
    return hipGetLastError();
}

// -- host side --------------------------------------------------------------------------
static int elem_size(int dtype) { return elem_bytes(dtype); }

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
        if (m[i].kind == TTX_BATCH_DENSE) continue;
        if (m[i].kind != p.family || (m[i].p3 && !vec)) continue;
        bool dup = false;
        for (const auto& s : shapes) dup |= s.ta == m[i].p1 && s.tb == m[i].p2;
        if (!dup) shapes.push_back(TileShape{m[i].p1, m[i].p2});
    }
    return default_config_from(p, shapes.data(), int(shapes.size()), staged.data(), int(staged.size()), true);
}

ttx_status batch_describe(const Problem& p, const ttx_config* forced, bool beta0, const void* A,
                          const void* Bsrc, void* Bdst, double alpha, double beta, BatchDesc* d,
                          ttx_config* used) {
    std::memset(d, 0, sizeof(*d));
    d->dtype = p.dtype;
    d->variant = -1;
    if (dtype_complex(p.dtype) || p.dtype_a != p.dtype)
        return fail(TTX_EUNSUPPORTED, "batched execution takes FP32 and FP64 problems only");
    if (p.family == TTX_FAMILY_EMPTY) {
        if (used) *used = default_config(p);
        return TTX_OK;
    }
    const bool vec = vector_ok(p, A, beta0 ? nullptr : Bsrc, Bdst);
    // the persistent kernel's variants run 256 threads with one element of
    // LDS padding: a config for another workgroup shape takes the heuristic
    ttx_config c = forced && !config_needs_jit(p, *forced) ? *forced : batch_default(p, vec);
    if (c.family != p.family) return fail(TTX_EINVAL, "config family does not match the problem");
    if (config_is_wide(c)) return fail(TTX_EINVAL, "whole-unit rows are for per-call launches only");
    c.flags &= ~TTX_CFG_XCD_SWIZZLE;  // tile ids are global in the persistent launch
    // the menu entry for a config (-1: none); flat configs get their tile here
    auto resolve = [&](ttx_config& k) -> int {
        if (p.family == TTX_FAMILY_FLAT) {
            k.tile_a = vec ? (p.dtype == TTX_F32 ? 4096 : 2048) : 1024;
            k.tile_b = 1;
            return batch_index(p.dtype, p.family, k.tile_a, 1, vec ? 1 : 0);
        }
        if (config_is_dense(k)) return dense_index(p.dtype);
        if (config_is_staged(k)) return staged_index(p.dtype, staged_lanes(p.dim[0].size), k.tile_a, k.tile_b);
        if (k.n_order != p.n) return -1;
        const int v = vec ? batch_index(p.dtype, p.family, k.tile_a, k.tile_b, 1) : -1;
        return v >= 0 ? v : batch_index(p.dtype, p.family, k.tile_a, k.tile_b, 0);
    };
    int idx = resolve(c);
    if (idx < 0 && forced) {
        // a tuned shape that only exists as a vector variant, now with
        // pointers that rule vectors out: fall back to the heuristic choice
        c = batch_default(p, false);
        c.flags &= ~TTX_CFG_XCD_SWIZZLE;
        idx = resolve(c);
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
        a.flags = 0;   // plain stores (the tile bodies below fix the store kind)
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
        a.flags = 0;   // plain stores (the tile bodies below fix the store kind)
        d->tiles = a.g.ntiles;
        std::memcpy(d->args, &a, sizeof(a));
    }
    d->variant = vclass * TTX_BATCH_MENU_SIZE + idx;
    if (used) *used = c;
    return TTX_OK;
}

void batch_set_output(BatchDesc* d, void* Bdst) {
    if (d->variant < 0) return;
    if (d->dtype == TTX_F32)
        reinterpret_cast<TileArgs<float>*>(d->args)->Bdst = static_cast<float*>(Bdst);
    else
        reinterpret_cast<TileArgs<double>*>(d->args)->Bdst = static_cast<double*>(Bdst);
}

int batch_candidates(const Problem& p, int max_candidates, ttx_config* out, int cap) {
    if (p.family == TTX_FAMILY_EMPTY) return 0;
    int n = 0;
    if (max_candidates == 0) max_candidates = 200;
    const int limit = max_candidates < 0 ? cap : (max_candidates < cap ? max_candidates : cap);
    if (p.family == TTX_FAMILY_FLAT) {   // one candidate: the persistent kernel stores plainly
        if (limit < 1) return 0;
        out[0] = default_config(p);
        out[0].flags = 0;
        return 1;
    }
    std::vector<ttx_config> all(1 << 17);
    int na = rank_candidates(p, -1, all.data(), nullptr, int(all.size()));
    // batched-menu candidates in cost order, and a quarter of the list kept
    // for each kind (menu, staged, dense tiles), as in rank_candidates
    std::vector<int> eligible, kind;
    for (int i = 0; i < na; ++i) {
        const ttx_config& c = all[i];
        if (c.flags & (TTX_CFG_XCD_SWIZZLE | TTX_CFG_WIDE | TTX_CFG_NT_STORE)) continue;
        int k = 0;
        if (config_is_dense(c)) {
            if (dense_index(p.dtype) < 0) continue;
            k = 2;
        } else if (config_is_staged(c)) {
            if (staged_index(p.dtype, staged_lanes(p.dim[0].size), c.tile_a, c.tile_b) < 0) continue;
            k = 1;
        } else if (batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 0) < 0 &&
                   batch_index(p.dtype, p.family, c.tile_a, c.tile_b, 1) < 0) {
            continue;
        }
        eligible.push_back(i);
        kind.push_back(k);
    }
    std::vector<char> taken(eligible.size(), 0);
    int per_kind[3] = {};
    const int quota = limit / 4;
    for (size_t j = 0; j < eligible.size() && n < limit; ++j)
        if (per_kind[kind[j]] < quota) {
            ++per_kind[kind[j]];
            taken[j] = 1;
            ++n;
        }
    for (size_t j = 0; j < eligible.size() && n < limit; ++j)
        if (!taken[j]) {
            taken[j] = 1;
            ++n;
        }
    n = 0;
    for (size_t j = 0; j < eligible.size(); ++j)
        if (taken[j]) out[n++] = all[eligible[j]];
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
    ttx_status st = make_problem(q.dtype, q.n, q.perm, q.size, q.has_outer_a ? q.outer_a : nullptr,
                                 q.has_outer_b ? q.outer_b : nullptr, p);
    if (st == TTX_OK && !dtype_complex(p->dtype) && (q.alpha_im != 0.0 || q.beta_im != 0.0))
        return fail(TTX_EINVAL, "complex alpha or beta for a real element type");
    return st;
}

static Scalar alpha_of(const ttx_problem& q) { return Scalar(q.alpha, q.alpha_im); }
static Scalar beta_of(const ttx_problem& q) { return Scalar(q.beta, q.beta_im); }

// Complex and mixed-precision problems run their per-call kernels (the
// persistent kernel's variants are FP32 and FP64 only).
static bool runs_per_call(const Problem& p) {
    return p.family != TTX_FAMILY_EMPTY && (dtype_complex(p.dtype) || p.dtype_a != p.dtype);
}

// Device work block of a batch: descriptors, chunk prefix, claim counter.
static constexpr size_t desc_bytes(int count) { return size_t(count) * sizeof(BatchDesc); }
static constexpr size_t prefix_offset(int count) { return desc_bytes(count); }
static constexpr size_t counter_offset(int count) { return (prefix_offset(count) + sizeof(uint32_t) * (count + 1) + 15) & ~size_t(15); }
static constexpr size_t work_bytes(int count) { return counter_offset(count) + 2 * sizeof(uint32_t); }

static const BatchDesc* work_desc(const ttx_batch* b) { return reinterpret_cast<const BatchDesc*>(b->d_work); }
static const uint32_t* work_prefix(const ttx_batch* b) {
    return reinterpret_cast<const uint32_t*>(b->d_work + prefix_offset(b->nk));
}
static uint32_t* work_counter(const ttx_batch* b) {
    return reinterpret_cast<uint32_t*>(b->d_work + counter_offset(b->nk));
}

static ttx_status describe_all(ttx_batch* b) {
    const int count = int(b->prob.size());
    std::vector<BatchDesc> desc(count);
    std::vector<int> kernel;
    uint64_t total = 0;
    b->bytes = 0;
    b->per_call.clear();
    for (int i = 0; i < count; ++i) {
        const ttx_problem& q = b->src[i];
        const Problem& p = b->prob[i];
        const bool beta0 = beta_is_zero(p.dtype, beta_of(q));
        b->bytes += p.elements * (elem_bytes(p.dtype_a) + elem_bytes(p.dtype) * (beta0 ? 1 : 2));
        if (runs_per_call(p)) {
            if (!b->forced[i] && !table_lookup(p, beta0, &b->cfg[i])) b->cfg[i] = default_config(p);
            b->per_call.push_back(i);
            continue;
        }
        const void* Bin = q.B_in ? q.B_in : q.B;
        ttx_config used;
        ttx_status st = batch_describe(p, b->forced[i] ? &b->cfg[i] : nullptr, beta0, q.A, Bin, q.B,
                                       q.alpha, q.beta, &desc[i], &used);
        if (st != TTX_OK) return st;
        b->cfg[i] = used;
        total += desc[i].tiles;
        if (total >= (uint64_t(1) << 32)) return fail(TTX_EUNSUPPORTED, "batch has too many tiles");
        kernel.push_back(i);
    }
    // largest problems first, so that the chunks claimed last are short ones
    b->order = kernel;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return b->prob[x].elements * elem_bytes(b->prob[x].dtype) >
               b->prob[y].elements * elem_bytes(b->prob[y].dtype);
    });
    b->nk = int(kernel.size());
    b->desc.resize(b->nk);
    for (int i = 0; i < b->nk; ++i) b->desc[i] = desc[b->order[i]];
    b->chunk_prefix.assign(b->nk + 1, 0);
    b->total = total;
    b->chunks = b->nk ? batch_layout(b->desc.data(), b->nk, b->chunk_prefix.data(), &b->grid) : 0;
    if (!b->nk) b->grid = 0;
    return TTX_OK;
}

// The per-call launches of a batch's complex and mixed-precision problems.
static hipError_t launch_per_call(const ttx_batch* b, hipStream_t stream) {
    for (int i : b->per_call) {
        const ttx_problem& q = b->src[i];
        const Problem& p = b->prob[i];
        const bool beta0 = beta_is_zero(p.dtype, beta_of(q));
        const void* Bin = q.B_in ? q.B_in : q.B;
        hipError_t e = launch_tiles(p, b->cfg[i], beta0, q.A, beta0 ? nullptr : Bin, q.B, alpha_of(q), beta_of(q),
                                    stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static ttx_status upload(ttx_batch* b, hipStream_t stream) {
    const int count = b->nk;
    const size_t need = work_bytes(count);
    if (!b->d_work) {
        if (hipMalloc(reinterpret_cast<void**>(&b->d_work), need) != hipSuccess)
            return fail(TTX_ENOMEM, "batch descriptor allocation failed");
        b->work_bytes = need;
        // the claim counter starts at zero; every launch leaves it at zero
        if (hipMemset(b->d_work + counter_offset(count), 0, 2 * sizeof(uint32_t)) != hipSuccess)
            return fail(TTX_EHIP, "batch counter initialisation failed");
    }
    if ((count && hipMemcpyAsync(b->d_work, b->desc.data(), desc_bytes(count), hipMemcpyHostToDevice, stream) !=
                      hipSuccess) ||
        hipMemcpyAsync(b->d_work + prefix_offset(count), b->chunk_prefix.data(), sizeof(uint32_t) * (count + 1),
                       hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(TTX_EHIP, "batch descriptor upload failed");
    return TTX_OK;
}

// Checks and plans every problem and builds the descriptor table, on the
// host only (no HIP call): what ttx_batch_create and ttx_batch_run_static
// share, so that both run the same configs.
static ttx_status prepare(ttx_batch* b, int count, const ttx_problem* problems) {
    b->prob.resize(count);
    b->src.assign(problems, problems + count);
    b->cfg.resize(count);
    b->forced.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        ttx_status st = problem_from(problems[i], &b->prob[i]);
        if (st == TTX_OK) {
            const bool beta0 = beta_is_zero(b->prob[i].dtype, beta_of(problems[i]));
            const void* Bin = problems[i].B_in ? problems[i].B_in : problems[i].B;
            st = check_pointers(b->prob[i], problems[i].A, Bin, problems[i].B, beta0);
            if (st == TTX_OK && b->prob[i].family != TTX_FAMILY_EMPTY && !runs_per_call(b->prob[i])) {
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
        if (st != TTX_OK) return fail(st, "problem " + std::to_string(i) + ": " + ttx_last_error());
    }
    return describe_all(b);
}

// -- allocation-free runs ----------------------------------------------------------------
// The work block of ttx_batch_run_static (descriptors, chunk prefix, claim
// counter of at most TTX_STATIC_BATCH_MAX problems) lives in this file-scope
// device array: each GPU the library runs on holds its own copy until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy (on the host it is only a stand-in symbol): it uses the device
// address that hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[work_bytes(TTX_STATIC_BATCH_MAX)];

static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[64];

static ttx_status scratch_address(unsigned char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TTX_EHIP, "no current device");
    if (dev < 0 || dev >= 64) return fail(TTX_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TTX_EHIP, std::string("scratch address lookup: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
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
    ttx_status st = prepare(b, count, problems);
    if (st != TTX_OK) {
        delete b;
        return st;
    }
    st = upload(b, nullptr);
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
        bool same = p.code == o.code && p.n == o.n && p.family == o.family && p.elements == o.elements;
        for (int d = 0; same && d < p.n; ++d)
            same = p.perm[d] == o.perm[d] && p.dim[d].size == o.dim[d].size &&
                   p.dim[d].sa == o.dim[d].sa && p.dim[d].sb == o.dim[d].sb;
        if (!same) return fail(TTX_EINVAL, "problem " + std::to_string(i) + " changed shape");
        const bool beta0 = beta_is_zero(p.dtype, beta_of(problems[i]));
        const void* Bin = problems[i].B_in ? problems[i].B_in : problems[i].B;
        st = check_pointers(p, problems[i].A, Bin, problems[i].B, beta0);
        if (st != TTX_OK) return st;
    }
    const uint32_t old_chunks = b->chunks;
    const int old_grid = b->grid;
    b->src.assign(problems, problems + count);
    for (int i = 0; i < count; ++i) b->forced[i] = b->prob[i].family != TTX_FAMILY_EMPTY;
    ttx_status st = describe_all(b);
    if (st != TTX_OK) return st;
    // per-call launches carry their pointers in the graph: capture again
    if (b->chunks != old_chunks || b->grid != old_grid || !b->per_call.empty()) drop_graph(b);
    return upload(b, stream);
}

// A tuned batched configuration replaces the current one only when it is
// faster by at least this fraction.
static constexpr double kBatchTuneMargin = 0.05;
// The tuned set must also win in context, by this much.
static constexpr double kBatchContextMargin = 0.01;

// Median time (ms) of `reps` persistent launches of the batch as described now.
static double time_launches(ttx_batch* b, hipStream_t s, int reps, hipEvent_t* ev) {
    std::vector<float> ms;
    for (int r = -1; r < reps; ++r) {   // r = -1: warm-up
        if (hipEventRecord(ev[0], s) != hipSuccess) return -1;
        if (launch_batch(work_desc(b), work_prefix(b), b->nk, b->chunks, b->grid, work_counter(b), s) != hipSuccess)
            return -1;
        if (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) return -1;
        float t = 0;
        if (hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess) return -1;
        if (r >= 0) ms.push_back(t);
    }
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

// Whether the configs now in `b` (the tuned set) run the whole persistent
// launch faster than `old_cfg` / `old_forced` (the set they replaced): both
// are timed in alternation on scratch copies of the batch's footprint (the
// kernel problems' A and B extents, each at its pointer's offset modulo 16
// bytes, so that every problem runs the same vector variant), never on the
// caller's tensors.  When the scratch cannot be allocated the tuned set is
// kept.  Leaves `b` described with the tuned set and the real pointers.
static bool tuned_set_wins(ttx_batch* b, const std::vector<ttx_config>& old_cfg, const std::vector<int>& old_forced,
                           int reps) {
    const std::vector<ttx_config> new_cfg = b->cfg;
    const std::vector<int> new_forced = b->forced;
    const std::vector<ttx_problem> real = b->src;
    std::vector<int64_t> off_a(b->prob.size(), -1), off_b(b->prob.size(), -1);
    int64_t total = 0;
    for (size_t i = 0; i < b->prob.size(); ++i) {
        const Problem& p = b->prob[i];
        if (p.family == TTX_FAMILY_EMPTY || runs_per_call(p)) continue;
        off_a[i] = total + int64_t(reinterpret_cast<uintptr_t>(real[i].A) & 15);
        total += (p.extent_a + 16 + 255) / 256 * 256;
        off_b[i] = total + int64_t(reinterpret_cast<uintptr_t>(real[i].B) & 15);
        total += (p.extent_b + 16 + 255) / 256 * 256;
    }
    unsigned char* scratch = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ok = total > 0 && hipMalloc(reinterpret_cast<void**>(&scratch), size_t(total)) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
    ok = ok && hipMemsetAsync(scratch, 0, size_t(total), s) == hipSuccess;
    double t_new = 0, t_old = 0;
    if (ok) {
        for (size_t i = 0; i < b->prob.size(); ++i) {
            if (off_a[i] < 0) continue;
            b->src[i].A = scratch + off_a[i];
            b->src[i].B = scratch + off_b[i];
            b->src[i].B_in = nullptr;
        }
        for (int round = 0; round < 2 && ok; ++round) {
            for (int set = 0; set < 2 && ok; ++set) {
                b->cfg = set == 0 ? new_cfg : old_cfg;
                b->forced = set == 0 ? new_forced : old_forced;
                ok = describe_all(b) == TTX_OK && upload(b, s) == TTX_OK;
                const double t = ok ? time_launches(b, s, reps, ev) : -1;
                ok = ok && t > 0;
                (set == 0 ? t_new : t_old) += t;
            }
        }
    }
    if (!ok) (void)hipGetLastError();   // no in-context check: the tuned set stays
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    if (s) (void)hipStreamDestroy(s);
    if (scratch) (void)hipFree(scratch);
    b->src = real;
    b->cfg = new_cfg;
    b->forced = new_forced;
    clear_error();
    return !ok || t_new < t_old * (1.0 - kBatchContextMargin);
}

ttx_status ttx_batch_tune(ttx_batch* b, int max_candidates, int reps) {
    if (!b) return fail(TTX_EINVAL, "NULL batch");
    if (max_candidates == 0) max_candidates = 16;
    // the batch's descriptors are rewritten below: no earlier launch of it may still read them
    const hipError_t idle = hipDeviceSynchronize();
    if (idle != hipSuccess) return fail(TTX_EHIP, std::string("hipDeviceSynchronize: ") + hipGetErrorString(idle));
    // a one-problem work block: descriptor, chunk prefix, claim counter
    const size_t need = work_bytes(1);
    unsigned char* d_blk = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&d_blk), need) != hipSuccess)
        return fail(TTX_ENOMEM, "tuner descriptor allocation failed");
    if (hipMemset(d_blk + counter_offset(1), 0, 2 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(d_blk);
        return fail(TTX_EHIP, "tuner counter initialisation failed");
    }
    BatchDesc* d_one = reinterpret_cast<BatchDesc*>(d_blk);
    uint32_t* d_pre = reinterpret_cast<uint32_t*>(d_blk + prefix_offset(1));
    uint32_t* d_cnt = reinterpret_cast<uint32_t*>(d_blk + counter_offset(1));
    ttx_status result = TTX_OK;
    std::vector<ttx_config> cands(4096);
    const std::vector<ttx_config> old_cfg = b->cfg;
    const std::vector<int> old_forced = b->forced;
    std::vector<std::string> added;   // per-shape table keys this call adds
    bool changed = false;             // a kernel problem's config differs from the one it started with
    for (size_t i = 0; i < b->prob.size() && result == TTX_OK; ++i) {
        const Problem& p = b->prob[i];
        if (p.family == TTX_FAMILY_EMPTY) continue;
        const ttx_problem& q = b->src[i];
        const bool beta0 = beta_is_zero(p.dtype, beta_of(q));
        if (runs_per_call(p)) {   // the per-call tuner and tune table
            ttx_config best;
            result = tune_problem(p, beta0, max_candidates, reps, &best, nullptr);
            if (result == TTX_OK) {
                b->cfg[i] = best;
                b->forced[i] = 1;
            }
            continue;
        }
        const void* Bin = q.B_in ? q.B_in : q.B;
        const int vec = vector_ok(p, q.A, beta0 ? nullptr : Bin, q.B);
        const std::string key = batch_key(p, beta0, vec);
        {
            std::lock_guard<std::mutex> lock(g_btab_mu);
            auto it = g_btab.find(key);
            if (it != g_btab.end()) {
                changed = changed || std::memcmp(&b->cfg[i], &it->second, sizeof(ttx_config)) != 0;
                b->cfg[i] = it->second;
                b->forced[i] = 1;
                continue;
            }
        }
        // candidate 0: the configuration the batch runs now (the heuristic
        // choice), then the ranked batched-menu candidates
        cands[0] = b->cfg[i];
        int nc = batch_candidates(p, max_candidates, cands.data() + 1, int(cands.size()) - 1);
        if (nc <= 0) continue;
        ++nc;
        // scratch pointers keep the real pointers' offsets modulo 16 bytes, so
        // that each candidate runs the same vector variant it will run for real
        const uintptr_t offa = reinterpret_cast<uintptr_t>(q.A) & 15;
        const uintptr_t offb = reinterpret_cast<uintptr_t>(q.B) & 15;
        int best_i = -1;
        double best_us = 0;
        std::vector<double> us(nc, 0.0);
        result = time_candidates(p, beta0, nc, reps,
            [&](int c, const void* A, void* B, hipStream_t s) -> hipError_t {
                BatchDesc one;
                const void* a = static_cast<const char*>(A) + offa;
                void* bb = static_cast<char*>(B) + offb;
                if (batch_describe(p, &cands[c], beta0, a, bb, bb, 1.0, beta0 ? 0.0 : 1.0, &one, nullptr) != TTX_OK)
                    return hipErrorInvalidValue;
                uint32_t pre[2];
                int grid = 0;
                const uint32_t chunks = batch_layout(&one, 1, pre, &grid);
                hipError_t e = hipMemcpyAsync(d_one, &one, sizeof(one), hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipMemcpyAsync(d_pre, pre, sizeof(pre), hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return e;
                return launch_batch(d_one, d_pre, 1, chunks, grid, d_cnt, s);
            },
            &best_i, &best_us, us.data());
        // another configuration only when it is clearly faster than the
        // current one (timing one problem alone ranks close candidates
        // differently from the full batch)
        if (result == TTX_OK && best_i > 0 && best_us < us[0] * (1.0 - kBatchTuneMargin)) {
            b->cfg[i] = cands[best_i];
            b->forced[i] = 1;
            changed = true;
            std::lock_guard<std::mutex> lock(g_btab_mu);
            g_btab[key] = cands[best_i];
            added.push_back(key);
        }
    }
    (void)hipFree(d_blk);
    if (result != TTX_OK) return result;
    // Timing one problem alone ranks close candidates differently from the
    // full batch, so the tuned set must also win in context; otherwise the
    // kernel problems go back to the configs they started with (per-call
    // problems keep their tuned configs: they run alone in any case).
    if (changed && b->nk > 0 && !tuned_set_wins(b, old_cfg, old_forced, std::max(reps, 5))) {
        for (size_t i = 0; i < b->prob.size(); ++i)
            if (!runs_per_call(b->prob[i])) {
                b->cfg[i] = old_cfg[i];
                b->forced[i] = old_forced[i];
            }
        std::lock_guard<std::mutex> lock(g_btab_mu);
        for (const std::string& k : added) g_btab.erase(k);
    }
    ttx_status st = describe_all(b);
    if (st != TTX_OK) return st;
    drop_graph(b);   // descriptors, chunk count or grid may have changed
    return upload(b, nullptr);
}

ttx_status ttx_batch_execute_direct(ttx_batch* b, hipStream_t stream) {
    if (!b) return fail(TTX_EINVAL, "NULL batch");
    hipError_t e = b->chunks ? launch_batch(work_desc(b), work_prefix(b), b->nk, b->chunks, b->grid,
                                            work_counter(b), stream)
                             : hipSuccess;
    if (e == hipSuccess) e = launch_per_call(b, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
}

ttx_status ttx_batch_execute(ttx_batch* b, hipStream_t stream) {
    if (!b) return fail(TTX_EINVAL, "NULL batch");
    if (b->chunks == 0 && b->per_call.empty()) return TTX_OK;
    if (!b->captured) {
        drop_graph(b);
        if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(TTX_EHIP, "capture stream creation failed");
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(TTX_EHIP, "stream capture failed to start");
        hipError_t e = b->chunks ? launch_batch(work_desc(b), work_prefix(b), b->nk, b->chunks, b->grid,
                                                work_counter(b), b->cap_stream)
                                 : hipSuccess;
        if (e == hipSuccess) e = launch_per_call(b, b->cap_stream);
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

ttx_status ttx_batch_run_static(int count, const ttx_problem* problems, hipStream_t stream) {
    if (count < 0 || (count > 0 && !problems)) return fail(TTX_EINVAL, "bad batch arguments");
    if (count > TTX_STATIC_BATCH_MAX)
        return fail(TTX_EINVAL, "at most " + std::to_string(TTX_STATIC_BATCH_MAX) +
                                    " problems per allocation-free run, got " + std::to_string(count));
    ttx_batch b;   // host bookkeeping only: it owns no device memory and no graph
    ttx_status st = prepare(&b, count, problems);
    if (st != TTX_OK) return st;
    hipError_t e = hipSuccess;
    if (b.chunks) {
        unsigned char* base = nullptr;
        st = scratch_address(&base);
        if (st != TTX_OK) return st;
        // one host block: descriptors, chunk prefix and a zeroed claim
        // counter, copied in one transfer ordered on the stream (a copy from
        // pageable memory has read the block when the call returns)
        std::vector<unsigned char> host(work_bytes(b.nk), 0);
        std::memcpy(host.data(), b.desc.data(), desc_bytes(b.nk));
        std::memcpy(host.data() + prefix_offset(b.nk), b.chunk_prefix.data(), sizeof(uint32_t) * (b.nk + 1));
        e = hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = launch_batch(reinterpret_cast<const BatchDesc*>(base),
                             reinterpret_cast<const uint32_t*>(base + prefix_offset(b.nk)), b.nk, b.chunks, b.grid,
                             reinterpret_cast<uint32_t*>(base + counter_offset(b.nk)), stream);
    }
    if (e == hipSuccess) e = launch_per_call(&b, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, std::string("static batch launch: ") + hipGetErrorString(e));
}

ttx_status ttx_batch_get_info(const ttx_batch* b, ttx_batch_info* info) {
    if (!b || !info) return fail(TTX_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->count = int(b->prob.size());
    info->total_tiles = int64_t(b->total);
    info->chunks = b->chunks;
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
    info->per_call = int(b->per_call.size());
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
        const bool beta0 = beta_is_zero(p.dtype, beta_of(problems[i]));
        const void* Bin = problems[i].B_in ? problems[i].B_in : problems[i].B;
        st = check_pointers(p, problems[i].A, Bin, problems[i].B, beta0);
        if (st != TTX_OK) return st;
        if (runs_per_call(p)) {
            if (!table_lookup(p, beta0, &configs[i])) configs[i] = default_config(p);
            tiles[i] = 0;
            continue;
        }
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
    if (b->d_work) (void)hipFree(b->d_work);
    delete b;
    return TTX_OK;
}

}  // extern "C"
