// Host-side launch of one planned transposition, the flat kernel, and the
// bandwidth-ceiling kernels used for measurement.
#include <cstdio>
#include <mutex>
#include <new>
#include <type_traits>

#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

static constexpr uint32_t kMaxGrid = 1u << 20;

static int device_cus() {
    static std::mutex mu;
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

// Calls f with values of B's and A's element types for a data-type code.
template <typename F>
static hipError_t with_types(int code, F&& f) {
    switch (code) {
        case TTX_F32: return f(float{}, float{});
        case TTX_F64: return f(double{}, double{});
        case TTX_C32: return f(cf32{}, cf32{});
        case TTX_C64: return f(cf64{}, cf64{});
        case TTX_F32_F64: return f(double{}, float{});
        case TTX_F64_F32: return f(float{}, double{});
        case TTX_C32_C64: return f(cf64{}, cf32{});
        case TTX_C64_C32: return f(cf32{}, cf64{});
        default: return hipErrorInvalidValue;
    }
}

template <typename T, typename S>
static hipError_t launch_flat(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                              const void* Bsrc, void* Bdst, const Scalar& alpha, const Scalar& beta,
                              hipStream_t stream) {
    FlatArgs<T, S> a;
    a.A = static_cast<const S*>(A);
    a.Bsrc = static_cast<const T*>(Bsrc);
    a.Bdst = static_cast<T*>(Bdst);
    a.alpha = scalar_as<T>(alpha);
    a.beta = scalar_as<T>(beta);
    a.n = p.dim[0].size;
    a.sa = p.dim[0].sa;
    a.sb = p.dim[0].sb;
    a.flags = kernel_flags(p, c, A, beta0 ? nullptr : Bsrc, Bdst);
    constexpr int V = kVec<T> < kVec<S> ? kVec<T> : kVec<S>;
    const int64_t per_block = int64_t(kThreads) * ((a.flags & KF_VEC_A) ? V * 4 : 1);
    int64_t blocks = (a.n + per_block - 1) / per_block;
    const int64_t cap = int64_t(device_cus()) * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    const dim3 g(static_cast<uint32_t>(blocks)), b(kThreads);
    const bool nt = (a.flags & KF_NT_STORE) != 0;
    if constexpr (std::is_same<T, S>::value) {
        if (beta0 && nt) hipLaunchKernelGGL((k_flat<T, true, true>), g, b, 0, stream, a);
        else if (beta0) hipLaunchKernelGGL((k_flat<T, true, false>), g, b, 0, stream, a);
        else if (nt) hipLaunchKernelGGL((k_flat<T, false, true>), g, b, 0, stream, a);
        else hipLaunchKernelGGL((k_flat<T, false, false>), g, b, 0, stream, a);
    } else {
        if (beta0 && nt) hipLaunchKernelGGL((k_flat_x<T, S, true, true>), g, b, 0, stream, a);
        else if (beta0) hipLaunchKernelGGL((k_flat_x<T, S, true, false>), g, b, 0, stream, a);
        else if (nt) hipLaunchKernelGGL((k_flat_x<T, S, false, true>), g, b, 0, stream, a);
        else hipLaunchKernelGGL((k_flat_x<T, S, false, false>), g, b, 0, stream, a);
    }
    return hipGetLastError();
}

// Calls f with values of B's and A's element types for any element code,
// the internal wide units included.
template <typename F>
static bool with_all_types(int code, F&& f) {
    switch (code) {
        case kWideF32x4: f(f32x4{}, f32x4{}); return true;
        case kWideF64x2: f(f64x2{}, f64x2{}); return true;
        case kWideF32x2: f(f32x2{}, f32x2{}); return true;
        default: return with_types(code, [&](auto t, auto s) { f(t, s); return hipSuccess; }) == hipSuccess;
    }
}

template <typename T, typename S>
static void fill_args(const Problem& p, const ttx_config& c, bool beta0, const void* A, const void* Bsrc,
                      void* Bdst, const Scalar& alpha, const Scalar& beta, TiledLaunch* L) {
    static_assert(sizeof(TileArgs<T, S>) <= sizeof(L->args), "argument block too small");
    TileArgs<T, S>* a = new (L->args) TileArgs<T, S>();
    build_grid(p, c, a);
    a->A = static_cast<const S*>(A);
    a->Bsrc = static_cast<const T*>(Bsrc);
    a->Bdst = static_cast<T*>(Bdst);
    a->alpha = scalar_as<T>(alpha);
    a->beta = scalar_as<T>(beta);
    a->flags = kernel_flags(p, c, A, beta0 ? nullptr : Bsrc, Bdst);
    L->args_bytes = sizeof(TileArgs<T, S>);
    L->flags = a->flags;
    L->ntiles = a->g.ntiles;
}

static bool aligned_to(const void* ptr, uintptr_t n) { return reinterpret_cast<uintptr_t>(ptr) % n == 0; }

bool prepare_tiled(const Problem& p, const ttx_config& c, bool beta0, const void* A, const void* Bsrc,
                   void* Bdst, const Scalar& alpha, const Scalar& beta, TiledLaunch* L) {
    if (p.family != TTX_FAMILY_MOVED && p.family != TTX_FAMILY_PRESERVED) return false;
    if (beta0) Bsrc = nullptr;
    if (config_is_wide(c)) {
        // dense tiles over whole units of the kept rows: one element per unit
        Problem w;
        if (!widen(p, &w)) return false;
        const uintptr_t ub = uintptr_t(elem_bytes(w.dtype));
        if (!aligned_to(A, ub) || !aligned_to(Bdst, ub) || (Bsrc && !aligned_to(Bsrc, ub)))
            return prepare_tiled(p, default_config_elementwise(p), beta0, A, Bsrc, Bdst, alpha, beta, L);
        L->p = w;
        L->c = c;
        L->c.flags &= ~TTX_CFG_WIDE;
    } else {
        L->p = p;
        L->c = c;
    }
    L->beta0 = beta0;
    const Problem& q = L->p;
    const ttx_config& k = L->c;
    if (!with_all_types(q.code, [&](auto t, auto s) {
            fill_args<decltype(t), decltype(s)>(q, k, beta0, A, Bsrc, Bdst, alpha, beta, L);
        }))
        return false;
    const int VA = 16 / elem_bytes(q.dtype_a), VB = 16 / elem_bytes(q.dtype);
    L->va = L->vb = 1;
    L->n0 = 0;
    L->cap = 0;
    uint32_t limit = kMaxGrid;
    if (config_is_dense(k)) {
        L->kind = kTileDense;
        L->cap = dense_cap(q.dtype);
        limit = dense_grid(q.code, beta0);
    } else if (config_is_staged(k)) {
        L->kind = kTileStaged;
        L->n0 = staged_lanes(q.dim[0].size);
    } else if (q.family == TTX_FAMILY_MOVED) {
        L->kind = kTileMoved;
        if ((L->flags & KF_VEC_A) && VA > 1 && k.tile_a % VA == 0) L->va = VA;
        if ((L->flags & KF_VEC_B) && VB > 1 && k.tile_b % VB == 0) L->vb = VB;
    } else {
        L->kind = kTilePreserved;
        const int V = VA < VB ? VA : VB;
        if ((L->flags & KF_VEC_A) && (L->flags & KF_VEC_B) && V > 1 && k.tile_a % V == 0) L->va = L->vb = V;
    }
    L->grid = L->ntiles < limit ? L->ntiles : limit;
    return true;
}

// The generic (pre-instantiated) kernel for a prepared launch.
static hipError_t launch_prepared(const TiledLaunch& L, hipStream_t stream) {
    const ttx_config& c = L.c;
    const bool nt = (L.flags & KF_NT_STORE) != 0;
    if (L.kind == kTileDense) return dense_launcher(L.p.code, L.beta0, nt)(L.args, L.grid, stream);
    if (L.kind == kTileStaged) {
        const StagedRow* rows;
        const int nr = staged_rows(L.p.code, L.beta0, &rows);
        for (int i = 0; i < nr; ++i)
            if (rows[i].n0_max == L.n0 && rows[i].tx == c.tile_a && rows[i].ty == c.tile_b)
                return rows[i].fn[nt ? 1 : 0](L.args, L.grid, stream);
        return hipErrorInvalidValue;
    }
    const LauncherRow* table;
    const int n = L.kind == kTileMoved ? moved_rows(L.p.code, L.beta0, &table) : preserved_rows(L.p.code, L.beta0, &table);
    const int variant = (L.flags & (KF_VEC_A | KF_VEC_B)) | (nt ? 4 : 0);
    for (int i = 0; i < n; ++i)
        if (table[i].ta == c.tile_a && table[i].tb == c.tile_b) return table[i].fn[variant](L.args, L.grid, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_tiles(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                        const void* Bsrc, void* Bdst, const Scalar& alpha, const Scalar& beta,
                        hipStream_t stream) {
    if (p.family == TTX_FAMILY_EMPTY) return hipSuccess;
    if (p.family == TTX_FAMILY_FLAT) {
        return with_types(p.code, [&](auto t, auto s) {
            return launch_flat<decltype(t), decltype(s)>(p, c, beta0, A, Bsrc, Bdst, alpha, beta, stream);
        });
    }
    TiledLaunch L;
    if (!prepare_tiled(p, c, beta0, A, Bsrc, Bdst, alpha, beta, &L)) return hipErrorInvalidValue;
    if (config_needs_jit(L.p, L.c)) {
        // no pre-compiled kernel for this workgroup size or LDS padding: the
        // size-specialised one (compiled on first use, then cached)
        const JitKernel* k = nullptr;
        if (jit_kernel(L, &k) != TTX_OK) return hipErrorInvalidImage;
        return jit_launch(*k, L, stream);
    }
    return launch_prepared(L, stream);
}

const char* element_type_name(int dtype) {
    switch (dtype) {
        case TTX_F32: return "float";
        case TTX_F64: return "double";
        case TTX_C32: return "ttx::cf32";
        case TTX_C64: return "ttx::cf64";
        case kWideF32x4: return "ttx::f32x4";
        case kWideF64x2: return "ttx::f64x2";
        case kWideF32x2: return "ttx::f32x2";
        default: return "?";
    }
}

std::string kernel_name(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                        const void* Bsrc, const void* Bdst) {
    if (p.family == TTX_FAMILY_EMPTY) return "";
    // the same-type kernels are k_<kind><T, ...>; mixed ones k_<kind>_x<T, S, ...>
    auto types = [](const Problem& q) {
        std::string ts = q.dtype_a != q.dtype ? "_x<" : "<";
        ts += element_type_name(q.dtype);
        if (q.dtype_a != q.dtype) ts += std::string(", ") + element_type_name(q.dtype_a);
        return ts;
    };
    const char* z = beta0 ? "true" : "false";
    char buf[160];
    if (p.family == TTX_FAMILY_FLAT) {
        const int f = kernel_flags(p, c, A, beta0 ? nullptr : Bsrc, Bdst);
        std::snprintf(buf, sizeof(buf), "k_flat%s, %s, %s>", types(p).c_str(), z,
                      (f & KF_NT_STORE) ? "true" : "false");
        return buf;
    }
    TiledLaunch L;
    if (!prepare_tiled(p, c, beta0, A, Bsrc, const_cast<void*>(Bdst), Scalar(1.0), Scalar(0.0), &L)) return "";
    if (config_needs_jit(L.p, L.c)) return jit_entry_name(L);
    const std::string ts = types(L.p);
    const char* nt = (L.flags & KF_NT_STORE) ? "true" : "false";
    switch (L.kind) {
        case kTileDense:
            std::snprintf(buf, sizeof(buf), "k_dense%s, %s, %d, %s>", ts.c_str(), z, L.cap, nt);
            break;
        case kTileMoved:
            std::snprintf(buf, sizeof(buf), "k_moved%s, %s, %d, %d, %d, %d, %s>", ts.c_str(), z, L.c.tile_a,
                          L.c.tile_b, L.va, L.vb, nt);
            break;
        case kTileStaged:
            std::snprintf(buf, sizeof(buf), "k_staged%s, %s, %d, %d, %d, %s>", ts.c_str(), z, L.n0, L.c.tile_a,
                          L.c.tile_b, nt);
            break;
        default:
            std::snprintf(buf, sizeof(buf), "k_preserved%s, %s, %d, %d, %d, %s>", ts.c_str(), z, L.c.tile_a,
                          L.c.tile_b, L.va, nt);
    }
    return buf;
}

// Zero fill of a strided region (the padding of a ragged packed panel), in
// 4-byte words: word w of row r is at dst + r*pitch + 4*w.
__global__ __launch_bounds__(kThreads) void k_fill_zero(uint32_t* __restrict__ dst, int64_t words,
                                                        int64_t height, int64_t pitch_words) {
    const int64_t total = words * height;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < total; i += int64_t(gridDim.x) * kThreads) {
        const int64_t r = i / words, w = i - r * words;
        dst[r * pitch_words + w] = 0u;
    }
}

hipError_t launch_fill_zero(void* dst, int64_t width, int64_t height, int64_t pitch, hipStream_t stream) {
    const int64_t words = width / 4, total = words * height;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + kThreads - 1) / kThreads;
    const int64_t cap = int64_t(device_cus()) * 8;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_fill_zero, dim3(uint32_t(blocks)), dim3(kThreads), 0, stream, static_cast<uint32_t*>(dst),
                       words, height, pitch / 4);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Ceiling kernels: a 16-byte-vector copy and an unfused axpby (the SAXPY
// peak of Sec. 3).  One pass: thread i moves vector i, and the grid covers
// the array, so the workgroups running at any moment sweep one contiguous
// stretch of memory.  (Grid-stride loops with several vectors in flight per
// thread touch addresses a whole grid apart and reach 4.2-4.8 TB/s on an
// MI355X; this form reaches about 6.1 TB/s, above hipMemcpy's 5.1.)
__global__ __launch_bounds__(kThreads) void k_copy16(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, int64_t nvec) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < nvec) dst[i] = src[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpby(const T* __restrict__ x, T* __restrict__ y,
                                                    int64_t n, T alpha, T beta) {
    constexpr int V = kVec<T>;
    const int64_t nv = n / V;
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < nv) {
        const vec_t<T, V> a = ld<T, V>(x + i * V);
        const vec_t<T, V> b = ld<T, V>(y + i * V);
        st<T, V, false>(y + i * V, epilogue<T, V, false>(a, b, alpha, beta));
    }
    const int64_t t = nv * V + i;   // the last n % V elements, one per thread
    if (i < V && t < n) y[t] = epilogue<T, 1, false>(x[t], y[t], alpha, beta);
}

hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t stream) {
    const int64_t nvec = bytes / 16;
    const int64_t blocks = nvec > 0 ? (nvec + kThreads - 1) / kThreads : 1;
    if (blocks > int64_t(0x7fffffff)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), nvec);
    return hipGetLastError();
}

hipError_t launch_axpby(int dtype, int64_t n, double alpha, const void* x, double beta, void* y,
                        hipStream_t stream) {
    const int V = dtype == TTX_F32 ? 4 : 2;
    const int64_t nv = n / V;
    const int64_t blocks = nv > 0 ? (nv + kThreads - 1) / kThreads : 1;
    if (blocks > int64_t(0x7fffffff)) return hipErrorInvalidValue;
    if (dtype == TTX_F32)
        hipLaunchKernelGGL((k_axpby<float>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                           static_cast<const float*>(x), static_cast<float*>(y), n, float(alpha), float(beta));
    else
        hipLaunchKernelGGL((k_axpby<double>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                           static_cast<const double*>(x), static_cast<double*>(y), n, alpha, beta);
    return hipGetLastError();
}

}  // namespace ttx
