// Host-side launch of one planned transposition, the flat kernel, and the
// bandwidth-ceiling kernels used for measurement.
#include <cstdio>
#include <mutex>
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
    if constexpr (std::is_same<T, S>::value) {
        if (beta0)
            hipLaunchKernelGGL((k_flat<T, true>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream, a);
        else
            hipLaunchKernelGGL((k_flat<T, false>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream, a);
    } else {
        if (beta0)
            hipLaunchKernelGGL((k_flat_x<T, S, true>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream, a);
        else
            hipLaunchKernelGGL((k_flat_x<T, S, false>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream, a);
    }
    return hipGetLastError();
}

template <typename T, typename S>
static hipError_t launch_tiled(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                               const void* Bsrc, void* Bdst, const Scalar& alpha, const Scalar& beta,
                               hipStream_t stream) {
    TileArgs<T, S> a;
    build_grid(p, c, &a);
    a.A = static_cast<const S*>(A);
    a.Bsrc = static_cast<const T*>(Bsrc);
    a.Bdst = static_cast<T*>(Bdst);
    a.alpha = scalar_as<T>(alpha);
    a.beta = scalar_as<T>(beta);
    a.flags = kernel_flags(p, c, A, beta0 ? nullptr : Bsrc, Bdst);
    if (config_is_dense(c)) {
        const uint32_t full = dense_grid(p.code, beta0);
        const uint32_t grid = a.g.ntiles < full ? a.g.ntiles : full;
        return dense_launcher(p.code, beta0)(&a, grid, stream);
    }
    if (config_is_staged(c)) {
        const StagedRow* rows;
        const int nr = staged_rows(p.code, beta0, &rows);
        const int lanes = staged_lanes(p.dim[0].size);
        for (int i = 0; i < nr; ++i) {
            if (rows[i].n0_max == lanes && rows[i].tx == c.tile_a && rows[i].ty == c.tile_b) {
                uint32_t grid = a.g.ntiles < kMaxGrid ? a.g.ntiles : kMaxGrid;
                return rows[i].fn(&a, grid, stream);
            }
        }
        return hipErrorInvalidValue;
    }
    const LauncherRow* table;
    int n;
    if (p.family == TTX_FAMILY_MOVED) {
        n = moved_rows(p.code, beta0, &table);
    } else {
        n = preserved_rows(p.code, beta0, &table);
    }
    const int variant = a.flags & (KF_VEC_A | KF_VEC_B);
    for (int i = 0; i < n; ++i) {
        if (table[i].ta == c.tile_a && table[i].tb == c.tile_b) {
            uint32_t grid = a.g.ntiles < kMaxGrid ? a.g.ntiles : kMaxGrid;
            return table[i].fn[variant](&a, grid, stream);
        }
    }
    return hipErrorInvalidValue;
}

static bool aligned_to(const void* ptr, uintptr_t n) { return reinterpret_cast<uintptr_t>(ptr) % n == 0; }

hipError_t launch_tiles(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                        const void* Bsrc, void* Bdst, const Scalar& alpha, const Scalar& beta,
                        hipStream_t stream) {
    if (p.family == TTX_FAMILY_EMPTY) return hipSuccess;
    if (config_is_wide(c)) {
        // dense tiles over whole units of the kept rows: one element per unit
        Problem w;
        if (!widen(p, &w)) return hipErrorInvalidValue;
        const uintptr_t ub = uintptr_t(elem_bytes(w.dtype));
        if (!aligned_to(A, ub) || !aligned_to(Bdst, ub) || (Bsrc && !aligned_to(Bsrc, ub)))
            return launch_tiles(p, default_config_elementwise(p), beta0, A, Bsrc, Bdst, alpha, beta, stream);
        ttx_config cw = c;
        cw.flags &= ~TTX_CFG_WIDE;
        switch (w.code) {
            case kWideF32x4: return launch_tiled<f32x4, f32x4>(w, cw, beta0, A, Bsrc, Bdst, alpha, beta, stream);
            case kWideF64x2: return launch_tiled<f64x2, f64x2>(w, cw, beta0, A, Bsrc, Bdst, alpha, beta, stream);
            default: return launch_tiled<f32x2, f32x2>(w, cw, beta0, A, Bsrc, Bdst, alpha, beta, stream);
        }
    }
    return with_types(p.code, [&](auto t, auto s) {
        using T = decltype(t);
        using S = decltype(s);
        if (p.family == TTX_FAMILY_FLAT) return launch_flat<T, S>(p, c, beta0, A, Bsrc, Bdst, alpha, beta, stream);
        return launch_tiled<T, S>(p, c, beta0, A, Bsrc, Bdst, alpha, beta, stream);
    });
}

std::string kernel_name(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                        const void* Bsrc, const void* Bdst) {
    if (p.family == TTX_FAMILY_EMPTY) return "";
    if (config_is_wide(c)) {
        Problem w;
        const uintptr_t ub = widen(p, &w) ? uintptr_t(elem_bytes(w.dtype)) : 0;
        if (!ub || !aligned_to(A, ub) || !aligned_to(Bdst, ub) || (Bsrc && !aligned_to(Bsrc, ub)))
            return kernel_name(p, default_config_elementwise(p), beta0, A, Bsrc, Bdst);
        static const char* const kWideName[] = {"ttx::f32x4", "ttx::f64x2", "ttx::f32x2"};
        char buf[96];
        std::snprintf(buf, sizeof(buf), "k_dense<%s, %s, %d>", kWideName[w.dtype - kWideF32x4],
                      beta0 ? "true" : "false", dense_cap(w.dtype));
        return buf;
    }
    static const char* const kTypeName[] = {"float", "double", "ttx::cf32", "ttx::cf64"};
    // the same-type kernels are k_<kind><T, ...>; mixed ones k_<kind>_x<T, S, ...>
    char ts[64];
    const bool mixed = p.dtype_a != p.dtype;
    if (mixed)
        std::snprintf(ts, sizeof(ts), "_x<%s, %s", kTypeName[p.dtype], kTypeName[p.dtype_a]);
    else
        std::snprintf(ts, sizeof(ts), "<%s", kTypeName[p.dtype]);
    const char* z = beta0 ? "true" : "false";
    const int VA = 16 / elem_bytes(p.dtype_a), VB = 16 / elem_bytes(p.dtype);
    const int V = VA < VB ? VA : VB;
    const int f = kernel_flags(p, c, A, beta0 ? nullptr : Bsrc, Bdst);
    char buf[160];
    if (p.family == TTX_FAMILY_FLAT) {
        std::snprintf(buf, sizeof(buf), "k_flat%s, %s>", ts, z);
    } else if (config_is_dense(c)) {
        std::snprintf(buf, sizeof(buf), "k_dense%s, %s, %d>", ts, z, dense_cap(p.dtype));
    } else if (p.family == TTX_FAMILY_MOVED) {
        const int va = (f & KF_VEC_A) && VA > 1 && c.tile_a % VA == 0 ? VA : 1;
        const int vb = (f & KF_VEC_B) && VB > 1 && c.tile_b % VB == 0 ? VB : 1;
        std::snprintf(buf, sizeof(buf), "k_moved%s, %s, %d, %d, %d, %d>", ts, z, c.tile_a, c.tile_b, va, vb);
    } else if (config_is_staged(c)) {
        std::snprintf(buf, sizeof(buf), "k_staged%s, %s, %d, %d, %d>", ts, z, staged_lanes(p.dim[0].size),
                      c.tile_a, c.tile_b);
    } else {
        const int v = (f & KF_VEC_A) && V > 1 && c.tile_a % V == 0 ? V : 1;
        std::snprintf(buf, sizeof(buf), "k_preserved%s, %s, %d, %d, %d>", ts, z, c.tile_a, c.tile_b, v);
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
// peak of Sec. 3).  Grid-stride loops with 4 vectors in flight per thread.
__global__ __launch_bounds__(kThreads) void k_copy16(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, int64_t nvec) {
    constexpr int U = 4;
    const int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t G = int64_t(gridDim.x) * kThreads;
    for (int64_t base = gid; base < nvec; base += G * U) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * G < nvec) v[u] = src[base + u * G];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * G < nvec) dst[base + u * G] = v[u];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpby(const T* __restrict__ x, T* __restrict__ y,
                                                    int64_t n, T alpha, T beta) {
    constexpr int V = kVec<T>;
    constexpr int U = 4;
    const int64_t nv = n / V;
    const int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t G = int64_t(gridDim.x) * kThreads;
    for (int64_t base = gid; base < nv; base += G * U) {
        vec_t<T, V> a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * G < nv) {
                a[u] = ld<T, V>(x + (base + u * G) * V);
                b[u] = ld<T, V>(y + (base + u * G) * V);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * G < nv)
                st<T, V>(y + (base + u * G) * V, epilogue<T, V, false>(a[u], b[u], alpha, beta), false);
    }
    const int64_t i = nv * V + gid;
    if (i < n) y[i] = epilogue<T, 1, false>(x[i], y[i], alpha, beta);
}

hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t stream) {
    const int64_t nvec = bytes / 16;
    int64_t blocks = (nvec + kThreads * 4 - 1) / (kThreads * 4);
    const int64_t cap = int64_t(device_cus()) * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy16, dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), nvec);
    return hipGetLastError();
}

hipError_t launch_axpby(int dtype, int64_t n, double alpha, const void* x, double beta, void* y,
                        hipStream_t stream) {
    const int V = dtype == TTX_F32 ? 4 : 2;
    int64_t blocks = (n / V + kThreads * 4 - 1) / (kThreads * 4);
    const int64_t cap = int64_t(device_cus()) * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (dtype == TTX_F32)
        hipLaunchKernelGGL((k_axpby<float>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                           static_cast<const float*>(x), static_cast<float*>(y), n, float(alpha), float(beta));
    else
        hipLaunchKernelGGL((k_axpby<double>), dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                           static_cast<const double*>(x), static_cast<double*>(y), n, alpha, beta);
    return hipGetLastError();
}

}  // namespace ttx
