// Dense-tile kernel instantiations (the dense capacity of B's element type,
// for every data-type code, and for the whole-unit types of kept rows).
#include <mutex>
#include <type_traits>

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, typename S, bool B0, int CAP, bool NT>
static hipError_t launch_dense(const void* args, uint32_t grid, hipStream_t stream) {
    const TileArgs<T, S>& a = *static_cast<const TileArgs<T, S>*>(args);
    if constexpr (std::is_same<T, S>::value)
        hipLaunchKernelGGL((k_dense<T, B0, CAP, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_dense_x<T, S, B0, CAP, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

// (both store kinds of a dense kernel use the same resources)
template <typename T, typename S, bool B0, int CAP>
static hipError_t dense_occupancy(int* nb) {
    if constexpr (std::is_same<T, S>::value)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_dense<T, B0, CAP, false>, kThreads, 0);
    else
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_dense_x<T, S, B0, CAP, false>, kThreads, 0);
}

// Workgroups of a full wave of the dense kernel on the current device: the
// kernel loops over tiles (pipelined), so that each workgroup computes its
// per-slot offsets once and streams many tiles.
template <typename T, typename S, bool B0, int CAP>
static uint32_t resident(int dev) {
    static std::mutex mu;
    static uint32_t cache[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) dev = 0;
    if (!cache[dev]) {
        int nb = 0, cus = 0;
        if (dense_occupancy<T, S, B0, CAP>(&nb) != hipSuccess || nb <= 0)
            nb = 4;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = uint32_t(nb) * uint32_t(cus);
    }
    return cache[dev];
}

uint32_t dense_grid(int code, bool beta0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    switch (code) {
        case TTX_F32:
            return beta0 ? resident<float, float, true, TTX_DENSE_CAP_F32>(dev) : resident<float, float, false, TTX_DENSE_CAP_F32>(dev);
        case TTX_F64:
            return beta0 ? resident<double, double, true, TTX_DENSE_CAP_F64>(dev) : resident<double, double, false, TTX_DENSE_CAP_F64>(dev);
        case TTX_C32:
            return beta0 ? resident<cf32, cf32, true, TTX_DENSE_CAP_C32>(dev) : resident<cf32, cf32, false, TTX_DENSE_CAP_C32>(dev);
        case TTX_C64:
            return beta0 ? resident<cf64, cf64, true, TTX_DENSE_CAP_C64>(dev) : resident<cf64, cf64, false, TTX_DENSE_CAP_C64>(dev);
        case TTX_F32_F64:
            return beta0 ? resident<double, float, true, TTX_DENSE_CAP_F64>(dev) : resident<double, float, false, TTX_DENSE_CAP_F64>(dev);
        case TTX_F64_F32:
            return beta0 ? resident<float, double, true, TTX_DENSE_CAP_F32>(dev) : resident<float, double, false, TTX_DENSE_CAP_F32>(dev);
        case TTX_C32_C64:
            return beta0 ? resident<cf64, cf32, true, TTX_DENSE_CAP_C64>(dev) : resident<cf64, cf32, false, TTX_DENSE_CAP_C64>(dev);
        case TTX_C64_C32:
            return beta0 ? resident<cf32, cf64, true, TTX_DENSE_CAP_C32>(dev) : resident<cf32, cf64, false, TTX_DENSE_CAP_C32>(dev);
        case kWideF32x4:
            return beta0 ? resident<f32x4, f32x4, true, TTX_DENSE_CAP_W16>(dev)
                         : resident<f32x4, f32x4, false, TTX_DENSE_CAP_W16>(dev);
        case kWideF64x2:
            return beta0 ? resident<f64x2, f64x2, true, TTX_DENSE_CAP_W16>(dev)
                         : resident<f64x2, f64x2, false, TTX_DENSE_CAP_W16>(dev);
        case kWideF32x2:
            return beta0 ? resident<f32x2, f32x2, true, TTX_DENSE_CAP_W8>(dev)
                         : resident<f32x2, f32x2, false, TTX_DENSE_CAP_W8>(dev);
        default: return 0;
    }
}

template <typename T, typename S, int CAP>
static TileLaunchFn pick_dense(bool beta0, bool nt) {
    if (beta0) return nt ? launch_dense<T, S, true, CAP, true> : launch_dense<T, S, true, CAP, false>;
    return nt ? launch_dense<T, S, false, CAP, true> : launch_dense<T, S, false, CAP, false>;
}

TileLaunchFn dense_launcher(int code, bool beta0, bool nt) {
    switch (code) {
        case TTX_F32: return pick_dense<float, float, TTX_DENSE_CAP_F32>(beta0, nt);
        case TTX_F64: return pick_dense<double, double, TTX_DENSE_CAP_F64>(beta0, nt);
        case TTX_C32: return pick_dense<cf32, cf32, TTX_DENSE_CAP_C32>(beta0, nt);
        case TTX_C64: return pick_dense<cf64, cf64, TTX_DENSE_CAP_C64>(beta0, nt);
        case TTX_F32_F64: return pick_dense<double, float, TTX_DENSE_CAP_F64>(beta0, nt);
        case TTX_F64_F32: return pick_dense<float, double, TTX_DENSE_CAP_F32>(beta0, nt);
        case TTX_C32_C64: return pick_dense<cf64, cf32, TTX_DENSE_CAP_C64>(beta0, nt);
        case TTX_C64_C32: return pick_dense<cf32, cf64, TTX_DENSE_CAP_C32>(beta0, nt);
        case kWideF32x4: return pick_dense<f32x4, f32x4, TTX_DENSE_CAP_W16>(beta0, nt);
        case kWideF64x2: return pick_dense<f64x2, f64x2, TTX_DENSE_CAP_W16>(beta0, nt);
        case kWideF32x2: return pick_dense<f32x2, f32x2, TTX_DENSE_CAP_W8>(beta0, nt);
        default: return nullptr;
    }
}

}  // namespace ttx
