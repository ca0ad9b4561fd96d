// Dense-tile kernel instantiations (one capacity per element type).
#include <mutex>

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, bool B0, int CAP>
static hipError_t launch_dense(const void* args, uint32_t grid, hipStream_t stream) {
    const TileArgs<T>& a = *static_cast<const TileArgs<T>*>(args);
    hipLaunchKernelGGL((k_dense<T, B0, CAP>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

// Workgroups of a full wave of the dense kernel on the current device: the
// kernel loops over tiles (pipelined), so that each workgroup computes its
// per-slot offsets once and streams many tiles.
template <typename T, bool B0, int CAP>
static uint32_t resident(int dev) {
    static std::mutex mu;
    static uint32_t cache[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) dev = 0;
    if (!cache[dev]) {
        int nb = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dense<T, B0, CAP>, kThreads, 0) != hipSuccess ||
            nb <= 0)
            nb = 4;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = uint32_t(nb) * uint32_t(cus);
    }
    return cache[dev];
}

uint32_t dense_grid(int dtype, bool beta0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    switch (dtype) {
        case TTX_F32:
            return beta0 ? resident<float, true, TTX_DENSE_CAP_F32>(dev) : resident<float, false, TTX_DENSE_CAP_F32>(dev);
        case TTX_F64:
            return beta0 ? resident<double, true, TTX_DENSE_CAP_F64>(dev) : resident<double, false, TTX_DENSE_CAP_F64>(dev);
        case TTX_C32:
            return beta0 ? resident<cf32, true, TTX_DENSE_CAP_C32>(dev) : resident<cf32, false, TTX_DENSE_CAP_C32>(dev);
        default:
            return beta0 ? resident<cf64, true, TTX_DENSE_CAP_C64>(dev) : resident<cf64, false, TTX_DENSE_CAP_C64>(dev);
    }
}

TileLaunchFn dense_launcher(int dtype, bool beta0) {
    switch (dtype) {
        case TTX_F32:
            return beta0 ? launch_dense<float, true, TTX_DENSE_CAP_F32> : launch_dense<float, false, TTX_DENSE_CAP_F32>;
        case TTX_F64:
            return beta0 ? launch_dense<double, true, TTX_DENSE_CAP_F64> : launch_dense<double, false, TTX_DENSE_CAP_F64>;
        case TTX_C32:
            return beta0 ? launch_dense<cf32, true, TTX_DENSE_CAP_C32> : launch_dense<cf32, false, TTX_DENSE_CAP_C32>;
        default:
            return beta0 ? launch_dense<cf64, true, TTX_DENSE_CAP_C64> : launch_dense<cf64, false, TTX_DENSE_CAP_C64>;
    }
}

}  // namespace ttx
