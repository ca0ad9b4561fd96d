// Dense-tile kernel instantiations (one capacity per dtype).
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

TileLaunchFn dense_launcher(int dtype, bool beta0) {
    if (dtype == TTX_F32)
        return beta0 ? launch_dense<float, true, TTX_DENSE_CAP_F32> : launch_dense<float, false, TTX_DENSE_CAP_F32>;
    return beta0 ? launch_dense<double, true, TTX_DENSE_CAP_F64> : launch_dense<double, false, TTX_DENSE_CAP_F64>;
}

}  // namespace ttx
