// Moved-family kernel instantiations: float, beta == 0.
#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <int TA, int TB, int VA, int VB>
static hipError_t launch(const void* args, uint32_t grid, hipStream_t stream) {
    constexpr int V = kVec<float>;
    constexpr int va = (VA > 1 && TA % V == 0) ? V : 1;
    constexpr int vb = (VB > 1 && TB % V == 0) ? V : 1;
    const TileArgs<float>& a = *static_cast<const TileArgs<float>*>(args);
    hipLaunchKernelGGL((k_moved<float, true, TA, TB, va, vb>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

#define TTX_ENTRY(ta, tb) {ta, tb, {launch<ta, tb, 1, 1>, launch<ta, tb, 2, 1>, launch<ta, tb, 1, 2>, launch<ta, tb, 2, 2>}},
static const LauncherRow kRows[] = {TTX_MOVED_MENU_F32(TTX_ENTRY)};
#undef TTX_ENTRY

int moved_rows_f32_beta0(const LauncherRow** out) {
    *out = kRows;
    return int(sizeof(kRows) / sizeof(kRows[0]));
}

}  // namespace ttx
