// Preserved-family kernel instantiations (one per tile shape of the menu).
#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, bool B0, int TA, int TR, int VEC>
static hipError_t launch(const void* args, uint32_t grid, hipStream_t stream) {
    constexpr int V = (VEC == 3 && TA % kVec<T> == 0) ? kVec<T> : 1;
    const TileArgs<T>& a = *static_cast<const TileArgs<T>*>(args);
    hipLaunchKernelGGL((k_preserved<T, B0, TA, TR, V>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

#define TTX_ROW(T, B0, ta, tr) \
    {ta, tr, {launch<T, B0, ta, tr, 0>, launch<T, B0, ta, tr, 0>, launch<T, B0, ta, tr, 0>, launch<T, B0, ta, tr, 3>}},
#define TTX_F32_B(ta, tr) TTX_ROW(float, false, ta, tr)
#define TTX_F32_Z(ta, tr) TTX_ROW(float, true, ta, tr)
#define TTX_F64_B(ta, tr) TTX_ROW(double, false, ta, tr)
#define TTX_F64_Z(ta, tr) TTX_ROW(double, true, ta, tr)
static const LauncherRow kF32B[] = {TTX_PRESERVED_MENU_F32(TTX_F32_B)};
static const LauncherRow kF32Z[] = {TTX_PRESERVED_MENU_F32(TTX_F32_Z)};
static const LauncherRow kF64B[] = {TTX_PRESERVED_MENU_F64(TTX_F64_B)};
static const LauncherRow kF64Z[] = {TTX_PRESERVED_MENU_F64(TTX_F64_Z)};

int preserved_rows(int dtype, bool beta0, const LauncherRow** out) {
    if (dtype == TTX_F32) {
        *out = beta0 ? kF32Z : kF32B;
        return int(sizeof(kF32B) / sizeof(kF32B[0]));
    }
    *out = beta0 ? kF64Z : kF64B;
    return int(sizeof(kF64B) / sizeof(kF64B[0]));
}

}  // namespace ttx
