// Preserved-family kernel instantiations (one per tile shape of the menu).
#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, bool B0, int TA, int TR, int VEC>
static hipError_t launch(const void* args, uint32_t grid, hipStream_t stream) {
    constexpr int V = (VEC == 3 && kVec<T> > 1 && TA % kVec<T> == 0) ? kVec<T> : 1;
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
#define TTX_C32_B(ta, tr) TTX_ROW(cf32, false, ta, tr)
#define TTX_C32_Z(ta, tr) TTX_ROW(cf32, true, ta, tr)
#define TTX_C64_B(ta, tr) TTX_ROW(cf64, false, ta, tr)
#define TTX_C64_Z(ta, tr) TTX_ROW(cf64, true, ta, tr)
static const LauncherRow kF32B[] = {TTX_PRESERVED_MENU_F32(TTX_F32_B)};
static const LauncherRow kF32Z[] = {TTX_PRESERVED_MENU_F32(TTX_F32_Z)};
static const LauncherRow kF64B[] = {TTX_PRESERVED_MENU_F64(TTX_F64_B)};
static const LauncherRow kF64Z[] = {TTX_PRESERVED_MENU_F64(TTX_F64_Z)};
static const LauncherRow kC32B[] = {TTX_PRESERVED_MENU_F64(TTX_C32_B)};
static const LauncherRow kC32Z[] = {TTX_PRESERVED_MENU_F64(TTX_C32_Z)};
static const LauncherRow kC64B[] = {TTX_PRESERVED_MENU_C64(TTX_C64_B)};
static const LauncherRow kC64Z[] = {TTX_PRESERVED_MENU_C64(TTX_C64_Z)};

#define TTX_PICK(B, Z) return *out = beta0 ? Z : B, int(sizeof(B) / sizeof(B[0]))
int preserved_rows(int dtype, bool beta0, const LauncherRow** out) {
    switch (dtype) {
        case TTX_F32: TTX_PICK(kF32B, kF32Z);
        case TTX_F64: TTX_PICK(kF64B, kF64Z);
        case TTX_C32: TTX_PICK(kC32B, kC32Z);
        default: TTX_PICK(kC64B, kC64Z);
    }
}

}  // namespace ttx
