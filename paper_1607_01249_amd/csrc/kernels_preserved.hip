// Preserved-family kernel instantiations (one per tile shape of the menu of
// B's element type, for every data-type code).
#include <type_traits>

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

// V counts elements of both A and B: the smaller of their 16-byte widths.
template <typename T, typename S, bool B0, int TA, int TR, int VEC, bool NT>
static hipError_t launch(const void* args, uint32_t grid, hipStream_t stream) {
    constexpr int W = kVec<T> < kVec<S> ? kVec<T> : kVec<S>;
    constexpr int V = (VEC == 3 && W > 1 && TA % W == 0) ? W : 1;
    const TileArgs<T, S>& a = *static_cast<const TileArgs<T, S>*>(args);
    if constexpr (std::is_same<T, S>::value)
        hipLaunchKernelGGL((k_preserved<T, B0, TA, TR, V, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_preserved_x<T, S, B0, TA, TR, V, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

#define TTX_ROW(T, S, B0, ta, tr) \
    {ta, tr, {launch<T, S, B0, ta, tr, 0, false>, launch<T, S, B0, ta, tr, 0, false>,             \
              launch<T, S, B0, ta, tr, 0, false>, launch<T, S, B0, ta, tr, 3, false>,             \
              launch<T, S, B0, ta, tr, 0, true>, launch<T, S, B0, ta, tr, 0, true>,               \
              launch<T, S, B0, ta, tr, 0, true>, launch<T, S, B0, ta, tr, 3, true>}},
#define TTX_F32_B(ta, tr) TTX_ROW(float, float, false, ta, tr)
#define TTX_F32_Z(ta, tr) TTX_ROW(float, float, true, ta, tr)
#define TTX_F64_B(ta, tr) TTX_ROW(double, double, false, ta, tr)
#define TTX_F64_Z(ta, tr) TTX_ROW(double, double, true, ta, tr)
#define TTX_C32_B(ta, tr) TTX_ROW(cf32, cf32, false, ta, tr)
#define TTX_C32_Z(ta, tr) TTX_ROW(cf32, cf32, true, ta, tr)
#define TTX_C64_B(ta, tr) TTX_ROW(cf64, cf64, false, ta, tr)
#define TTX_C64_Z(ta, tr) TTX_ROW(cf64, cf64, true, ta, tr)
#define TTX_SD_B(ta, tr) TTX_ROW(double, float, false, ta, tr)
#define TTX_SD_Z(ta, tr) TTX_ROW(double, float, true, ta, tr)
#define TTX_DS_B(ta, tr) TTX_ROW(float, double, false, ta, tr)
#define TTX_DS_Z(ta, tr) TTX_ROW(float, double, true, ta, tr)
#define TTX_CZ_B(ta, tr) TTX_ROW(cf64, cf32, false, ta, tr)
#define TTX_CZ_Z(ta, tr) TTX_ROW(cf64, cf32, true, ta, tr)
#define TTX_ZC_B(ta, tr) TTX_ROW(cf32, cf64, false, ta, tr)
#define TTX_ZC_Z(ta, tr) TTX_ROW(cf32, cf64, true, ta, tr)
static const LauncherRow kF32B[] = {TTX_PRESERVED_MENU_F32(TTX_F32_B)};
static const LauncherRow kF32Z[] = {TTX_PRESERVED_MENU_F32(TTX_F32_Z)};
static const LauncherRow kF64B[] = {TTX_PRESERVED_MENU_F64(TTX_F64_B)};
static const LauncherRow kF64Z[] = {TTX_PRESERVED_MENU_F64(TTX_F64_Z)};
static const LauncherRow kC32B[] = {TTX_PRESERVED_MENU_F64(TTX_C32_B)};
static const LauncherRow kC32Z[] = {TTX_PRESERVED_MENU_F64(TTX_C32_Z)};
static const LauncherRow kC64B[] = {TTX_PRESERVED_MENU_C64(TTX_C64_B)};
static const LauncherRow kC64Z[] = {TTX_PRESERVED_MENU_C64(TTX_C64_Z)};
static const LauncherRow kSDB[] = {TTX_PRESERVED_MENU_F64(TTX_SD_B)};
static const LauncherRow kSDZ[] = {TTX_PRESERVED_MENU_F64(TTX_SD_Z)};
static const LauncherRow kDSB[] = {TTX_PRESERVED_MENU_F32(TTX_DS_B)};
static const LauncherRow kDSZ[] = {TTX_PRESERVED_MENU_F32(TTX_DS_Z)};
static const LauncherRow kCZB[] = {TTX_PRESERVED_MENU_C64(TTX_CZ_B)};
static const LauncherRow kCZZ[] = {TTX_PRESERVED_MENU_C64(TTX_CZ_Z)};
static const LauncherRow kZCB[] = {TTX_PRESERVED_MENU_F64(TTX_ZC_B)};
static const LauncherRow kZCZ[] = {TTX_PRESERVED_MENU_F64(TTX_ZC_Z)};

#define TTX_PICK(B, Z) return *out = beta0 ? Z : B, int(sizeof(B) / sizeof(B[0]))
int preserved_rows(int code, bool beta0, const LauncherRow** out) {
    switch (code) {
        case TTX_F32: TTX_PICK(kF32B, kF32Z);
        case TTX_F64: TTX_PICK(kF64B, kF64Z);
        case TTX_C32: TTX_PICK(kC32B, kC32Z);
        case TTX_C64: TTX_PICK(kC64B, kC64Z);
        case TTX_F32_F64: TTX_PICK(kSDB, kSDZ);
        case TTX_F64_F32: TTX_PICK(kDSB, kDSZ);
        case TTX_C32_C64: TTX_PICK(kCZB, kCZZ);
        case TTX_C64_C32: TTX_PICK(kZCB, kZCZ);
        default: return 0;
    }
}

}  // namespace ttx
