// Staged preserved-family kernel instantiations (one per shape of the staged
// menu of B's element type, for every data-type code).
#include <type_traits>

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, typename S, bool B0, int N0, int TX, int TY>
static hipError_t launch(const void* args, uint32_t grid, hipStream_t stream) {
    const TileArgs<T, S>& a = *static_cast<const TileArgs<T, S>*>(args);
    if constexpr (std::is_same<T, S>::value)
        hipLaunchKernelGGL((k_staged<T, B0, N0, TX, TY>), dim3(grid), dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_staged_x<T, S, B0, N0, TX, TY>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

#define TTX_F32_B(n0, tx, ty) {n0, tx, ty, launch<float, float, false, n0, tx, ty>},
#define TTX_F32_Z(n0, tx, ty) {n0, tx, ty, launch<float, float, true, n0, tx, ty>},
#define TTX_F64_B(n0, tx, ty) {n0, tx, ty, launch<double, double, false, n0, tx, ty>},
#define TTX_F64_Z(n0, tx, ty) {n0, tx, ty, launch<double, double, true, n0, tx, ty>},
#define TTX_C32_B(n0, tx, ty) {n0, tx, ty, launch<cf32, cf32, false, n0, tx, ty>},
#define TTX_C32_Z(n0, tx, ty) {n0, tx, ty, launch<cf32, cf32, true, n0, tx, ty>},
#define TTX_C64_B(n0, tx, ty) {n0, tx, ty, launch<cf64, cf64, false, n0, tx, ty>},
#define TTX_C64_Z(n0, tx, ty) {n0, tx, ty, launch<cf64, cf64, true, n0, tx, ty>},
#define TTX_SD_B(n0, tx, ty) {n0, tx, ty, launch<double, float, false, n0, tx, ty>},
#define TTX_SD_Z(n0, tx, ty) {n0, tx, ty, launch<double, float, true, n0, tx, ty>},
#define TTX_DS_B(n0, tx, ty) {n0, tx, ty, launch<float, double, false, n0, tx, ty>},
#define TTX_DS_Z(n0, tx, ty) {n0, tx, ty, launch<float, double, true, n0, tx, ty>},
#define TTX_CZ_B(n0, tx, ty) {n0, tx, ty, launch<cf64, cf32, false, n0, tx, ty>},
#define TTX_CZ_Z(n0, tx, ty) {n0, tx, ty, launch<cf64, cf32, true, n0, tx, ty>},
#define TTX_ZC_B(n0, tx, ty) {n0, tx, ty, launch<cf32, cf64, false, n0, tx, ty>},
#define TTX_ZC_Z(n0, tx, ty) {n0, tx, ty, launch<cf32, cf64, true, n0, tx, ty>},
static const StagedRow kF32B[] = {TTX_STAGED_MENU_F32(TTX_F32_B)};
static const StagedRow kF32Z[] = {TTX_STAGED_MENU_F32(TTX_F32_Z)};
static const StagedRow kF64B[] = {TTX_STAGED_MENU_F64(TTX_F64_B)};
static const StagedRow kF64Z[] = {TTX_STAGED_MENU_F64(TTX_F64_Z)};
static const StagedRow kC32B[] = {TTX_STAGED_MENU_F64(TTX_C32_B)};
static const StagedRow kC32Z[] = {TTX_STAGED_MENU_F64(TTX_C32_Z)};
static const StagedRow kC64B[] = {TTX_STAGED_MENU_C64(TTX_C64_B)};
static const StagedRow kC64Z[] = {TTX_STAGED_MENU_C64(TTX_C64_Z)};
static const StagedRow kSDB[] = {TTX_STAGED_MENU_F64(TTX_SD_B)};
static const StagedRow kSDZ[] = {TTX_STAGED_MENU_F64(TTX_SD_Z)};
static const StagedRow kDSB[] = {TTX_STAGED_MENU_F32(TTX_DS_B)};
static const StagedRow kDSZ[] = {TTX_STAGED_MENU_F32(TTX_DS_Z)};
static const StagedRow kCZB[] = {TTX_STAGED_MENU_C64(TTX_CZ_B)};
static const StagedRow kCZZ[] = {TTX_STAGED_MENU_C64(TTX_CZ_Z)};
static const StagedRow kZCB[] = {TTX_STAGED_MENU_F64(TTX_ZC_B)};
static const StagedRow kZCZ[] = {TTX_STAGED_MENU_F64(TTX_ZC_Z)};

#define TTX_PICK(B, Z) return *out = beta0 ? Z : B, int(sizeof(B) / sizeof(B[0]))
int staged_rows(int code, bool beta0, const StagedRow** out) {
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
