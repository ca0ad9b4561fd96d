// Staged preserved-family kernel instantiations (one per menu shape).
#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, bool B0, int N0, int TX, int TY>
static hipError_t launch(const void* args, uint32_t grid, hipStream_t stream) {
    const TileArgs<T>& a = *static_cast<const TileArgs<T>*>(args);
    hipLaunchKernelGGL((k_staged<T, B0, N0, TX, TY>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

#define TTX_F32_B(n0, tx, ty) {n0, tx, ty, launch<float, false, n0, tx, ty>},
#define TTX_F32_Z(n0, tx, ty) {n0, tx, ty, launch<float, true, n0, tx, ty>},
#define TTX_F64_B(n0, tx, ty) {n0, tx, ty, launch<double, false, n0, tx, ty>},
#define TTX_F64_Z(n0, tx, ty) {n0, tx, ty, launch<double, true, n0, tx, ty>},
#define TTX_C32_B(n0, tx, ty) {n0, tx, ty, launch<cf32, false, n0, tx, ty>},
#define TTX_C32_Z(n0, tx, ty) {n0, tx, ty, launch<cf32, true, n0, tx, ty>},
#define TTX_C64_B(n0, tx, ty) {n0, tx, ty, launch<cf64, false, n0, tx, ty>},
#define TTX_C64_Z(n0, tx, ty) {n0, tx, ty, launch<cf64, true, n0, tx, ty>},
static const StagedRow kF32B[] = {TTX_STAGED_MENU_F32(TTX_F32_B)};
static const StagedRow kF32Z[] = {TTX_STAGED_MENU_F32(TTX_F32_Z)};
static const StagedRow kF64B[] = {TTX_STAGED_MENU_F64(TTX_F64_B)};
static const StagedRow kF64Z[] = {TTX_STAGED_MENU_F64(TTX_F64_Z)};
static const StagedRow kC32B[] = {TTX_STAGED_MENU_F64(TTX_C32_B)};
static const StagedRow kC32Z[] = {TTX_STAGED_MENU_F64(TTX_C32_Z)};
static const StagedRow kC64B[] = {TTX_STAGED_MENU_C64(TTX_C64_B)};
static const StagedRow kC64Z[] = {TTX_STAGED_MENU_C64(TTX_C64_Z)};

#define TTX_PICK(B, Z) return *out = beta0 ? Z : B, int(sizeof(B) / sizeof(B[0]))
int staged_rows(int dtype, bool beta0, const StagedRow** out) {
    switch (dtype) {
        case TTX_F32: TTX_PICK(kF32B, kF32Z);
        case TTX_F64: TTX_PICK(kF64B, kF64Z);
        case TTX_C32: TTX_PICK(kC32B, kC32Z);
        default: TTX_PICK(kC64B, kC64Z);
    }
}

}  // namespace ttx
