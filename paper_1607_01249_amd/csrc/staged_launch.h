// Staged preserved-family launcher rows (one per shape of the staged menu of
// B's element type) for one pair of element types; each translation unit
// kernels_staged_<types>.hip instantiates both beta classes of one pair.
#pragma once

#include <type_traits>

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, typename S, bool B0, int N0, int TX, int TY, bool NT>
static hipError_t launch_staged(const void* args, uint32_t grid, hipStream_t stream) {
    const TileArgs<T, S>& a = *static_cast<const TileArgs<T, S>*>(args);
    if constexpr (std::is_same<T, S>::value)
        hipLaunchKernelGGL((k_staged<T, B0, N0, TX, TY, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_staged_x<T, S, B0, N0, TX, TY, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ttx

// One row: shape (n0, tx, ty) with plain and with nontemporal stores.
#define TTX_STAGED_ENTRY(T, S, B0, n0, tx, ty) \
    {n0, tx, ty, {launch_staged<T, S, B0, n0, tx, ty, false>, launch_staged<T, S, B0, n0, tx, ty, true>}},

// int fn(bool beta0, const StagedRow**) over MENU for element types (T, S).
#define TTX_STAGED_TABLE(fn, T, S, MENU)                                                        \
    namespace ttx {                                                                              \
    int fn(bool beta0, const StagedRow** out) {                                                  \
        static const StagedRow b[] = {MENU(TTX_ENTRY_B)};                                        \
        static const StagedRow z[] = {MENU(TTX_ENTRY_Z)};                                        \
        *out = beta0 ? z : b;                                                                    \
        return int(sizeof(b) / sizeof(b[0]));                                                    \
    }                                                                                            \
    }
