// Moved-family launcher rows for one pair of element types and beta class.
// Each translation unit kernels_moved_<types>_<beta>.hip instantiates one
// table (the moved kernels are the largest share of the code, so they
// compile in parallel).  A vector variant a shape cannot use (its edge is
// not a multiple of the side's vector width, or the element is already 16
// bytes) falls back to single elements on that side.
#pragma once

#include <type_traits>

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

// T: B's element type, S: A's (the same unless mixed precision).
template <typename T, typename S, bool B0, int TA, int TB, int VA, int VB, bool NT>
static hipError_t launch_moved(const void* args, uint32_t grid, hipStream_t stream) {
    constexpr int va = (VA > 1 && kVec<S> > 1 && TA % kVec<S> == 0) ? kVec<S> : 1;
    constexpr int vb = (VB > 1 && kVec<T> > 1 && TB % kVec<T> == 0) ? kVec<T> : 1;
    const TileArgs<T, S>& a = *static_cast<const TileArgs<T, S>*>(args);
    if constexpr (std::is_same<T, S>::value)
        hipLaunchKernelGGL((k_moved<T, B0, TA, TB, va, vb, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_moved_x<T, S, B0, TA, TB, va, vb, NT>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ttx

// One row: the four vector variants of shape (ta, tb), with plain and with
// nontemporal stores.
#define TTX_MOVED_ENTRY(T, S, B0, ta, tb)                                                       \
    {ta, tb, {launch_moved<T, S, B0, ta, tb, 1, 1, false>, launch_moved<T, S, B0, ta, tb, 2, 1, false>, \
              launch_moved<T, S, B0, ta, tb, 1, 2, false>, launch_moved<T, S, B0, ta, tb, 2, 2, false>, \
              launch_moved<T, S, B0, ta, tb, 1, 1, true>, launch_moved<T, S, B0, ta, tb, 2, 1, true>,   \
              launch_moved<T, S, B0, ta, tb, 1, 2, true>, launch_moved<T, S, B0, ta, tb, 2, 2, true>}},

// int fn(const LauncherRow**) over MENU, whose entries expand through the
// including file's TTX_ENTRY(ta, tb).
#define TTX_MOVED_TABLE(fn, MENU)                                                               \
    namespace ttx {                                                                              \
    int fn(const LauncherRow** out) {                                                            \
        static const LauncherRow rows[] = {MENU(TTX_ENTRY)};                                     \
        *out = rows;                                                                             \
        return int(sizeof(rows) / sizeof(rows[0]));                                              \
    }                                                                                            \
    }
