// Moved-family launcher rows for one element type and beta class.  Each
// translation unit kernels_moved_<type>_<beta>.hip instantiates one table
// (the moved kernels are the largest share of the code, so they compile in
// parallel).  A vector variant a shape cannot use (its edge is not a
// multiple of the vector width, or the element is already 16 bytes) falls
// back to single elements on that side.
#pragma once

#include "menu.h"
#include "registry.h"
#include "tile_kernels.h"

namespace ttx {

template <typename T, bool B0, int TA, int TB, int VA, int VB>
static hipError_t launch_moved(const void* args, uint32_t grid, hipStream_t stream) {
    constexpr int V = kVec<T>;
    constexpr int va = (VA > 1 && V > 1 && TA % V == 0) ? V : 1;
    constexpr int vb = (VB > 1 && V > 1 && TB % V == 0) ? V : 1;
    const TileArgs<T>& a = *static_cast<const TileArgs<T>*>(args);
    hipLaunchKernelGGL((k_moved<T, B0, TA, TB, va, vb>), dim3(grid), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ttx

// One row: the four vector variants of shape (ta, tb).
#define TTX_MOVED_ENTRY(T, B0, ta, tb)                                                          \
    {ta, tb, {launch_moved<T, B0, ta, tb, 1, 1>, launch_moved<T, B0, ta, tb, 2, 1>,             \
              launch_moved<T, B0, ta, tb, 1, 2>, launch_moved<T, B0, ta, tb, 2, 2>}},

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
