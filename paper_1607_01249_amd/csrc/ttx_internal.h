// Internal types shared by the planner, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <functional>
#include <string>
#include <type_traits>

#include "../../include/ttx.h"
#include "device_types.h"
#include "menu.h"

namespace ttx {

static_assert(kMaxDims == TTX_MAX_DIMS, "rank limit of the C ABI");

// A data-type code (ttx_dtype) names the element types of A and B; they
// differ for the mixed-precision codes.
inline bool dtype_valid(int code) { return code >= TTX_F32 && code <= TTX_C64_C32; }
// Internal element types (never accepted from callers): whole units of a
// kept stride-1 row, moved as one element each (configs with TTX_CFG_WIDE).
enum : int {
    kWideF32x4 = 8,   // four FP32 elements (16 bytes)
    kWideF64x2 = 9,   // two FP64 elements (16 bytes)
    kWideF32x2 = 10,  // two FP32 elements (8 bytes)
};
inline int dtype_b_of(int code) {
    static const int b[] = {TTX_F32, TTX_F64, TTX_C32, TTX_C64, TTX_F64, TTX_F32, TTX_C64, TTX_C32,
                            kWideF32x4, kWideF64x2, kWideF32x2};
    return b[code];
}
inline int dtype_a_of(int code) {
    static const int a[] = {TTX_F32, TTX_F64, TTX_C32, TTX_C64, TTX_F32, TTX_F64, TTX_C32, TTX_C64,
                            kWideF32x4, kWideF64x2, kWideF32x2};
    return a[code];
}
inline bool dtype_complex(int dtype) { return dtype == TTX_C32 || dtype == TTX_C64; }
inline int elem_bytes(int dtype) {
    static const int e[] = {4, 8, 8, 16, 0, 0, 0, 0, 16, 16, 8};
    return e[dtype];
}
inline const char* dtype_name(int dtype) {
    return dtype == TTX_F32 ? "f32" : dtype == TTX_F64 ? "f64" : dtype == TTX_C32 ? "c32" : "c64";
}

// A scalar alpha or beta as the caller passed it (the imaginary part is zero
// for the real element types).
struct Scalar {
    double re = 0.0, im = 0.0;
    Scalar() = default;
    Scalar(double r) : re(r) {}
    Scalar(double r, double i) : re(r), im(i) {}
};

// The scalar rounded to the element type's scalar.
template <typename T>
inline T scalar_as(const Scalar& s) {
    if constexpr (std::is_same<T, cf32>::value) {
        return T{float(s.re), float(s.im)};
    } else if constexpr (std::is_same<T, cf64>::value) {
        return T{s.re, s.im};
    } else if constexpr (WideOf<T>::lanes > 0) {
        T t;
        for (int i = 0; i < WideOf<T>::lanes; ++i) t.v[i] = typename WideOf<T>::lane_t(s.re);
        return t;
    } else {
        return T(s.re);
    }
}


// A merged problem (planner output), A order.
struct Dim {
    int64_t size;
    int64_t sa;   // stride in A
    int64_t sb;   // stride in B
};

struct Problem {
    int dtype = 0;              // B's element type (TTX_F32 .. TTX_C64)
    int dtype_a = 0;            // A's element type
    int code = 0;               // the ttx_dtype code the problem was made with
    int n = 0;                  // merged rank
    Dim dim[kMaxDims];
    int perm[kMaxDims];         // merged gather perm: B position k holds merged dim perm[k]
    int family = TTX_FAMILY_EMPTY;
    int64_t elements = 0;
    int64_t extent_a = 0;       // bytes
    int64_t extent_b = 0;
    // original (unmerged) problem, kept for keys and descriptions
    int n_orig = 0;
};

struct TileShape { int ta, tb; };

// Status with a thread-local message.
ttx_status fail(ttx_status s, const std::string& msg);
void clear_error();

// beta == 0 after rounding to the element type (complex: both parts); then B is not read.
bool beta_is_zero(int dtype, const Scalar& beta);
// Pointer checks shared by every entry point: NULL, element alignment, and
// overlap of A with B_out and of B_in with B_out (unless they are equal).
ttx_status check_pointers(const Problem& p, const void* A, const void* Bin, const void* Bout,
                          bool beta0);

// The per-call path with the plan cache; B_in may differ from B_out.
ttx_status transpose_cached(int dtype, int n, const int* perm, const int64_t* size,
                            const int64_t* outer_a, const int64_t* outer_b, const Scalar& alpha,
                            const void* A, const Scalar& beta, const void* Bin, void* Bout,
                            hipStream_t stream);

// Planner (host only).
ttx_status make_problem(int dtype, int n, const int* perm, const int64_t* size,
                        const int64_t* outer_a, const int64_t* outer_b, Problem* out);
// The same from element strides (sa[m], sb[m]: A's and B's stride of A index m)
// that the caller has already checked (n, perm, sizes valid; B's addressed
// elements distinct).
ttx_status make_problem_strided(int dtype, int n, const int* perm, const int64_t* size,
                                const int64_t* sa, const int64_t* sb, Problem* out);
// Validates a config against a problem; fills *why on rejection.
bool config_valid(const Problem& p, const ttx_config& c, std::string* why);
// The heuristic default config (best-ranked candidate).
ttx_config default_config(const Problem& p);
// The same without whole-unit rows (for pointers not aligned to the unit).
ttx_config default_config_elementwise(const Problem& p);
// The same greedy choice restricted to the given tile shapes; staged tiles
// (preserved family, short rows) come from `staged` entries packed as
// {lanes * 65536 + tile_x, tile_y}, or from the whole staged menu when
// nstaged < 0; dense tiles are considered when `dense` is set, and dense
// tiles over whole units of the rows (TTX_CFG_WIDE) also when `wide` is.
ttx_config default_config_from(const Problem& p, const TileShape* shapes, int ns,
                               const TileShape* staged, int nstaged, bool dense, bool wide = false);
// Candidate enumeration with estimated costs (sorted ascending).
int rank_candidates(const Problem& p, int max_candidates, ttx_config* out, double* cost, int cap);
// Builds the kernel-side grid, strides and index groups for a config.
void build_grid(const Problem& p, const ttx_config& c, TileArgsHost* h);
// Flags for the vector paths given the pointers in use.
int kernel_flags(const Problem& p, const ttx_config& c, const void* A, const void* Bsrc,
                 const void* Bdst);

// Kernel menu (tile shapes the library instantiates), per dtype and family.
int tile_menu(int dtype, int family, const TileShape** shapes);
bool tile_in_menu(int dtype, int family, int ta, int tb);
// The larger moved-family tiles that exist only as run-time compiled kernels.
int large_tile_menu(int dtype, const TileShape** shapes);
bool tile_in_large_menu(int dtype, int ta, int tb);
// Staged preserved tiles: row-lane count for a row length (16, 32 or 64; 0 if
// the rows are too long to stage) and whether (n0_max, tx, ty) is instantiated.
int staged_lanes(int64_t n0);
bool staged_in_menu(int dtype, int n0_max, int tx, int ty);
// A preserved-family config with index groups selects the staged tiles
// (the padded-lane kind unless dense).
inline bool config_is_dense(const ttx_config& c) { return (c.flags & TTX_CFG_DENSE) != 0; }
inline bool config_is_staged(const ttx_config& c) {
    return c.family == TTX_FAMILY_PRESERVED && (c.group_a > 1 || c.group_b > 1) && !config_is_dense(c);
}
// Elements per dense tile.
inline int dense_cap(int dtype) {
    static const int cap[] = {TTX_DENSE_CAP_F32, TTX_DENSE_CAP_F64, TTX_DENSE_CAP_C32, TTX_DENSE_CAP_C64,
                              0, 0, 0, 0, TTX_DENSE_CAP_W16, TTX_DENSE_CAP_W16, TTX_DENSE_CAP_W8};
    return cap[dtype];
}
inline bool config_is_wide(const ttx_config& c) { return (c.flags & TTX_CFG_WIDE) != 0; }
// Whether the config's tile passes through LDS in rows of a fixed length
// (moved menu tiles and staged tiles): the tiles that lds_pad pads.
inline bool config_uses_pad(const ttx_config& c) {
    return !config_is_dense(c) && (c.family == TTX_FAMILY_MOVED || config_is_staged(c));
}
// The LDS row padding in effect (1, the pre-compiled kernels', where none applies).
inline int config_pad(const ttx_config& c) { return config_uses_pad(c) ? c.lds_pad : 1; }
// Whether the config runs outside the pre-compiled kernels (another
// workgroup size or LDS padding, line-aligned A runs, a pipelined persistent
// grid): then it always runs a size-specialised kernel, compiled on first use.
inline bool config_needs_jit(const ttx_config& c) {
    return c.threads != kThreads || config_pad(c) != 1 || (c.flags & (TTX_CFG_ALIGN_A | TTX_CFG_PIPELINED));
}
// The same, also true for a moved tile of the run-time-only list (a shape
// outside the pre-compiled menu).
inline bool config_needs_jit(const Problem& p, const ttx_config& c) {
    return config_needs_jit(c) || (p.family == TTX_FAMILY_MOVED && !config_is_dense(c) &&
                                   !tile_in_menu(p.dtype, p.family, c.tile_a, c.tile_b));
}
// Elements of A per 128-byte line for line-aligned A runs (TTX_CFG_ALIGN_A; 0 when off).
inline int config_align_elems(const ttx_config& c, int elem_bytes_a) {
    return (c.flags & TTX_CFG_ALIGN_A) ? 128 / elem_bytes_a : 0;
}
// Workgroup variants of a valid config (threads per workgroup x LDS row
// padding), the config itself first; returns how many were written.
int workgroup_variants(const Problem& p, const ttx_config& base, ttx_config* out, int cap);
// Steps of the first grid position per group of the grouped tile order.
constexpr uint32_t kGroupedSteps = 8;
// The problem over whole units of the kept stride-1 rows (TTX_CFG_WIDE):
// FP32/FP64 one-type preserved problems whose row length and other strides
// are multiples of the unit and whose rows hold at least two units.  Fills
// *w and returns true when there is one.
bool widen(const Problem& p, Problem* w);

// The matrix-core GEMM over packed panels (gemm.hip).
hipError_t launch_gemm_panels(int dtype, int panel, int64_t m, int64_t n, int64_t k, const void* Pa,
                              const void* Pb, void* C, int64_t ldc, hipStream_t stream);

// Launchers (kernels.hip).  They return hipSuccess or the launch error.
hipError_t launch_tiles(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                        const void* Bsrc, void* Bdst, const Scalar& alpha, const Scalar& beta,
                        hipStream_t stream);

// What launch_tiles runs for a tiled (moved or preserved family) problem,
// resolved for a set of pointers: the problem and config the tile kernel
// runs on (over whole units of the kept rows for wide configs, or the
// element-wise fallback when the pointers are not aligned to the unit), the
// tile kind with its vector widths, row lanes or slot count, the grid, and
// the kernel's argument block (a TileArgs<T, S>).
enum : int { kTileMoved = 0, kTilePreserved = 1, kTileStaged = 2, kTileDense = 3 };
struct TiledLaunch {
    Problem p;
    ttx_config c;
    bool beta0;
    int kind;
    int va, vb;          // vector widths (moved: A and B sides; preserved: both the same)
    int n0;              // staged tiles: row lanes
    int cap;             // dense tiles: slots
    int flags;           // kernel flags (KF_*)
    uint32_t ntiles, grid;
    size_t args_bytes;
    alignas(16) unsigned char args[sizeof(TileArgs<cf64, cf64>)];
};
// Fills *L; false for empty and flat problems (nothing tiled) and for
// element codes without tile kernels.
bool prepare_tiled(const Problem& p, const ttx_config& c, bool beta0, const void* A, const void* Bsrc,
                   void* Bdst, const Scalar& alpha, const Scalar& beta, TiledLaunch* L);
// Size-specialised kernels (jit.cpp): the kernel a prepared launch runs,
// compiled at run time with the problem's arguments as constants.
struct JitKernel;
// Finds or compiles (hipRTC) and loads the kernel for L on the current device.
ttx_status jit_kernel(const TiledLaunch& L, const JitKernel** out);
// The translation unit jit_kernel compiles for L, and its kernel's name.
std::string jit_source(const TiledLaunch& L);
std::string jit_entry_name(const TiledLaunch& L);
// True when k runs what L launches (same device, kernel, flags and arguments).
bool jit_matches(const JitKernel& k, const TiledLaunch& L);
// The kernel's name as profilers print it.
const std::string& jit_name(const JitKernel& k);
hipError_t jit_launch(const JitKernel& k, const TiledLaunch& L, hipStream_t stream);
// C++ spelling of an element type ("float", "ttx::cf32", "ttx::f32x4", ...).
const char* element_type_name(int dtype);

// The kernel launch_tiles would use, spelled as profilers print it.
std::string kernel_name(const Problem& p, const ttx_config& c, bool beta0, const void* A,
                        const void* Bsrc, const void* Bdst);

// Zero bytes [0, width) of `height` rows that start `pitch` bytes apart
// (dispatch.hip; width and pitch multiples of 4, dst 4-byte aligned).
hipError_t launch_fill_zero(void* dst, int64_t width, int64_t height, int64_t pitch, hipStream_t stream);

// Ceiling kernels (dispatch.hip).
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t stream);
hipError_t launch_axpby(int dtype, int64_t n, double alpha, const void* x, double beta, void* y,
                        hipStream_t stream);

// Tune table (tune.cpp).
ttx_status tune_problem(const Problem& p, bool beta0, int max_candidates, int reps, ttx_config* best,
                        int* n_timed);
// The same with every candidate compiled as a size-specialised kernel and
// timed in that form (default 24 candidates).
ttx_status tune_problem_specialised(const Problem& p, bool beta0, int max_candidates, int reps, ttx_config* best,
                                    int* n_timed);
// specialised: the entries for size-specialised execution (ttx_tune_specialised).
bool table_lookup(const Problem& p, bool beta0, ttx_config* out, bool specialised = false);
void table_store(const Problem& p, bool beta0, const ttx_config& c, double usec, bool specialised = false);
uint64_t table_generation();
// Times `count` candidates on tuner-owned scratch buffers sized for p (minimum
// of `reps` runs, the 1 GiB flush area cleared before each) and returns the
// fastest; launch(i, A, B, stream) runs candidate i.  all_us (may be NULL)
// receives every candidate's time.
ttx_status time_candidates(const Problem& p, bool beta0, int count, int reps,
                           const std::function<hipError_t(int, const void*, void*, hipStream_t)>& launch,
                           int* best_i, double* best_us, double* all_us = nullptr);

// -- batched execution (batch.hip) ------------------------------------------
// One entry of the device descriptor table read by the persistent kernel:
// the tile variant (an index into the batched menu for the dtype and beta
// class, or -1 when there is nothing to do), the tile count, and the
// arguments of the tile body (a TileArgs<float> or TileArgs<double>).
struct alignas(16) BatchDesc {
    int variant;
    int dtype;
    uint32_t tiles;
    uint32_t chunk;     // tiles per claimed chunk (set by batch_layout)
    alignas(16) unsigned char args[sizeof(TileArgs<double>)];
};

// Fills *d for one problem: a tuned config when `forced` is non-NULL (it
// must name a batched-menu shape), else the heuristic choice among the
// batched-menu shapes.  *used receives the config.  Host only.
ttx_status batch_describe(const Problem& p, const ttx_config* forced, bool beta0, const void* A,
                          const void* Bsrc, void* Bdst, double alpha, double beta, BatchDesc* d,
                          ttx_config* used);
// Points a described problem at another output tensor (same alignment class).
void batch_set_output(BatchDesc* d, void* Bdst);
// Batched-menu configs for a problem, best heuristic first (for tuning).
int batch_candidates(const Problem& p, int max_candidates, ttx_config* out, int cap);
// Work layout of a persistent launch over `count` descriptors: sets each
// descriptor's chunk size and fills chunk_prefix[0..count] (chunks of
// problem i are chunk_prefix[i] .. chunk_prefix[i+1]-1).  Returns the total
// chunk count and sets *grid to the workgroup count.  Host only.
uint32_t batch_layout(BatchDesc* desc, int count, uint32_t* chunk_prefix, int* grid);
// Workgroups of the persistent launch for `chunks` chunks.
int batch_grid(uint32_t chunks);
// The persistent kernel over count descriptors.  `counter` is two words of
// device memory that are zero before the launch; the launch leaves them zero
// again (the last workgroup to finish resets them), so launches that use
// the same counter must not overlap.
hipError_t launch_batch(const BatchDesc* d_desc, const uint32_t* d_chunk_prefix, int count,
                        uint32_t chunks, int grid, uint32_t* counter, hipStream_t stream);

}  // namespace ttx
