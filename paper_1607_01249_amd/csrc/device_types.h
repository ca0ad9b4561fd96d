// Types shared by the host planner and the device tile code: element
// types, the index-division helper, and the kernel argument blocks.  This
// header is also compiled at run time (hipRTC) for size-specialised kernels,
// so it includes nothing beyond the standard integer and trait headers.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif
#include <cstdint>
#include <type_traits>

namespace ttx {

// Largest tensor rank (the C ABI's TTX_MAX_DIMS).
constexpr int kMaxDims = 16;
// Threads per workgroup of every tile kernel.
constexpr int kThreads = 256;

// Complex elements: interleaved (re, im) pairs, aligned to their size so
// that one element is one 8- or 16-byte access.
struct alignas(8) cf32 {
    float re, im;
};
struct alignas(16) cf64 {
    double re, im;
};

// Units of a kept row (the internal wide element types).
struct alignas(16) f32x4 {
    float v[4];
};
struct alignas(16) f64x2 {
    double v[2];
};
struct alignas(8) f32x2 {
    float v[2];
};
template <typename T>
struct WideOf {
    static constexpr int lanes = 0;
};
template <>
struct WideOf<f32x4> {
    static constexpr int lanes = 4;
    using lane_t = float;
};
template <>
struct WideOf<f64x2> {
    static constexpr int lanes = 2;
    using lane_t = double;
};
template <>
struct WideOf<f32x2> {
    static constexpr int lanes = 2;
    using lane_t = float;
};

// Division by a run-time invariant 32-bit divisor with a multiply and a
// shift (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994): for d >= 1, l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1 give n / d = (mulhi(n, m) + n) >> l for
// every 32-bit n (the sum is formed in 64 bits).
struct FastDiv {
    uint32_t d;
    uint32_t m;
    uint32_t l;

    constexpr FastDiv() : d(1), m(1), l(0) {}
    explicit constexpr FastDiv(uint32_t divisor) : d(1), m(1), l(0) { init(divisor); }

    constexpr void init(uint32_t divisor) {
        d = divisor ? divisor : 1;
        l = 0;
        while ((uint64_t(1) << l) < d) ++l;
        m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    }

    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
        uint64_t hi = (uint64_t(n) * m) >> 32;
        return uint32_t((hi + n) >> l);
    }
};

// Description of the tiled iteration space shared by the tile kernels.
// Tile ids enumerate the merged indices in `order` (fastest first); position
// p has count[p] steps, and one step moves the tile origin by stepA[p] /
// stepB[p] elements.  Positions pa and pb hold the two tile indices; their
// full extents bound the edge tiles.
struct TileGrid {
    int nd;
    int pa, pb;
    int pz;                        // dense tiles: position of the third tiled index (-1: none)
    uint32_t ntiles;
    int64_t ext_a, ext_b;          // extents along the two tile indices
    int64_t ext_z;                 // and along the third (dense tiles)
    uint32_t count[kMaxDims];
    FastDiv div[kMaxDims];
    int64_t stepA[kMaxDims];
    int64_t stepB[kMaxDims];
    // Grouped order (gk > 0): within each plane of the first two positions,
    // ids walk groups of gk steps of position 0 across all of position 1, so
    // the tiles in flight together are neighbours along both.  dvg divides by
    // gk * count[1], dvp by count[0] * count[1].
    uint32_t gk;
    FastDiv dvg, dvp;

    // The plane-major id of the tile that grouped id t names (a bijection on
    // [0, ntiles)).
    __host__ __device__ __forceinline__ uint32_t grouped(uint32_t t) const {
        const uint32_t c0 = count[0], c1 = count[1];
        const uint32_t q = dvp.div(t), r = t - q * (c0 * c1);
        const uint32_t g = dvg.div(r), first0 = g * gk;
        const uint32_t gsz = c0 - first0 < gk ? c0 - first0 : gk;
        const uint32_t rr = r - g * gk * c1;
        const uint32_t p1 = rr / gsz, p0 = first0 + (rr - p1 * gsz);
        return q * (c0 * c1) + p0 + p1 * c0;
    }
};

// Kernel-side flags (separate from TTX_CFG_*, which describe a config).
enum : int {
    KF_VEC_A = 1,      // 16-byte vector accesses along the tile index of A
    KF_VEC_B = 2,      // 16-byte vector accesses along the tile index of B
    KF_NT_STORE = 4,   // non-temporal stores to B
    KF_SWIZZLE = 8,    // XCD-aware tile id mapping
};

// A super index: ng consecutive merged indices tiled as one.  The offset of
// position y in the other tensor is sum_k digit_k(y) * stride[k] with
// digit_k = (y / prod_{j<k} size_j) % size_k (index 0 fastest).  With several
// members the extent is below 2^31 and digits come from 32-bit divisions.
constexpr int kMaxGroup = 4;
struct Group {
    int ng;
    FastDiv div[kMaxGroup - 1];   // sizes of all members but the last
    int64_t stride[kMaxGroup];

    __host__ __device__ __forceinline__ int64_t offset(int64_t y) const {
        if (ng == 1) return y * stride[0];
        uint32_t rem = uint32_t(y);
        int64_t off = 0;
        for (int k = 0; k + 1 < ng; ++k) {
            const uint32_t q = div[k].div(rem);
            off += int64_t(rem - q * div[k].d) * stride[k];
            rem = q;
        }
        return off + int64_t(rem) * stride[ng - 1];
    }
};

// The dtype-independent part of a tile kernel's arguments (built by the planner;
// ConstArgs in tile_kernels.h mirrors every member).
struct TileArgsHost {
    TileGrid g;
    int64_t sAa, sAb;   // A strides of the two tile (leader) indices
    int64_t sBa, sBb;   // B strides of the two tile (leader) indices
    Group gA;           // B offsets of the A-side super index (moved and staged tiles)
    Group gB;           // A offsets of the B-side super index (moved and staged tiles)
    int64_t s0A, s0B;   // staged tiles: strides of the shared row index in A and B
    int n0;             // staged tiles: row length
    // dense tiles: rows of dn0 elements (1 for the moved family), tx x ty rows
    // per tile; an A run holds runA = dn0*tx elements, a B run runB = dn0*ty;
    // the LDS tile has ty rows of ldr >= runA elements
    int dn0, tx, ty, ldr;
    uint32_t runA, runB;
    FastDiv dv0, dvA, dvB;
    // and tz planes along a third index (strides sAz, sBz); a plane holds
    // planeA = runA*ty (A order) or planeB = runB*tx (B order) elements
    int tz;
    int64_t sAz, sBz;
    uint32_t planeA, planeB;
    FastDiv dvPA, dvPB;
};

// T: B's element type (the arithmetic and LDS type); S: A's (converted to T
// on load when the precisions differ).
template <typename T, typename S = T>
struct TileArgs : TileArgsHost {
    const S* A;
    const T* Bsrc;      // read when beta != 0
    T* Bdst;
    T alpha, beta;
    int flags;
};

template <typename T, typename S = T>
struct FlatArgs {
    const S* A;
    const T* Bsrc;
    T* Bdst;
    T alpha, beta;
    int64_t n;          // element count
    int64_t sa, sb;     // strides of the single index
    int flags;
};

}  // namespace ttx
