// Device code for the transposition kernels (gfx950, wave64).
//
// Sec. 2.2 splits an N-D transposition into independent 2D transpositions
// ("macro-tiles") that run in parallel, one per thread block on GPUs, each
// staged through on-chip memory.  Here one workgroup (256 threads in the
// pre-compiled kernels; 64 to 512 in size-specialised ones) handles one
// tile at a time:
//   - moved family (A's stride-1 index moves): the tile is TA elements along
//     A's stride-1 index times TB elements along B's stride-1 index.  A is
//     read along its stride-1 index with 16-byte vector loads, the tile is
//     transposed through LDS (rows padded, by one element in the
//     pre-compiled kernels, so that the column-wise reads of the store
//     phase spread over the banks), and B
//     is written along its stride-1 index with 16-byte vector stores;
//   - preserved family (the stride-1 index stays in place, Sec. 3.2): rows
//     are contiguous in both tensors, so they are copied directly with
//     vector loads and stores, no LDS; short rows are staged through LDS
//     with whole rows inside the tile (StagedTile);
//   - dense tiles (either family): run-time tile extents, rows packed
//     without padding, several small planes per tile (DenseTile);
//   - flat: one merged index, a strided axpby.
// Edge tiles are predicated (the remainder of Sec. 2.3).  The epilogue is
// Eqn. 1: alpha*a when beta == 0 (B is never read), otherwise
// alpha*a + beta*b with both products and the sum rounded separately.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif
#include <type_traits>

#include "device_types.h"

#pragma clang fp contract(off)

namespace ttx {

template <typename T>
struct IsComplex : std::false_type {};
template <>
struct IsComplex<cf32> : std::true_type {};
template <>
struct IsComplex<cf64> : std::true_type {};

// Two single complex elements: one 16-byte vector.
struct alignas(16) cf32x2 {
    cf32 e[2];
    __device__ __forceinline__ cf32& operator[](int j) { return e[j]; }
    __device__ __forceinline__ const cf32& operator[](int j) const { return e[j]; }
};

template <typename T, int N>
struct VecOf {
    using type = T __attribute__((ext_vector_type(N)));
};
template <typename T>
struct VecOf<T, 1> {
    using type = T;
};
template <>
struct VecOf<cf32, 2> {
    using type = cf32x2;
};
template <typename T, int N>
using vec_t = typename VecOf<T, N>::type;

// The same bytes as a vector of a built-in type, for loads and stores.
template <typename T, int N>
struct RawOf {
    using type = vec_t<T, N>;
};
template <>
struct RawOf<cf32, 1> {
    using type = float __attribute__((ext_vector_type(2)));
};
template <>
struct RawOf<cf32, 2> {
    using type = float __attribute__((ext_vector_type(4)));
};
template <>
struct RawOf<cf64, 1> {
    using type = double __attribute__((ext_vector_type(2)));
};
template <>
struct RawOf<f32x4, 1> {
    using type = float __attribute__((ext_vector_type(4)));
};
template <>
struct RawOf<f64x2, 1> {
    using type = double __attribute__((ext_vector_type(2)));
};
template <>
struct RawOf<f32x2, 1> {
    using type = float __attribute__((ext_vector_type(2)));
};

template <typename T>
constexpr int kVec = 16 / int(sizeof(T));

template <typename T, int N>
__device__ __forceinline__ T lane(const vec_t<T, N>& v, int j) {
    if constexpr (N == 1)
        return v;
    else
        return v[j];
}

template <typename T, int N>
__device__ __forceinline__ void set_lane(vec_t<T, N>& v, int j, T x) {
    if constexpr (N == 1)
        v = x;
    else
        v[j] = x;
}

template <typename T, int N>
__device__ __forceinline__ vec_t<T, N> ld(const T* p) {
    using R = typename RawOf<T, N>::type;
    return __builtin_bit_cast(vec_t<T, N>, *reinterpret_cast<const R*>(p));
}

// NT: nontemporal store.  The store kind is a template parameter: a run-time
// choice between the two stores, which differ only in their cache hint, is
// merged by the compiler into one plain store.
template <typename T, int N, bool NT>
__device__ __forceinline__ void st(T* p, const vec_t<T, N>& v) {
    using R = typename RawOf<T, N>::type;
    const R r = __builtin_bit_cast(R, v);
    if constexpr (NT)
        __builtin_nontemporal_store(r, reinterpret_cast<R*>(p));
    else
        *reinterpret_cast<R*>(p) = r;
}

// The same bytes with only the element's alignment: a 16-byte vector that
// starts at any element boundary (global memory takes dword-aligned
// multi-dword accesses, so these are still single 16-byte instructions).
template <typename T, int N>
struct RawU {
    using type = typename RawOf<T, N>::type;
};
template <>
struct RawU<float, 4> {
    typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct RawU<float, 2> {
    typedef float type __attribute__((ext_vector_type(2), aligned(4)));
};
template <>
struct RawU<double, 2> {
    typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct RawU<cf32, 2> {
    typedef float type __attribute__((ext_vector_type(4), aligned(8)));
};

// Up to N elements at p (element-aligned): the whole vector when n >= N,
// else elements 0..n-1 one by one (the rest of v is left as it was), so that
// a run whose length is not a multiple of N never reads or writes past it.
template <typename T, int N>
__device__ __forceinline__ void ld_part(vec_t<T, N>& v, const T* p, int n) {
    if constexpr (N == 1) {
        v = ld<T, 1>(p);
    } else {
        using R = typename RawU<T, N>::type;
        if (n >= N) {
            v = __builtin_bit_cast(vec_t<T, N>, *reinterpret_cast<const R*>(p));
        } else {
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (j < n) set_lane<T, N>(v, j, p[j]);
        }
    }
}

template <typename T, int N, bool NT>
__device__ __forceinline__ void st_part(T* p, const vec_t<T, N>& v, int n) {
    if constexpr (N == 1) {
        st<T, 1, NT>(p, v);
    } else {
        using R = typename RawU<T, N>::type;
        if (n >= N) {
            const R r = __builtin_bit_cast(R, v);
            if constexpr (NT)
                __builtin_nontemporal_store(r, reinterpret_cast<R*>(p));
            else
                *reinterpret_cast<R*>(p) = r;
        } else {
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (j < n) p[j] = lane<T, N>(v, j);
        }
    }
}

// Complex product s*x: re = s.re*x.re - s.im*x.im, im = s.re*x.im + s.im*x.re,
// every product and sum rounded on its own (contraction is off in this file).
template <typename C>
__device__ __forceinline__ C cmul(const C& s, const C& x) {
    const auto t1 = s.re * x.re, t2 = s.im * x.im, t3 = s.re * x.im, t4 = s.im * x.re;
    return C{t1 - t2, t3 + t4};
}

// Eqn. 1 on one vector: alpha*a, or alpha*a + beta*b (unfused; complex
// elements add the two complex products part by part).
template <typename T, int N, bool BETA0>
__device__ __forceinline__ vec_t<T, N> epilogue(const vec_t<T, N>& a, const vec_t<T, N>& b,
                                                T alpha, T beta) {
    if constexpr (WideOf<T>::lanes > 0) {
        // a unit of a kept row: Eqn. 1 on each of its elements
        static_assert(N == 1, "units are whole vectors");
        T r;
#pragma unroll
        for (int i = 0; i < WideOf<T>::lanes; ++i) {
            if constexpr (BETA0) {
                r.v[i] = alpha.v[i] * a.v[i];
            } else {
                const auto pa = alpha.v[i] * a.v[i];
                const auto pb = beta.v[i] * b.v[i];
                r.v[i] = pa + pb;
            }
        }
        return r;
    } else if constexpr (IsComplex<T>::value) {
        vec_t<T, N> r;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const T x = lane<T, N>(a, j);
            const T pa = cmul(alpha, x);
            if constexpr (BETA0) {
                set_lane<T, N>(r, j, pa);
            } else {
                const T pb = cmul(beta, lane<T, N>(b, j));
                set_lane<T, N>(r, j, T{pa.re + pb.re, pa.im + pb.im});
            }
        }
        return r;
    } else if constexpr (BETA0) {
        return alpha * a;
    } else {
        vec_t<T, N> pa = alpha * a;
        vec_t<T, N> pb = beta * b;
        return pa + pb;
    }
}

// Mixed precision: an A element (type S) converted to B's type T (widening
// exact, narrowing to nearest, part by part for complex elements).
template <typename T, typename S>
__device__ __forceinline__ T conv(const S& x) {
    if constexpr (std::is_same<T, S>::value)
        return x;
    else if constexpr (IsComplex<T>::value)
        return T{decltype(T::re)(x.re), decltype(T::im)(x.im)};
    else
        return T(x);
}

template <typename T, typename S, int V>
__device__ __forceinline__ vec_t<T, V> conv_vec(const vec_t<S, V>& v) {
    if constexpr (std::is_same<T, S>::value)
        return v;
    else if constexpr (V == 1)
        return conv<T, S>(v);
    else
        return __builtin_convertvector(v, vec_t<T, V>);
}

// XCD-aware tile mapping.  Workgroups are dispatched round-robin over the
// 8 XCDs of an MI355X, each with its own L2.  This bijection on [0, G) gives
// XCD x the consecutive ids [start(x), start(x) + count(x)), so that tiles
// that share cache lines or DRAM pages run under one L2.
__device__ __forceinline__ uint32_t swizzle_id(uint32_t bid, uint32_t G) {
    const uint32_t per = G >> 3, rem = G & 7;
    const uint32_t x = bid & 7, local = bid >> 3;
    const uint32_t start = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return start + local;
}

struct TileCoord {
    int64_t oa, ob;     // origin offsets (moved family: without the group cross terms)
    int64_t x0, y0;     // origin along the two tile (super) indices
    int ea, eb;         // extents of this (maybe edge) tile
    int ez;             // dense tiles: planes along the third index
};

// Tile id -> origin offsets in A and B and the extents of this (maybe edge)
// tile; TC is the tile extent along the third index of dense tiles.
__device__ __forceinline__ TileCoord decode_tile(const TileGrid& g, uint32_t t, int TA, int TB, int TC = 1) {
    TileCoord c{0, 0, 0, 0, TA, TB, TC};
    if (g.gk) t = g.grouped(t);
    uint32_t rem = t;
    for (int q = 0; q < g.nd; ++q) {
        const uint32_t next = g.div[q].div(rem);
        const uint32_t r = rem - next * g.count[q];
        rem = next;
        c.oa += int64_t(r) * g.stepA[q];
        c.ob += int64_t(r) * g.stepB[q];
        if (q == g.pa) {
            c.x0 = int64_t(r) * TA;
            c.ea = int(min(int64_t(TA), g.ext_a - c.x0));
        }
        if (q == g.pb) {
            c.y0 = int64_t(r) * TB;
            c.eb = int(min(int64_t(TB), g.ext_b - c.y0));
        }
        if (q == g.pz) c.ez = int(min(int64_t(TC), g.ext_z - int64_t(r) * TC));
    }
    return c;
}

constexpr int pow2_ceil(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Thread layout used for both sides of a tile: a run of TA elements is
// covered by P = pow2_ceil(TA / V) threads (the last P - TA/V idle when
// TA / V is not a power of two), so NT / P runs are handled per pass and a
// thread's address advances by a fixed stride from one pass to the next.

// The tile bodies are split into phases so that a workgroup working through
// several tiles can overlap them: tile k+1's loads are issued before tile
// k's stores, so waiting for those loads never waits for the stores (memory
// operations retire in order), and the stores drain while the next tile is
// transposed.  `tile_loop` runs tiles t, t + step, ... < end that way.

// Whether a tile stores to B nontemporally: fixed by the tile's NTS (0 or 1;
// the generic kernels are instantiated once per store kind and the host
// picks the instance from KF_NT_STORE), or, with NTS < 0, the KF_NT_STORE
// bit of an argument block whose flags are a compile-time constant (the
// size-specialised kernels).
template <int NTS, typename Args>
constexpr bool nt_of() {
    if constexpr (NTS >= 0)
        return NTS == 1;
    else
        return (Args::flags & KF_NT_STORE) != 0;
}

// One moved-family tile over the A-side super index x (A's first group_a
// indices, contiguous in A) and the B-side super index y (B's first group_b
// indices, contiguous in B): element (x0 + x, y0 + y) for x < ea, y < eb is
// A[oa + x*sAa + gB.offset(y0 + y)] -> B[ob + y*sBb + gA.offset(x0 + x)].
// VA / VB are the vector widths along x in A and along y in B (VA > 1
// implies sAa == 1, VB > 1 implies sBb == 1); vectors need only element
// alignment, and a vector that would run past the end of the super index is
// moved element by element.  The LDS tile has TB rows of TA + PAD elements
// (the pre-compiled kernels pad by one, so that the column-wise reads of the
// store phase fall in distinct banks); NTH threads share the tile.
//
// Line-aligned A runs (ALN > 0, the elements of one 128-byte line of A;
// A's super index contiguous, sAa == 1): the tile's x range is shifted down
// so that it starts on a line boundary (of device addresses) in the A row
// of its first y,
// [x0 - s, x0 - s + TA) with s = that row's element offset modulo ALN, and
// clipped to [0, ext_a); the grid holds one more x tile to cover the shift.
// Rows whose length is not a multiple of the line then cost whole lines
// only, instead of sharing the lines at each tile boundary with the
// neighbouring tile.  With ALN == 0 the tile is [x0, x0 + TA).
template <typename T, bool BETA0, int TA, int TB, int VA, int VB, typename S = T, int NTS = -1,
          int NTH = kThreads, int PAD = 1, int ALN = 0>
struct MovedTile {
    static constexpr bool kUsesLds = true;
    static constexpr int kTA = TA, kTB = TB;
    static constexpr int NT = NTH, LDR = TA + PAD;
    static_assert(ALN == 0 || (ALN & (ALN - 1)) == 0, "line length in elements is a power of two");

    // The tile's x range: origin x0 (the tile covers x0 .. x0 + TA - 1), the
    // A offset of element x0 of its first row, and the valid positions
    // lo <= x < hi relative to x0.
    struct Span {
        int64_t x0, oa;
        int lo, hi;
    };
    template <typename Args>
    __device__ __forceinline__ static Span span(const Args& a, const TileCoord& c) {
        if constexpr (ALN == 0) {
            return Span{c.x0, c.oa, 0, c.ea};
        } else {
            // A element index (from address 0) of (x = 0, y0): the tile's
            // origin offset without its x term, plus A's base in elements
            const int64_t row = c.oa - c.x0 + a.gB.offset(c.y0) +
                                int64_t(reinterpret_cast<uintptr_t>(a.A) / sizeof(S));
            const int s = int(row & (ALN - 1));
            const int64_t x0 = c.x0 - s, rem = a.g.ext_a - x0;
            return Span{x0, c.oa - s, x0 < 0 ? int(-x0) : 0, int(rem < TA ? (rem < 0 ? 0 : rem) : TA)};
        }
    }
    template <typename Args>
    __device__ static int ext_a(const Args&) { return TA; }
    template <typename Args>
    __device__ static int ext_b(const Args&) { return TB; }
    template <typename Args>
    __device__ static int ext_c(const Args&) { return 1; }
    template <typename Args>
    __device__ __forceinline__ void init(const Args&) {}
    // A side: columns (fixed y) of TA elements along x
    static constexpr int LA = TA / VA, PA = pow2_ceil(LA), RA = NT / PA, NA = (TB + RA - 1) / RA;
    // B side: rows (fixed x) of TB elements along y
    static constexpr int LB = TB / VB, PB = pow2_ceil(LB), RB = NT / PB, NB = (TA + RB - 1) / RB;
    static_assert(PA <= NT && PB <= NT, "tile edge too long for the workgroup");

    vec_t<S, VA> ra[NA];
    vec_t<T, VB> rb[NB];
    vec_t<T, VB> out[NB];

    template <typename Args>
    __device__ __forceinline__ void load(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
        const Span sp = span(a, c);
        const int xa = (tid % PA) * VA, ya = tid / PA;
        const bool live_a = (tid % PA) < LA && xa < sp.hi && xa + VA > sp.lo;
        const S* pa = a.A + sp.oa + int64_t(xa) * a.sAa;
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (live_a && ya + i * RA < c.eb) {
                const S* p = pa + a.gB.offset(c.y0 + ya + i * RA);
                if constexpr (ALN == 0) {
                    ld_part<S, VA>(ra[i], p, sp.hi - xa);
                } else if (xa >= sp.lo) {
                    ld_part<S, VA>(ra[i], p, sp.hi - xa);
                } else {   // a vector that starts before x = 0: its elements from x = 0 on
#pragma unroll
                    for (int j = 0; j < VA; ++j)
                        if (xa + j >= sp.lo && xa + j < sp.hi) set_lane<S, VA>(ra[i], j, p[j]);
                }
            }
        if constexpr (!BETA0) {
            const int yb = (tid % PB) * VB, xb = tid / PB;
            const bool live_b = (tid % PB) < LB && yb < c.eb;
            const int64_t off_b = c.ob + int64_t(yb) * a.sBb;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int x = xb + i * RB;
                if (live_b && x >= sp.lo && x < sp.hi)
                    ld_part<T, VB>(rb[i], a.Bsrc + off_b + a.gA.offset(sp.x0 + x), c.eb - yb);
            }
        }
    }

    template <typename Args>
    __device__ __forceinline__ void to_lds(T* __restrict__ lds, const Args&, const TileCoord& c) {
        const int tid = threadIdx.x;
        const int xa = (tid % PA) * VA, ya = tid / PA;
        if ((tid % PA) >= LA) return;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int y = ya + i * RA;
            if (y < TB) {
#pragma unroll
                for (int j = 0; j < VA; ++j) lds[y * LDR + xa + j] = conv<T, S>(lane<S, VA>(ra[i], j));
            }
        }
    }

    template <typename Args>
    __device__ __forceinline__ void from_lds(const T* __restrict__ lds, const Args& a,
                                             const TileCoord& c) {
        const int tid = threadIdx.x;
        const Span sp = span(a, c);
        const int yb = (tid % PB) * VB, xb = tid / PB;
        const bool live_b = (tid % PB) < LB && yb < c.eb;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int x = xb + i * RB;
            if (live_b && x >= sp.lo && x < sp.hi) {
                vec_t<T, VB> v;
#pragma unroll
                for (int j = 0; j < VB; ++j) set_lane<T, VB>(v, j, lds[(yb + j) * LDR + x]);
                out[i] = epilogue<T, VB, BETA0>(v, rb[i], a.alpha, a.beta);
            }
        }
    }

    template <typename Args>
    __device__ __forceinline__ void store(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
        const Span sp = span(a, c);
        const int yb = (tid % PB) * VB, xb = tid / PB;
        const bool live_b = (tid % PB) < LB && yb < c.eb;
        constexpr bool nt = nt_of<NTS, Args>();
        const int64_t off_b = c.ob + int64_t(yb) * a.sBb;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int x = xb + i * RB;
            if (live_b && x >= sp.lo && x < sp.hi)
                st_part<T, VB, nt>(a.Bdst + off_b + a.gA.offset(sp.x0 + x), out[i], c.eb - yb);
        }
    }

    // from_lds and store in one pass (no tile held in registers in between)
    template <typename Args>
    __device__ __forceinline__ void read_store(const T* __restrict__ lds, const Args& a,
                                               const TileCoord& c) {
        const int tid = threadIdx.x;
        const Span sp = span(a, c);
        const int yb = (tid % PB) * VB, xb = tid / PB;
        const bool live_b = (tid % PB) < LB && yb < c.eb;
        constexpr bool nt = nt_of<NTS, Args>();
        const int64_t off_b = c.ob + int64_t(yb) * a.sBb;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int x = xb + i * RB;
            if (live_b && x >= sp.lo && x < sp.hi) {
                vec_t<T, VB> v;
#pragma unroll
                for (int j = 0; j < VB; ++j) set_lane<T, VB>(v, j, lds[(yb + j) * LDR + x]);
                st_part<T, VB, nt>(a.Bdst + off_b + a.gA.offset(sp.x0 + x), epilogue<T, VB, BETA0>(v, rb[i], a.alpha, a.beta),
                               c.eb - yb);
            }
        }
    }
};

// One preserved-family tile: rows of ea elements contiguous in A and B.
// Row y < eb starts at A[oa + y*sAb] and B[ob + y*sBb]; element x of a row is
// at x*sAa / x*sBa (V > 1 implies sAa == sBa == 1).  No LDS.  NTH threads.
template <typename T, bool BETA0, int TA, int TR, int V, typename S = T, int NTS = -1, int NTH = kThreads>
struct PreservedTile {
    static constexpr bool kUsesLds = false;
    static constexpr int kTA = TA, kTB = TR;
    static constexpr int NT = NTH;
    template <typename Args>
    __device__ static int ext_a(const Args&) { return TA; }
    template <typename Args>
    __device__ static int ext_b(const Args&) { return TR; }
    template <typename Args>
    __device__ static int ext_c(const Args&) { return 1; }
    template <typename Args>
    __device__ __forceinline__ void init(const Args&) {}
    static constexpr int L = TA / V, P = pow2_ceil(L), R = NT / P, N = (TR + R - 1) / R;
    static_assert(P <= NT, "row too long for the workgroup");

    vec_t<S, V> ra[N];
    vec_t<T, V> rb[N];
    vec_t<T, V> out[N];

    template <typename Args>
    __device__ __forceinline__ void load(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
        const int x = (tid % P) * V, y0 = tid / P;
        const bool live = (tid % P) < L && x < c.ea;
        const int64_t off_a = c.oa + int64_t(x) * a.sAa + int64_t(y0) * a.sAb;
        const int64_t off_b = c.ob + int64_t(x) * a.sBa + int64_t(y0) * a.sBb;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if (live && y0 + i * R < c.eb) {
                ld_part<S, V>(ra[i], a.A + off_a + i * int64_t(R) * a.sAb, c.ea - x);
                if constexpr (!BETA0) ld_part<T, V>(rb[i], a.Bsrc + off_b + i * int64_t(R) * a.sBb, c.ea - x);
            }
        }
    }

    template <typename Args>
    __device__ __forceinline__ void finish(const Args& a, const TileCoord& c) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = epilogue<T, V, BETA0>(conv_vec<T, S, V>(ra[i]), rb[i], a.alpha, a.beta);
    }

    template <typename Args>
    __device__ __forceinline__ void store(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
        const int x = (tid % P) * V, y0 = tid / P;
        const bool live = (tid % P) < L && x < c.ea;
        constexpr bool nt = nt_of<NTS, Args>();
        const int64_t off_b = c.ob + int64_t(x) * a.sBa + int64_t(y0) * a.sBb;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (live && y0 + i * R < c.eb) st_part<T, V, nt>(a.Bdst + off_b + i * int64_t(R) * a.sBb, out[i], c.ea - x);
    }

    // finish and store in one pass
    template <typename Args>
    __device__ __forceinline__ void finish_store(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
        const int x = (tid % P) * V, y0 = tid / P;
        const bool live = (tid % P) < L && x < c.ea;
        constexpr bool nt = nt_of<NTS, Args>();
        const int64_t off_b = c.ob + int64_t(x) * a.sBa + int64_t(y0) * a.sBb;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (live && y0 + i * R < c.eb)
                st_part<T, V, nt>(a.Bdst + off_b + i * int64_t(R) * a.sBb,
                              epilogue<T, V, BETA0>(conv_vec<T, S, V>(ra[i]), rb[i], a.alpha, a.beta), c.ea - x);
    }
};

// One staged preserved-family tile, for short stride-1 rows: rows of n0
// (<= N0) elements are contiguous in both tensors; the tile holds TX rows
// along A's super index x (A's indices after the row index, contiguous in A)
// for each of TY rows along B's super index y (B's indices after the row
// index, contiguous in B).  Element (i, x0 + x, y0 + y) is
//   A[oa + i*s0A + x*sAa + gB.offset(y0 + y)] -> B[ob + i*s0B + y*sBb + gA.offset(x0 + x)].
// A is read in runs of n0*TX elements and B written in runs of n0*TY; the
// tile passes through LDS as [y][x][i] (row length TX*N0 + PAD).  NTH threads.
template <typename T, bool BETA0, int N0, int TX, int TY, typename S = T, int NTS = -1, int NTH = kThreads,
          int PAD = 1>
struct StagedTile {
    static constexpr bool kUsesLds = true;
    static constexpr int kTA = TX, kTB = TY;
    static constexpr int NT = NTH, LDR = TX * N0 + PAD;
    template <typename Args>
    __device__ static int ext_a(const Args&) { return TX; }
    template <typename Args>
    __device__ static int ext_b(const Args&) { return TY; }
    template <typename Args>
    __device__ static int ext_c(const Args&) { return 1; }
    template <typename Args>
    __device__ __forceinline__ void init(const Args&) {}
    // padded runs: N0 lanes per row, TX rows per A run, TY rows per B run
    static constexpr int PA = N0 * TX, PB = N0 * TY;
    static constexpr int NA = PA * TY / NT, NB = PB * TX / NT;
    static_assert((N0 & (N0 - 1)) == 0 && (PA & (PA - 1)) == 0 && (PB & (PB - 1)) == 0, "powers of two");
    static_assert(PA * TY % NT == 0, "whole passes");

    S ra[NA];
    T rb[NB];
    T out[NB];
    int n0_ = 0;

    template <typename Args>
    __device__ __forceinline__ void load(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x, n0 = a.n0;
        n0_ = n0;
        const S* A0 = a.A + c.oa;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + i * NT, r = e % PA, y = e / PA;
            const int iv = r % N0, x = r / N0;
            if (iv < n0 && x < c.ea && y < c.eb)
                ra[i] = A0[int64_t(iv) * a.s0A + int64_t(x) * a.sAa + a.gB.offset(c.y0 + y)];
        }
        if constexpr (!BETA0) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int e = tid + i * NT, r = e % PB, x = e / PB;
                const int iv = r % N0, y = r / N0;
                if (iv < n0 && y < c.eb && x < c.ea)
                    rb[i] = a.Bsrc[c.ob + int64_t(iv) * a.s0B + int64_t(y) * a.sBb + a.gA.offset(c.x0 + x)];
            }
        }
    }

    template <typename Args>
    __device__ __forceinline__ void to_lds(T* __restrict__ lds, const Args&, const TileCoord& c) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + i * NT, r = e % PA, y = e / PA;
            const int iv = r % N0, x = r / N0;
            if (iv < n0_) lds[y * LDR + x * N0 + iv] = conv<T, S>(ra[i]);
        }
    }

    template <typename Args>
    __device__ __forceinline__ void from_lds(const T* __restrict__ lds, const Args& a,
                                             const TileCoord& c) {
        const int tid = threadIdx.x, n0 = a.n0;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * NT, r = e % PB, x = e / PB;
            const int iv = r % N0, y = r / N0;
            if (iv < n0 && y < c.eb && x < c.ea)
                out[i] = epilogue<T, 1, BETA0>(lds[y * LDR + x * N0 + iv], rb[i], a.alpha, a.beta);
        }
    }

    template <typename Args>
    __device__ __forceinline__ void store(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x, n0 = a.n0;
        constexpr bool nt = nt_of<NTS, Args>();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * NT, r = e % PB, x = e / PB;
            const int iv = r % N0, y = r / N0;
            if (iv < n0 && y < c.eb && x < c.ea)
                st<T, 1, nt>(a.Bdst + c.ob + int64_t(iv) * a.s0B + int64_t(y) * a.sBb + a.gA.offset(c.x0 + x),
                         out[i]);
        }
    }

    // from_lds and store in one pass
    template <typename Args>
    __device__ __forceinline__ void read_store(const T* __restrict__ lds, const Args& a,
                                               const TileCoord& c) {
        const int tid = threadIdx.x, n0 = a.n0;
        constexpr bool nt = nt_of<NTS, Args>();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * NT, r = e % PB, x = e / PB;
            const int iv = r % N0, y = r / N0;
            if (iv < n0 && y < c.eb && x < c.ea) {
                const T v = lds[y * LDR + x * N0 + iv];
                st<T, 1, nt>(a.Bdst + c.ob + int64_t(iv) * a.s0B + int64_t(y) * a.sBb + a.gA.offset(c.x0 + x),
                         epilogue<T, 1, BETA0>(v, rb[i], a.alpha, a.beta));
            }
        }
    }
};

// One dense tile: rows of n0 = dn0 elements (the shared stride-1 index of
// the preserved family; n0 = 1 for the moved family), tx rows along A's super
// index x and ty rows along B's super index y, and tz planes along a third
// index z, with tx, ty, tz run-time values and n0 * tx * ty * tz <= CAP.
// Element (i, x0 + x, y0 + y, z) is
//   A[oa + i*s0A + x*sAa + gB.offset(y0 + y) + z*sAz]
//     -> B[ob + i*s0B + y*sBb + gA.offset(x0 + x) + z*sBz].
// Slot e of the tile (e = tid + s*NT) is read in A order (i, x, y, z: plane
// z = e / planeA, then y and i + n0*x within runs of runA) and written in B
// order (i, y, x, z: runs of runB), so that both sides run along their
// contiguous index without padding lanes to a power of two.  The tile passes
// through LDS as [z][y][x][i], rows of ldr >= runA elements (odd when possible).
// NTH threads, CAP / NTH slots each.
template <typename T, bool BETA0, int CAP, typename S = T, int NTS = -1, int NTH = kThreads>
struct DenseTile {
    static constexpr bool kUsesLds = true;
    static constexpr int NT = NTH, NS = CAP / NT;
    static_assert(CAP % NT == 0 && CAP <= 1024, "whole passes; slot coordinates packed in 11+11+10 bits");
    template <typename Args>
    __device__ static int ext_a(const Args& a) { return a.tx; }
    template <typename Args>
    __device__ static int ext_b(const Args& a) { return a.ty; }
    template <typename Args>
    __device__ static int ext_c(const Args& a) { return a.tz; }

    S ra[NS];
    T rb[NS];
    T out[NS];
    // Per-slot constants (the same for every tile of a problem): offsets
    // within the tile in A and B (a group with one member is linear and is
    // folded in), LDS indices, and the slot's (x, y, z) packed as
    // x | y << 11 | z << 22 (all ones: beyond the tile).
    int32_t relA[NS], relB[NS];
    uint32_t la[NS], lb[NS];
    uint32_t pa[NS], pb[NS];

    template <typename Args>
    __device__ __forceinline__ void init(const Args& a) {
        const uint32_t tid = threadIdx.x;
        const uint32_t count = a.planeA * uint32_t(a.tz);
        const int64_t ya = a.gB.ng == 1 ? a.gB.stride[0] : 0;   // A stride of y when linear
        const int64_t xb = a.gA.ng == 1 ? a.gA.stride[0] : 0;   // B stride of x when linear
        const uint32_t n0 = uint32_t(a.dn0), ty = uint32_t(a.ty), ldr = uint32_t(a.ldr);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint32_t e = tid + s * NT;
            // A order: i fastest, then x (runs of runA), y, z
            uint32_t z = a.dvPA.div(e);
            uint32_t rem = e - z * a.planeA;
            uint32_t y = a.dvA.div(rem);
            uint32_t r = rem - y * a.runA;
            uint32_t x = a.dv0.div(r);
            uint32_t i = r - x * n0;
            la[s] = (z * ty + y) * ldr + r;
            relA[s] = int32_t(int64_t(i) * a.s0A + int64_t(x) * a.sAa + int64_t(z) * a.sAz + int64_t(y) * ya);
            pa[s] = e < count ? (x | y << 11 | z << 22) : 0xffffffffu;
            // B order: i fastest, then y (runs of runB), x, z
            z = a.dvPB.div(e);
            rem = e - z * a.planeB;
            x = a.dvB.div(rem);
            r = rem - x * a.runB;
            y = a.dv0.div(r);
            i = r - y * n0;
            lb[s] = (z * ty + y) * ldr + x * n0 + i;
            relB[s] = int32_t(int64_t(i) * a.s0B + int64_t(y) * a.sBb + int64_t(z) * a.sBz + int64_t(x) * xb);
            pb[s] = e < count ? (x | y << 11 | z << 22) : 0xffffffffu;
        }
    }
    __device__ __forceinline__ static bool inside(const TileCoord& c, uint32_t p) {
        return (p & 2047u) < uint32_t(c.ea) && ((p >> 11) & 2047u) < uint32_t(c.eb) && (p >> 22) < uint32_t(c.ez);
    }
    // A and B addresses of slot s in tile c
    template <typename Args>
    __device__ __forceinline__ const S* a_ptr(const Args& a, const TileCoord& c, int s) const {
        if (a.gB.ng == 1) return a.A + (c.oa + c.y0 * a.gB.stride[0]) + relA[s];
        return a.A + c.oa + relA[s] + a.gB.offset(c.y0 + ((pa[s] >> 11) & 2047u));
    }
    template <typename Args>
    __device__ __forceinline__ int64_t b_off(const Args& a, const TileCoord& c, int s) const {
        if (a.gA.ng == 1) return c.ob + c.x0 * a.gA.stride[0] + relB[s];
        return c.ob + relB[s] + a.gA.offset(c.x0 + (pb[s] & 2047u));
    }

    template <typename Args>
    __device__ __forceinline__ void load(const Args& a, const TileCoord& c) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (inside(c, pa[s])) ra[s] = *a_ptr(a, c, s);
        if constexpr (!BETA0) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (inside(c, pb[s])) rb[s] = a.Bsrc[b_off(a, c, s)];
        }
    }

    template <typename Args>
    __device__ __forceinline__ void to_lds(T* __restrict__ lds, const Args&, const TileCoord& c) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (inside(c, pa[s])) lds[la[s]] = conv<T, S>(ra[s]);
    }

    template <typename Args>
    __device__ __forceinline__ void from_lds(const T* __restrict__ lds, const Args& a,
                                             const TileCoord& c) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (inside(c, pb[s])) out[s] = epilogue<T, 1, BETA0>(lds[lb[s]], rb[s], a.alpha, a.beta);
    }

    template <typename Args>
    __device__ __forceinline__ void store(const Args& a, const TileCoord& c) {
        constexpr bool nt = nt_of<NTS, Args>();
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (inside(c, pb[s])) st<T, 1, nt>(a.Bdst + b_off(a, c, s), out[s]);
    }

    template <typename Args>
    __device__ __forceinline__ void read_store(const T* __restrict__ lds, const Args& a,
                                               const TileCoord& c) {
        constexpr bool nt = nt_of<NTS, Args>();
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (inside(c, pb[s]))
                st<T, 1, nt>(a.Bdst + b_off(a, c, s), epilogue<T, 1, BETA0>(lds[lb[s]], rb[s], a.alpha, a.beta));
    }
};

// LDS elements of a dense tile: tz*ty rows of ldr <= runA + 1 elements, with
// runA * ty * tz <= CAP.
constexpr int dense_lds_elems(int cap) { return 2 * cap; }

// One flat tile (everything merged into one index): TF consecutive elements,
// V-element vectors (V > 1 needs unit strides and an element count that is
// a multiple of V), U vectors per thread.  No LDS.
template <typename T, bool BETA0, int V, int U, int NTS = -1>
struct FlatTile {
    static constexpr bool kUsesLds = false;
    static constexpr int NT = kThreads, TF = NT * V * U;
    template <typename Args>
    __device__ static int ext_a(const Args&) { return TF; }
    template <typename Args>
    __device__ static int ext_b(const Args&) { return 1; }
    template <typename Args>
    __device__ static int ext_c(const Args&) { return 1; }
    template <typename Args>
    __device__ __forceinline__ void init(const Args&) {}

    vec_t<T, V> ra[U];
    vec_t<T, V> rb[U];
    vec_t<T, V> out[U];

    template <typename Args>
    __device__ __forceinline__ void load(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = (tid + u * NT) * V;
            if (k < c.ea) {
                ra[u] = ld<T, V>(a.A + c.oa + int64_t(k) * a.sAa);
                if constexpr (!BETA0) rb[u] = ld<T, V>(a.Bsrc + c.ob + int64_t(k) * a.sBa);
            }
        }
    }
    template <typename Args>
    __device__ __forceinline__ void finish(const Args& a, const TileCoord&) {
#pragma unroll
        for (int u = 0; u < U; ++u) out[u] = epilogue<T, V, BETA0>(ra[u], rb[u], a.alpha, a.beta);
    }
    template <typename Args>
    __device__ __forceinline__ void store(const Args& a, const TileCoord& c) {
        const int tid = threadIdx.x;
        constexpr bool nt = nt_of<NTS, Args>();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = (tid + u * NT) * V;
            if (k < c.ea) st<T, V, nt>(a.Bdst + c.ob + int64_t(k) * a.sBa, out[u]);
        }
    }
    template <typename Args>
    __device__ __forceinline__ void finish_store(const Args& a, const TileCoord& c) {
        finish(a, c);
        store(a, c);
    }
};

// Tiles t, t + step, ... < end of one problem.  With PIPE, tile k+1's loads
// are issued between tile k's LDS read and its stores, as described above;
// this holds two tiles' data in registers at once, so it is used where the
// register budget allows.  Every thread of the workgroup runs the same trip
// count (t, end, step are uniform), so the barriers are reached by all.
template <class Tile, bool PIPE, typename T, typename Args>
__device__ __forceinline__ void tile_loop(T* __restrict__ lds, const Args& a, uint32_t t,
                                          uint32_t end, uint32_t step) {
    Tile tile;
    tile.init(a);
    if constexpr (!PIPE) {
        for (uint64_t u = t; u < end; u += step) {
            const TileCoord c = decode_tile(a.g, uint32_t(u), Tile::ext_a(a), Tile::ext_b(a), Tile::ext_c(a));
            tile.load(a, c);
            if constexpr (Tile::kUsesLds) {
                tile.to_lds(lds, a, c);
                __syncthreads();
                tile.read_store(lds, a, c);
                __syncthreads();   // the next tile rewrites the LDS tile
            } else {
                tile.finish_store(a, c);
            }
        }
    } else {
        TileCoord c = decode_tile(a.g, t, Tile::ext_a(a), Tile::ext_b(a), Tile::ext_c(a));
        tile.load(a, c);
        while (true) {
            if constexpr (Tile::kUsesLds) {
                tile.to_lds(lds, a, c);
                __syncthreads();
                tile.from_lds(lds, a, c);
            } else {
                tile.finish(a, c);
            }
            const uint64_t tn = uint64_t(t) + step;
            const bool more = tn < end;
            TileCoord cn = c;
            if (more) {
                cn = decode_tile(a.g, uint32_t(tn), Tile::ext_a(a), Tile::ext_b(a), Tile::ext_c(a));
                tile.load(a, cn);
            }
            tile.store(a, c);
            if constexpr (Tile::kUsesLds) __syncthreads();   // the LDS tile is rewritten next
            if (!more) break;
            c = cn;
            t = uint32_t(tn);
        }
    }
}

// The kernel body shared by the generic kernels and the size-specialised
// ones: workgroup b takes tiles b, b + G, ... (G workgroups; ids permuted
// XCD-aware when KF_SWIZZLE is set).
template <typename Tile, bool PIPE, typename T, typename Args>
__device__ __forceinline__ void run_grid(T* lds, const Args& a) {
    const uint32_t G = gridDim.x;
    const uint32_t first = (a.flags & KF_SWIZZLE) ? swizzle_id(blockIdx.x, G) : blockIdx.x;
    if (first < a.g.ntiles) tile_loop<Tile, PIPE>(lds, a, first, a.g.ntiles, G);
}

// Arguments of a size-specialised kernel (compiled at run time for one
// problem): the problem-dependent part is the compile-time constant H, so
// every extent, stride, tile count and divisor that the tile code reads
// folds into the instructions, and loops over merged indices and group
// members unroll; the pointers and scalars are run-time values.  The
// members mirror TileArgs (a member added to TileArgsHost is added here).
template <const TileArgsHost& H, typename T, typename S, int FLAGS>
struct ConstArgs {
    static constexpr const TileGrid& g = H.g;
    static constexpr int64_t sAa = H.sAa, sAb = H.sAb, sBa = H.sBa, sBb = H.sBb;
    static constexpr const Group& gA = H.gA;
    static constexpr const Group& gB = H.gB;
    static constexpr int64_t s0A = H.s0A, s0B = H.s0B;
    static constexpr int n0 = H.n0, dn0 = H.dn0, tx = H.tx, ty = H.ty, ldr = H.ldr;
    static constexpr uint32_t runA = H.runA, runB = H.runB;
    static constexpr const FastDiv& dv0 = H.dv0;
    static constexpr const FastDiv& dvA = H.dvA;
    static constexpr const FastDiv& dvB = H.dvB;
    static constexpr int tz = H.tz;
    static constexpr int64_t sAz = H.sAz, sBz = H.sBz;
    static constexpr uint32_t planeA = H.planeA, planeB = H.planeB;
    static constexpr const FastDiv& dvPA = H.dvPA;
    static constexpr const FastDiv& dvPB = H.dvPB;
    static constexpr int flags = FLAGS;
    const S* A;
    const T* Bsrc;
    T* Bdst;
    T alpha, beta;
};

// Body of a size-specialised kernel: the generic body over ConstArgs.
template <typename Tile, bool PIPE, const TileArgsHost& H, int FLAGS, typename T, typename S>
__device__ __forceinline__ void run_specialised(T* lds, const TileArgs<T, S>& in) {
    const ConstArgs<H, T, S, FLAGS> a{in.A, in.Bsrc, in.Bdst, in.alpha, in.beta};
    run_grid<Tile, PIPE>(lds, a);
}

// Vector widths are template parameters so that each variant gets its own
// register allocation: the scalar fallbacks need many more address
// registers than the 16-byte paths and would otherwise lower the occupancy
// of every variant.  Scalar variants ask for at least 4 waves per SIMD.
template <typename T, bool BETA0, int TA, int TB, int VA, int VB, bool NT>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(VA == 1 || VB == 1 ? 4 : 1)))
void k_moved(TileArgs<T> a) {
    __shared__ T lds[TB * (TA + 1)];
    run_grid<MovedTile<T, BETA0, TA, TB, VA, VB, T, NT>, false>(lds, a);
}

template <typename T, bool BETA0, int TA, int TR, int V, bool NT>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(V == 1 ? 4 : 1)))
void k_preserved(TileArgs<T> a) {
    run_grid<PreservedTile<T, BETA0, TA, TR, V, T, NT>, false>(static_cast<T*>(nullptr), a);
}

// Launched with about one wave of workgroups, each looping over tiles
// (pipelined): the per-slot offsets are computed once per workgroup.
template <typename T, bool BETA0, int CAP, bool NT>
__global__ __launch_bounds__(kThreads) void k_dense(TileArgs<T> a) {
    __shared__ T lds[dense_lds_elems(CAP)];
    run_grid<DenseTile<T, BETA0, CAP, T, NT>, true>(lds, a);
}

template <typename T, bool BETA0, int N0, int TX, int TY, bool NT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_staged(TileArgs<T> a) {
    __shared__ T lds[TY * (TX * N0 + 1)];
    run_grid<StagedTile<T, BETA0, N0, TX, TY, T, NT>, false>(lds, a);
}

// Mixed precision (A of type S, B of type T): the same tiles, converting
// A's elements to T as they are loaded.
template <typename T, typename S, bool BETA0, int TA, int TB, int VA, int VB, bool NT>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(VA == 1 || VB == 1 ? 4 : 1)))
void k_moved_x(TileArgs<T, S> a) {
    __shared__ T lds[TB * (TA + 1)];
    run_grid<MovedTile<T, BETA0, TA, TB, VA, VB, S, NT>, false>(lds, a);
}

template <typename T, typename S, bool BETA0, int TA, int TR, int V, bool NT>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(V == 1 ? 4 : 1)))
void k_preserved_x(TileArgs<T, S> a) {
    run_grid<PreservedTile<T, BETA0, TA, TR, V, S, NT>, false>(static_cast<T*>(nullptr), a);
}

template <typename T, typename S, bool BETA0, int CAP, bool NT>
__global__ __launch_bounds__(kThreads) void k_dense_x(TileArgs<T, S> a) {
    __shared__ T lds[dense_lds_elems(CAP)];
    run_grid<DenseTile<T, BETA0, CAP, S, NT>, true>(lds, a);
}

template <typename T, typename S, bool BETA0, int N0, int TX, int TY, bool NT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_staged_x(TileArgs<T, S> a) {
    __shared__ T lds[TY * (TX * N0 + 1)];
    run_grid<StagedTile<T, BETA0, N0, TX, TY, S, NT>, false>(lds, a);
}

// Flat: one index of n elements with strides sa, sb.  The vector path
// (contiguous, aligned) moves 4 vectors per thread per iteration; the
// remaining n % V elements are handled one per thread.  V counts elements
// of both A and B (the smaller of their 16-byte widths).
template <typename T, typename S, bool BETA0, bool NT>
__device__ __forceinline__ void flat_body(const FlatArgs<T, S>& a) {
    constexpr int V = kVec<T> < kVec<S> ? kVec<T> : kVec<S>;
    constexpr int U = 4;
    constexpr bool nt = NT;
    const int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t G = int64_t(gridDim.x) * kThreads;
    if (a.flags & KF_VEC_A) {
        const int64_t nv = a.n / V;
        for (int64_t base = gid; base < nv; base += G * U) {
            vec_t<S, V> va[U];
            vec_t<T, V> vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * G;
                if (i < nv) {
                    va[u] = ld<S, V>(a.A + i * V);
                    if constexpr (!BETA0) vb[u] = ld<T, V>(a.Bsrc + i * V);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * G;
                if (i < nv)
                    st<T, V, nt>(a.Bdst + i * V, epilogue<T, V, BETA0>(conv_vec<T, S, V>(va[u]), vb[u], a.alpha, a.beta));
            }
        }
        const int64_t i = nv * V + gid;
        if (i < a.n) {
            T b{};
            if constexpr (!BETA0) b = a.Bsrc[i];
            a.Bdst[i] = epilogue<T, 1, BETA0>(conv<T, S>(a.A[i]), b, a.alpha, a.beta);
        }
        return;
    }
    for (int64_t i = gid; i < a.n; i += G) {
        T b{};
        if constexpr (!BETA0) b = a.Bsrc[i * a.sb];
        a.Bdst[i * a.sb] = epilogue<T, 1, BETA0>(conv<T, S>(a.A[i * a.sa]), b, a.alpha, a.beta);
    }
}

template <typename T, bool BETA0, bool NT>
__global__ __launch_bounds__(kThreads) void k_flat(FlatArgs<T> a) {
    flat_body<T, T, BETA0, NT>(a);
}

template <typename T, typename S, bool BETA0, bool NT>
__global__ __launch_bounds__(kThreads) void k_flat_x(FlatArgs<T, S> a) {
    flat_body<T, S, BETA0, NT>(a);
}

}  // namespace ttx
