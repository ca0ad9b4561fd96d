// A GEMM over matrix-core operand panels (ttx_pack with TTX_PACK_MFMA_A /
// TTX_PACK_MFMA_B): the consumer that the packing of Sec. 2.1 (Fig. 3)
// prepares operands for, and the contraction step of a transpose-transpose-
// GEMM-transpose tensor contraction.
//
// Each wave computes WM x WN panel x panel blocks of C with the gfx950
// matrix instructions: for every block of kb = 64 / panel values of k, lane
// l loads element l of each left panel's block and element l of each right
// panel's block (64 consecutive elements each, already in the instruction's
// operand order) and issues one instruction per C block.  The instruction
// is given the right panel as its first operand and the left panel as its
// second, so it forms C^T: the result registers then run down C's columns
// (lane l holds row l mod panel of the block), and each store of one
// register writes whole column segments of the column-major C.  Result
// order of C^T (checked on the device with a unique value per element):
//   16 x 16 x 4 FP32: register r of lane l is C^T(4*(l/16) + r, l%16);
//   16 x 16 x 4 FP64: register r of lane l is C^T(l/16 + 4*r, l%16);
//   32 x 32 x 2 FP32: register r of lane l is C^T(8*(r/4) + 4*(l/32) + r%4, l%32).
// The k loop runs in chunks of kUnroll blocks whose operands are loaded one
// chunk ahead, so the loads of the next chunk are in flight while the
// current chunk's instructions run.  The products are accumulated in the
// element type by the matrix cores.
#include <cstdint>

#include "ttx_internal.h"

namespace ttx {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int kGemmWaves = 4;   // waves per workgroup
constexpr int kUnroll = 4;      // k blocks per chunk

template <typename T, int PANEL>
struct Mfma;
template <>
struct Mfma<float, 16> {
    using Acc = f32x4_t;
    static constexpr int kRegs = 4;
    __device__ static Acc step(float x, float y, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0); }
    // (row, column) of C held by register r of lane l
    __device__ static int row(int l, int) { return l & 15; }
    __device__ static int col(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mfma<float, 32> {
    using Acc = f32x16_t;
    static constexpr int kRegs = 16;
    __device__ static Acc step(float x, float y, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, c, 0, 0, 0); }
    __device__ static int row(int l, int) { return l & 31; }
    __device__ static int col(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
};
template <>
struct Mfma<double, 16> {
    using Acc = f64x4_t;
    static constexpr int kRegs = 4;
    __device__ static Acc step(double x, double y, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }
    __device__ static int row(int l, int) { return l & 15; }
    __device__ static int col(int l, int r) { return (l >> 4) + 4 * r; }
};

// Wave w of the grid takes the C blocks (pw*WM + i, qw*WN + j), i < WM,
// j < WN, with pw = w % mpw, qw = w / mpw; blocks past the panel counts
// (mp, nq) are skipped.  K is k rounded up to whole blocks of 64 / PANEL.
template <typename T, int PANEL, int WM, int WN>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm_panels(const T* __restrict__ Pa, const T* __restrict__ Pb,
                                                                 T* __restrict__ C, int64_t m, int64_t n, int64_t K,
                                                                 int64_t ldc, int64_t mp, int64_t nq, int64_t mpw,
                                                                 int64_t waves) {
    using M = Mfma<T, PANEL>;
    const int lane = threadIdx.x & 63;
    const int64_t w = int64_t(blockIdx.x) * kGemmWaves + (threadIdx.x >> 6);
    if (w >= waves) return;   // a whole wave leaves: no barrier follows
    const int64_t p0 = (w % mpw) * WM, q0 = (w / mpw) * WN;
    const T* a[WM];
    const T* b[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) a[i] = Pa + (p0 + i < mp ? p0 + i : p0) * PANEL * K + lane;
#pragma unroll
    for (int j = 0; j < WN; ++j) b[j] = Pb + (q0 + j < nq ? q0 + j : q0) * PANEL * K + lane;
    typename M::Acc acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < M::kRegs; ++r) acc[i][j][r] = T(0);
    const int64_t nblk = K / (64 / PANEL), nfull = nblk / kUnroll * kUnroll;
    T xa[kUnroll][WM], xb[kUnroll][WN];
    if (nfull > 0) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int i = 0; i < WM; ++i) xa[u][i] = a[i][64 * u];
#pragma unroll
            for (int j = 0; j < WN; ++j) xb[u][j] = b[j][64 * u];
        }
    }
    for (int64_t s = 0; s < nfull; s += kUnroll) {
        T ca[kUnroll][WM], cb[kUnroll][WN];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int i = 0; i < WM; ++i) ca[u][i] = xa[u][i];
#pragma unroll
            for (int j = 0; j < WN; ++j) cb[u][j] = xb[u][j];
        }
        if (s + kUnroll < nfull) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
                for (int i = 0; i < WM; ++i) xa[u][i] = a[i][64 * (s + kUnroll + u)];
#pragma unroll
                for (int j = 0; j < WN; ++j) xb[u][j] = b[j][64 * (s + kUnroll + u)];
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) acc[i][j] = M::step(cb[u][j], ca[u][i], acc[i][j]);
    }
    for (int64_t s = nfull; s < nblk; ++s) {
        T ca[WM], cb[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i) ca[i] = a[i][64 * s];
#pragma unroll
        for (int j = 0; j < WN; ++j) cb[j] = b[j][64 * s];
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) acc[i][j] = M::step(cb[j], ca[i], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int64_t row = (p0 + i) * PANEL + M::row(lane, 0);
        if (p0 + i >= mp || row >= m) continue;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (q0 + j >= nq) continue;
#pragma unroll
            for (int r = 0; r < M::kRegs; ++r) {
                const int64_t col = (q0 + j) * PANEL + M::col(lane, r);
                if (col < n) C[row + col * ldc] = acc[i][j][r];
            }
        }
    }
}

template <typename T, int PANEL, int WM, int WN>
hipError_t launch_gemm_as(int64_t m, int64_t n, int64_t K, const void* Pa, const void* Pb, void* C, int64_t ldc,
                          hipStream_t stream) {
    const int64_t mp = (m + PANEL - 1) / PANEL, nq = (n + PANEL - 1) / PANEL;
    const int64_t mpw = (mp + WM - 1) / WM, waves = mpw * ((nq + WN - 1) / WN);
    const int64_t grid = (waves + kGemmWaves - 1) / kGemmWaves;
    if (grid > int64_t(0x7fffffff)) return hipErrorInvalidValue;
    const dim3 g{uint32_t(grid)}, t{64 * kGemmWaves};
    hipLaunchKernelGGL((k_gemm_panels<T, PANEL, WM, WN>), g, t, 0, stream, static_cast<const T*>(Pa),
                       static_cast<const T*>(Pb), static_cast<T*>(C), m, n, K, ldc, mp, nq, mpw, waves);
    return hipGetLastError();
}

// 2 x 2 blocks per wave where that still leaves at least kBlockedWaves
// waves (four per SIMD); otherwise one block per wave, for parallelism.
constexpr int64_t kBlockedWaves = 4096;

template <typename T, int PANEL>
hipError_t launch_gemm_panel(int64_t m, int64_t n, int64_t K, const void* Pa, const void* Pb, void* C, int64_t ldc,
                             hipStream_t stream) {
    const int64_t mp = (m + PANEL - 1) / PANEL, nq = (n + PANEL - 1) / PANEL;
    if (((mp + 1) / 2) * ((nq + 1) / 2) >= kBlockedWaves)
        return launch_gemm_as<T, PANEL, 2, 2>(m, n, K, Pa, Pb, C, ldc, stream);
    return launch_gemm_as<T, PANEL, 1, 1>(m, n, K, Pa, Pb, C, ldc, stream);
}

hipError_t launch_gemm_panels(int dtype, int panel, int64_t m, int64_t n, int64_t k, const void* Pa,
                              const void* Pb, void* C, int64_t ldc, hipStream_t stream) {
    const int64_t kb = 64 / panel, K = (k + kb - 1) / kb * kb;
    if (dtype == TTX_F32 && panel == 16) return launch_gemm_panel<float, 16>(m, n, K, Pa, Pb, C, ldc, stream);
    if (dtype == TTX_F32 && panel == 32) return launch_gemm_panel<float, 32>(m, n, K, Pa, Pb, C, ldc, stream);
    if (dtype == TTX_F64 && panel == 16) return launch_gemm_panel<double, 16>(m, n, K, Pa, Pb, C, ldc, stream);
    return hipErrorInvalidValue;
}

}  // namespace ttx

using namespace ttx;

extern "C" ttx_status ttx_gemm_panels(ttx_dtype dtype, int panel, int64_t m, int64_t n, int64_t k, const void* Pa,
                                      const void* Pb, void* C, int64_t ldc, hipStream_t stream) {
    if (!((dtype == TTX_F32 && (panel == 16 || panel == 32)) || (dtype == TTX_F64 && panel == 16)))
        return fail(TTX_EUNSUPPORTED, "matrix-core GEMM: FP32 with panels of 16 or 32, FP64 with panels of 16");
    if (m < 0 || n < 0 || k < 0 || ldc < (m > 1 ? m : 1)) return fail(TTX_EINVAL, "negative extent or ldc < m");
    if (m == 0 || n == 0) return TTX_OK;
    if (!Pa || !Pb || !C) return fail(TTX_EINVAL, "NULL pointer");
    const uintptr_t es = uintptr_t(elem_bytes(dtype));
    if (reinterpret_cast<uintptr_t>(Pa) % es || reinterpret_cast<uintptr_t>(Pb) % es ||
        reinterpret_cast<uintptr_t>(C) % es)
        return fail(TTX_EINVAL, "pointer not aligned to the element size");
    const hipError_t e = launch_gemm_panels(dtype, panel, m, n, k, Pa, Pb, C, ldc, stream);
    return e == hipSuccess ? TTX_OK : fail(TTX_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
}
