// A GEMM over matrix-core operand panels (ttx_pack with TTX_PACK_MFMA_A /
// TTX_PACK_MFMA_B): the consumer that the packing of Sec. 2.1 (Fig. 3)
// prepares operands for, and the contraction step of a transpose-transpose-
// GEMM-transpose tensor contraction.
//
// Each wave computes one panel x panel block of C with the gfx950 matrix
// instructions: for every block of kb = 64 / panel values of k, lane l loads
// element l of the left panel's block and element l of the right panel's
// block (64 consecutive elements each, already in the instruction's operand
// order) and issues one instruction.  Output registers hold C in the
// instructions' result order (checked on the device with a unique value per
// element of C):
//   16 x 16 x 4 FP32: register r of lane l is C(4*(l/16) + r, l%16);
//   16 x 16 x 4 FP64: register r of lane l is C(l/16 + 4*r, l%16);
//   32 x 32 x 2 FP32: register r of lane l is C(8*(r/4) + 4*(l/32) + r%4, l%32).
// The products are accumulated in the element type by the matrix cores.
#include <cstdint>

#include "ttx_internal.h"

namespace ttx {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int kGemmWaves = 4;   // waves (C blocks) per workgroup

// C blocks: p along m (panels of Pa), q along n (panels of Pb); block id
// = q * mp + p.  K is k rounded up to whole blocks of 64 / PANEL.
template <typename T, int PANEL>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm_panels(const T* __restrict__ Pa, const T* __restrict__ Pb,
                                                                 T* __restrict__ C, int64_t m, int64_t n, int64_t K,
                                                                 int64_t ldc, int64_t mp, int64_t blocks) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = int64_t(blockIdx.x) * kGemmWaves + (threadIdx.x >> 6);
    if (blk >= blocks) return;   // a whole wave leaves: no barrier follows
    const int64_t p = blk % mp, q = blk / mp;
    const T* a = Pa + p * PANEL * K + lane;
    const T* b = Pb + q * PANEL * K + lane;
    const int64_t nblk = K / (64 / PANEL);
    if constexpr (PANEL == 16) {
        using Acc = typename std::conditional<std::is_same<T, float>::value, f32x4_t, f64x4_t>::type;
        Acc acc = {0, 0, 0, 0};
        for (int64_t s = 0; s < nblk; ++s) {
            if constexpr (std::is_same<T, float>::value)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[64 * s], b[64 * s], acc, 0, 0, 0);
            else
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[64 * s], b[64 * s], acc, 0, 0, 0);
        }
        const int64_t col = q * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = std::is_same<T, float>::value ? p * 16 + 4 * (lane >> 4) + r
                                                              : p * 16 + (lane >> 4) + 4 * r;
            if (row < m && col < n) C[row + col * ldc] = acc[r];
        }
    } else {
        static_assert(PANEL == 32 && std::is_same<T, float>::value, "32 x 32 x 2 is an FP32 instruction");
        f32x16_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
        for (int64_t s = 0; s < nblk; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[64 * s], b[64 * s], acc, 0, 0, 0);
        const int64_t col = q * 32 + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = p * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (row < m && col < n) C[row + col * ldc] = acc[r];
        }
    }
}

hipError_t launch_gemm_panels(int dtype, int panel, int64_t m, int64_t n, int64_t k, const void* Pa,
                              const void* Pb, void* C, int64_t ldc, hipStream_t stream) {
    const int64_t kb = 64 / panel, K = (k + kb - 1) / kb * kb;
    const int64_t mp = (m + panel - 1) / panel, nq = (n + panel - 1) / panel, blocks = mp * nq;
    const int64_t grid = (blocks + kGemmWaves - 1) / kGemmWaves;
    if (grid > int64_t(0x7fffffff)) return hipErrorInvalidValue;
    const dim3 g{uint32_t(grid)}, t{64 * kGemmWaves};
    if (dtype == TTX_F32 && panel == 16)
        hipLaunchKernelGGL((k_gemm_panels<float, 16>), g, t, 0, stream, static_cast<const float*>(Pa),
                           static_cast<const float*>(Pb), static_cast<float*>(C), m, n, K, ldc, mp, blocks);
    else if (dtype == TTX_F32 && panel == 32)
        hipLaunchKernelGGL((k_gemm_panels<float, 32>), g, t, 0, stream, static_cast<const float*>(Pa),
                           static_cast<const float*>(Pb), static_cast<float*>(C), m, n, K, ldc, mp, blocks);
    else if (dtype == TTX_F64 && panel == 16)
        hipLaunchKernelGGL((k_gemm_panels<double, 16>), g, t, 0, stream, static_cast<const double*>(Pa),
                           static_cast<const double*>(Pb), static_cast<double*>(C), m, n, K, ldc, mp, blocks);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
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
