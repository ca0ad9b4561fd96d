// Kernel launcher tables: one row per instantiated tile shape.
#pragma once

#include "ttx_internal.h"

namespace ttx {

using TileLaunchFn = hipError_t (*)(const void* args, uint32_t grid, hipStream_t stream);

// fn[v]: v = vector variant, bit 0 = 16-byte accesses along A's tile index,
// bit 1 = along B's tile index (the preserved family uses 0 and 3 only),
// bit 2 = nontemporal stores to B.
// A variant a shape cannot use (its tile edge is not a multiple of the
// vector width) is instantiated with scalar accesses on that side.
struct LauncherRow {
    int ta, tb;
    TileLaunchFn fn[8];
};

int moved_rows_f32_beta(const LauncherRow** out);
int moved_rows_f32_beta0(const LauncherRow** out);
int moved_rows_f64_beta(const LauncherRow** out);
int moved_rows_f64_beta0(const LauncherRow** out);
int moved_rows_c32_beta(const LauncherRow** out);
int moved_rows_c32_beta0(const LauncherRow** out);
int moved_rows_c64_beta(const LauncherRow** out);
int moved_rows_c64_beta0(const LauncherRow** out);
int moved_rows_sd_beta(const LauncherRow** out);
int moved_rows_sd_beta0(const LauncherRow** out);
int moved_rows_ds_beta(const LauncherRow** out);
int moved_rows_ds_beta0(const LauncherRow** out);
int moved_rows_cz_beta(const LauncherRow** out);
int moved_rows_cz_beta0(const LauncherRow** out);
int moved_rows_zc_beta(const LauncherRow** out);
int moved_rows_zc_beta0(const LauncherRow** out);
// Rows for a data-type code (ttx_dtype: the element types of A and B).
inline int moved_rows(int code, bool beta0, const LauncherRow** out) {
    switch (code) {
        case TTX_F32: return beta0 ? moved_rows_f32_beta0(out) : moved_rows_f32_beta(out);
        case TTX_F64: return beta0 ? moved_rows_f64_beta0(out) : moved_rows_f64_beta(out);
        case TTX_C32: return beta0 ? moved_rows_c32_beta0(out) : moved_rows_c32_beta(out);
        case TTX_C64: return beta0 ? moved_rows_c64_beta0(out) : moved_rows_c64_beta(out);
        case TTX_F32_F64: return beta0 ? moved_rows_sd_beta0(out) : moved_rows_sd_beta(out);
        case TTX_F64_F32: return beta0 ? moved_rows_ds_beta0(out) : moved_rows_ds_beta(out);
        case TTX_C32_C64: return beta0 ? moved_rows_cz_beta0(out) : moved_rows_cz_beta(out);
        case TTX_C64_C32: return beta0 ? moved_rows_zc_beta0(out) : moved_rows_zc_beta(out);
        default: return 0;
    }
}
int preserved_rows(int code, bool beta0, const LauncherRow** out);

struct StagedRow {
    int n0_max, tx, ty;
    TileLaunchFn fn[2];   // [nontemporal stores]
};
int staged_rows_f32(bool beta0, const StagedRow** out);
int staged_rows_f64(bool beta0, const StagedRow** out);
int staged_rows_c32(bool beta0, const StagedRow** out);
int staged_rows_c64(bool beta0, const StagedRow** out);
int staged_rows_sd(bool beta0, const StagedRow** out);
int staged_rows_ds(bool beta0, const StagedRow** out);
int staged_rows_cz(bool beta0, const StagedRow** out);
int staged_rows_zc(bool beta0, const StagedRow** out);
inline int staged_rows(int code, bool beta0, const StagedRow** out) {
    switch (code) {
        case TTX_F32: return staged_rows_f32(beta0, out);
        case TTX_F64: return staged_rows_f64(beta0, out);
        case TTX_C32: return staged_rows_c32(beta0, out);
        case TTX_C64: return staged_rows_c64(beta0, out);
        case TTX_F32_F64: return staged_rows_sd(beta0, out);
        case TTX_F64_F32: return staged_rows_ds(beta0, out);
        case TTX_C32_C64: return staged_rows_cz(beta0, out);
        case TTX_C64_C32: return staged_rows_zc(beta0, out);
        default: return 0;
    }
}

// The dense-tile kernel for a data-type code and beta class, and the
// workgroups that fill the device with it (its launches loop over the tiles).
TileLaunchFn dense_launcher(int code, bool beta0, bool nt);
uint32_t dense_grid(int code, bool beta0);

}  // namespace ttx
