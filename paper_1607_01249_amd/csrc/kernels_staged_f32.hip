// Staged preserved-family kernel instantiations: FP32.
#include "staged_launch.h"

#define TTX_ENTRY_B(n0, tx, ty) TTX_STAGED_ENTRY(float, float, false, n0, tx, ty)
#define TTX_ENTRY_Z(n0, tx, ty) TTX_STAGED_ENTRY(float, float, true, n0, tx, ty)
TTX_STAGED_TABLE(staged_rows_f32, float, float, TTX_STAGED_MENU_F32)
