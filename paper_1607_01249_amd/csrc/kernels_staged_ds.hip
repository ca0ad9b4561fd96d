// Staged preserved-family kernel instantiations: A FP64, B FP32.
#include "staged_launch.h"

#define TTX_ENTRY_B(n0, tx, ty) TTX_STAGED_ENTRY(float, double, false, n0, tx, ty)
#define TTX_ENTRY_Z(n0, tx, ty) TTX_STAGED_ENTRY(float, double, true, n0, tx, ty)
TTX_STAGED_TABLE(staged_rows_ds, float, double, TTX_STAGED_MENU_F32)
