// Staged preserved-family kernel instantiations: A FP32, B FP64.
#include "staged_launch.h"

#define TTX_ENTRY_B(n0, tx, ty) TTX_STAGED_ENTRY(double, float, false, n0, tx, ty)
#define TTX_ENTRY_Z(n0, tx, ty) TTX_STAGED_ENTRY(double, float, true, n0, tx, ty)
TTX_STAGED_TABLE(staged_rows_sd, double, float, TTX_STAGED_MENU_F64)
