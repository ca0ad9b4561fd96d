// Staged preserved-family kernel instantiations: FP64.
#include "staged_launch.h"

#define TTX_ENTRY_B(n0, tx, ty) TTX_STAGED_ENTRY(double, double, false, n0, tx, ty)
#define TTX_ENTRY_Z(n0, tx, ty) TTX_STAGED_ENTRY(double, double, true, n0, tx, ty)
TTX_STAGED_TABLE(staged_rows_f64, double, double, TTX_STAGED_MENU_F64)
