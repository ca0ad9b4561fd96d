// Staged preserved-family kernel instantiations: double complex.
#include "staged_launch.h"

#define TTX_ENTRY_B(n0, tx, ty) TTX_STAGED_ENTRY(cf64, cf64, false, n0, tx, ty)
#define TTX_ENTRY_Z(n0, tx, ty) TTX_STAGED_ENTRY(cf64, cf64, true, n0, tx, ty)
TTX_STAGED_TABLE(staged_rows_c64, cf64, cf64, TTX_STAGED_MENU_C64)
