// Staged preserved-family kernel instantiations: A single complex, B double complex.
#include "staged_launch.h"

#define TTX_ENTRY_B(n0, tx, ty) TTX_STAGED_ENTRY(cf64, cf32, false, n0, tx, ty)
#define TTX_ENTRY_Z(n0, tx, ty) TTX_STAGED_ENTRY(cf64, cf32, true, n0, tx, ty)
TTX_STAGED_TABLE(staged_rows_cz, cf64, cf32, TTX_STAGED_MENU_C64)
