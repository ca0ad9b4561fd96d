// Moved-family kernel instantiations: A single complex, B double complex, beta == 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(cf64, cf32, true, ta, tb)
TTX_MOVED_TABLE(moved_rows_cz_beta0, TTX_MOVED_MENU_C64)
