// Moved-family kernel instantiations: A double complex, B single complex, beta != 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(cf32, cf64, false, ta, tb)
TTX_MOVED_TABLE(moved_rows_zc_beta, TTX_MOVED_MENU_F64)
