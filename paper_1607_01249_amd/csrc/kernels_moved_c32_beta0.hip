// Moved-family kernel instantiations: single complex, beta == 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(cf32, cf32, true, ta, tb)
TTX_MOVED_TABLE(moved_rows_c32_beta0, TTX_MOVED_MENU_F64)
