// Moved-family kernel instantiations: double complex, beta == 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(cf64, cf64, true, ta, tb)
TTX_MOVED_TABLE(moved_rows_c64_beta0, TTX_MOVED_MENU_C64)
