// Moved-family kernel instantiations: FP64, beta == 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(double, double, true, ta, tb)
TTX_MOVED_TABLE(moved_rows_f64_beta0, TTX_MOVED_MENU_F64)
