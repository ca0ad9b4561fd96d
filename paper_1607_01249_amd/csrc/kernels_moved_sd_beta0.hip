// Moved-family kernel instantiations: A FP32, B FP64, beta == 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(double, float, true, ta, tb)
TTX_MOVED_TABLE(moved_rows_sd_beta0, TTX_MOVED_MENU_F64)
