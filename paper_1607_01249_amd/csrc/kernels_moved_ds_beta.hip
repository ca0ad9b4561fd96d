// Moved-family kernel instantiations: A FP64, B FP32, beta != 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(float, double, false, ta, tb)
TTX_MOVED_TABLE(moved_rows_ds_beta, TTX_MOVED_MENU_F32)
