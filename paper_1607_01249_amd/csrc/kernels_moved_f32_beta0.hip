// Moved-family kernel instantiations: FP32, beta == 0.
#include "moved_launch.h"

#define TTX_ENTRY(ta, tb) TTX_MOVED_ENTRY(float, float, true, ta, tb)
TTX_MOVED_TABLE(moved_rows_f32_beta0, TTX_MOVED_MENU_F32)
