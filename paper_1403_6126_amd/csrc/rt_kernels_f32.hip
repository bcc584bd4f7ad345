// Step kernels with FP32 intensities and per-angle arithmetic (the
// temperature Newton solve, the per-cell sums across waves and the totals
// stay FP64).
#define RT_S float
#define RT_SUFFIX f32
#define RT_PACKED 1
#include "rt_kernels.inc"
