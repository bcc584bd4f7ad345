// Step kernels with FP64 intensities and arithmetic.  No packed persistent
// kernel: its FP64 instances spill registers; the serving runtime runs FP64
// requests through the per-step launches.
#define RT_S double
#define RT_SUFFIX f64
#define RT_PACKED 0
#include "rt_kernels.inc"
