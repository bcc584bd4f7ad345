// Wave-group step kernels, FP64 intensities, 2 angle groups per wave.
#define RT_S double
#define RT_SUFFIX f64
#define RT_NG 2
#define RT_PACKED 0
#include "rt_step3_inst.inc"
