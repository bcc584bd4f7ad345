// Wave-group step kernels, FP32 intensities, 2 angle groups per wave.
#define RT_S float
#define RT_SUFFIX f32
#define RT_NG 2
#define RT_PACKED 1
#include "rt_step3_inst.inc"
