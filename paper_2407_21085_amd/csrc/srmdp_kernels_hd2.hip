// The sweep for d = 13..16 (the paper's Tables LP1d13, LP1d14 and LP1d15_19
// up to d = 16); d = 7, 9..12 are in srmdp_kernels_hd.hip and d = 17..19 in
// srmdp_kernels_hd3.hip.
#define HD_DIMS(X) X(13) X(14) X(15) X(16)
#define HD_FN(name) name##2
#define HD_NEXT(name) name##3
#define HD_KERNEL sweep_step_hd2_kernel
#define HD_IMPL launch_hd2_impl

#include "srmdp_hd_body.hpp"
