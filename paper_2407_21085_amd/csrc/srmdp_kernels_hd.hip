// The sweep for the dimensions without the LDS kernel, d = 7, 9, 10, 11 and 12
// (the paper's Tables LP0d11, LP1d11 and LP1d12); d = 13..16 are in
// srmdp_kernels_hd2.hip and d = 17..19 in srmdp_kernels_hd3.hip.  Binary32
// only, clouds streamed through LDS (at these dimensions and the paper's M the
// LP1 clouds are hundreds of KB per stratum), look-up modes Y and YZ, and every
// kernel around the sweep in both precisions.
#define HD_DIMS(X) X(7) X(9) X(10) X(11) X(12)
#define HD_FN(name) name
#define HD_NEXT(name) name##2
#define HD_KERNEL sweep_step_hd_kernel
#define HD_IMPL launch_hd_impl
#include "srmdp_hd_body.hpp"

namespace srmdp {

bool hd_dimension_compiled(int d)
{
    switch (d) {
    case 7: case 9: case 10: case 11: case 12: case 13: case 14: case 15: case 16: case 17: case 18: case 19:
        return true;
    default: return false;
    }
}

}  // namespace srmdp
