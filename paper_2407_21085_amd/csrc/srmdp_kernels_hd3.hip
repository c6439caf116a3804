// The sweep for d = 17..19 (the paper's Table LP1d15_19 from d = 17 on); the
// other dimensions without the LDS kernel are in srmdp_kernels_hd.hip and
// srmdp_kernels_hd2.hip.
#define HD_DIMS(X) X(17) X(18) X(19)
#define HD_FN(name) name##3
#define HD_NEXT(name) hd_none_##name
#define HD_KERNEL sweep_step_hd3_kernel
#define HD_IMPL launch_hd3_impl

#include <hip/hip_runtime.h>

namespace srmdp {
// Past the last high-dimension file: no such dimension.
template <typename R, typename... A>
static hipError_t hd_none(A...) { return hipErrorInvalidValue; }
}  // namespace srmdp
#define hd_none_launch_step_gr_hd hd_none
#define hd_none_launch_face_flags_hd hd_none
#define hd_none_launch_lookup_rows_hd hd_none
#define hd_none_launch_root_hd hd_none
#define hd_none_launch_eval_hd hd_none
#define hd_none_launch_draw_hd hd_none

#include "srmdp_hd_body.hpp"
