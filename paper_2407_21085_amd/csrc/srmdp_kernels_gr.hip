// Equal-size cells on the global-cloud kernels of srmdp_gr.hpp; the
// equal-probability grid goes to srmdp_kernels_ep.hip.
#include "srmdp_gr.hpp"

namespace srmdp {

template <typename R>
hipError_t launch_step_gr(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    if (a.equal_prob) return launch_step_ep<R>(d, a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
    switch (d) {
#define X(DD) \
    case DD: return dispatch_gr_d<R, DD, false>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        SRMDP_GR_FOR_EACH_D(X)
#undef X
    default: return launch_step_gr_hd<R>(d, a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
    }
}

template hipError_t launch_step_gr<float>(int, const StepArgs<float> &, const LaunchShape &, int, int, const void *,
                                          const void *, void *, void *, void *, hipStream_t);
template hipError_t launch_step_gr<double>(int, const StepArgs<double> &, const LaunchShape &, int, int,
                                           const void *, const void *, void *, void *, void *, hipStream_t);

}  // namespace srmdp
