// The backward step on equal-probability cells (the second example of
// hypercubes under assumption (A_Strat): cells cut at the logistic quantiles,
// every cube of nu-probability 1/K), for the dimensions of the LDS kernels, in
// both precisions and every look-up mode; always with the clouds in global
// memory, so that the LDS kernels keep no code of this grid.
#include "srmdp_gr.hpp"

namespace srmdp {

template <typename R>
hipError_t launch_step_ep(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return dispatch_gr_d<R, DD, true>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        SRMDP_GR_FOR_EACH_D(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_step_ep<float>(int, const StepArgs<float> &, const LaunchShape &, int, int, const void *,
                                          const void *, void *, void *, void *, hipStream_t);
template hipError_t launch_step_ep<double>(int, const StepArgs<double> &, const LaunchShape &, int, int,
                                           const void *, const void *, void *, void *, void *, hipStream_t);

}  // namespace srmdp
