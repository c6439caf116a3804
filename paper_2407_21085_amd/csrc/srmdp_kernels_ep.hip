// The backward step on equal-probability cells (the second example of
// hypercubes under assumption (A_Strat): cells cut at the logistic quantiles,
// every cube of nu-probability 1/K), for the dimensions of the LDS kernels, in
// both precisions and every look-up mode: the clouds in LDS
// (sweep_step_ep_kernel) or, when they do not fit, streamed (the body
// of srmdp_gr.hpp).  The other dimensions run the high-dimension kernels'
// equal-probability form.  The equal-size kernels keep no code of this grid.
#include "srmdp_gr.hpp"

namespace srmdp {

template <typename R, int D, int NB, int LK, int PF = 0>
__global__ void __launch_bounds__(256) sweep_step_ep_kernel(const StepArgs<R> a,
                                                           const CellF<R> *__restrict__ cellF,
                                                           const R *__restrict__ bsig, R *__restrict__ lk,
                                                           R *__restrict__ table,
                                                           unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<R, D, NB, LK, false, false, true, BuiltinModel, PF>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF,
                                                                    bsig, lk, table, counters, smem);
}

template <typename R, int D, int NB, int LK, int PF>
static hipError_t launch_ep_lds_pf(const StepArgs<R> &a, const LaunchShape &s, const void *cellF, const void *bsig,
                                   void *lk, void *table, void *counters, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_step_ep_kernel<R, D, NB, LK, PF>), dim3(s.blocks), dim3(s.threads), s.lds_bytes, st,
                       a, (const CellF<R> *)cellF, (const R *)bsig, (R *)lk, (R *)table,
                       (unsigned long long *)counters);
    return hipGetLastError();
}

template <typename R, int D, int NB, int LK>
static hipError_t launch_ep_lds_impl(const StepArgs<R> &a, const LaunchShape &s, const void *cellF,
                                     const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    // At most one gather in flight: the longer cell location of these cells
    // (a logistic CDF and a table read per coordinate) keeps the SIMDs busier,
    // and the third wavefront per SIMD is worth more than the second gather
    // (67.4 against 67.7 ms per sweep of the d = 8, K = 4^8, M = 64, N = 50
    // workload).
    if constexpr (sizeof(R) == 4) {
        if (prefetch_depth<R, D, NB, LK>(a) >= 1)
            return launch_ep_lds_pf<R, D, NB, LK, 1>(a, s, cellF, bsig, lk, table, counters, st);
    }
    return launch_ep_lds_pf<R, D, NB, LK, 0>(a, s, cellF, bsig, lk, table, counters, st);
}

template <typename R, int D>
static hipError_t dispatch_ep_lds_d(const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                                    const void *cf, const void *bs, void *lk, void *tab, void *ctr, hipStream_t st)
{
    if (basis == 0) {
        if (lkmode == kLookupY) return launch_ep_lds_impl<R, D, 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
        if (lkmode == kLookupYZ) return launch_ep_lds_impl<R, D, 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
        return launch_ep_lds_impl<R, D, 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
    }
    if (lkmode == kLookupY) return launch_ep_lds_impl<R, D, D + 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
    if (lkmode == kLookupYZ) return launch_ep_lds_impl<R, D, D + 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
    return launch_ep_lds_impl<R, D, D + 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
}

template <typename R>
hipError_t launch_step_ep_lds(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                              const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                              hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return dispatch_ep_lds_d<R, DD>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        SRMDP_GR_FOR_EACH_D(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_step_ep_lds<float>(int, const StepArgs<float> &, const LaunchShape &, int, int,
                                              const void *, const void *, void *, void *, void *, hipStream_t);
template hipError_t launch_step_ep_lds<double>(int, const StepArgs<double> &, const LaunchShape &, int, int,
                                               const void *, const void *, void *, void *, void *, hipStream_t);

template <typename R>
hipError_t launch_step_ep(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return dispatch_gr_d<R, DD, true>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        SRMDP_GR_FOR_EACH_D(X)
#undef X
    default: return launch_step_gr_hd<R>(d, a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
    }
}

template hipError_t launch_step_ep<float>(int, const StepArgs<float> &, const LaunchShape &, int, int, const void *,
                                          const void *, void *, void *, void *, hipStream_t);
template hipError_t launch_step_ep<double>(int, const StepArgs<double> &, const LaunchShape &, int, int,
                                           const void *, const void *, void *, void *, void *, hipStream_t);

}  // namespace srmdp
