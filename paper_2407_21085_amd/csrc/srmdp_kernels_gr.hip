// Backward-step kernels for clouds too large for LDS: the same body as
// sweep_step_kernel (Algorithm SRMDP, eq. (PsiM)), with each stratum's cloud
// rows and chunk sums in global memory and the launch covering a range of
// strata (StepArgs::k0 .. k_end).  Per stratum the rows are written once and
// read by the regression phases; against the path simulation that produced
// them this traffic is small (a few per cent at M in the thousands).
#include "srmdp_sweep.hpp"

namespace srmdp {

template <typename R, int D, int NB, int LK>
__global__ void __launch_bounds__(256) sweep_step_gr_kernel(const StepArgs<R> a,
                                                           const CellF<R> *__restrict__ cellF,
                                                           const R *__restrict__ bsig, R *__restrict__ lk,
                                                           R *__restrict__ table,
                                                           unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<R, D, NB, LK, false, true>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF, bsig, lk, table,
                                           counters, smem);
}

template <typename R, int D, int NB, int LK>
static hipError_t launch_gr_impl(const StepArgs<R> &a, const LaunchShape &s, const void *cellF, const void *bsig,
                                 void *lk, void *table, void *counters, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_step_gr_kernel<R, D, NB, LK>), dim3(s.blocks), dim3(s.threads), s.lds_bytes, st, a,
                       (const CellF<R> *)cellF, (const R *)bsig, (R *)lk, (R *)table,
                       (unsigned long long *)counters);
    return hipGetLastError();
}

#define SRMDP_GR_FOR_EACH_D(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8)

template <typename R, int D>
static hipError_t dispatch_gr_d(const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode, const void *cf,
                                const void *bs, void *lk, void *tab, void *ctr, hipStream_t st)
{
    if (basis == 0) {
        if (lkmode == kLookupY) return launch_gr_impl<R, D, 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
        if (lkmode == kLookupYZ) return launch_gr_impl<R, D, 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
        return launch_gr_impl<R, D, 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
    }
    if (lkmode == kLookupY) return launch_gr_impl<R, D, D + 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
    if (lkmode == kLookupYZ) return launch_gr_impl<R, D, D + 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
    return launch_gr_impl<R, D, D + 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
}

template <typename R>
hipError_t launch_step_gr(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return dispatch_gr_d<R, DD>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
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
