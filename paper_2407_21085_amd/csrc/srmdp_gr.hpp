// Backward-step kernels for clouds too large for LDS: the same body as
// sweep_step_kernel (Algorithm SRMDP, eq. (PsiM)), with each stratum's cloud
// streamed through an LDS window in rounds (sweep_group, GR), S' and y_{i+1}
// of its samples in global memory, and the launch covering a range of strata
// (StepArgs::k0 .. k_end).
// Instantiated for equal-size cells in srmdp_kernels_gr.hip and for
// equal-probability cells (EP) in srmdp_kernels_ep.hip.
#pragma once
#include "srmdp_sweep.hpp"

namespace srmdp {

template <typename R, int D, int NB, int LK, bool EP>
__global__ void __launch_bounds__(256) sweep_step_gr_kernel(const StepArgs<R> a,
                                                           const CellF<R> *__restrict__ cellF,
                                                           const R *__restrict__ bsig, R *__restrict__ lk,
                                                           R *__restrict__ table,
                                                           unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<R, D, NB, LK, false, true, EP>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF, bsig, lk, table,
                                           counters, smem);
}

template <typename R, int D, int NB, int LK, bool EP>
static hipError_t launch_gr_impl(const StepArgs<R> &a, const LaunchShape &s, const void *cellF, const void *bsig,
                                 void *lk, void *table, void *counters, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_step_gr_kernel<R, D, NB, LK, EP>), dim3(s.blocks), dim3(s.threads), s.lds_bytes, st, a,
                       (const CellF<R> *)cellF, (const R *)bsig, (R *)lk, (R *)table,
                       (unsigned long long *)counters);
    return hipGetLastError();
}

#define SRMDP_GR_FOR_EACH_D(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8)

template <typename R, int D, bool EP>
static hipError_t dispatch_gr_d(const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode, const void *cf,
                                const void *bs, void *lk, void *tab, void *ctr, hipStream_t st)
{
    if (basis == 0) {
        if (lkmode == kLookupY) return launch_gr_impl<R, D, 1, kLookupY, EP>(a, s, cf, bs, lk, tab, ctr, st);
        if (lkmode == kLookupYZ) return launch_gr_impl<R, D, 1, kLookupYZ, EP>(a, s, cf, bs, lk, tab, ctr, st);
        return launch_gr_impl<R, D, 1, kLookupFull, EP>(a, s, cf, bs, lk, tab, ctr, st);
    }
    if (lkmode == kLookupY) return launch_gr_impl<R, D, D + 1, kLookupY, EP>(a, s, cf, bs, lk, tab, ctr, st);
    if (lkmode == kLookupYZ) return launch_gr_impl<R, D, D + 1, kLookupYZ, EP>(a, s, cf, bs, lk, tab, ctr, st);
    return launch_gr_impl<R, D, D + 1, kLookupFull, EP>(a, s, cf, bs, lk, tab, ctr, st);
}

}  // namespace srmdp
