// Body of the high-dimension files (included by srmdp_kernels_hd.hip and
// srmdp_kernels_hd2.hip, which split the dimensions between two translation
// units so that they compile in parallel).  The including file defines
//   HD_DIMS(X)    the dimensions it compiles,
//   HD_FN(name)   the names of its launchers,
//   HD_NEXT(name) the launchers that take the other dimensions,
//   HD_KERNEL, HD_IMPL  names of its kernel and launch helper.
// Binary32 sweeps with streamed clouds, look-up modes Y and YZ, on equal-size
// or equal-probability cells; every kernel around the sweep in both
// precisions.
#include <type_traits>

#include "srmdp_aux.hpp"

namespace srmdp {

template <typename R, int D, int NB, int LK, bool EP>
__global__ void __launch_bounds__(256) HD_KERNEL(const StepArgs<R> a,
                                                           const CellF<R> *__restrict__ cellF,
                                                           const R *__restrict__ bsig, R *__restrict__ lk,
                                                           R *__restrict__ table,
                                                           unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<R, D, NB, LK, false, true, EP>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF, bsig, lk, table,
                                               counters, smem);
}

// Equal-size or equal-probability cells (StepArgs::equal_prob).
template <int D, int NB, int LK>
static hipError_t HD_IMPL(const StepArgs<float> &a, const LaunchShape &s, const void *cellF, const void *bsig,
                                 void *lk, void *table, void *counters, hipStream_t st)
{
    if (a.equal_prob)
        hipLaunchKernelGGL((HD_KERNEL<float, D, NB, LK, true>), dim3(s.blocks), dim3(s.threads), s.lds_bytes, st,
                           a, (const CellF<float> *)cellF, (const float *)bsig, (float *)lk, (float *)table,
                           (unsigned long long *)counters);
    else
        hipLaunchKernelGGL((HD_KERNEL<float, D, NB, LK, false>), dim3(s.blocks), dim3(s.threads), s.lds_bytes, st,
                           a, (const CellF<float> *)cellF, (const float *)bsig, (float *)lk, (float *)table,
                           (unsigned long long *)counters);
    return hipGetLastError();
}

template <typename R>
hipError_t HD_FN(launch_step_gr_hd)(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                             const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                             hipStream_t st)
{
    if constexpr (!std::is_same<R, float>::value) {
        return hipErrorInvalidValue;
    } else {
        if (lkmode != kLookupY && lkmode != kLookupYZ) return hipErrorInvalidValue;
        switch (d) {
#define X(DD)                                                                                                \
    case DD:                                                                                                 \
        if (basis == 0)                                                                                      \
            return lkmode == kLookupY ? HD_IMPL<DD, 1, kLookupY>(a, s, cellF, bsig, lk, table, counters, st) \
                                      : HD_IMPL<DD, 1, kLookupYZ>(a, s, cellF, bsig, lk, table, counters, st); \
        return lkmode == kLookupY ? HD_IMPL<DD, DD + 1, kLookupY>(a, s, cellF, bsig, lk, table, counters, st) \
                                  : HD_IMPL<DD, DD + 1, kLookupYZ>(a, s, cellF, bsig, lk, table, counters, st);
            HD_DIMS(X)
#undef X
        default: return HD_NEXT(launch_step_gr_hd)<R>(d, a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        }
    }
}

template <typename R>
hipError_t HD_FN(launch_face_flags_hd)(int d, int basis, const StepArgs<R> &a, const void *cellF, const void *bsig,
                                void *counters, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                              \
    case DD:                                                                               \
        if (basis == 0) return launch_face_flags_impl<R, DD, 1>(a, cellF, bsig, counters, st); \
        return launch_face_flags_impl<R, DD, DD + 1>(a, cellF, bsig, counters, st);
        HD_DIMS(X)
#undef X
    default: return HD_NEXT(launch_face_flags_hd)<R>(d, basis, a, cellF, bsig, counters, st);
    }
}

template <typename R>
hipError_t HD_FN(launch_lookup_rows_hd)(int d, int basis, int lkmode, const void *table, void *lk, uint32_t K, int i_lo,
                                 int i_hi, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                                                    \
    case DD:                                                                                                     \
        if (basis == 0) {                                                                                        \
            if (lkmode == kLookupY) return launch_lookup_rows_impl<R, DD, 1, kLookupY>(table, lk, K, i_lo, i_hi, st);   \
            if (lkmode == kLookupYZ) return launch_lookup_rows_impl<R, DD, 1, kLookupYZ>(table, lk, K, i_lo, i_hi, st); \
            return launch_lookup_rows_impl<R, DD, 1, kLookupFull>(table, lk, K, i_lo, i_hi, st);               \
        }                                                                                                        \
        if (lkmode == kLookupY) return launch_lookup_rows_impl<R, DD, DD + 1, kLookupY>(table, lk, K, i_lo, i_hi, st);   \
        if (lkmode == kLookupYZ) return launch_lookup_rows_impl<R, DD, DD + 1, kLookupYZ>(table, lk, K, i_lo, i_hi, st); \
        return launch_lookup_rows_impl<R, DD, DD + 1, kLookupFull>(table, lk, K, i_lo, i_hi, st);
        HD_DIMS(X)
#undef X
    default: return HD_NEXT(launch_lookup_rows_hd)<R>(d, basis, lkmode, table, lk, K, i_lo, i_hi, st);
    }
}

template <typename R>
hipError_t HD_FN(launch_root_hd)(int d, int basis, int lkmode, const StepArgs<R> &a, const void *bsig, const void *lk,
                          const RootPoint &x0, int M_root, int nblocks, double *partial, double *out, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                                                   \
    case DD:                                                                                                    \
        if (basis == 0) {                                                                                       \
            if (lkmode == kLookupY)                                                                             \
                return launch_root_impl<R, DD, 1, kLookupY>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
            if (lkmode == kLookupYZ)                                                                            \
                return launch_root_impl<R, DD, 1, kLookupYZ>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
            return launch_root_impl<R, DD, 1, kLookupFull>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
        }                                                                                                       \
        if (lkmode == kLookupY)                                                                                 \
            return launch_root_impl<R, DD, DD + 1, kLookupY>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
        if (lkmode == kLookupYZ)                                                                                \
            return launch_root_impl<R, DD, DD + 1, kLookupYZ>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
        return launch_root_impl<R, DD, DD + 1, kLookupFull>(a, bsig, lk, x0, M_root, nblocks, partial, out, st);
        HD_DIMS(X)
#undef X
    default: return HD_NEXT(launch_root_hd)<R>(d, basis, lkmode, a, bsig, lk, x0, M_root, nblocks, partial, out, st);
    }
}

template <typename R>
hipError_t HD_FN(launch_eval_hd)(int d, int basis, const StepArgs<R> &a, const void *table, const double *x, int64_t n,
                          double *y, double *z, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                                    \
    case DD:                                                                                     \
        if (basis == 0) return launch_eval_impl<R, DD, 1>(a, table, x, n, y, z, st);             \
        return launch_eval_impl<R, DD, DD + 1>(a, table, x, n, y, z, st);
        HD_DIMS(X)
#undef X
    default: return HD_NEXT(launch_eval_hd)<R>(d, basis, a, table, x, n, y, z, st);
    }
}

template <typename R>
hipError_t HD_FN(launch_draw_hd)(int d, const StepArgs<R> &a, const SetupArgs &sa, int kind, uint32_t k0, uint32_t nk,
                          uint32_t m0, uint32_t nm, int count, double *out, hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return launch_draw_impl<R, DD>(a, sa, kind, k0, nk, m0, nm, count, out, st);
        HD_DIMS(X)
#undef X
    default: return HD_NEXT(launch_draw_hd)<R>(d, a, sa, kind, k0, nk, m0, nm, count, out, st);
    }
}

#define SRMDP_HD_INSTANTIATE(R)                                                                                     \
    template hipError_t HD_FN(launch_step_gr_hd)<R>(int, const StepArgs<R> &, const LaunchShape &, int, int, const void *, \
                                             const void *, void *, void *, void *, hipStream_t);                    \
    template hipError_t HD_FN(launch_face_flags_hd)<R>(int, int, const StepArgs<R> &, const void *, const void *, void *, \
                                                hipStream_t);                                                      \
    template hipError_t HD_FN(launch_lookup_rows_hd)<R>(int, int, int, const void *, void *, uint32_t, int, int,          \
                                                 hipStream_t);                                                     \
    template hipError_t HD_FN(launch_root_hd)<R>(int, int, int, const StepArgs<R> &, const void *, const void *,          \
                                          const RootPoint &, int, int, double *, double *, hipStream_t);           \
    template hipError_t HD_FN(launch_eval_hd)<R>(int, int, const StepArgs<R> &, const void *, const double *, int64_t,    \
                                          double *, double *, hipStream_t);                                        \
    template hipError_t HD_FN(launch_draw_hd)<R>(int, const StepArgs<R> &, const SetupArgs &, int, uint32_t, uint32_t,    \
                                          uint32_t, uint32_t, int, double *, hipStream_t);

SRMDP_HD_INSTANTIATE(float)
SRMDP_HD_INSTANTIATE(double)

}  // namespace srmdp
