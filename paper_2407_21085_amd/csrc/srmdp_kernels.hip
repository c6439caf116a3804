// HIP kernels (gfx950) of the SRMDP backward sweep, Algorithm SRMDP of the
// paper (Section 3.1, eq. (PsiM)), and its read-outs.
//
// Mapping (differs from the paper's one-thread-per-stratum design): a group of
// L lanes handles one stratum; lane t simulates the stratum's paths
// m = t, t + L, ...  Paths never touch memory: the start point, the Euler steps
// and the response accumulation live in registers, and only what the two
// regressions need (phi(X_i), dW_i, S', y_{i+1}(X_{i+1})) goes to LDS.  The
// Gram matrix and right-hand sides are then formed lane-parallel over their
// entries with binary64 accumulators, the Gram matrix is inverted in binary64
// by Gauss-Jordan elimination (its pivots are the squared diagonal of the
// Cholesky factor, which the singular test reads), the coefficients are the
// inverse times the right-hand sides, and the stratum's record is written once
// to the coefficient table and once, projected on what the driver needs, to a
// compact look-up row that later steps gather from L2/MALL.
#include <algorithm>

#include "srmdp_aux.hpp"

namespace srmdp {

// ------------------------------------------------------------- setup kernel
// (sampler constants: cell_constants in srmdp_aux.hpp)
template <typename R>
__global__ void setup_kernel(SetupArgs a, CellF<R> *cellF, R *bsig)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.d * a.cmax) {
        const int l = t / a.cmax, c = t % a.cmax;
        cellF[t] = c < a.cells[l] ? cell_constants<R>(a, l, c) : CellF<R>{};
    }
    if (t < a.d) bsig[t] = (R)a.b[t];
    if (t < a.d) bsig[a.d + a.d * a.q + t] = (R)a.b_lin[t];
    if (t < a.d) bsig[2 * a.d + a.d * a.q + t] = (R)a.sigma_lin[t];
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

// Look-up rows, TABLE and ROOT read-outs and the generator check live in
// srmdp_aux.hpp, shared with the high-dimension file.

// --------------------------------------------------------- instantiation

template <typename R, int D, int NB, int LK, int PF>
static hipError_t launch_step_pf(const StepArgs<R> &a, const LaunchShape &s, const void *cellF, const void *bsig,
                                 void *lk, void *table, void *counters, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_step_kernel<R, D, NB, LK, false, PF>), dim3(s.blocks), dim3(s.threads), s.lds_bytes,
                       st, a, (const CellF<R> *)cellF, (const R *)bsig, (R *)lk, (R *)table,
                       (unsigned long long *)counters);
    return hipGetLastError();
}

template <typename R, int D, int NB, int LK>
static hipError_t launch_step_impl(const StepArgs<R> &a, const LaunchShape &s, const void *cellF,
                                   const void *bsig, void *lk, void *table, void *counters,
                                   hipStream_t st)
{
    if constexpr (sizeof(R) == 4) {
        const int depth = prefetch_depth<R, D, NB, LK>(a);
        if constexpr (LK != kLookupFull)
            if (depth == 2) return launch_step_pf<R, D, NB, LK, 2>(a, s, cellF, bsig, lk, table, counters, st);
        if (depth >= 1) return launch_step_pf<R, D, NB, LK, 1>(a, s, cellF, bsig, lk, table, counters, st);
    }
    return launch_step_pf<R, D, NB, LK, 0>(a, s, cellF, bsig, lk, table, counters, st);
}

template <typename R>
static hipError_t launch_setup_impl(const SetupArgs &s, const double *sigma, void *cellF, void *bsig,
                                    hipStream_t st)
{
    const int n = s.d * s.cmax > s.d ? s.d * s.cmax : s.d;
    hipLaunchKernelGGL((setup_kernel<R>), dim3((n + 255) / 256), dim3(256), 0, st, s,
                       (CellF<R> *)cellF, (R *)bsig);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // sigma (row-major d x q) in the working precision after b
    R v[kMaxDim * kMaxDim];
    for (int t = 0; t < s.d * s.q; ++t) v[t] = (R)sigma[t];
    return launch_upload((R *)bsig + s.d, v, sizeof(R) * s.d * s.q, st);
}

// Dispatch tables over the compiled dimensions.
#define SRMDP_FOR_EACH_D(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8)

template <typename R, int D>
static hipError_t dispatch_step_d(const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                                  const void *cf, const void *bs, void *lk, void *tab, void *ctr,
                                  hipStream_t st)
{
    if (basis == 0) {
        if (lkmode == kLookupY) return launch_step_impl<R, D, 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
        if (lkmode == kLookupYZ) return launch_step_impl<R, D, 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
        return launch_step_impl<R, D, 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
    }
    if (lkmode == kLookupY) return launch_step_impl<R, D, D + 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
    if (lkmode == kLookupYZ) return launch_step_impl<R, D, D + 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
    return launch_step_impl<R, D, D + 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
}

template <typename R>
hipError_t launch_step(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                       const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                       hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return dispatch_step_d<R, DD>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_face_flags(int d, int basis, const StepArgs<R> &a, const void *cellF, const void *bsig,
                             void *counters, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                              \
    case DD:                                                                               \
        if (basis == 0) return launch_face_flags_impl<R, DD, 1>(a, cellF, bsig, counters, st); \
        return launch_face_flags_impl<R, DD, DD + 1>(a, cellF, bsig, counters, st);
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return launch_face_flags_hd<R>(d, basis, a, cellF, bsig, counters, st);
    }
}

template <typename R>
hipError_t launch_lookup_rows(int d, int basis, int lkmode, const void *table, void *lk, uint32_t K,
                              int i_lo, int i_hi, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                                         \
    case DD:                                                                                          \
        if (basis == 0) {                                                                             \
            if (lkmode == kLookupY) return launch_lookup_rows_impl<R, DD, 1, kLookupY>(table, lk, K, i_lo, i_hi, st);   \
            if (lkmode == kLookupYZ) return launch_lookup_rows_impl<R, DD, 1, kLookupYZ>(table, lk, K, i_lo, i_hi, st); \
            return launch_lookup_rows_impl<R, DD, 1, kLookupFull>(table, lk, K, i_lo, i_hi, st);    \
        }                                                                                             \
        if (lkmode == kLookupY) return launch_lookup_rows_impl<R, DD, DD + 1, kLookupY>(table, lk, K, i_lo, i_hi, st);   \
        if (lkmode == kLookupYZ) return launch_lookup_rows_impl<R, DD, DD + 1, kLookupYZ>(table, lk, K, i_lo, i_hi, st); \
        return launch_lookup_rows_impl<R, DD, DD + 1, kLookupFull>(table, lk, K, i_lo, i_hi, st);
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return launch_lookup_rows_hd<R>(d, basis, lkmode, table, lk, K, i_lo, i_hi, st);
    }
}

template <typename R>
hipError_t launch_root(int d, int basis, int lkmode, const StepArgs<R> &a, const void *bsig,
                       const void *lk, const RootPoint &x0, int M_root, int nblocks, double *partial,
                       double *out, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                                         \
    case DD:                                                                                          \
        if (basis == 0) {                                                                             \
            if (lkmode == kLookupY) return launch_root_impl<R, DD, 1, kLookupY>(a, bsig, lk, x0, M_root, nblocks, partial, out, st);   \
            if (lkmode == kLookupYZ) return launch_root_impl<R, DD, 1, kLookupYZ>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
            return launch_root_impl<R, DD, 1, kLookupFull>(a, bsig, lk, x0, M_root, nblocks, partial, out, st);    \
        }                                                                                             \
        if (lkmode == kLookupY) return launch_root_impl<R, DD, DD + 1, kLookupY>(a, bsig, lk, x0, M_root, nblocks, partial, out, st);   \
        if (lkmode == kLookupYZ) return launch_root_impl<R, DD, DD + 1, kLookupYZ>(a, bsig, lk, x0, M_root, nblocks, partial, out, st); \
        return launch_root_impl<R, DD, DD + 1, kLookupFull>(a, bsig, lk, x0, M_root, nblocks, partial, out, st);
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return launch_root_hd<R>(d, basis, lkmode, a, bsig, lk, x0, M_root, nblocks, partial, out, st);
    }
}

template <typename R>
hipError_t launch_eval(int d, int basis, const StepArgs<R> &a, const void *table, const double *x,
                       int64_t n, double *y, double *z, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                  \
    case DD:                                                                   \
        if (basis == 0) return launch_eval_impl<R, DD, 1>(a, table, x, n, y, z, st); \
        return launch_eval_impl<R, DD, DD + 1>(a, table, x, n, y, z, st);
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return launch_eval_hd<R>(d, basis, a, table, x, n, y, z, st);
    }
}

template <typename R>
hipError_t launch_raw_basis(int d, int q, const StepArgs<R> &a, const void *table, void *raw, hipStream_t st)
{
    const size_t records = (size_t)a.N * a.K * (size_t)(1 + q);
    const size_t blocks = std::min<size_t>((records + 255) / 256, 65536);
    hipLaunchKernelGGL((raw_basis_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, st, a, d, 1 + q,
                       (const R *)table, (R *)raw, records);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_draw(int d, const StepArgs<R> &a, const SetupArgs &sa, int kind, uint32_t k0,
                       uint32_t nk, uint32_t m0, uint32_t nm, int count, double *out, hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return launch_draw_impl<R, DD>(a, sa, kind, k0, nk, m0, nm, count, out, st);
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return launch_draw_hd<R>(d, a, sa, kind, k0, nk, m0, nm, count, out, st);
    }
}

template <typename R>
hipError_t launch_setup(const SetupArgs &s, const double *sigma, void *cellF, void *bsig, hipStream_t st)
{
    return launch_setup_impl<R>(s, sigma, cellF, bsig, st);
}

bool lds_dimension_compiled(int d)
{
    switch (d) {
#define X(DD) case DD: return true;
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return false;
    }
}

bool dimension_compiled(int d) { return lds_dimension_compiled(d) || hd_dimension_compiled(d); }

// Cloud rows of a stratum (16-byte aligned) and its chunk sums.
static size_t cube_row_bytes(int prec_is_float, int d, int nb, int M, bool cv)
{
    const size_t rsz = prec_is_float ? 4 : 8;
    // with the control variate, one spare row for the lanes past the last simulation
    const size_t rows = (size_t)(cv ? M + 1 : M) * (nb + d + 2 + (cv ? 2 : 0)) * rsz;
    return (rows + 15) & ~(size_t)15;
}
static size_t cube_part_bytes(int d, int nb, int M)
{
    const int nch = (M + kChunk - 1) / kChunk;
    return nch > 1 ? (size_t)(nb * (nb + 1) / 2 + d * nb) * nch * sizeof(double) : 0;
}

// The stratum's cell constants (CellF, four values of the working precision per
// dimension), first in a stratum's LDS.
static size_t cube_cell_bytes(int prec_is_float, int d)
{
    return ((size_t)d * 4 * (prec_is_float ? 4 : 8) + 15) & ~(size_t)15;
}

size_t cube_lds_bytes(int prec_is_float, int d, int nb, int M, bool cv)
{
    const size_t small = (size_t)(2 * nb * nb + 2 * (1 + d) * nb + 2 + nb) * sizeof(double);
    return cube_cell_bytes(prec_is_float, d) + cube_row_bytes(prec_is_float, d, nb, M, cv) + small +
           cube_part_bytes(d, nb, M);
}

size_t cube_stream_lds_bytes(int prec_is_float, int d, int nb, int L, int pb)
{
    const size_t rsz = prec_is_float ? 4 : 8;
    const size_t small = (size_t)(2 * nb * nb + 2 * (1 + d) * nb + 2 + nb) * sizeof(double);
    const size_t part = (size_t)(nb * (nb + 1) / 2 + d * nb) * pb * sizeof(double);
    const int RS = L >= kChunk ? L : kChunk;
    return cube_cell_bytes(prec_is_float, d) + ((small + part + 15) & ~(size_t)15) +
           (size_t)RS * (nb + d + 2) * rsz;
}

int cube_stream_chunks(int prec_is_float, int d, int nb, int L, size_t cap)
{
    const int RS = L >= kChunk ? L : kChunk;
    int pb = RS / kChunk;
    while (pb > 1 && cube_stream_lds_bytes(prec_is_float, d, nb, L, pb) > cap) --pb;
    return cube_stream_lds_bytes(prec_is_float, d, nb, L, pb) <= cap ? pb : 0;
}

size_t cube_global_bytes(int prec_is_float, int M)
{
    const size_t rsz = prec_is_float ? 4 : 8;
    return ((size_t)M * 2 * rsz + 255) & ~(size_t)255;  // S' and y_{i+1}(X_{i+1}) per sample
}

#define SRMDP_INSTANTIATE(R)                                                                        \
    template hipError_t launch_step<R>(int, const StepArgs<R> &, const LaunchShape &, int, int,     \
                                       const void *, const void *, void *, void *, void *,           \
                                       hipStream_t);                                                 \
    template hipError_t launch_face_flags<R>(int, int, const StepArgs<R> &, const void *,           \
                                             const void *, void *, hipStream_t);                     \
    template hipError_t launch_lookup_rows<R>(int, int, int, const void *, void *, uint32_t, int,   \
                                              int, hipStream_t);                                     \
    template hipError_t launch_root<R>(int, int, int, const StepArgs<R> &, const void *,            \
                                       const void *, const RootPoint &, int, int, double *,         \
                                       double *, hipStream_t);                                       \
    template hipError_t launch_eval<R>(int, int, const StepArgs<R> &, const void *, const double *, \
                                       int64_t, double *, double *, hipStream_t);                    \
    template hipError_t launch_raw_basis<R>(int, int, const StepArgs<R> &, const void *, void *,    \
                                            hipStream_t);                                            \
    template hipError_t launch_draw<R>(int, const StepArgs<R> &, const SetupArgs &, int, uint32_t,  \
                                       uint32_t, uint32_t, uint32_t, int, double *, hipStream_t);    \
    template hipError_t launch_setup<R>(const SetupArgs &, const double *, void *, void *, hipStream_t);

SRMDP_INSTANTIATE(float)
SRMDP_INSTANTIATE(double)

}  // namespace srmdp
