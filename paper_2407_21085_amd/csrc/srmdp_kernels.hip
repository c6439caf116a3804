// HIP kernels (gfx950) of the SRMDP backward sweep, Algorithm SRMDP of the
// paper (Section 3.1, eq. (PsiM)), and its read-outs.
//
// Mapping (differs from the paper's one-thread-per-stratum design): a group of
// L lanes handles one stratum; lane t simulates the stratum's paths
// m = t, t + L, ...  Paths never touch memory: the start point, the Euler steps
// and the response accumulation live in registers, and only what the two
// regressions need (phi(X_i), dW_i, S', y_{i+1}(X_{i+1})) goes to LDS.  The
// Gram matrix and right-hand sides are then formed lane-parallel over their
// entries with binary64 accumulators, the Cholesky factor and the solves run
// in binary64, and the stratum's record is written once to the coefficient
// table and once, projected on what the driver needs, to a compact look-up row
// that later steps gather from L2/MALL.
#include "srmdp_sweep.hpp"

namespace srmdp {

// ------------------------------------------------------------- setup kernel
// Sampler constants of cell c along dimension l, computed in binary64 and
// stored in the working precision.
template <typename R>
__device__ __forceinline__ CellF<R> cell_constants(const SetupArgs &a, int l, int c)
{
    CellF<R> v{};
    const double h = (a.hi[l] - a.lo[l]) / (double)a.cells[l];
    const double xm = a.lo[l] + c * h, xp = xm + h, xc = xm + 0.5 * h;
    const double F_m = 1.0 / (1.0 + exp(-a.mu * xm)), F_p = 1.0 / (1.0 + exp(-a.mu * xp));
    const double G_m = 1.0 / (1.0 + exp(a.mu * xm)), G_p = 1.0 / (1.0 + exp(a.mu * xp));  // 1 - F
    const double F_c = 1.0 / (1.0 + exp(-a.mu * xc)), G_c = 1.0 / (1.0 + exp(a.mu * xc));
    // F differences from the side where F (or 1 - F) is small, to avoid cancellation
    const double delta = xm >= 0.0 ? G_m - G_p : F_p - F_m;
    const double to_c = xm >= 0.0 ? G_m - G_c : F_c - F_m;
    v.uc = (R)(to_c / delta);
    v.rp = (R)(delta / F_c);
    v.rs = (R)(delta / G_c);
    v.centre = (R)xc;
    return v;
}

template <typename R>
__global__ void setup_kernel(SetupArgs a, CellF<R> *cellF, R *bsig)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.d * a.cmax) {
        const int l = t / a.cmax, c = t % a.cmax;
        cellF[t] = c < a.cells[l] ? cell_constants<R>(a, l, c) : CellF<R>{};
    }
    if (t < a.d) bsig[t] = (R)a.b[t];
    if (t < a.d * a.q) bsig[a.d + t] = (R)a.sigma[t];
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

// Rebuilds look-up rows [i_lo, i_hi] from the coefficient table (resume).
template <typename R, int D, int NB, int LK>
__global__ void lookup_rows_kernel(const R *__restrict__ table, R *__restrict__ lk, uint32_t K,
                                   int i_lo, int i_hi)
{
    constexpr int REC = (1 + D) * NB;
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    const size_t n = (size_t)(i_hi - i_lo + 1) * K;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t row = (size_t)i_lo * K + g;
        const R *rec = table + row * REC;
        R *out = lk + row * W;
        for (int e = 0; e < W; ++e) {
            R v = (R)0;
            if constexpr (LK == kLookupFull) {
                if (e < REC) v = rec[e];
            } else {
                if (e < NB) {
                    v = rec[e];
                } else if (LK == kLookupYZ && e < 2 * NB) {
                    const int b = e - NB;
                    double acc = 0.0;
                    for (int c = 0; c < D; ++c) acc += (double)rec[(1 + c) * NB + b];
                    v = (R)acc;
                }
            }
            out[e] = v;
        }
    }
}

// ----------------------------------------------------------------- eval
template <typename R, int D, int NB>
__global__ void eval_kernel(const StepArgs<R> a, const R *__restrict__ table, const double *__restrict__ x,
                            int64_t n, double *__restrict__ y, double *__restrict__ z)
{
    constexpr int REC = (1 + D) * NB;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        R xi[D];
        uint32_t k = 0;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const R xv = (R)x[p * D + l];
            const R tt = (xv - a.lo[l]) * a.scale[l];
            const R c = RealOps<R>::clamp_cell(tt, a.cmax_f[l]);
            xi[l] = (R)2 * (tt - c) - (R)1;
            k += (uint32_t)c * a.stride[l];
        }
        const R *rec = table + ((size_t)a.i * a.K + k) * REC;
#pragma unroll
        for (int c = 0; c <= D; ++c) {
            R v = rec[c * NB];
            if constexpr (NB > 1) {
#pragma unroll
                for (int l = 0; l < D; ++l) v += rec[c * NB + 1 + l] * xi[l];
            }
            if (c == 0) {
                if (y) y[p] = (double)clamp_level<R>(v, a.clamp_y);
            } else {
                if (z) z[p * D + c - 1] = (double)clamp_level<R>(v, a.clamp_z);
            }
        }
    }
}

// ------------------------------------------------------------- ROOT read-out
// Paths from the fixed point x0 at step 0 (counter stratum SRMDP_ROOT_STRATUM).
// Per-block binary64 partial sums of S', y_1(X_1) and S' dW_0,l are written in
// block order; root_finish_kernel reduces them in a fixed order.
template <typename R, int D, int NB, int LK>
__global__ void __launch_bounds__(256) root_paths_kernel(const StepArgs<R> a, const R *__restrict__ bsig,
                                                        const R *__restrict__ lk, RootPoint x0, int M_root,
                                                        double *__restrict__ partial)
{
    constexpr int NP = D + 2;
    __shared__ double red[256 * NP];
    double acc[NP];
#pragma unroll
    for (int v = 0; v < NP; ++v) acc[v] = 0.0;
    const Key key{a.key0, a.key1};
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < M_root; m += gridDim.x * blockDim.x) {
        R x[D];
#pragma unroll
        for (int l = 0; l < D; ++l) x[l] = (R)x0.x[l];
        NormalStream<R, D> ns;
        ns.init(key, (uint32_t)m, 0xFFFFFFFFu, a.tag, a.sqrt_dt);
        R dW0[D], y1, Sp;
        run_path<R, D, NB, LK>(a, bsig, lk, ns, x, dW0, y1, Sp);
        acc[0] += (double)Sp;
        acc[1] += (double)y1;
#pragma unroll
        for (int l = 0; l < D; ++l) acc[2 + l] += (double)Sp * (double)dW0[l];
    }
#pragma unroll
    for (int v = 0; v < NP; ++v) red[threadIdx.x * NP + v] = acc[v];
    __syncthreads();
    if (threadIdx.x < NP) {
        double s = 0.0;
        for (int u = 0; u < (int)blockDim.x; ++u) s += red[u * NP + threadIdx.x];
        partial[(size_t)blockIdx.x * NP + threadIdx.x] = s;
    }
}

// y0 = mean(S') + dt * mean f(0, x0, y1, z0) (both built-in drivers are affine
// in y for a fixed z), z0 = mean(S' dW_0) / dt, truncated.
template <typename R, int D>
__global__ void root_finish_kernel(const StepArgs<R> a, const double *__restrict__ partial, int nblocks,
                                   int M_root, double *__restrict__ out)
{
    constexpr int NP = D + 2;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[NP];
    for (int v = 0; v < NP; ++v) s[v] = 0.0;
    for (int b = 0; b < nblocks; ++b)
        for (int v = 0; v < NP; ++v) s[v] += partial[(size_t)b * NP + v];
    double zsum = 0.0;
    for (int l = 0; l < D; ++l) {
        double zl = s[2 + l] / M_root / (double)a.dt;
        zl = fmin(fmax(zl, -(double)a.clamp_z), (double)a.clamp_z);
        out[1 + l] = zl;
        zsum += zl;
    }
    const double mean_S = s[0] / M_root, mean_y1 = s[1] / M_root;
    double fbar;
    if (a.driver == 1)
        fbar = zsum * (mean_y1 - (double)a.c_logistic);
    else
        fbar = (double)a.kappa * zsum - (double)a.r * mean_y1;
    out[0] = mean_S + fbar * (double)a.dt;
}

// ----------------------------------------------------------------- draws
template <typename R, int D>
__global__ void draw_kernel(const StepArgs<R> a, const SetupArgs sa, int kind,
                            uint32_t k0, uint32_t nk, uint32_t m0, uint32_t nm, int count,
                            double *__restrict__ out)
{
    const Key key{a.key0, a.key1};
    const size_t total = (size_t)nk * nm;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const uint32_t k = k0 + (uint32_t)(g / nm), m = m0 + (uint32_t)(g % nm);
        double *o = out + g * count;
        if (kind == 0) {
            for (int u = 0; u < count; ++u)
                o[u] = (double)open_uniform<R>(stream_word(key, m, k, a.tag, (uint32_t)u));
        } else if (kind == 1) {
            NormalStream<R, D> ns;
            ns.init(key, m, k, a.tag, (R)1);
            for (int s = 0; s * D < count; ++s) {
                R v[D];
                ns.step((uint32_t)s, v);
                for (int l = 0; l < D && s * D + l < count; ++l) o[s * D + l] = (double)v[l];
            }
        } else {
            for (int l = 0; l < D; ++l) {
                const uint32_t cell = (k / a.stride[l]) % a.cells[l];
                const R u = open_uniform<R>(stream_word(key, m, k, a.tag, (uint32_t)l));
                const CellF<R> cf = cell_constants<R>(sa, l, (int)cell);
                o[l] = (double)(cf.centre + stratified_offset<R>(cf, u, a.inv_mu));
            }
        }
    }
}

// --------------------------------------------------------- instantiation

template <typename R, int D, int NB, int LK>
static hipError_t launch_step_impl(const StepArgs<R> &a, const LaunchShape &s, const void *cellF,
                                   const void *bsig, void *lk, void *table, void *counters,
                                   hipStream_t st)
{
    hipLaunchKernelGGL((sweep_step_kernel<R, D, NB, LK, false>), dim3(s.blocks), dim3(s.threads),
                       s.lds_bytes, st, a, (const CellF<R> *)cellF, (const R *)bsig, (R *)lk,
                       (R *)table, (unsigned long long *)counters);
    return hipGetLastError();
}

template <typename R, int D, int NB>
static hipError_t launch_face_flags_impl(const StepArgs<R> &a, const void *cellF, const void *bsig,
                                         void *counters, hipStream_t st)
{
    hipLaunchKernelGGL((face_flags_kernel<R, D, NB>), dim3(a.K), dim3(64), 0, st, a,
                       (const CellF<R> *)cellF, (const R *)bsig, (unsigned long long *)counters);
    return hipGetLastError();
}

template <typename R, int D, int NB, int LK>
static hipError_t launch_lookup_rows_impl(const void *table, void *lk, uint32_t K, int i_lo, int i_hi,
                                          hipStream_t st)
{
    const size_t n = (size_t)(i_hi - i_lo + 1) * K;
    const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL((lookup_rows_kernel<R, D, NB, LK>), dim3(blocks), dim3(256), 0, st,
                       (const R *)table, (R *)lk, K, i_lo, i_hi);
    return hipGetLastError();
}

template <typename R, int D, int NB, int LK>
static hipError_t launch_root_impl(const StepArgs<R> &a, const void *bsig, const void *lk,
                                   const RootPoint &x0, int M_root, int nblocks, double *partial,
                                   double *out, hipStream_t st)
{
    hipLaunchKernelGGL((root_paths_kernel<R, D, NB, LK>), dim3(nblocks), dim3(256), 0, st, a,
                       (const R *)bsig, (const R *)lk, x0, M_root, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((root_finish_kernel<R, D>), dim3(1), dim3(64), 0, st, a, partial, nblocks,
                       M_root, out);
    return hipGetLastError();
}

template <typename R, int D, int NB>
static hipError_t launch_eval_impl(const StepArgs<R> &a, const void *table, const double *x,
                                   int64_t n, double *y, double *z, hipStream_t st)
{
    const int64_t blocks64 = (n + 255) / 256;
    const int blocks = (int)(blocks64 < 16384 ? (blocks64 > 0 ? blocks64 : 1) : 16384);
    hipLaunchKernelGGL((eval_kernel<R, D, NB>), dim3(blocks), dim3(256), 0, st, a, (const R *)table,
                       x, n, y, z);
    return hipGetLastError();
}

template <typename R, int D>
static hipError_t launch_draw_impl(const StepArgs<R> &a, const SetupArgs &sa, int kind, uint32_t k0,
                                   uint32_t nk, uint32_t m0, uint32_t nm, int count, double *out,
                                   hipStream_t st)
{
    const size_t total = (size_t)nk * nm;
    const int blocks = (int)((total + 255) / 256 < 16384 ? (total + 255) / 256 : 16384);
    hipLaunchKernelGGL((draw_kernel<R, D>), dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, a,
                       sa, kind, k0, nk, m0, nm, count, out);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_setup_impl(const SetupArgs &s, void *cellF, void *bsig, hipStream_t st)
{
    const int n = s.d * s.cmax > s.d * s.q ? s.d * s.cmax : s.d * s.q;
    hipLaunchKernelGGL((setup_kernel<R>), dim3((n + 255) / 256), dim3(256), 0, st, s,
                       (CellF<R> *)cellF, (R *)bsig);
    return hipGetLastError();
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
    default: return hipErrorInvalidValue;
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
    default: return hipErrorInvalidValue;
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
    default: return hipErrorInvalidValue;
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
    default: return hipErrorInvalidValue;
    }
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
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_setup(const SetupArgs &s, void *cellF, void *bsig, hipStream_t st)
{
    return launch_setup_impl<R>(s, cellF, bsig, st);
}

bool dimension_compiled(int d)
{
    switch (d) {
#define X(DD) case DD: return true;
        SRMDP_FOR_EACH_D(X)
#undef X
    default: return false;
    }
}

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

size_t cube_lds_bytes(int prec_is_float, int d, int nb, int M, bool cv, bool grows)
{
    const size_t small = (size_t)(2 * nb * nb + 2 * (1 + d) * nb + 2 + nb) * sizeof(double);
    if (grows) {  // binary64 arrays, then the window of rows
        const size_t rsz = prec_is_float ? 4 : 8;
        return ((small + 15) & ~(size_t)15) +
               (size_t)cube_stage_chunks(prec_is_float, d, nb, M) * kChunk * (nb + d + 2) * rsz;
    }
    return cube_row_bytes(prec_is_float, d, nb, M, cv) + small + cube_part_bytes(d, nb, M);
}

int cube_stage_chunks(int prec_is_float, int d, int nb, int M)
{
    const size_t rsz = prec_is_float ? 4 : 8;
    const int fit = (int)(kStageBytes / ((size_t)kChunk * (nb + d + 2) * rsz));
    const int nch = (M + kChunk - 1) / kChunk;
    return fit < 1 ? 1 : (fit < nch ? fit : nch);
}

size_t cube_global_bytes(int prec_is_float, int d, int nb, int M)
{
    const size_t b = cube_row_bytes(prec_is_float, d, nb, M, false) + cube_part_bytes(d, nb, M);
    return (b + 255) & ~(size_t)255;
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
    template hipError_t launch_draw<R>(int, const StepArgs<R> &, const SetupArgs &, int, uint32_t,  \
                                       uint32_t, uint32_t, uint32_t, int, double *, hipStream_t);    \
    template hipError_t launch_setup<R>(const SetupArgs &, void *, void *, hipStream_t);

SRMDP_INSTANTIATE(float)
SRMDP_INSTANTIATE(double)

}  // namespace srmdp
