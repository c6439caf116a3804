// Kernels around the sweep (look-up rows for resuming, the TABLE and ROOT
// read-outs, the generator check) and their launchers, for every compiled
// dimension.
#pragma once
#include "srmdp_sweep.hpp"

namespace srmdp {

// Sampler constants of cell c along dimension l, computed in binary64 and
// stored in the working precision.
template <typename R>
__device__ __forceinline__ CellF<R> cell_constants(const SetupArgs &a, int l, int c)
{
    CellF<R> v{};
    if (a.equal_prob) {
        // F = c / n and (c + 1) / n at the edges, (c + 1/2) / n at the centre (the
        // cell's nu-median); the outer cells are unbounded, which the inverse-CDF
        // offset from the centre does not see
        const double n = (double)a.cells[l], lo_n = c + 0.5, hi_n = n - c - 0.5;
        v.uc = (R)0.5;
        v.rp = (R)(1.0 / lo_n);
        v.rs = (R)(1.0 / hi_n);
        v.centre = (R)(log(lo_n / hi_n) / a.mu);
        return v;
    }
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
template <typename R, int D, int NB, bool EP>
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
            const R c = cell_and_xi<R, EP>(a, l, (R)x[p * D + l], xi[l]);
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
template <typename R, int D, int NB, int LK, bool EP>
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
        run_path<R, D, NB, LK, false, EP>(a, bsig, lk, ns, x, dW0, y1, Sp);
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

// Table records in the raw basis (1, x_1..x_d) (srmdp_to_raw_basis): one
// record (step, stratum, component) per thread, alpha_l = 2 s_l beta_l and
// alpha_0 = beta_0 - sum_l alpha_l m_l in binary64, m_l the cell's centre or
// nu-median and s_l = scale_l (the LP1 coordinate 2 s_l (x_l - m_l)).  Every
// value of a record is read before it is written, so raw may alias table.
template <typename R>
__global__ void raw_basis_kernel(const StepArgs<R> a, int d, int q1, const R *table, R *raw, size_t records)
{
    const int nb = d + 1;
    for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < records;
         r += (size_t)gridDim.x * blockDim.x) {
        const R *b = table + r * nb;
        R *o = raw + r * nb;
        const uint32_t k = (uint32_t)((r / (size_t)q1) % a.K);
        double a0 = (double)b[0];
        for (int l = 0; l < d; ++l) {
            const double c = (double)((k / a.stride[l]) % a.cells[l]);
            const double s = (double)a.scale[l];
            const double m = a.equal_prob ? log((c + 0.5) / ((double)a.cells[l] - c - 0.5)) / (s + s)
                                           : (double)a.lo[l] + (c + 0.5) / s;
            a0 -= 2.0 * s * (double)b[1 + l] * m;
        }
        for (int l = 0; l < d; ++l) o[1 + l] = (R)(2.0 * (double)a.scale[l] * (double)b[1 + l]);
        o[0] = (R)a0;
    }
}

// ------------------------------------------------------------- launchers

template <typename R, int D, int NB>
static hipError_t launch_face_flags_impl(const StepArgs<R> &a, const void *cellF, const void *bsig,
                                         void *counters, hipStream_t st)
{
    if (a.equal_prob) {
        hipLaunchKernelGGL((face_flags_kernel<R, D, NB, true>), dim3(a.K), dim3(64), 0, st, a,
                           (const CellF<R> *)cellF, (const R *)bsig, (unsigned long long *)counters);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((face_flags_kernel<R, D, NB, false>), dim3(a.K), dim3(64), 0, st, a,
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
    if (a.equal_prob) {
        hipLaunchKernelGGL((root_paths_kernel<R, D, NB, LK, true>), dim3(nblocks), dim3(256), 0, st, a,
                           (const R *)bsig, (const R *)lk, x0, M_root, partial);
    } else {
        hipLaunchKernelGGL((root_paths_kernel<R, D, NB, LK, false>), dim3(nblocks), dim3(256), 0, st, a,
                           (const R *)bsig, (const R *)lk, x0, M_root, partial);
    }
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
    if (a.equal_prob) {
        hipLaunchKernelGGL((eval_kernel<R, D, NB, true>), dim3(blocks), dim3(256), 0, st, a, (const R *)table, x,
                           n, y, z);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((eval_kernel<R, D, NB, false>), dim3(blocks), dim3(256), 0, st, a, (const R *)table,
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

}  // namespace srmdp
