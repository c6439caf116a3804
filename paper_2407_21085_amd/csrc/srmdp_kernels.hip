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
#include "srmdp_device.hpp"
#include "srmdp_internal.hpp"

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

// --------------------------------------------------------- sweep step kernel

// Loads one look-up record (W values, 16-byte aligned) of the working precision.
template <typename R, int W>
__device__ __forceinline__ void load_record(const R *__restrict__ p, R *rec)
{
    if constexpr (sizeof(R) == 4) {
        static_assert(W % 4 == 0, "float records are padded to 4");
        const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
        for (int v = 0; v < W / 4; ++v) {
            const float4 f = q[v];
            rec[4 * v] = f.x;
            rec[4 * v + 1] = f.y;
            rec[4 * v + 2] = f.z;
            rec[4 * v + 3] = f.w;
        }
    } else {
        static_assert(W % 2 == 0, "double records are padded to 2");
        const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
        for (int v = 0; v < W / 2; ++v) {
            const double2 f = q[v];
            rec[2 * v] = f.x;
            rec[2 * v + 1] = f.y;
        }
    }
}

template <typename R>
struct RealOps;
// Cell of a coordinate along one dimension: floor((x - lo) * cells/(hi - lo))
// clamped to [0, cells - 1] (points outside the domain use the boundary cell).
template <>
struct RealOps<float> {
    // v_med3_f32 also maps +-inf into [0, cmax]; a NaN stays NaN and the index
    // conversion then yields stratum 0
    static __device__ __forceinline__ float clamp_cell(float t, float cmax)
    {
        return __builtin_amdgcn_fmed3f(floorf(t), 0.0f, cmax);
    }
};
template <>
struct RealOps<double> {
    static __device__ __forceinline__ double clamp_cell(double t, double cmax)
    {
        return fmin(fmax(floor(t), 0.0), cmax);
    }
};

// Fitted y_{j}(x) and sum_l z_{j,l}(x) from the look-up row j.
// True when the point with cell coordinate t (in cell widths from lo) lies
// within eps of a face between two cells of the grid (not the domain's outer
// faces, where the clamped cell does not change).
template <typename R>
__device__ __forceinline__ bool near_interior_face(R t, R c, R cmax, R eps)
{
    const R frac = t - c;
    return (frac < eps && c > (R)0 && t >= (R)0) || (frac > (R)1 - eps && c < cmax);
}

template <typename R, int D>
__device__ __forceinline__ bool near_face(const StepArgs<R> &a, const R *x)
{
    bool near = false;
    for (int l = 0; l < D; ++l) {
        const R t = (x[l] - a.lo[l]) * a.scale[l];
        near |= near_interior_face<R>(t, RealOps<R>::clamp_cell(t, a.cmax_f[l]), a.cmax_f[l],
                                      a.face_eps);
    }
    return near;
}

// Cell of x per dimension: floor((x - lo) cells / (hi - lo)) clamped to the
// grid, xi = 2 (t - cell) - 1, and the offset of the stratum's look-up record
// in a row.  The stratum index is accumulated in the working precision, exact
// because K <= 2^24; K W < 2^32 so the offset is a 24-bit product.
template <typename R, int D, int NB, int LK>
__device__ __forceinline__ uint32_t locate(const StepArgs<R> &a, const R *x, R *xi)
{
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    R kf = (R)0;
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const R t = (x[l] - a.lo[l]) * a.scale[l];
        const R c = RealOps<R>::clamp_cell(t, a.cmax_f[l]);
        xi[l] = (R)2 * (t - c) - (R)1;
        kf = c * a.stride_f[l] + kf;
    }
    return __umul24((uint32_t)kf, (uint32_t)W);
}

// Fitted y_j(x) (truncated) and sum_l z_{j,l}(x) from a look-up record.
template <typename R, int D, int NB, int LK>
__device__ __forceinline__ void eval_record(const StepArgs<R> &a, const R *rec, const R *xi, R &y,
                                            R &zsum)
{
    R yv = rec[0];
    if constexpr (NB > 1) {
#pragma unroll
        for (int l = 0; l < D; ++l) yv += rec[1 + l] * xi[l];
    }
    y = clamp_level<R>(yv, a.clamp_y);
    if constexpr (LK == kLookupY) {
        zsum = (R)0;
    } else if constexpr (LK == kLookupYZ) {
        R zv = rec[NB];
        if constexpr (NB > 1) {
#pragma unroll
            for (int l = 0; l < D; ++l) zv += rec[NB + 1 + l] * xi[l];
        }
        zsum = zv;
    } else {
        R acc = (R)0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            R zv = rec[(1 + c) * NB];
            if constexpr (NB > 1) {
#pragma unroll
                for (int l = 0; l < D; ++l) zv += rec[(1 + c) * NB + 1 + l] * xi[l];
            }
            acc += clamp_level<R>(zv, a.clamp_z);
        }
        zsum = acc;
    }
}

template <typename R, int D, int NB, int LK>
__device__ __forceinline__ void lookup_eval(const StepArgs<R> &a, const R *__restrict__ row, const R *x,
                                            R &y, R &zsum)
{
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    R xi[D], rec[W];
    load_record<R, W>(row + locate<R, D, NB, LK>(a, x, xi), rec);
    eval_record<R, D, NB, LK>(a, rec, xi, y, zsum);
}

// X_{j+1} = X_j + b dt + sigma dW_j (Algorithm "Euler dynamics", read with the
// time index of the current step; exact for the constant coefficients here).
template <typename R, int D>
__device__ __forceinline__ void euler_step(const StepArgs<R> &a, const R *__restrict__ bsig,
                                           const R *x, const R *dW, R *xn)
{
    if (a.identity_sigma) {
#pragma unroll
        for (int l = 0; l < D; ++l) xn[l] = x[l] + dW[l];
    } else {
#pragma unroll
        for (int l = 0; l < D; ++l) {
            R acc = x[l];
#pragma unroll
            for (int c = 0; c < D; ++c) acc += bsig[D + l * D + c] * dW[c];
            xn[l] = acc;
        }
    }
    if (a.has_drift) {
#pragma unroll
        for (int l = 0; l < D; ++l) xn[l] += bsig[l] * a.dt;
    }
}

template <typename R, int D>
__device__ __forceinline__ R terminal_at(const StepArgs<R> &a, const R *x)
{
    R s = (R)0;
#pragma unroll
    for (int l = 0; l < D; ++l) s += x[l];
    return terminal_g<R>(a.terminal, a.T, s);
}

// One simulation from X_i = x (eq. (PsiM)): the Euler scheme to X_N with the
// fitted rows i+1..N-1, returning dW_i, y_{i+1}(X_{i+1}) (g(X_N) when
// i + 1 = N) and the tail response
//   S' = g(X_N) + sum_{j=i+1}^{N-1} f_j(X_j, y_{j+1}(X_{j+1}), z_j(X_j)) dt.
// The first and last steps are peeled off so that the steady loop has no
// branch that depends on j.
template <typename R, int D, int NB, int LK>
__device__ __forceinline__ void run_path(const StepArgs<R> &a, const R *__restrict__ bsig,
                                         const R *__restrict__ lk, NormalStream<R, D> &ns, R *x,
                                         R *dWi_out, R &y1, R &Sp)
{
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    const int i = a.i, N = a.N;
    const size_t row_elems = (size_t)a.K * W;
    const R dt = a.dt;
    R dW[D], xn[D];
    ns.step(0u, dW);
    euler_step<R, D>(a, bsig, x, dW, xn);
    R zsum_cur = (R)0;
    if (i + 1 < N) {
        lookup_eval<R, D, NB, LK>(a, lk + (size_t)(i + 1) * row_elems, xn, y1, zsum_cur);
    } else {
        y1 = terminal_at<R, D>(a, xn);
    }
#pragma unroll
    for (int l = 0; l < D; ++l) {
        dWi_out[l] = dW[l];
        x[l] = xn[l];
    }
    R S = (R)0;
    for (int j = i + 1; j < N - 1; ++j) {
        ns.step((uint32_t)(j - i), dW);
        euler_step<R, D>(a, bsig, x, dW, xn);
        R yn, zn;
        lookup_eval<R, D, NB, LK>(a, lk + (size_t)(j + 1) * row_elems, xn, yn, zn);
        S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
        zsum_cur = zn;
#pragma unroll
        for (int l = 0; l < D; ++l) x[l] = xn[l];
    }
    R gN;
    if (i < N - 1) {
        ns.step((uint32_t)(N - 1 - i), dW);
        euler_step<R, D>(a, bsig, x, dW, xn);
        gN = terminal_at<R, D>(a, xn);
        S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, gN, zsum_cur) * dt;
    } else {
        gN = y1;
    }
    Sp = gN + S;
}

// One simulation of stratum k from step i: X_i ~ nu_k by Algorithm
// "stratify" (phi(X_i) to full precision from the centred offset), then
// run_path.  phi(X_i) and dW_i go to the stratum's LDS row as soon as they are
// known, so they do not occupy registers during the path.
template <typename R, int D, int NB>
__device__ __forceinline__ void sample_start(const StepArgs<R> &a, const CellF<R> *__restrict__ cellF,
                                             uint32_t k, uint32_t m, R *x, R *phi_out)
{
    const Key key{a.key0, a.key1};
#pragma unroll
    for (int b = 0; b < (D + 3) / 4; ++b) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)b, m, k, a.tag), key);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int l = 4 * b + t;
            if (l < D) {
                const uint32_t cell = (k / a.stride[l]) % a.cells[l];
                const CellF<R> cf = cellF[l * a.cmax + cell];
                const R off = stratified_offset<R>(cf, open_uniform<R>(ws[t]), a.inv_mu);
                x[l] = cf.centre + off;
                // xi = 2 (x - c) / h, and 1/h = scale
                if constexpr (NB > 1) phi_out[1 + l] = (off + off) * a.scale[l];
            }
        }
    }
    phi_out[0] = (R)1;
}

template <typename R, int D, int NB, int LK>
__device__ __forceinline__ void simulate_path(const StepArgs<R> &a, const CellF<R> *__restrict__ cellF,
                                              const R *__restrict__ bsig, const R *__restrict__ lk,
                                              uint32_t k, uint32_t m, R *phi_out, R *dWi_out,
                                              R &Sp, R &y1)
{
    R x[D];
    sample_start<R, D, NB>(a, cellF, k, m, x, phi_out);
    NormalStream<R, D> ns;
    ns.init(Key{a.key0, a.key1}, m, k, a.tag, a.sqrt_dt);
    run_path<R, D, NB, LK>(a, bsig, lk, ns, x, dWi_out, y1, Sp);
}

// Near-face diagnostic of step i: the positions of a simulation do not depend
// on the fitted rows, so they are recomputed here with the same draws and the
// same Euler steps as the sweep, and stratum k is marked when one of its
// simulations reaches a look-up point within face_eps of an interior face.
// One wavefront per stratum.
template <typename R, int D, int NB>
__global__ void __launch_bounds__(64) face_flags_kernel(const StepArgs<R> a,
                                                       const CellF<R> *__restrict__ cellF,
                                                       const R *__restrict__ bsig,
                                                       unsigned long long *__restrict__ counters)
{
    const uint32_t k = blockIdx.x;
    int count = 0;
    for (int m = threadIdx.x; m < a.M; m += 64) {
        R x[D], phi[NB], dW[D], xn[D];
        sample_start<R, D, NB>(a, cellF, k, (uint32_t)m, x, phi);
        NormalStream<R, D> ns;
        ns.init(Key{a.key0, a.key1}, (uint32_t)m, k, a.tag, a.sqrt_dt);
        bool near = false;
        for (int j = a.i; j < a.N - 1; ++j) {
            ns.step((uint32_t)(j - a.i), dW);
            euler_step<R, D>(a, bsig, x, dW, xn);
            near |= near_face<R, D>(a, xn);
#pragma unroll
            for (int l = 0; l < D; ++l) x[l] = xn[l];
        }
        count += near ? 1 : 0;
    }
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    if (count) atomicAdd(&total, count);
    __syncthreads();
    if (threadIdx.x == 0) {
        a.face_flags[(size_t)a.i * a.K + k] = total ? 1 : 0;
        if (total) atomicAdd(counters + kCounterNearFace, (unsigned long long)total);
    }
}

// LDS layout of one stratum: path rows [M][SW] in the working precision
// (phi: NB, dW_i: D, S': 1, y1: 1), then the binary64 block
// G[NB*NB] | H[NB*NB] (the two buffers of the in-place inversion)
// | RHS[(1+D)*NB] (y first, then z_1..z_D) | beta[(1+D)*NB] | flag[2]
// | zsum[NB] (sum over l of the z_l coefficients).
template <typename R, int D, int NB>
struct CubeLds {
    static constexpr int SW = NB + D + 2;
    static constexpr int F64 = 2 * NB * NB + 2 * (1 + D) * NB + 2 + NB;
    static __host__ __device__ size_t bytes(int M)
    {
        size_t rows = (size_t)M * SW * sizeof(R);
        rows = (rows + 15) & ~(size_t)15;
        return rows + (size_t)F64 * sizeof(double);
    }
};

// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so block b
// runs on XCD b % 8.  Give each XCD a contiguous range of strata so that
// neighbouring strata, whose paths gather the same look-up records, share an
// L2.  Bijective on the complete rounds, identity on the tail.
__device__ __forceinline__ uint32_t xcd_block_order(uint32_t b, uint32_t n)
{
    const uint32_t full = n - n % 8u;
    if (b >= full) return b;
    return (b % 8u) * (full / 8u) + b / 8u;
}

template <typename R, int D, int NB, int LK>
__global__ void __launch_bounds__(256) sweep_step_kernel(const StepArgs<R> a,
                                                        const CellF<R> *__restrict__ cellF,
                                                        const R *__restrict__ bsig,
                                                        R *__restrict__ lk, R *__restrict__ table,
                                                        unsigned long long *__restrict__ counters)
{
    using Lay = CubeLds<R, D, NB>;
    constexpr int SW = Lay::SW;
    constexpr int REC = (1 + D) * NB;
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    extern __shared__ __align__(16) unsigned char smem[];

    const int L = a.lanes;
    const int cpw = blockDim.x / L;
    const int slot = threadIdx.x / L;
    const int t = threadIdx.x % L;
    const int M = a.M;

    const uint32_t k = xcd_block_order(blockIdx.x, gridDim.x) * (uint32_t)cpw + (uint32_t)slot;
    const bool live = k < a.K;

    unsigned char *base = smem + (size_t)slot * a.lds_per_cube;
    R *rows = reinterpret_cast<R *>(base);
    double *f64 = reinterpret_cast<double *>(base + (((size_t)M * SW * sizeof(R) + 15) & ~(size_t)15));
    double *G = f64;
    double *H = G + NB * NB;
    double *RHS = H + NB * NB;
    double *beta = RHS + REC;
    double *flag = beta + REC;
    double *zsum = flag + 2;

    // 1. the cloud C_{i,k}: paths in registers, regression inputs to LDS
    if (live) {
        for (int m = t; m < M; m += L) {
            R *row = rows + (size_t)m * SW;
            R Sp, y1;
            simulate_path<R, D, NB, LK>(a, cellF, bsig, lk, k, (uint32_t)m, row, row + NB, Sp, y1);
            row[NB + D] = Sp;
            row[NB + D + 1] = y1;
        }
    }
    __syncthreads();

    // 2. Gram entries (a <= b) and z right-hand sides, one entry per lane,
    //    binary64 sums over the M samples in sample order.
    constexpr int NG = NB * (NB + 1) / 2;
    constexpr int NE = NG + D * NB;
    if (live) {
        for (int e = t; e < NE; e += L) {
            double acc = 0.0;
            if (e < NG) {
                int r = 0, rem = e;
                while (rem >= NB - r) {
                    rem -= NB - r;
                    ++r;
                }
                const int c = r + rem;
                for (int m = 0; m < M; ++m) {
                    const R *row = rows + (size_t)m * SW;
                    acc += (double)row[r] * (double)row[c];
                }
                G[r * NB + c] = acc;
                G[c * NB + r] = acc;
            } else {
                const int l = (e - NG) / NB, b = (e - NG) % NB;
                for (int m = 0; m < M; ++m) {
                    const R *row = rows + (size_t)m * SW;
                    acc += (double)row[b] * ((double)row[NB + D] * (double)row[NB + l]);
                }
                RHS[(1 + l) * NB + b] = acc * a.inv_dt;
            }
        }
    }
    __syncthreads();

    // 3. G^{-1} by Gauss-Jordan elimination without pivoting (G is symmetric
    //    positive definite), binary64, one entry per lane per pivot, two LDS
    //    buffers.  The pivots are the Schur complements, i.e. the squared
    //    diagonal of the Cholesky factor; a pivot <= 1e-12 trace(G) marks the
    //    stratum singular and it falls back to the LP0 mean.
    double tol = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) tol += G[b * NB + b];
    tol *= 1e-12;
    bool ok = live;
    double *src = G, *dst = H;
    for (int p = 0; p < NB; ++p) {
        const double piv = src[p * NB + p];
        ok = ok && piv > tol;
        const double inv = 1.0 / piv;
        if (live) {
            for (int e = t; e < NB * NB; e += L) {
                const int r = e / NB, c = e % NB;
                double v;
                if (r == p && c == p) v = inv;
                else if (r == p) v = src[p * NB + c] * inv;
                else if (c == p) v = -src[r * NB + p] * inv;
                else v = src[r * NB + c] - src[r * NB + p] * src[p * NB + c] * inv;
                dst[e] = v;
            }
        }
        __syncthreads();
        double *tmp = src;
        src = dst;
        dst = tmp;
    }
    const double *Ginv = src;
    if (live && !ok && t == 0) atomicAdd(counters + kCounterSingular, 1ull);

    // 4. z regressions: beta_{z_l} = G^{-1} RHS_{z_l}, one coefficient per lane
    if (live) {
        for (int e = t; e < D * NB; e += L) {
            const int c = e / NB, b = e % NB;
            const double *rhs = RHS + (1 + c) * NB;
            double v;
            if (ok) {
                v = 0.0;
#pragma unroll
                for (int u = 0; u < NB; ++u) v += Ginv[b * NB + u] * rhs[u];
            } else {
                v = b == 0 ? rhs[0] / M : 0.0;
            }
            beta[(1 + c) * NB + b] = v;
        }
    }
    __syncthreads();

    // 5. y responses S_Y = S' + f_i(X_i, y_{i+1}(X_{i+1}), z_i(X_i)) dt with the
    //    just-fitted (truncated) z_i, written over S' in LDS.  Without z
    //    truncation sum_l z_l(X_i) = (sum_l beta_{z_l}) . phi(X_i).
    const bool z_clamped = LK == kLookupFull;
    if (live && !z_clamped) {
        for (int b = t; b < NB; b += L) {
            double acc = 0.0;
            for (int c = 0; c < D; ++c) acc += beta[(1 + c) * NB + b];
            zsum[b] = acc;
        }
    }
    __syncthreads();
    if (live) {
        for (int m = t; m < M; m += L) {
            R *row = rows + (size_t)m * SW;
            R zs = (R)0;
            if (!z_clamped) {
#pragma unroll
                for (int b = 0; b < NB; ++b) zs += (R)zsum[b] * row[b];
            } else {
#pragma unroll 1
                for (int c = 0; c < D; ++c) {
                    R v = (R)0;
#pragma unroll
                    for (int b = 0; b < NB; ++b) v += (R)beta[(1 + c) * NB + b] * row[b];
                    zs += clamp_level<R>(v, a.clamp_z);
                }
            }
            row[NB + D] += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, row[NB + D + 1], zs) * a.dt;
        }
    }
    __syncthreads();

    // 6. y right-hand side and solve
    if (live) {
        for (int b = t; b < NB; b += L) {
            double acc = 0.0;
            for (int m = 0; m < M; ++m) {
                const R *row = rows + (size_t)m * SW;
                acc += (double)row[b] * (double)row[NB + D];
            }
            RHS[b] = acc;
        }
    }
    __syncthreads();
    if (live) {
        for (int b = t; b < NB; b += L) {
            double v;
            if (ok) {
                v = 0.0;
#pragma unroll
                for (int u = 0; u < NB; ++u) v += Ginv[b * NB + u] * RHS[u];
            } else {
                v = b == 0 ? RHS[0] / M : 0.0;
            }
            beta[b] = v;
        }
    }
    __syncthreads();

    // 7. store the record and its look-up projection
    if (live) {
        R *out = table + ((size_t)a.i * a.K + k) * REC;
        for (int e = t; e < REC; e += L) {
            const double v = beta[e];
            out[e] = (R)v;
            if (a.check_finite && !isfinite(v)) atomicAdd(counters + kCounterNonFinite, 1ull);
        }
        R *lrow = lk + ((size_t)a.i * a.K + k) * W;
        for (int e = t; e < W; e += L) {
            double v = 0.0;
            if constexpr (LK == kLookupFull) {
                if (e < REC) v = beta[e];
            } else {
                if (e < NB) {
                    v = beta[e];
                } else if (LK == kLookupYZ && e < 2 * NB) {
                    const int b = e - NB;
                    for (int c = 0; c < D; ++c) v += beta[(1 + c) * NB + b];
                }
            }
            lrow[e] = (R)v;
        }
    }
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
    hipLaunchKernelGGL((sweep_step_kernel<R, D, NB, LK>), dim3(s.blocks), dim3(s.threads),
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

size_t cube_lds_bytes(int prec_is_float, int d, int nb, int M)
{
    const size_t rsz = prec_is_float ? 4 : 8;
    size_t rows = (size_t)M * (nb + d + 2) * rsz;
    rows = (rows + 15) & ~(size_t)15;
    return rows + (size_t)(2 * nb * nb + 2 * (1 + d) * nb + 2 + nb) * sizeof(double);
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
