// Device code of one backward step of the SRMDP sweep (Algorithm SRMDP,
// Section 3.1, eq. (PsiM)): simulation of the clouds, responses with table
// look-ups, the per-stratum regressions and the table writes.  Included by the
// translation units that instantiate the sweep kernels (with and without the
// learned control variate).
#pragma once

#include "srmdp_device.hpp"
#include "srmdp_internal.hpp"
#include "srmdp_mlp.hpp"

namespace srmdp {

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
// Equal-probability cells (the cells of dimension l cut at the logistic
// quantiles F^{-1}(c / n)): the coordinate is t = n F(x), F(x) = 1/(1 + e^{-mu x}),
// and mu times the offset of x from the nu-median of cell c is
// mu x - log((c + 1/2) / (n - c - 1/2)).
template <>
struct RealOps<float> {
    // v_med3_f32 also maps +-inf into [0, cmax]; a NaN stays NaN and the index
    // conversion then yields stratum 0
    static __device__ __forceinline__ float clamp_cell(float t, float cmax)
    {
        return __builtin_amdgcn_fmed3f(floorf(t), 0.0f, cmax);
    }
    static __device__ __forceinline__ float prob_coord(float x, float mu, float n)
    {
        return __fdividef(n, 1.0f + __expf(-mu * x));  // n / inf = 0 far below the grid
    }
    static __device__ __forceinline__ float median_offset(float x, float mu, float c, float n)
    {
        return mu * x - __logf(__fdividef(c + 0.5f, n - c - 0.5f));
    }
};
template <>
struct RealOps<double> {
    static __device__ __forceinline__ double clamp_cell(double t, double cmax)
    {
        return fmin(fmax(floor(t), 0.0), cmax);
    }
    static __device__ __forceinline__ double prob_coord(double x, double mu, double n)
    {
        return n / (1.0 + exp(-mu * x));
    }
    static __device__ __forceinline__ double median_offset(double x, double mu, double c, double n)
    {
        return mu * x - log((c + 0.5) / (n - c - 0.5));
    }
};

// Coordinate of x along dimension l in cell widths: (x - lo) cells / (hi - lo)
// for equal-size cells, n F(x) for equal-probability cells (EP).  The grid
// kind is a template parameter so that the equal-size kernels carry none of
// the other kind's code.
template <typename R, bool EP>
__device__ __forceinline__ R cell_coord(const StepArgs<R> &a, int l, R x)
{
    if constexpr (EP) return RealOps<R>::prob_coord(x, a.scale[l] + a.scale[l], a.cmax_f[l] + (R)1);
    return (x - a.lo[l]) * a.scale[l];
}

// Clamped cell c of x along dimension l and the LP1 coordinate xi of x in it
// (2 (t - c) - 1 for equal-size cells, mu (x - median) for equal-probability
// ones).
template <typename R, bool EP>
__device__ __forceinline__ R cell_and_xi(const StepArgs<R> &a, int l, R x, R &xi)
{
    const R t = cell_coord<R, EP>(a, l, x);
    const R c = RealOps<R>::clamp_cell(t, a.cmax_f[l]);
    if constexpr (EP)
        xi = RealOps<R>::median_offset(x, a.scale[l] + a.scale[l], c, a.cmax_f[l] + (R)1);
    else
        xi = (R)2 * (t - c) - (R)1;
    return c;
}

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

template <typename R, int D, bool EP>
__device__ __forceinline__ bool near_face(const StepArgs<R> &a, const R *x)
{
    bool near = false;
    for (int l = 0; l < D; ++l) {
        const R t = cell_coord<R, EP>(a, l, x[l]);
        near |= near_interior_face<R>(t, RealOps<R>::clamp_cell(t, a.cmax_f[l]), a.cmax_f[l],
                                      a.face_eps);
    }
    return near;
}

// Cell of x per dimension, clamped to the grid (equal-size cells:
// floor((x - lo) cells / (hi - lo)), xi = 2 (t - cell) - 1; equal-probability
// cells: t = C F(x), xi = mu (x - m_c) with the cell's nu-median m_c read from
// the sampler's table instead of its logarithm), and the offset of the
// stratum's look-up record in a row.  The stratum index is accumulated in the
// working precision, exact because K <= 2^24; K W < 2^32 so the offset is a
// 24-bit product.
template <typename R, int D, int NB, int LK, bool EP>
__device__ __forceinline__ uint32_t locate(const StepArgs<R> &a, const R *x, R *xi)
{
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    R kf = (R)0;
    if constexpr (EP) {
        const CellF<R> *med = (const CellF<R> *)a.cell_table;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const R mu = a.scale[l] + a.scale[l];
            const R c = RealOps<R>::clamp_cell(cell_coord<R, true>(a, l, x[l]), a.cmax_f[l]);
            xi[l] = mu * (x[l] - med[l * a.cmax + (int)c].centre);
            kf = c * a.stride_f[l] + kf;
        }
    } else {
#pragma unroll
        for (int l = 0; l < D; ++l) kf = cell_and_xi<R, false>(a, l, x[l], xi[l]) * a.stride_f[l] + kf;
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

template <typename R, int D, int NB, int LK, bool EP>
__device__ __forceinline__ void lookup_eval(const StepArgs<R> &a, const R *__restrict__ row, const R *x,
                                            R &y, R &zsum)
{
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    R xi[D], rec[W];
    load_record<R, W>(row + locate<R, D, NB, LK, EP>(a, x, xi), rec);
    eval_record<R, D, NB, LK>(a, rec, xi, y, zsum);
}

// Fitted y_j(x) and every z_{j,c}(x), each truncated, from a whole record
// (look-up mode Full): what a model's own driver f(t, x, y, z) reads.
template <typename R, int D, int NB, bool EP>
__device__ __forceinline__ void lookup_eval_full(const StepArgs<R> &a, const R *__restrict__ row, const R *x,
                                                 R &y, R *z)
{
    constexpr int W = LookupWidth<R, D, NB, kLookupFull>::value;
    R xi[D], rec[W];
    load_record<R, W>(row + locate<R, D, NB, kLookupFull, EP>(a, x, xi), rec);
#pragma unroll
    for (int c = 0; c <= D; ++c) {
        R v = rec[c * NB];
        if constexpr (NB > 1) {
#pragma unroll
            for (int l = 0; l < D; ++l) v += rec[c * NB + 1 + l] * xi[l];
        }
        if (c == 0)
            y = clamp_level<R>(v, a.clamp_y);
        else
            z[c - 1] = clamp_level<R>(v, a.clamp_z);
    }
}

// X_{j+1} = X_j + b(X_j) dt + sigma dW_j (Algorithm "Euler dynamics", read with
// the time index of the current step), with b(x)_l = b_l + b_lin_l x_l: exact
// for constant b, the Euler scheme of the Ornstein-Uhlenbeck drift otherwise.
// bsig holds b [D], sigma [D][D] and b_lin [D].
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
    if (a.has_lin_drift) {
#pragma unroll
        for (int l = 0; l < D; ++l) xn[l] += bsig[D + D * D + l] * x[l] * a.dt;
    }
    if (a.has_lin_sigma) {  // sigma(X_j) = sigma + diag(sigma_lin) X_j
#pragma unroll
        for (int l = 0; l < D; ++l) xn[l] += bsig[2 * D + D * D + l] * x[l] * dW[l];
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

// The problem data of eq. (fbsde): drift, diffusion, driver and terminal
// condition.  BuiltinModel is the compiled families (drift and diffusion
// affine in the state, the linear and logistic drivers through sum_l z_l, the
// cos and logistic terminals), read from StepArgs and the bsig block.  A model
// compiled at run time from a caller's source (srmdp_model) has kUser = true
// and supplies
//   step(a, p, t, x, dW, xn)      X_{j+1} = X_j + b(t_j, X_j) dt + sigma(t_j, X_j) dW_j,
//   driver(a, p, t, x, y, z)      f(t, x, y, z) with every component of z,
//   terminal(a, p, x)             g(x),
// with p its parameters (in the bsig block); its look-ups read whole records.
struct BuiltinModel {
    static constexpr bool kUser = false;
};

template <typename R, int D, class Model>
__device__ __forceinline__ void model_step(const StepArgs<R> &a, const R *__restrict__ bsig, int j, const R *x,
                                           const R *dW, R *xn)
{
    if constexpr (Model::kUser)
        Model::template step<R, D>(a, bsig, (R)j * a.dt, x, dW, xn);
    else
        euler_step<R, D>(a, bsig, x, dW, xn);
}

template <typename R, int D, class Model>
__device__ __forceinline__ R model_terminal(const StepArgs<R> &a, const R *__restrict__ bsig, const R *x)
{
    if constexpr (Model::kUser)
        return Model::template terminal<R, D>(a, bsig, x);
    else
        return terminal_at<R, D>(a, x);
}

// The control-variate network as one wavefront sees it (unused without it).
struct CvWave {
    MlpWeights w;
    int lane;
};

// One simulation from X_i = x (eq. (PsiM)): the Euler scheme to X_N with the
// fitted rows i+1..N-1, returning dW_i, y_{i+1}(X_{i+1}) (g(X_N) when
// i + 1 = N) and the tail response
//   S' = g(X_N) + sum_{j=i+1}^{N-1} f_j(X_j, y_{j+1}(X_{j+1}), z_j(X_j)) dt.
// With the control variate (CV), S' also loses the martingale increments
// sum_{j=i+1}^{N-1} z_theta(t_j', X_j') . dW_j, whose conditional mean given
// X_i is zero (j' = i + stride floor((j - i) / stride): the network is
// evaluated every `cv_stride` steps and its last value weighs the increments
// in between), and cvi = z_theta(t_i, X_i) . dW_i is returned for the y
// response; every lane of the wavefront must then run the same steps.
// The first and last steps are peeled off so that the steady loop has no
// branch that depends on j.
// PF, the depth of the gather pipeline (built-in problems without the control
// variate): the positions do not depend on the fitted rows, so with PF = 1
// X_{j+2} is formed and its record requested while the record of X_{j+1} is
// evaluated (one gather in flight across a step's arithmetic), and with PF = 2
// X_{j+3} while the records of X_{j+1} and X_{j+2} are held (two in flight).
// The same operations in the same order as the plain loop: PF = 1 compiles
// to the same bits, PF = 2 (whose loop the compiler unrolls) agrees with them
// to rounding.
template <typename R, int D, int NB, int LK, bool CV = false, bool EP = false, class Model = BuiltinModel,
          int PF = 0>
__device__ __forceinline__ void run_path(const StepArgs<R> &a, const R *__restrict__ bsig,
                                         const R *__restrict__ lk, NormalStream<R, D> &ns, R *x,
                                         R *dWi_out, R &y1, R &Sp, const CvWave *cv = nullptr,
                                         R *cvi = nullptr)
{
    static_assert(!CV || sizeof(R) == 4, "the control variate runs in binary32");
    static_assert(!Model::kUser || (LK == kLookupFull && !CV), "a model's driver reads whole records");
    constexpr int W = LookupWidth<R, D, NB, LK>::value;
    const int i = a.i, N = a.N;
    const size_t row_elems = (size_t)a.K * W;
    const R dt = a.dt;
    R dW[D], xn[D];
    R cv_tail = (R)0;
    R zc[CV ? D : 1];  // the network's last value
    auto cv_dot = [&](const R *dw) {
        R s = (R)0;
#pragma unroll
        for (int l = 0; l < D; ++l) s += zc[l] * dw[l];
        return s;
    };
    ns.step(0u, dW);
    if constexpr (CV) {
        mlp_eval_z<D, D>(cv->w, cv->lane, (R)i * dt, x, zc);
        *cvi = cv_dot(dW);
    }
    model_step<R, D, Model>(a, bsig, i, x, dW, xn);
    R zsum_cur = (R)0;
    R zv_cur[Model::kUser ? D : 1];  // z_j(X_j), every component (a model's driver)
    if (i + 1 < N) {
        if constexpr (Model::kUser)
            lookup_eval_full<R, D, NB, EP>(a, lk + (size_t)(i + 1) * row_elems, xn, y1, zv_cur);
        else
            lookup_eval<R, D, NB, LK, EP>(a, lk + (size_t)(i + 1) * row_elems, xn, y1, zsum_cur);
    } else {
        y1 = model_terminal<R, D, Model>(a, bsig, xn);
    }
#pragma unroll
    for (int l = 0; l < D; ++l) {
        dWi_out[l] = dW[l];
        x[l] = xn[l];
    }
    R S = (R)0;
    if constexpr (PF == 2 && !CV && !Model::kUser) {
        constexpr int V = LookupWidth<R, D, NB, LK>::value;
        // Records of X_{j+1} (A) and X_{j+2} (B) in flight while X_{j+3} is formed
        // and its record (C) requested: two gathers stay in flight across a step.
        const int nf = N - i - 2;  // driver terms f_j, j = i+1..N-2, from rows i+2..N-1
        if (nf >= 1) {
            R xiA[D], recA[V], xiB[D], recB[V];
            ns.step(1u, dW);
            model_step<R, D, Model>(a, bsig, i + 1, x, dW, xn);
            load_record<R, V>(lk + (size_t)(i + 2) * row_elems + locate<R, D, NB, LK, EP>(a, xn, xiA), recA);
#pragma unroll
            for (int l = 0; l < D; ++l) x[l] = xn[l];
            if (nf >= 2) {
                ns.step(2u, dW);
                model_step<R, D, Model>(a, bsig, i + 2, x, dW, xn);
                load_record<R, V>(lk + (size_t)(i + 3) * row_elems + locate<R, D, NB, LK, EP>(a, xn, xiB), recB);
#pragma unroll
                for (int l = 0; l < D; ++l) x[l] = xn[l];
            }
            for (int j = i + 1; j < N - 3; ++j) {
                // X_{j+3} from X_{j+2}, and its record requested
                ns.step((uint32_t)(j + 2 - i), dW);
                model_step<R, D, Model>(a, bsig, j + 2, x, dW, xn);
                R xiC[D], recC[V];
                load_record<R, V>(lk + (size_t)(j + 3) * row_elems + locate<R, D, NB, LK, EP>(a, xn, xiC), recC);
                // f_j from the record of X_{j+1}
                R yn, zn;
                eval_record<R, D, NB, LK>(a, recA, xiA, yn, zn);
                S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
                zsum_cur = zn;
#pragma unroll
                for (int l = 0; l < D; ++l) {
                    x[l] = xn[l];
                    xiA[l] = xiB[l];
                    xiB[l] = xiC[l];
                }
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    recA[v] = recB[v];
                    recB[v] = recC[v];
                }
            }
            // the last one or two terms, f_{N-3} and f_{N-2}, from the records in flight
            R yn, zn;
            eval_record<R, D, NB, LK>(a, recA, xiA, yn, zn);
            S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
            zsum_cur = zn;
            if (nf >= 2) {
                eval_record<R, D, NB, LK>(a, recB, xiB, yn, zn);
                S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
                zsum_cur = zn;
            }
        }
    } else if constexpr (PF == 1 && !CV && !Model::kUser) {
        constexpr int V = LookupWidth<R, D, NB, LK>::value;
        if (i + 1 < N - 1) {
            // X_{i+2} and the request of its record (row i+2)
            ns.step(1u, dW);
            model_step<R, D, Model>(a, bsig, i + 1, x, dW, xn);
            R xi[D], rec[V];
            load_record<R, V>(lk + (size_t)(i + 2) * row_elems + locate<R, D, NB, LK, EP>(a, xn, xi), rec);
#pragma unroll
            for (int l = 0; l < D; ++l) x[l] = xn[l];
            for (int j = i + 1; j < N - 2; ++j) {
                // X_{j+2} from X_{j+1}, and its record requested
                ns.step((uint32_t)(j + 1 - i), dW);
                model_step<R, D, Model>(a, bsig, j + 1, x, dW, xn);
                R xi2[D], rec2[V];
                load_record<R, V>(lk + (size_t)(j + 2) * row_elems + locate<R, D, NB, LK, EP>(a, xn, xi2), rec2);
                // f_j from the record of X_{j+1}
                R yn, zn;
                eval_record<R, D, NB, LK>(a, rec, xi, yn, zn);
                S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
                zsum_cur = zn;
#pragma unroll
                for (int l = 0; l < D; ++l) {
                    x[l] = xn[l];
                    xi[l] = xi2[l];
                }
#pragma unroll
                for (int v = 0; v < V; ++v) rec[v] = rec2[v];
            }
            // f_{N-2} from the record of X_{N-1}
            R yn, zn;
            eval_record<R, D, NB, LK>(a, rec, xi, yn, zn);
            S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
            zsum_cur = zn;
        }
    } else
    for (int j = i + 1; j < N - 1; ++j) {
        ns.step((uint32_t)(j - i), dW);
        if constexpr (CV) {
            if ((j - i) % a.cv_stride == 0) mlp_eval_z<D, D>(cv->w, cv->lane, (R)j * dt, x, zc);
            cv_tail += cv_dot(dW);
        }
        model_step<R, D, Model>(a, bsig, j, x, dW, xn);
        if constexpr (Model::kUser) {
            R yn, zn[D];
            lookup_eval_full<R, D, NB, EP>(a, lk + (size_t)(j + 1) * row_elems, xn, yn, zn);
            S += Model::template driver<R, D>(a, bsig, (R)j * dt, x, yn, zv_cur) * dt;
#pragma unroll
            for (int l = 0; l < D; ++l) zv_cur[l] = zn[l];
        } else {
            R yn, zn;
            lookup_eval<R, D, NB, LK, EP>(a, lk + (size_t)(j + 1) * row_elems, xn, yn, zn);
            S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, yn, zsum_cur) * dt;
            zsum_cur = zn;
        }
#pragma unroll
        for (int l = 0; l < D; ++l) x[l] = xn[l];
    }
    R gN;
    if (i < N - 1) {
        ns.step((uint32_t)(N - 1 - i), dW);
        if constexpr (CV) {
            if ((N - 1 - i) % a.cv_stride == 0) mlp_eval_z<D, D>(cv->w, cv->lane, (R)(N - 1) * dt, x, zc);
            cv_tail += cv_dot(dW);
        }
        model_step<R, D, Model>(a, bsig, N - 1, x, dW, xn);
        gN = model_terminal<R, D, Model>(a, bsig, xn);
        if constexpr (Model::kUser)
            S += Model::template driver<R, D>(a, bsig, (R)(N - 1) * dt, x, gN, zv_cur) * dt;
        else
            S += driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, gN, zsum_cur) * dt;
    } else {
        gN = y1;
    }
    Sp = gN + S - cv_tail;
}

// One simulation of stratum k from step i: X_i ~ nu_k by Algorithm
// "stratify" (phi(X_i) to full precision from the centred offset), then
// run_path.  phi(X_i) and dW_i go to the stratum's LDS row as soon as they are
// known, so they do not occupy registers during the path.
template <typename R, int D, int NB, typename CellAt>
__device__ __forceinline__ void sample_start_with(const StepArgs<R> &a, CellAt cell_at, uint32_t k, uint32_t m,
                                                  R *x, R *phi_out)
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
                const CellF<R> cf = cell_at(l);
                const R off = stratified_offset<R>(cf, open_uniform<R>(ws[t]), a.inv_mu);
                x[l] = cf.centre + off;
                // xi = 2 scale (x - centre): 2 (x - c) / h, or mu times the offset
                // from the cell's nu-median (the centre of an equal-probability cell)
                if constexpr (NB > 1) phi_out[1 + l] = (off + off) * a.scale[l];
            }
        }
    }
    phi_out[0] = (R)1;
}

// The cell constants of stratum k along dimension l.
template <typename R>
__device__ __forceinline__ CellF<R> stratum_cell(const StepArgs<R> &a, const CellF<R> *__restrict__ cellF, uint32_t k,
                                                 int l)
{
    return cellF[l * a.cmax + (k / a.stride[l]) % a.cells[l]];
}

// Start point from the sampler's table (cell of each dimension from k).
template <typename R, int D, int NB>
__device__ __forceinline__ void sample_start(const StepArgs<R> &a, const CellF<R> *__restrict__ cellF,
                                             uint32_t k, uint32_t m, R *x, R *phi_out)
{
    sample_start_with<R, D, NB>(a, [&](int l) { return stratum_cell<R>(a, cellF, k, l); }, k, m, x, phi_out);
}

// Start point from the stratum's own cell constants scf[0..D-1] (stratum_cell
// of every dimension, formed once per stratum in LDS by the sweep).
template <typename R, int D, int NB>
__device__ __forceinline__ void sample_start_cached(const StepArgs<R> &a, const CellF<R> *scf, uint32_t k,
                                                    uint32_t m, R *x, R *phi_out)
{
    sample_start_with<R, D, NB>(a, [&](int l) { return scf[l]; }, k, m, x, phi_out);
}

// With the control variate and z_center, *centre = y_{i+1}(X_i) (g(X_i) when
// i + 1 = N): the fitted row i+1 of the stratum itself (X_i lies in it),
// truncated, whose product with dW_i / dt has conditional mean zero.
// scf: the stratum's cell constants (sample_start_cached).
template <typename R, int D, int NB, int LK, bool CV, bool EP, class Model = BuiltinModel, int PF = 0>
__device__ __forceinline__ void simulate_path(const StepArgs<R> &a, const CellF<R> *scf,
                                              const R *__restrict__ bsig, const R *__restrict__ lk,
                                              uint32_t k, uint32_t m, R *phi_out, R *dWi_out,
                                              R &Sp, R &y1, const CvWave *cv, R *cvi, R *centre)
{
    R x[D];
    sample_start_cached<R, D, NB>(a, scf, k, m, x, phi_out);
    if constexpr (CV) {
        R c = (R)0;
        if (a.z_center) {
            if (a.i + 1 < a.N) {
                constexpr int W = LookupWidth<R, D, NB, LK>::value;
                const R *rec = lk + ((size_t)(a.i + 1) * a.K + k) * W;
#pragma unroll
                for (int b = 0; b < NB; ++b) c += rec[b] * phi_out[b];
                c = clamp_level<R>(c, a.clamp_y);
            } else {
                c = terminal_at<R, D>(a, x);
            }
        }
        *centre = c;
    }
    NormalStream<R, D> ns;
    ns.init(Key{a.key0, a.key1}, m, k, a.tag, a.sqrt_dt);
    run_path<R, D, NB, LK, CV, EP, Model, PF>(a, bsig, lk, ns, x, dWi_out, y1, Sp, cv, cvi);
}

// Near-face diagnostic of step i: the positions of a simulation do not depend
// on the fitted rows, so they are recomputed here with the same draws and the
// same Euler steps as the sweep, and stratum k is marked when one of its
// simulations reaches a look-up point within face_eps of an interior face.
// One wavefront per stratum.
template <typename R, int D, int NB, bool EP, class Model = BuiltinModel>
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
            model_step<R, D, Model>(a, bsig, j, x, dW, xn);
            near |= near_face<R, D, EP>(a, xn);
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
// LDS of one stratum: M rows of (phi, dW_i, S', y_{i+1}(X_{i+1}) [, cvi,
// centre]) in the working precision, then the binary64 Gram, its inverse,
// right-hand sides, coefficients, flags and the summed z coefficients.  With
// the control variate the S' column holds S' - centre, the z response's
// numerator.
template <typename R, int D, int NB, bool CV = false>
struct CubeLds {
    static constexpr int SW = NB + D + 2 + (CV ? 2 : 0);
    static constexpr int F64 = 2 * NB * NB + 2 * (1 + D) * NB + 2 + NB;
    static constexpr int NE = NB * (NB + 1) / 2 + D * NB;  // Gram and z right-hand-side entries
};

// Sums over the samples run in chunks of kChunk in sample order; with more
// than one chunk the chunk sums (one per lane and entry, in parallel) are
// added in chunk order.  The order depends on M only, not on the lanes.
constexpr int kChunk = 64;

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

// One group of strata of backward step a.i: the workgroup's cpw = blockDim / L
// strata k = group * cpw + slot, L = a.lanes lanes each.  Shared by the
// per-step kernel and the batched (several instances) kernel.
//
// Clouds in LDS (GR = false): the M rows of regression inputs of a stratum are
// held in LDS, then the sums run over them.
// Streamed clouds (GR = true, clouds too large for LDS): the samples are
// simulated in rounds of RS = max(L, kChunk) (whole chunks); a round's rows
// live in an LDS window, their chunk sums are added to running sums in chunk
// order (the same additions, in the same order, as the LDS form), and only
// S' and y_{i+1}(X_{i+1}) of each sample go to global memory (a.grows,
// a.grow_bytes per stratum).  The y pass draws X_i and phi(X_i) again from the
// same counter and reads S', y_{i+1} back.  The launch covers strata
// a.k0 .. a.k_end-1.
template <typename R, int D, int NB, int LK, bool CV, bool GR = false, bool EP = false, class Model = BuiltinModel,
          int PF = 0>
__device__ __forceinline__ void sweep_group(const StepArgs<R> &a, uint32_t group,
                                            const CellF<R> *__restrict__ cellF,
                                            const R *__restrict__ bsig, R *__restrict__ lk,
                                            R *__restrict__ table,
                                            unsigned long long *__restrict__ counters,
                                            unsigned char *smem)
{
    static_assert(!(GR && CV), "streamed clouds run without the control variate");
    using Lay = CubeLds<R, D, NB, CV>;
    constexpr int SW = Lay::SW;
    constexpr int REC = (1 + D) * NB;
    constexpr int W = LookupWidth<R, D, NB, LK>::value;

    const int L = a.lanes;
    const int cpw = blockDim.x / L;
    const int slot = threadIdx.x / L;
    const int t = threadIdx.x % L;
    const int M = a.M;

    const uint32_t k = (GR ? a.k0 : 0u) + group * (uint32_t)cpw + (uint32_t)slot;
    const bool live = k < (GR ? a.k_end : a.K);

    // With the control variate the workgroup first copies the network's
    // forward weights to LDS; the strata follow them.
    CvWave cv;
    if constexpr (CV) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.cv_packed);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (int v = threadIdx.x; v < (int)(kPackedFwdBytes / 16); v += blockDim.x) dst[v] = src[v];
        cv.w.bias = reinterpret_cast<const float *>(smem);
        cv.w.frag = reinterpret_cast<const bf16x8 *>(smem + kPackedBiasBytes);
        cv.lane = threadIdx.x & 63;
        __syncthreads();
    }
    unsigned char *base = smem + (CV ? kPackedFwdBytes : 0) + (size_t)slot * a.lds_per_cube;
    // The stratum's cell constants along each dimension, formed once here for
    // every start point of the stratum (slots past the last stratum: K - 1).
    CellF<R> *scf = reinterpret_cast<CellF<R> *>(base);
    base += (D * sizeof(CellF<R>) + 15) & ~(size_t)15;
    {
        // compile-time dimension indices: the batched kernel holds `a` in
        // registers, where a run-time index would put it in scratch memory
        const uint32_t ks = live ? k : a.K - 1;
#pragma unroll
        for (int l = 0; l < D; ++l)
            if (l % L == t) scf[l] = stratum_cell<R>(a, cellF, ks, l);
    }
    __syncthreads();
    const size_t row_bytes = ((size_t)(CV ? M + 1 : M) * SW * sizeof(R) + 15) & ~(size_t)15;
    constexpr int NG = NB * (NB + 1) / 2;
    constexpr int NE = Lay::NE;
    // LDS form: rows [M][SW], then the binary64 arrays, then the chunk sums.
    // Streamed form: the binary64 arrays, the partial sums of a.stage_chunks
    // chunks, then the window of RS rows; S', y1 per sample in global memory.
    R *rows;
    double *f64;
    R *sy = nullptr;
    if constexpr (GR) {
        sy = reinterpret_cast<R *>(a.grows + (size_t)(group * (uint32_t)cpw + (uint32_t)slot) * a.grow_bytes);
        f64 = reinterpret_cast<double *>(base);
        rows = reinterpret_cast<R *>(base + ((sizeof(double) * ((size_t)Lay::F64 + (size_t)NE * a.stage_chunks) +
                                              15) & ~(size_t)15));
    } else {
        rows = reinterpret_cast<R *>(base);
        f64 = reinterpret_cast<double *>(base + row_bytes);
    }
    double *G = f64;
    double *H = G + NB * NB;
    double *RHS = H + NB * NB;
    double *beta = RHS + REC;
    double *flag = beta + REC;
    double *zsum = flag + 2;
    // [entries][chunks] partial sums when M > kChunk (streamed: [entries][a.stage_chunks])
    double *part = zsum + NB;
    const int nch = (M + kChunk - 1) / kChunk;

    constexpr int kSumUnroll = 8;  // per-sample sums: loads of later samples issue ahead
    // Gram entries (a <= b) and z right-hand sides: binary64 sums over samples
    // m0..m1-1 of a block of rows, in sample order.
    auto gram_sum = [&](const R *rb, int e, int m0, int m1) {
        double acc = 0.0;
        if (e < NG) {
            int r = 0, rem = e;
            while (rem >= NB - r) {
                rem -= NB - r;
                ++r;
            }
            const int c = r + rem;
            // the additions stay in sample order
#pragma unroll kSumUnroll
            for (int m = m0; m < m1; ++m) {
                const R *row = rb + (size_t)m * SW;
                acc += (double)row[r] * (double)row[c];
            }
        } else {
            const int l = (e - NG) / NB, b = (e - NG) % NB;
#pragma unroll kSumUnroll
            for (int m = m0; m < m1; ++m) {
                const R *row = rb + (size_t)m * SW;
                acc += (double)row[b] * ((double)row[NB + D] * (double)row[NB + l]);
            }
        }
        return acc;
    };
    // Work items of the Gram and z right-hand-side sums: up to three entries
    // that share a column value v_m = row[x] row[y] and take their other
    // factor from row[a_k]; each entry sums row[a_k] v_m in binary64 over the
    // samples, in sample order.
    //   Gram entry (r, c), r <= c: v = row[c] row[0], which is row[c] exactly
    //   (phi_0 = 1), a = r; items run down a column c, rows 3j..3j+2 <= c.
    //   z right-hand side (l, b): v = S' dW_l, a = b; items take b = 3j..3j+2.
    // One item per lane (entry triples share the loads and the product of v);
    // the sums are those of one entry per lane, operation for operation, so
    // both forms give the same bits.  The items take more registers, so they
    // run only where they save rounds of the lanes: the streamed-cloud kernels
    // of LP1 at d >= 12 (two to seven rounds of entries per chunk set before,
    // one to three after), and the binary32 kernels with clouds in LDS when
    // there are more entries than 64 (LP1 at d >= 6: at d = 8, 117 entries in
    // two divergent rounds against 42 items in one) and the lanes of the launch
    // take fewer rounds of items than of entries.  There the samples of an
    // item unroll by four: by eight the headline kernel's plain path loop went
    // from 94 to 111 VGPRs, one wavefront per SIMD fewer.  The others, and the
    // control variate, sum one entry per lane.
    constexpr bool kItems = GR && NB >= 13;
    constexpr bool kItemsLds = !GR && !CV && NE > 64 && sizeof(R) == 4;
    constexpr int kItemUnroll = GR ? kSumUnroll : 4;
    constexpr int NTR3 = (NB + 2) / 3;  // right-hand-side items per component
    constexpr int NTG = [] {
        int n = 0;
        for (int c = 0; c < NB; ++c) n += (c + 3) / 3;
        return n;
    }();
    constexpr int NT = NTG + D * NTR3;
    struct SumItem {
        int x, y, a[3], e[3], n;
    };
    auto sum_item = [&](int w) {
        SumItem it;
        if (w < NTG) {
            int c = 0, j = w;
            while (j >= (c + 3) / 3) {
                j -= (c + 3) / 3;
                ++c;
            }
            it.x = c;
            it.y = 0;
            it.n = min(3, c + 1 - 3 * j);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int r = 3 * j + (k < it.n ? k : 0);
                it.a[k] = r;
                it.e[k] = r * NB - r * (r - 1) / 2 + (c - r);  // packed upper triangle
            }
        } else {
            const int l = (w - NTG) / NTR3, j = (w - NTG) % NTR3;
            it.x = NB + D;
            it.y = NB + l;
            it.n = min(3, NB - 3 * j);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int b = 3 * j + (k < it.n ? k : 0);
                it.a[k] = b;
                it.e[k] = NG + l * NB + b;
            }
        }
        return it;
    };
    auto item_sums = [&](const R *rb, const SumItem &it, int m0, int m1, double *acc) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll kItemUnroll
        for (int m = m0; m < m1; ++m) {
            const R *row = rb + (size_t)m * SW;
            const double v = (double)row[it.x] * (double)row[it.y];
            s0 += (double)row[it.a[0]] * v;
            s1 += (double)row[it.a[1]] * v;
            s2 += (double)row[it.a[2]] * v;
        }
        acc[0] = s0;
        acc[1] = s1;
        acc[2] = s2;
    };
    // Where entry e is kept: the upper triangle of G, or the z right-hand side.
    auto entry_slot = [&](int e) -> double * {
        if (e < NG) {
            int r = 0, rem = e;
            while (rem >= NB - r) {
                rem -= NB - r;
                ++r;
            }
            return G + r * NB + r + rem;
        }
        const int l = (e - NG) / NB, b = (e - NG) % NB;
        return RHS + (1 + l) * NB + b;
    };
    auto gram_store = [&](int e, double acc) {
        if (e < NG) {
            int r = 0, rem = e;
            while (rem >= NB - r) {
                rem -= NB - r;
                ++r;
            }
            const int c = r + rem;
            const double g = k == a.debug_singular ? 0.0 : acc;
            G[r * NB + c] = g;
            G[c * NB + r] = g;
        } else {
            const int l = (e - NG) / NB, b = (e - NG) % NB;
            RHS[(1 + l) * NB + b] = acc * a.inv_dt;
        }
    };

    if constexpr (GR) {
        // 1-2 (streamed). Rounds of RS samples: simulate into the window, then
        //    add the round's chunk sums (a.stage_chunks chunks at a time) to the
        //    running sums kept in place, in chunk order.
        const int RS = L >= kChunk ? L : kChunk;
        const int pb = a.stage_chunks;
        if (live) {
            for (int e = t; e < NB * NB; e += L) G[e] = 0.0;
            for (int e = t; e < REC; e += L) RHS[e] = 0.0;
        }
        for (int r0 = 0; r0 < M; r0 += RS) {
            const int rn = min(RS, M - r0);
            if (live) {
                for (int u = t; u < rn; u += L) {
                    const int m = r0 + u;
                    R *row = rows + (size_t)u * SW;
                    R Sp, y1, cvi, centre;
                    simulate_path<R, D, NB, LK, false, EP, Model>(a, scf, bsig, lk, k, (uint32_t)m, row, row + NB,
                                                                  Sp, y1, &cv, &cvi, &centre);
                    row[NB + D] = Sp;
                    row[NB + D + 1] = y1;
                    sy[2 * (size_t)m] = Sp;
                    sy[2 * (size_t)m + 1] = y1;
                }
            }
            __syncthreads();
            const int rc = (rn + kChunk - 1) / kChunk;
            for (int c0 = 0; c0 < rc; c0 += pb) {
                const int nbc = min(pb, rc - c0);
                // consecutive lanes take different entries (items) of one
                // chunk: rows kChunk apart would fall in the same LDS bank
                if (live) {
                    if constexpr (kItems) {
                        for (int w = t; w < NT * nbc; w += L) {
                            const int c = w / NT;
                            const SumItem it = sum_item(w % NT);
                            double acc[3];
                            item_sums(rows, it, (c0 + c) * kChunk, min(rn, (c0 + c + 1) * kChunk), acc);
#pragma unroll
                            for (int k = 0; k < 3; ++k)
                                if (k < it.n) part[it.e[k] * nbc + c] = acc[k];
                        }
                    } else {
                        for (int w = t; w < NE * nbc; w += L) {
                            const int e = w % NE, c = w / NE;
                            part[e * nbc + c] =
                                gram_sum(rows, e, (c0 + c) * kChunk, min(rn, (c0 + c + 1) * kChunk));
                        }
                    }
                }
                __syncthreads();
                if (live)
                    for (int e = t; e < NE; e += L) {
                        double *acc = entry_slot(e);
                        double v = *acc;
                        for (int c = 0; c < nbc; ++c) v += part[e * nbc + c];
                        *acc = v;
                    }
                __syncthreads();
            }
        }
        if (live)
            for (int e = t; e < NE; e += L) gram_store(e, *entry_slot(e));
    } else {
        // 1. the cloud C_{i,k}: paths in registers, regression inputs to LDS.  The
        //    network needs every lane of a wavefront, so with the control variate
        //    the slots past the last stratum simulate stratum K-1 and discard it,
        //    and every lane makes ceil(M / L) trips: the lanes past simulation M-1
        //    simulate one more (index >= M, a stream of its own) into the spare
        //    row M, which nothing reads.
        if (live || CV) {
            const uint32_t ks = live ? k : a.K - 1;
            const int mend = CV ? (M + L - 1) / L * L : M;
            for (int m = t; m < mend; m += L) {
                R *row = rows + (size_t)(CV ? (m < M ? m : M) : m) * SW;
                R Sp, y1, cvi, centre;
                simulate_path<R, D, NB, LK, CV, EP, Model, PF>(a, scf, bsig, lk, ks, (uint32_t)m, row, row + NB, Sp,
                                                           y1, &cv, &cvi, &centre);
                row[NB + D + 1] = y1;
                if constexpr (CV) {
                    row[NB + D] = Sp - centre;
                    row[NB + D + 2] = cvi;
                    row[NB + D + 3] = centre;
                } else {
                    row[NB + D] = Sp;
                }
            }
        }
        __syncthreads();

        // 2. Gram entries and z right-hand sides over the M samples, one
        //    (entry, chunk) pair per lane, then the chunks in order.
        // work items where they take fewer rounds of the lanes than single entries
        const bool items = kItemsLds && (NT * nch + L - 1) / L < (NE * nch + L - 1) / L;
        if (nch == 1) {
            if (live) {
                if (items) {
                    for (int w = t; w < NT; w += L) {
                        const SumItem it = sum_item(w);
                        double acc[3];
                        item_sums(rows, it, 0, M, acc);
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            if (k < it.n) gram_store(it.e[k], acc[k]);
                    }
                } else {
                    for (int e = t; e < NE; e += L) gram_store(e, gram_sum(rows, e, 0, M));
                }
            }
        } else {
            if (live) {
                if (items) {
                    for (int w = t; w < NT * nch; w += L) {
                        const int c = w / NT;
                        const SumItem it = sum_item(w % NT);
                        double acc[3];
                        item_sums(rows, it, c * kChunk, min(M, (c + 1) * kChunk), acc);
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            if (k < it.n) part[it.e[k] * nch + c] = acc[k];
                    }
                } else {
                    for (int w = t; w < NE * nch; w += L) {
                        const int e = w % NE, c = w / NE;
                        part[e * nch + c] = gram_sum(rows, e, c * kChunk, min(M, (c + 1) * kChunk));
                    }
                }
            }
            __syncthreads();
            if (live)
                for (int e = t; e < NE; e += L) {
                    double acc = 0.0;
                    for (int c = 0; c < nch; ++c) acc += part[e * nch + c];
                    gram_store(e, acc);
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
    //    just-fitted (truncated) z_i.  Without z truncation
    //    sum_l z_l(X_i) = (sum_l beta_{z_l}) . phi(X_i).
    const bool z_clamped = LK == kLookupFull;
    if (live && !z_clamped) {
        for (int b = t; b < NB; b += L) {
            double acc = 0.0;
            for (int c = 0; c < D; ++c) acc += beta[(1 + c) * NB + b];
            zsum[b] = acc;
        }
    }
    __syncthreads();
    // S_Y of one sample from phi(X_i), S' and y_{i+1}(X_{i+1}) (built-in drivers)
    auto y_response = [&](const R *phi, R Sp, R y1) -> R {
        R zs = (R)0;
        if (!z_clamped) {
#pragma unroll
            for (int b = 0; b < NB; ++b) zs += (R)zsum[b] * phi[b];
        } else {
#pragma unroll 1
            for (int c = 0; c < D; ++c) {
                R v = (R)0;
#pragma unroll
                for (int b = 0; b < NB; ++b) v += (R)beta[(1 + c) * NB + b] * phi[b];
                zs += clamp_level<R>(v, a.clamp_z);
            }
        }
        return Sp + driver_f<R>(a.driver, a.r, a.kappa, a.c_logistic, y1, zs) * a.dt;
    };
    if constexpr (GR) {
        // 5-6 (streamed). Rounds again: X_i and phi(X_i) drawn again from the
        //    same counter, S' and y_{i+1} read back; rows (phi, S_Y) in the
        //    window; y right-hand side summed as the Gram sums.
        constexpr int YW = NB + 1;
        const int RS = L >= kChunk ? L : kChunk;
        const int pb = a.stage_chunks;
        if (live)
            for (int b = t; b < NB; b += L) RHS[b] = 0.0;
        for (int r0 = 0; r0 < M; r0 += RS) {
            const int rn = min(RS, M - r0);
            if (live) {
                for (int u = t; u < rn; u += L) {
                    const int m = r0 + u;
                    R x[D], phi[NB];
                    sample_start_cached<R, D, NB>(a, scf, k, (uint32_t)m, x, phi);
                    R *row = rows + (size_t)u * YW;
#pragma unroll
                    for (int b = 0; b < NB; ++b) row[b] = phi[b];
                    if constexpr (Model::kUser) {
                        // the model's driver at X_i with every z_{i,c}(X_i), as in
                        // the clouds held in LDS
                        R z[D];
#pragma unroll 1
                        for (int c = 0; c < D; ++c) {
                            R v = (R)0;
#pragma unroll
                            for (int b = 0; b < NB; ++b) v += (R)beta[(1 + c) * NB + b] * phi[b];
                            z[c] = clamp_level<R>(v, a.clamp_z);
                        }
                        R Sy = sy[2 * (size_t)m];
                        Sy += Model::template driver<R, D>(a, bsig, (R)a.i * a.dt, x, sy[2 * (size_t)m + 1], z) *
                              a.dt;
                        row[NB] = Sy;
                    } else {
                        row[NB] = y_response(phi, sy[2 * (size_t)m], sy[2 * (size_t)m + 1]);
                    }
                }
            }
            __syncthreads();
            const int rc = (rn + kChunk - 1) / kChunk;
            for (int c0 = 0; c0 < rc; c0 += pb) {
                const int nbc = min(pb, rc - c0);
                if (live)
                    for (int w = t; w < NB * nbc; w += L) {
                        const int b = w % NB, c = c0 + w / NB;
                        double acc = 0.0;
#pragma unroll kSumUnroll
                        for (int m = c * kChunk; m < min(rn, (c + 1) * kChunk); ++m) {
                            const R *row = rows + (size_t)m * YW;
                            acc += (double)row[b] * (double)row[NB];
                        }
                        part[b * nbc + (c - c0)] = acc;
                    }
                __syncthreads();
                if (live)
                    for (int b = t; b < NB; b += L) {
                        double v = RHS[b];
                        for (int c = 0; c < nbc; ++c) v += part[b * nbc + c];
                        RHS[b] = v;
                    }
                __syncthreads();
            }
        }
    } else {
        if constexpr (Model::kUser) {
            // a model's driver reads X_i itself: drawn again from the same
            // counter (bit-identical to the cloud's start), and every z_{i,c}(X_i)
            if (live) {
                for (int m = t; m < M; m += L) {
                    R *row = rows + (size_t)m * SW;
                    R x[D], phi[NB], z[D];
                    sample_start_cached<R, D, NB>(a, scf, k, (uint32_t)m, x, phi);
#pragma unroll 1
                    for (int c = 0; c < D; ++c) {
                        R v = (R)0;
#pragma unroll
                        for (int b = 0; b < NB; ++b) v += (R)beta[(1 + c) * NB + b] * row[b];
                        z[c] = clamp_level<R>(v, a.clamp_z);
                    }
                    row[NB + D] +=
                        Model::template driver<R, D>(a, bsig, (R)a.i * a.dt, x, row[NB + D + 1], z) * a.dt;
                }
            }
        } else if (live) {
            for (int m = t; m < M; m += L) {
                R *row = rows + (size_t)m * SW;
                R Sp = row[NB + D];
                if constexpr (CV) Sp += row[NB + D + 3];
                R SY = y_response(row, Sp, row[NB + D + 1]);
                if constexpr (CV) SY -= row[NB + D + 2];
                row[NB + D] = SY;
            }
        }
        __syncthreads();

        // 6. y right-hand side (chunked as the Gram sums)
        auto y_sum = [&](const R *rb, int b, int m0, int m1) {
            double acc = 0.0;
#pragma unroll kSumUnroll
            for (int m = m0; m < m1; ++m) {
                const R *row = rb + (size_t)m * SW;
                acc += (double)row[b] * (double)row[NB + D];
            }
            return acc;
        };
        if (nch == 1) {
            if (live)
                for (int b = t; b < NB; b += L) RHS[b] = y_sum(rows, b, 0, M);
        } else {
            if (live)
                for (int w = t; w < NB * nch; w += L) {
                    const int b = w % NB, c = w / NB;
                    part[b * nch + c] = y_sum(rows, b, c * kChunk, min(M, (c + 1) * kChunk));
                }
            __syncthreads();
            if (live)
                for (int b = t; b < NB; b += L) {
                    double acc = 0.0;
                    for (int c = 0; c < nch; ++c) acc += part[b * nch + c];
                    RHS[b] = acc;
                }
        }
    }
    __syncthreads();
    // y solve
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

template <typename R, int D, int NB, int LK, bool CV, int PF = 0>
__global__ void __launch_bounds__(256) sweep_step_kernel(const StepArgs<R> a,
                                                        const CellF<R> *__restrict__ cellF,
                                                        const R *__restrict__ bsig,
                                                        R *__restrict__ lk, R *__restrict__ table,
                                                        unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<R, D, NB, LK, CV, false, false, BuiltinModel, PF>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF,
                                                              bsig, lk, table,
                                  counters, smem);
}

}  // namespace srmdp
