// Internal interface between the host runtime (srmdp_host.cpp) and the HIP
// kernels (srmdp_kernels.hip).  Not part of the public ABI.
#pragma once

#if !defined(__HIPCC_RTC__)  // under hipRTC the runtime is built in; the run-time source declares the integer types
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#endif

#include "../../include/srmdp.h"

namespace srmdp {

constexpr int kMaxDim = 19;

#if !defined(__HIPCC_RTC__)
// Records the message returned by srmdp_last_error() on this thread (host
// runtime, srmdp_host.cpp) and returns `s`.
srmdp_status set_error(srmdp_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
#endif

// What a look-up row holds for each stratum: the y coefficients only (the
// driver does not use z), y and the sum of the z_l coefficients (both built-in
// drivers depend on z only through sum_l z_l, and without truncation
// sum_l z_l(x) = (sum_l beta_{z_l}) . phi(x)), or the whole record (z
// truncation needs each component).
enum LookupMode { kLookupY = 0, kLookupYZ = 1, kLookupFull = 2 };

enum CounterIndex { kCounterSingular = 0, kCounterNonFinite = 1, kCounterNearFace = 2, kCounterCount = 4 };

template <typename R, int D, int NB, int LK>
struct LookupWidth {
    static constexpr int raw = LK == kLookupY ? NB : LK == kLookupYZ ? 2 * NB : (1 + D) * NB;
    static constexpr int align = sizeof(R) == 4 ? 4 : 2;  // 16-byte records
    static constexpr int value = (raw + align - 1) / align * align;
};

inline int lookup_width(int prec_is_float, int d, int nb, int lk)
{
    const int raw = lk == kLookupY ? nb : lk == kLookupYZ ? 2 * nb : (1 + d) * nb;
    const int align = prec_is_float ? 4 : 2;
    return (raw + align - 1) / align * align;
}

// Kernel arguments of one backward step (passed by value).
template <typename R>
struct StepArgs {
    R lo[kMaxDim];        // domain lower corner (equal-size cells)
    R scale[kMaxDim];     // cells / (hi - lo), or mu / 2 for equal-probability cells: the LP1
                          // coordinate is 2 scale (x - centre of the cell) in both cases
    R cmax_f[kMaxDim];    // cells - 1
    R stride_f[kMaxDim];  // stride of the stratum index (exact: K <= 2^24)
    uint32_t stride[kMaxDim];
    uint32_t cells[kMaxDim];
    int cmax;             // max cells over the dimensions (row length of the cell table)
    uint32_t K;
    int M, i, N;
    uint32_t key0, key1, tag;
    R dt, sqrt_dt, T, inv_mu;
    double dt_d, inv_dt;
    int driver, terminal;
    R r, kappa, c_logistic, clamp_y, clamp_z;
    int identity_sigma, has_drift, has_lin_drift, has_lin_sigma;
    int equal_prob;       // cells cut at the logistic quantiles F^{-1}(c / cells)
    const void *cell_table;  // the sampler's CellF<R> [d][cmax] (centre = nu-median of an
                             // equal-probability cell), read by the sweep and ROOT paths
    int lanes;
    int check_finite;
    size_t lds_per_cube;
    uint8_t *face_flags;  // [N*K] near-face marks or nullptr
    R face_eps;           // in cell widths
    const unsigned char *cv_packed;  // control-variate network, packed (nullptr = none)
    int cv_stride;                   // network evaluated every cv_stride steps (>= 1)
    int z_center;                    // subtract y_{i+1}(X_i) from the z response's S'
    // Streamed-cloud launches (clouds too large for LDS): this launch runs
    // strata k0 .. k_end-1, each keeping S' and y_{i+1} of its samples in
    // grow_bytes of global memory from grows (slot = stratum - k0).
    uint32_t k0, k_end;
    unsigned char *grows;
    size_t grow_bytes;
    int stage_chunks;  // streamed clouds: chunks whose partial sums are formed together
    uint32_t debug_singular;  // stratum whose Gram is zeroed in this launch (test aid), or ~0u
};

// Arguments of the set-up kernel (cell constants and the coefficient block
// b | sigma | b_lin | sigma_lin).  The d x q diffusion matrix is not among
// them (at d = 19 it alone takes 2.9 KB of the kernel-argument block); it is
// uploaded next to them by launch_setup.
struct SetupArgs {
    double lo[kMaxDim], hi[kMaxDim];
    int cells[kMaxDim];
    double b[kMaxDim];
    double b_lin[kMaxDim];
    double sigma_lin[kMaxDim];
    int d, q, cmax;
    double mu;
    int equal_prob;
};

struct RootPoint {
    double x[kMaxDim];
};

struct LaunchShape {
    unsigned blocks, threads;  // groups of strata, threads per workgroup
    size_t lds_bytes;
    bool grows;                // streamed clouds, launches of `kc` strata
    uint32_t kc;
    size_t grow_bytes;         // global bytes per stratum
    int stage_chunks;          // streamed clouds: chunks whose partial sums are formed together
};

#if !defined(__HIPCC_RTC__)  // host launchers
// Depth of the path loop's gather pipeline (run_path, PF) for a launch whose
// paths gather from the look-up rows i+1..N-1.  Past 144 MiB of rows most
// gathers miss L2 and the launch time goes to gather latency: binary32 sweeps
// then keep one gather in flight across a step (one wavefront per SIMD less
// than the plain loop).  Past 176 MiB the rows no longer stay in the 256 MB
// last-level cache either, and two gathers in flight (a further wavefront per
// SIMD less) pay; whole records (look-up mode Full) keep one.  Measured at
// d = 8, K = 4^8, M = 64 (5.2 MB rows), per sweep: 60.2 ms with the plain
// loop everywhere, 56.3 ms with depth 1 from 29 rows on, 52.9 ms with depth 2
// from 29 rows on, which loses to depth 1 below 36 rows and gains up to 19 %
// per launch beyond.
constexpr size_t kPrefetchRowBytes = (size_t)144 << 20;
constexpr size_t kPrefetch2RowBytes = (size_t)176 << 20;

template <typename R, int D, int NB, int LK>
inline int prefetch_depth(const StepArgs<R> &a)
{
    const size_t rows = (size_t)(a.N - a.i - 1) * a.K * LookupWidth<R, D, NB, LK>::value * sizeof(R);
    if (sizeof(R) != 4 || rows < kPrefetchRowBytes) return 0;
    return rows >= kPrefetch2RowBytes && LK != kLookupFull ? 2 : 1;
}

template <typename R>
hipError_t launch_setup(const SetupArgs &s, const double *sigma, void *cellF, void *bsig, hipStream_t st);
template <typename R>
hipError_t launch_step(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                       const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                       hipStream_t st);
template <typename R>
hipError_t launch_face_flags(int d, int basis, const StepArgs<R> &a, const void *cellF, const void *bsig,
                             void *counters, hipStream_t st);
template <typename R>
hipError_t launch_lookup_rows(int d, int basis, int lkmode, const void *table, void *lk, uint32_t K,
                              int i_lo, int i_hi, hipStream_t st);
template <typename R>
hipError_t launch_root(int d, int basis, int lkmode, const StepArgs<R> &a, const void *bsig,
                       const void *lk, const RootPoint &x0, int M_root, int nblocks, double *partial,
                       double *out, hipStream_t st);
template <typename R>
hipError_t launch_raw_basis(int d, int q, const StepArgs<R> &a, const void *table, void *raw, hipStream_t st);
template <typename R>
hipError_t launch_eval(int d, int basis, const StepArgs<R> &a, const void *table, const double *x,
                       int64_t n, double *y, double *z, hipStream_t st);
template <typename R>
hipError_t launch_draw(int d, const StepArgs<R> &a, const SetupArgs &s, int kind, uint32_t k0,
                       uint32_t nk, uint32_t m0, uint32_t nm, int count, double *out, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t st);

// The dimensions of the high-dimension files (d = 7, 9, 10 and 11..19, the
// paper's Tables LP0d11 .. LP1d15_19): binary32 sweeps with streamed clouds
// and look-up modes Y and YZ, and every kernel around the sweep.
bool hd_dimension_compiled(int d);
template <typename R>
hipError_t launch_step_gr_hd(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                             const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                             hipStream_t st);
template <typename R>
hipError_t launch_face_flags_hd(int d, int basis, const StepArgs<R> &a, const void *cellF, const void *bsig,
                                void *counters, hipStream_t st);
template <typename R>
hipError_t launch_lookup_rows_hd(int d, int basis, int lkmode, const void *table, void *lk, uint32_t K,
                                 int i_lo, int i_hi, hipStream_t st);
template <typename R>
hipError_t launch_root_hd(int d, int basis, int lkmode, const StepArgs<R> &a, const void *bsig,
                          const void *lk, const RootPoint &x0, int M_root, int nblocks, double *partial,
                          double *out, hipStream_t st);
template <typename R>
hipError_t launch_eval_hd(int d, int basis, const StepArgs<R> &a, const void *table, const double *x,
                          int64_t n, double *y, double *z, hipStream_t st);
template <typename R>
hipError_t launch_draw_hd(int d, const StepArgs<R> &a, const SetupArgs &s, int kind, uint32_t k0,
                          uint32_t nk, uint32_t m0, uint32_t nm, int count, double *out, hipStream_t st);
// The same for the second high-dimension file.
template <typename R>
hipError_t launch_step_gr_hd2(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                             const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                             hipStream_t st);
template <typename R>
hipError_t launch_face_flags_hd2(int d, int basis, const StepArgs<R> &a, const void *cellF, const void *bsig,
                                void *counters, hipStream_t st);
template <typename R>
hipError_t launch_lookup_rows_hd2(int d, int basis, int lkmode, const void *table, void *lk, uint32_t K,
                                 int i_lo, int i_hi, hipStream_t st);
template <typename R>
hipError_t launch_root_hd2(int d, int basis, int lkmode, const StepArgs<R> &a, const void *bsig,
                          const void *lk, const RootPoint &x0, int M_root, int nblocks, double *partial,
                          double *out, hipStream_t st);
template <typename R>
hipError_t launch_eval_hd2(int d, int basis, const StepArgs<R> &a, const void *table, const double *x,
                          int64_t n, double *y, double *z, hipStream_t st);
template <typename R>
hipError_t launch_draw_hd2(int d, const StepArgs<R> &a, const SetupArgs &s, int kind, uint32_t k0,
                          uint32_t nk, uint32_t m0, uint32_t nm, int count, double *out, hipStream_t st);
// The same for the third high-dimension file.
template <typename R>
hipError_t launch_step_gr_hd3(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                             const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                             hipStream_t st);
template <typename R>
hipError_t launch_face_flags_hd3(int d, int basis, const StepArgs<R> &a, const void *cellF, const void *bsig,
                                void *counters, hipStream_t st);
template <typename R>
hipError_t launch_lookup_rows_hd3(int d, int basis, int lkmode, const void *table, void *lk, uint32_t K,
                                 int i_lo, int i_hi, hipStream_t st);
template <typename R>
hipError_t launch_root_hd3(int d, int basis, int lkmode, const StepArgs<R> &a, const void *bsig,
                          const void *lk, const RootPoint &x0, int M_root, int nblocks, double *partial,
                          double *out, hipStream_t st);
template <typename R>
hipError_t launch_eval_hd3(int d, int basis, const StepArgs<R> &a, const void *table, const double *x,
                          int64_t n, double *y, double *z, hipStream_t st);
template <typename R>
hipError_t launch_draw_hd3(int d, const StepArgs<R> &a, const SetupArgs &s, int kind, uint32_t k0,
                          uint32_t nk, uint32_t m0, uint32_t nm, int count, double *out, hipStream_t st);

#endif

// ------------------------------------------------------ batched sweeps
// One instance of a batched sweep, as the batched kernel reads it.  Global
// step g runs backward step i = N - 1 - g of every instance with N > g; the
// instances are sorted by N (descending), so the active ones are a prefix,
// and work item w of step g belongs to the last active instance whose
// first_item <= w.
template <typename R>
struct BatchInstance {
    StepArgs<R> a;
    const void *cellF, *bsig;
    void *lk, *table, *counters;
    uint32_t first_item;  // first work item (stratum group) of the instance
    uint32_t items;       // ceil(K / strata per workgroup)
    uint32_t instance;    // instance field of the counter tag
    uint32_t pad;
};

#if !defined(__HIPCC_RTC__)  // host launchers
template <typename R>
hipError_t launch_batch_step(int d, int basis, int lkmode, bool equal_prob, const void *inst, int n_active,
                             uint32_t total_items, int g, unsigned threads, size_t lds_bytes, hipStream_t st);
// Copies `bytes` from host memory to the device through kernel arguments (no
// staging buffer, nothing to keep alive after the call, capturable).
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st);

// Kernels of a problem's own model (srmdp_model), compiled at run time for the
// current device (srmdp_rtc.cpp): hipFunction_t of the step kernel and of the
// near-face diagnostic, for the grid kind (equal_prob) and the cloud storage
// (streamed: clouds streamed through LDS, LaunchShape::grows) of the shape.
struct ModelKernels {
    void *step = nullptr, *face_flags = nullptr;
};
srmdp_status model_kernels(const srmdp_model *m, int d, int nb, int is_float, bool equal_prob, bool streamed,
                           ModelKernels &out);
template <typename R>
hipError_t launch_model_step(const ModelKernels &k, const StepArgs<R> &a, const LaunchShape &s, const void *cellF,
                             const void *bsig, void *lk, void *table, void *counters, hipStream_t st);
template <typename R>
hipError_t launch_model_face_flags(const ModelKernels &k, const StepArgs<R> &a, const void *cellF, const void *bsig,
                                   void *counters, hipStream_t st);

// Dimensions with the LDS sweep kernel, and every dimension compiled at all.
bool lds_dimension_compiled(int d);
bool dimension_compiled(int d);
// LDS bytes of one stratum's regression with its cloud in LDS.
size_t cube_lds_bytes(int prec_is_float, int d, int nb, int M, bool cv = false);
// Streamed clouds (too large for LDS): LDS bytes of one stratum with L lanes
// and the partial sums of pb chunks at a time; the largest pb whose LDS fits
// in `cap` (0 if none); global bytes per stratum (S' and y_{i+1} per sample).
size_t cube_stream_lds_bytes(int prec_is_float, int d, int nb, int L, int pb);
int cube_stream_chunks(int prec_is_float, int d, int nb, int L, size_t cap);
size_t cube_global_bytes(int prec_is_float, int M);
template <typename R>
hipError_t launch_step_gr(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                          hipStream_t st);
// Equal-probability cells (srmdp_kernels_ep.hip): streamed clouds, and clouds in LDS.
template <typename R>
hipError_t launch_step_ep(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                          hipStream_t st);
template <typename R>
hipError_t launch_step_ep_lds(int d, const StepArgs<R> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                          hipStream_t st);

// ------------------------------------------------ learned control variate
// (srmdp_cv.hip; binary32 sweeps only)
struct MlpTrainArgs {
    int in, out;
    float *theta, *adam_m, *adam_v;  // [P] each
    int64_t adam_t0;                 // Adam steps taken before this call
    const float *x16, *z16;          // training pairs [S][16]
    int64_t S;
    int updates, batch;
    float lr, beta1, beta2, eps;
    unsigned char *packed_out;       // the packing of theta on entry, kept equal to it after each update
    float *loss;                     // [updates] or nullptr
};
bool cv_dimension_compiled(int d);
hipError_t launch_step_cv(int d, const StepArgs<float> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                          hipStream_t st);
hipError_t launch_cv_pairs(int d, int basis, const StepArgs<float> &a, const void *cellF, const void *table,
                           int64_t S, float *x16, float *z16, hipStream_t st);
hipError_t launch_mlp_pack(int in, int out, const float *theta, void *packed, hipStream_t st);
hipError_t launch_mlp_init(int in, int out, uint64_t seed, int zero_output_layer, float *theta,
                           hipStream_t st);
hipError_t launch_mlp_forward(int in, int out, const void *packed, const float *x, int64_t B, float *y,
                              hipStream_t st);
size_t mlp_backward_partials(int64_t B);
hipError_t launch_mlp_backward(int in, int out, const void *packed, const float *x, const float *dy,
                               int64_t B, float *partial, float *grad, hipStream_t st);
// Bytes of the per-workgroup gradient partials of one update at this batch.
size_t mlp_train_partial_bytes(int in, int out, int batch);
// t.updates Adam updates, two launches each; partial: mlp_train_partial_bytes.
hipError_t launch_mlp_train(const MlpTrainArgs &t, float *partial, hipStream_t st);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st);

#endif

}  // namespace srmdp
