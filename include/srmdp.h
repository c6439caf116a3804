/*
 * srmdp.h -- C ABI of the MI355X (gfx950) library for the backward
 * dynamic-programming sweep of the stratified regression Monte-Carlo scheme
 * (SRMDP) of Gobet, Lopez-Salas, Turkedjiev and Vazquez, "Stratified regression
 * Monte-Carlo scheme for semilinear PDEs and BSDEs with large scale
 * parallelization on GPUs", arXiv 2407.21085.
 *
 * The library solves the decoupled FBSDE of the paper's eq. (fbsde)-(eds)
 * (equivalently the semilinear PDE eq. (pde)) on the time grid t_i = i T/N with
 * the multistep-forward dynamic programming identity eq. (MDP:intro), by
 * Algorithm SRMDP (Section 3.1): for i = N-1 down to 0, every stratum H_k of a
 * uniform grid gets M fresh starting points drawn from the restricted logistic
 * law nu_k (assumption (A_nu), Algorithm "stratify"); each is simulated to t_N
 * (Algorithm "Euler dynamics"), and the responses of eq. (PsiM) are regressed on
 * the local space LP0 or LP1 of assumption (A_Strat).  Only the coefficient
 * table is kept.
 *
 * Conventions shared by every entry point
 *  - C99-compatible, no exceptions cross the ABI; every call returns a
 *    srmdp_status; srmdp_last_error() describes the last failure on the
 *    calling thread.
 *  - Device work is enqueued on `stream` (a hipStream_t passed as void*;
 *    NULL = the null stream) and is asynchronous unless a host output is
 *    requested (stats, read-outs), in which case the call synchronises the
 *    stream before returning.
 *  - The caller owns every buffer.  The library allocates no device memory in
 *    srmdp_solve/srmdp_eval/srmdp_root/srmdp_draw; scratch comes from the
 *    caller's workspace.  It keeps only cached hipGraph executables (flag
 *    SRMDP_F_GRAPH), released by srmdp_release_graphs().
 *  - Pointer kinds are stated per argument: "host" pointers are read during
 *    the call only; "device" pointers must stay valid until the enqueued work
 *    has finished.
 *  - Argument errors are detected before anything is enqueued and return
 *    SRMDP_E_INVALID (or SRMDP_E_WORKSPACE for an undersized workspace,
 *    SRMDP_E_UNSUPPORTED for a valid request outside what is compiled).
 */
#ifndef SRMDP_H
#define SRMDP_H

#if !defined(__HIPCC_RTC__)  /* device code compiled at run time has the types built in */
#include <stddef.h>
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define SRMDP_MAX_D 19          /* largest d = q compiled.  d = 1..6 and 8 run every
                                 * option; d = 7 and 9..19 run binary32 sweeps with
                                 * look-up modes Y and YZ (no z truncation), without
                                 * the control variate, on either grid kind; other
                                 * requests return SRMDP_E_UNSUPPORTED */
#define SRMDP_ROOT_STRATUM 0xFFFFFFFFu  /* counter stratum tag of ROOT paths */

typedef enum {
    SRMDP_OK = 0,
    SRMDP_E_INVALID = -1,      /* bad argument, nothing enqueued */
    SRMDP_E_UNSUPPORTED = -2,  /* valid request that this build does not cover */
    SRMDP_E_WORKSPACE = -3,    /* workspace smaller than srmdp_workspace_bytes() */
    SRMDP_E_HIP = -4,          /* a HIP runtime call failed (message in srmdp_last_error) */
    SRMDP_E_NUMERIC = -5       /* SRMDP_F_CHECK_FINITE found a non-finite coefficient */
} srmdp_status;

/* Local approximation spaces of assumption (A_Strat): LP0 = span{1_H}, nb = 1;
 * LP1 = span{1, x_1..x_d} on H, nb = d + 1. */
typedef enum { SRMDP_LP0 = 0, SRMDP_LP1 = 1 } srmdp_basis;

/* Arithmetic of the sweep.  FP64: everything in binary64.  FP32: paths,
 * responses and table look-ups in binary32; Gram and right-hand-side sums,
 * Cholesky factors and solves in binary64; coefficients stored in binary32. */
typedef enum { SRMDP_FP64 = 0, SRMDP_FP32 = 1 } srmdp_precision;

/* Driver f(t, x, y, z).  LINEAR: f = -r y + kappa sum_l z_l.  LOGISTIC: the
 * paper's benchmark (Section 5.1), f = (sum_l z_l)(y - (2 + q)/(2 q)). */
typedef enum { SRMDP_DRV_LINEAR = 0, SRMDP_DRV_LOGISTIC = 1 } srmdp_driver;

/* Terminal condition g.  COS_SUM: g = cos(sum_l x_l).  LOGISTIC: the paper's
 * benchmark, g = omega(T,x)/(1 + omega(T,x)), omega(t,x) = exp(t + sum_l x_l). */
typedef enum { SRMDP_G_COS_SUM = 0, SRMDP_G_LOGISTIC = 1 } srmdp_terminal;

/* A problem's own coefficients and data, compiled at run time (hipRTC, for
 * the device the sweep runs on) into the sweep kernels: general b(t, x),
 * sigma(t, x) through the Euler scheme of Section 2 (Algorithm "Euler
 * dynamics", at (t_j, X_j)) and general f(t, x, y, z), g(x) of eq.
 * (fbsde)-(MDP:intro).
 *  source   host, NUL-terminated HIP C++ device code.  It is compiled with
 *           `srmdp_real` (double for SRMDP_FP64 sweeps, float for SRMDP_FP32)
 *           and the macros SRMDP_D (= d) and SRMDP_Q (= q = d) defined, and
 *           must define
 *     __device__ void srmdp_b(srmdp_real t, const srmdp_real *x, const srmdp_real *p,
 *                             srmdp_real *out);                 out[SRMDP_D] = b(t, x)
 *     __device__ void srmdp_sigma_dw(srmdp_real t, const srmdp_real *x, const srmdp_real *dw,
 *                                    const srmdp_real *p, srmdp_real *out);   out[SRMDP_D] = sigma(t, x) dw
 *     __device__ srmdp_real srmdp_f(srmdp_real t, const srmdp_real *x, srmdp_real y,
 *                                   const srmdp_real *z, const srmdp_real *p);  f(t, x, y, z), z[SRMDP_Q]
 *     __device__ srmdp_real srmdp_g(const srmdp_real *x, const srmdp_real *p);    g(x)
 *           The Euler step is X_{j+1} = X_j + b(t_j, X_j) dt + sigma(t_j, X_j) dW_j
 *           with t_j = j dt, in that order of additions.
 *  params   host [n_params] or NULL: p[0..n_params-1] of the functions above,
 *           converted to srmdp_real (a new value needs no new compilation).
 *  n_params 0..64.
 * Kernels are compiled once per (device, source, d, basis, precision, grid
 * kind, cloud storage) and kept for the process.  A compilation error returns
 * SRMDP_E_INVALID with the compiler's log in srmdp_last_error().  Covered:
 * srmdp_solve (d <= 8, either grid kind, clouds in LDS or, for large M or with
 * SRMDP_F_GLOBAL_ROWS, streamed through it; no control variate or
 * autotuner), srmdp_eval; other entry points return SRMDP_E_UNSUPPORTED for a
 * problem with a model. */
typedef struct {
    const char *source;
    const double *params;
    int32_t n_params;
} srmdp_model;

/* Problem data (eq. (fbsde)-(eds)): the built-in families below, or a
 * compiled model (then driver, terminal, r, kappa, b, sigma, b_lin and
 * sigma_lin are not used and must be zero or NULL). */
typedef struct {
    int32_t d, q;          /* 1..SRMDP_MAX_D; the built-in f and g need q == d */
    double T;              /* horizon > 0 */
    int32_t N;             /* time steps, 1..65535; dt = T / N */
    const double *b;       /* host [d]: constant drift; NULL = 0 */
    const double *sigma;   /* host [d*q] row-major constant diffusion; NULL = identity */
    int32_t driver;        /* srmdp_driver */
    int32_t terminal;      /* srmdp_terminal */
    double r, kappa;       /* LINEAR driver parameters */
    double clamp_y, clamp_z; /* truncation levels C_y, C_z of eq. (TL), applied when a
                              * fitted function is evaluated; INFINITY = off */
    const double *b_lin;   /* host [d]: diagonal linear drift, so that the drift is
                            * b_l + b_lin_l x_l (Ornstein-Uhlenbeck dynamics, through the
                            * Euler scheme of Section 2); NULL = 0 */
    const double *sigma_lin; /* host [d]: diagonal part of the diffusion linear in the state,
                              * sigma(x)_{l,c} = sigma_{l,c} + [l = c] sigma_lin_l x_l, evaluated at
                              * X_j in the Euler scheme of Section 2 (geometric Brownian motion
                              * when sigma is zero); NULL = 0 */
    const srmdp_model *model; /* host or NULL: the problem's own coefficients (srmdp_model) */
} srmdp_problem;

/* Stratification: the two examples of hypercubes under assumption
 * (A_Strat), with the sampling law of assumption (A_nu).
 * SRMDP_GRID_EQUAL_SIZE: cells[l] half-open cells of equal width in
 *   [lo, hi); points outside are evaluated with the fit of the nearest
 *   boundary cell; only the K = prod(cells) bounded cells are sampled.
 * SRMDP_GRID_EQUAL_PROB: the cells of dimension l are cut at the logistic
 *   quantiles F^{-1}(c / cells[l]), F(x) = 1 / (1 + exp(-mu x)), so that each
 *   of the K cubes has nu-probability 1/K and they cover R^d (the two outer
 *   cells of each dimension are unbounded); lo and hi are ignored (may be
 *   NULL).  The LP1 coordinate of an equal-probability cell is mu (x - m),
 *   m the cell's nu-median F^{-1}((c + 1/2) / cells[l]); for an equal-size
 *   cell it is 2 (x - centre) / width.  Table coefficients are in these
 *   coordinates. */
typedef enum { SRMDP_GRID_EQUAL_SIZE = 0, SRMDP_GRID_EQUAL_PROB = 1 } srmdp_grid_kind;

typedef struct {
    const double *lo, *hi;   /* host [d], lo < hi (SRMDP_GRID_EQUAL_SIZE only) */
    const int32_t *cells;    /* host [d], >= 1; K = prod(cells) <= 2^24 */
    double mu;               /* logistic parameter > 0 */
    int32_t kind;            /* srmdp_grid_kind; 0 (a zero-initialised struct) = equal size */
} srmdp_grid;

/* Learned martingale control variate (not part of the paper's scheme).  A
 * network z_theta(t, x): (d+1) -> 64 -> 64 -> q, SiLU after both hidden
 * layers, bfloat16 weights and layer inputs, binary32 accumulation and biases,
 * evaluated on the matrix cores.  Each simulation of step i subtracts
 * sum_{j>i} z_theta(t_j, X_j) . dW_j from its response S' and, for the y
 * regression only, z_theta(t_i, X_i) . dW_i as well.  Every subtracted term has
 * conditional mean zero given X_i because dW_j is independent of X_j and of
 * the network, which is fixed during the step, so the regressions of eq.
 * (PsiM) keep their targets (the martingale representation behind eq.
 * (MDP:intro)) and only their variance changes.
 *   FROZEN: the network cv_params is used unchanged at every step.
 *   ONLINE: cv_params is the initial network; after each backward step i the
 *           network takes cv_train.updates_per_step Adam steps on pairs
 *           (t_i, X_i^(m), z_i(X_i^(m))) of that step's clouds (srmdp_cv_pairs)
 *           and is used from step i-1 on; cv_params holds the trained network
 *           when the call returns.
 * With cv_stride = s > 1 the network is evaluated at t_j for
 * j - i = 0, s, 2s, ... and its last value weighs dW_j in between (still
 * adapted, so still of mean zero), dividing its cost by s.  With
 * SRMDP_F_CV_CENTER_Z the z response S' dW_i / dt also loses
 * y_{i+1}(X_i) dW_i / dt (g(X_i) when i + 1 = N), of conditional mean zero too.
 * Binary32 sweeps only (any M >= nb, any lanes per stratum).  The ROOT
 * read-out does not use it. */
typedef enum { SRMDP_CV_NONE = 0, SRMDP_CV_FROZEN = 1, SRMDP_CV_ONLINE = 2 } srmdp_cv;

#define SRMDP_MLP_HIDDEN 64
#define SRMDP_CV_PAIR_STRATUM 0xFFFFFFFEu  /* counter stratum of the training-pair draws */

typedef struct {
    int32_t updates_per_step;  /* Adam steps after each backward step, 1..4096 */
    int32_t batch;             /* pairs per step of Adam: multiple of 256, <= 65536 */
    float lr, beta1, beta2, eps;  /* Adam (Kingma & Ba 2015); lr > 0, betas in [0, 1), eps > 0 */
} srmdp_mlp_train_config;

/* Option flags. */
#define SRMDP_F_GRAPH        0x1u  /* capture the N step launches in a cached hipGraph */
#define SRMDP_F_CHECK_FINITE 0x2u  /* fail with SRMDP_E_NUMERIC on a non-finite coefficient */
#define SRMDP_F_CV_CENTER_Z  0x4u  /* control variate: centre the z response (see srmdp_cv) */
#define SRMDP_F_AUTOTUNE     0x8u  /* lanes_per_cube == 0: use the autotuned value (srmdp_tune_lanes;
                                    * tuned once per shape and cached; not during capture) */
#define SRMDP_F_GLOBAL_ROWS  0x10u /* stream every stratum's cloud through an LDS window in
                                    * rounds, with S' and y_{i+1} per sample in global memory
                                    * (see global_rows_strata); automatic, without the control
                                    * variate, when a cloud does not fit in 64 KB of LDS */
#define SRMDP_F_DEBUG_SINGULAR 0x20u /* test aid: the Gram matrix of stratum debug_stratum at
                                      * step debug_step is replaced by zero, so that this
                                      * stratum takes the LP0 fallback of a singular Gram
                                      * (explicit LP0 solution, Section 4.1) and is counted
                                      * in srmdp_stats.singular_cubes; srmdp_solve only */

typedef struct {
    int32_t M;              /* simulations per stratum, >= nb (Definition of the clouds) */
    int32_t basis;          /* srmdp_basis */
    int32_t prec;           /* srmdp_precision */
    uint64_t seed;          /* Philox4x32-10 key = (seed mod 2^32, seed >> 32) */
    uint32_t instance;      /* counter tag, < 65536 */
    int32_t step_hi;        /* first backward step to run (-1 = N-1); rows > step_hi of the
                             * table must hold a previous run's coefficients (resume) */
    int32_t step_lo;        /* last backward step to run (-1 = 0) */
    int32_t lanes_per_cube; /* 0 = automatic (next power of two >= M, at most 256);
                             * else 8, 16, 32, 64, 128 or 256 */
    uint32_t flags;         /* SRMDP_F_* */
    uint8_t *face_flags;    /* device [N*K] or NULL.  When set, entry i*K + k of every step
                             * run becomes 1 if a simulation of stratum k at step i looked
                             * up a table row at a point within face_eps cell widths of an
                             * interior cell face (where binary32 and binary64 positions may
                             * pick different cells), else 0 */
    double face_eps;        /* distance in cell widths; <= 0 means 1e-5 */
    int32_t cv;             /* srmdp_cv */
    float *cv_params;       /* device [srmdp_mlp_param_count(d+1, q)] binary32 network
                             * parameters (layout of srmdp_mlp_param_count); read by FROZEN,
                             * read and overwritten by ONLINE; NULL when cv is NONE */
    srmdp_mlp_train_config cv_train;  /* ONLINE only */
    int32_t cv_stride;      /* network evaluated every cv_stride steps; <= 1 = every step */
    int32_t global_rows_strata; /* streamed clouds: strata per launch (rounded up to a
                                 * multiple of 8); 0 = as many as 2 GiB hold.  The workspace
                                 * then holds, per stratum of a launch, S' and y_{i+1}(X_{i+1})
                                 * of each of the M samples in the working precision */
    int32_t debug_step;     /* SRMDP_F_DEBUG_SINGULAR: step and stratum of the zeroed Gram */
    uint32_t debug_stratum;
} srmdp_options;

typedef struct {
    uint64_t singular_cubes;   /* strata whose Gram matrix fell back to LP0 */
    uint64_t path_steps;       /* Euler steps simulated */
    float ms_total;            /* device time of everything the call enqueued (hipEvents) */
    float ms_steps;            /* device time of the backward-step kernels alone (hipEvents
                                * around them); -1 when the steps ran from a hipGraph */
    int32_t step_launches;     /* backward-step kernels launched */
    int32_t lanes_per_cube;    /* lanes per stratum actually used */
    uint64_t near_face_paths;  /* simulations with a near-face look-up (face_flags set) */
    float cv_loss_first;       /* ONLINE: mean training loss over the updates after the first
                                * step run, and after the last one (0 otherwise) */
    float cv_loss_last;
} srmdp_stats;

/* Number of coefficients of the table: N * K * (1 + q) * nb.  Layout
 * table[i][k][c][b], i < N, k lexicographic with dimension 0 fastest,
 * c in {y, z_1..z_q}, b in {1, xi_1..xi_d} with the cube-centred, scaled
 * coordinate xi_l = 2 (x_l - centre_l) / h_l.  Returns 0 on invalid input. */
size_t srmdp_table_elems(const srmdp_problem *problem, const srmdp_grid *grid, int32_t basis);

/* Device workspace bytes srmdp_solve needs; 0 on invalid input. */
size_t srmdp_workspace_bytes(const srmdp_problem *problem, const srmdp_grid *grid,
                             const srmdp_options *opts);

/* Algorithm SRMDP (Section 3.1, eq. (PsiM)) for i = step_hi .. step_lo.
 *  table      device, (1+q)*nb*K*N values of the option's precision (double for
 *             FP64, float for FP32), layout as in srmdp_table_elems; rows
 *             step_lo..step_hi are written, rows > step_hi are read.
 *  workspace  device, ws_bytes >= srmdp_workspace_bytes(...).
 *  stats      host or NULL; when non-NULL the call synchronises `stream`.
 * Draws: stratum k, simulation m, step i uses Philox4x32-10 counter
 * (block, m, k, i | instance << 16); block 0..ceil(d/4)-1 words give the start
 * point (Algorithm "stratify"), later blocks give Box-Muller normals in pairs. */
srmdp_status srmdp_solve(const srmdp_problem *problem, const srmdp_grid *grid,
                         const srmdp_options *opts, void *table, void *workspace,
                         size_t ws_bytes, srmdp_stats *stats, void *stream);

/* Autotuner of the lanes per stratum: times one backward step (the middle of
 * step_hi..step_lo, whose table row it overwrites; rows above it are read as
 * for srmdp_solve) with 8, 16, 32, 64, 128 and 256 lanes (those that fit M and
 * the LDS budget), stores the fastest in *lanes and, if ms is non-NULL, the
 * time per launch of each candidate in ms[0..5] (-1 = not tried).  The result
 * is cached per shape and used by SRMDP_F_AUTOTUNE.  Synchronises `stream`. */
srmdp_status srmdp_tune_lanes(const srmdp_problem *problem, const srmdp_grid *grid,
                              const srmdp_options *opts, void *table, void *workspace,
                              size_t ws_bytes, int32_t *lanes, float *ms, void *stream);

/* Ragged batch: n independent instances (host arrays of n problems, grids and
 * options; same d, basis, precision and look-up mode; any K, M, N, seeds,
 * instance tags and driver parameters; full plain sweeps; lanes_per_cube 0
 * means one lane per simulation up to 256).  One launch per global step g = 0..max N - 1 runs backward step
 * N_b - 1 - g of every instance with N_b > g, over the flattened list of
 * their stratum groups; with SRMDP_F_GRAPH in opts[0].flags the launches are
 * replayed from a cached hipGraph.  tables: host array of n device tables
 * (layout of srmdp_table_elems); each equals what srmdp_solve returns for the
 * instance with the same lanes.  stats: host [n] or NULL (then the call does
 * not synchronise). */
size_t srmdp_workspace_bytes_batch(int32_t n, const srmdp_problem *problems, const srmdp_grid *grids,
                                   const srmdp_options *opts);
srmdp_status srmdp_solve_batch(int32_t n, const srmdp_problem *problems, const srmdp_grid *grids,
                               const srmdp_options *opts, void *const *tables, void *workspace,
                               size_t ws_bytes, srmdp_stats *stats, void *stream);

/* Evaluation of the fitted, truncated y_i and z_i (eq. (PsiM)'s y^M_i, z^M_i)
 * at n points.  table device (precision prec); x device [n*d] doubles;
 * y device [n] or NULL; z device [n*q] or NULL. */
srmdp_status srmdp_eval(const srmdp_problem *problem, const srmdp_grid *grid, int32_t basis,
                        int32_t prec, const void *table, int32_t i, const double *x, int64_t n,
                        double *y, double *z, void *stream);

/* The table in the paper's raw basis (1, x_1, .., x_d) of the local polynomials
 * of degree 1 (Section 4.1), record by record.  A table record holds the
 * coefficients beta on (1, xi_1, .., xi_d), xi_l = 2 s_l (x_l - m_l), with
 * m_l the centre of the cell (equal-size cells, s_l = cells_l / (hi_l - lo_l))
 * or its nu-median F^{-1}((c + 1/2) / cells_l) (equal-probability cells,
 * s_l = mu / 2).  The raw coefficients are alpha_l = 2 s_l beta_l and
 * alpha_0 = beta_0 - sum_l alpha_l m_l, so that alpha . (1, x) = beta . (1, xi).
 * LP0 records are copied.  table, raw: device, srmdp_table_elems values of
 * precision prec in the table layout; raw may be table (in place).  Far from
 * the origin the raw form loses digits to cancellation; the sweep and the
 * read-outs keep the centred form. */
srmdp_status srmdp_to_raw_basis(const srmdp_problem *problem, const srmdp_grid *grid, int32_t basis,
                                int32_t prec, const void *table, void *raw, void *stream);

/* ROOT read-out of y(0, x0), z(0, x0): the MDP identity with the initial law
 * delta_{x0} (the value functions do not depend on the initial law, Section 2),
 * i.e. an LP0 regression on the point x0 with M_root simulations (counter
 * stratum SRMDP_ROOT_STRATUM, step 0): z first, then y with the fitted z in the
 * i = 0 driver term.  table device (full, precision opts->prec); x0 host [d];
 * y0 host scalar; z0 host [q]; workspace as for srmdp_solve.  Synchronises. */
srmdp_status srmdp_root(const srmdp_problem *problem, const srmdp_grid *grid,
                        const srmdp_options *opts, const void *table, const double *x0,
                        int32_t M_root, double *y0, double *z0, void *workspace,
                        size_t ws_bytes, void *stream);

/* Random inputs of the sweep, for checking the generator (test access).
 * kind 0: the first `count` uniforms of each simulation's stream;
 * kind 1: the first `count` standard normals (before the sqrt(dt) scale);
 * kind 2: the starting point (count must equal d).
 * Simulations are (i, k0 + a, m0 + c) for a < nk, c < nm; out device doubles
 * [nk][nm][count], computed in precision prec and widened to double.
 * problem/grid/opts as for srmdp_solve (grid and problem only matter for
 * kinds 1 and 2). */
srmdp_status srmdp_draw(const srmdp_problem *problem, const srmdp_grid *grid,
                        const srmdp_options *opts, int32_t kind, int32_t i, uint32_t k0,
                        uint32_t nk, uint32_t m0, uint32_t nm, int32_t count, double *out,
                        void *stream);

/* Training pairs of the online control variate after step i: pair s draws a
 * stratum k = floor(K u0) and a simulation m = floor(M u1) from the 32-bit
 * words (u0, u1) of Philox4x32-10 counter (0, s, SRMDP_CV_PAIR_STRATUM,
 * i | instance << 16), rebuilds that simulation's start X_i^(m) (the draw of
 * the sweep) and takes the fitted, truncated z_i of stratum k there.
 * x16 device [n][16] floats: (t_i, X_i, zero padding); z16 device [n][16]:
 * (z_i, zero padding).  table device binary32 (opts->prec must be FP32), row i
 * written; workspace as for srmdp_solve. */
srmdp_status srmdp_cv_pairs(const srmdp_problem *problem, const srmdp_grid *grid,
                            const srmdp_options *opts, const void *table, int32_t i, int64_t n,
                            float *x16, float *z16, void *workspace, size_t ws_bytes, void *stream);

/* --- the control-variate network on its own (shapes in <= 16, out <= 16) ---
 * Parameters, binary32, row-major: W1 [64][in], b1 [64], W2 [64][64], b2 [64],
 * W3 [out][64], b3 [out].  The packed form (srmdp_mlp_packed_bytes() bytes,
 * device) holds the biases and the bf16 weight fragments the kernels read. */
int64_t srmdp_mlp_param_count(int32_t in, int32_t out);
size_t srmdp_mlp_packed_bytes(void);

/* Glorot-uniform weights from Philox4x32-10 (key = seed), zero biases; with
 * zero_output_layer the last layer's weights are zero too (z_theta = 0). */
srmdp_status srmdp_mlp_init(int32_t in, int32_t out, uint64_t seed, int32_t zero_output_layer,
                            float *params, void *stream);
srmdp_status srmdp_mlp_pack(int32_t in, int32_t out, const float *params, void *packed, void *stream);

/* y [n][out] = z_theta(x [n][in]) (device arrays). */
srmdp_status srmdp_mlp_forward(int32_t in, int32_t out, const void *packed, const float *x, int64_t n,
                               float *y, void *stream);

/* grad [P] = d/dtheta sum_s <dy_s, z_theta(x_s)> with bf16 operands as in the
 * forward pass (upstream and hidden-layer gradients rounded to bf16 where they
 * enter a matrix product; bias gradients in binary32).  Device arrays;
 * workspace of srmdp_mlp_backward_workspace(in, out, n) bytes. */
size_t srmdp_mlp_backward_workspace(int32_t in, int32_t out, int64_t n);
srmdp_status srmdp_mlp_backward(int32_t in, int32_t out, const void *packed, const float *x,
                                const float *dy, int64_t n, float *grad, void *workspace,
                                size_t ws_bytes, void *stream);

/* cfg->updates_per_step Adam steps on the mean over a batch of
 * sum_o (z_theta(x)_o - z_o)^2, batches taken cyclically from the n pairs
 * x16 / z16 ([n][16] floats, 16-byte aligned, n a multiple of 64); adam_m and
 * adam_v [P] are the moment estimates (zero before the first step) and adam_t0
 * the number of steps taken before.  params is updated in place; packed_out
 * receives the packed network; loss (device [updates] or NULL) the batch loss
 * before each step.  Each update is two launches: the batch's gradient over
 * batch / 256 workgroups (partial sums in the workspace, device,
 * srmdp_mlp_train_workspace_bytes() bytes), then the Adam step over the
 * parameters, which sums the partials in workgroup order. */
size_t srmdp_mlp_train_workspace_bytes(int32_t in, int32_t out, const srmdp_mlp_train_config *cfg);
srmdp_status srmdp_mlp_train(int32_t in, int32_t out, float *params, float *adam_m, float *adam_v,
                             int64_t adam_t0, const float *x16, const float *z16, int64_t n,
                             const srmdp_mlp_train_config *cfg, void *packed_out, float *loss,
                             void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes that srmdp_solve_noalloc serves: one library-owned device
 * array of this size on each GPU the library runs on, held until the process
 * ends. */
#define SRMDP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* srmdp_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same sweep with the same kernels and the same table; its workspace is the
 * library's own device array of SRMDP_NOALLOC_SCRATCH_BYTES on the current
 * device instead of a caller buffer.  The caller still owns `table` (device,
 * layout and precision as for srmdp_solve) and the stream (of the current
 * device, NULL = null stream).
 *  - Allocates nothing: no hipMalloc, hipFree, events or graphs.  The device
 *    address of the array is resolved once per device, on the first call there.
 *  - Asynchronous: no stats, never synchronises.  Rejects, before enqueuing
 *    anything, SRMDP_F_GRAPH, SRMDP_F_CHECK_FINITE and SRMDP_F_AUTOTUNE with
 *    lanes_per_cube == 0 (SRMDP_E_INVALID), and any request whose
 *    srmdp_workspace_bytes exceeds SRMDP_NOALLOC_SCRATCH_BYTES
 *    (SRMDP_E_WORKSPACE; e.g. d = 8, K = 4^8, N = 50 needs 262 MB of look-up
 *    rows).  Other argument errors as srmdp_solve.
 *  - Every call on a GPU uses that GPU's one array, which keeps the previous
 *    call's contents; the sweep zeroes its counters (with a kernel) and
 *    writes every other part before reading it.  Calls that overlap in time
 *    on one GPU (two streams, two threads) race on the array: serialise them. */
srmdp_status srmdp_solve_noalloc(const srmdp_problem *problem, const srmdp_grid *grid,
                                 const srmdp_options *opts, void *table, void *stream);

/* Releases cached hipGraph executables. */
void srmdp_release_graphs(void);

/* Description of the last failure on the calling thread ("" if none). */
const char *srmdp_last_error(void);

/* ABI version (major * 100 + minor). */
int32_t srmdp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SRMDP_H */
