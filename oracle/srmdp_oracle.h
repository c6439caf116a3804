/*
 * srmdp_oracle.h -- plain FP64 CPU oracle of the stratified regression
 * multistep-forward dynamic programming (SRMDP) backward sweep of
 * Gobet, Lopez-Salas, Turkedjiev, Vazquez, "Stratified regression Monte-Carlo
 * scheme for semilinear PDEs and BSDEs with large scale parallelization on
 * GPUs" (arXiv 2407.21085).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library.  It is
 * called from the test-suite, from the smoke check and from the CPU-baseline
 * leg of the benchmark, and from nothing else.  It shares no code, header,
 * constant table or helper with the GPU library; the only thing both sides
 * agree on is the published definition of the Philox4x32-10 generator and the
 * way the paper's random inputs are mapped onto its counter (documented below).
 *
 * Everything is computed in IEEE binary64, without fast-math, in one plain code
 * path, following the paper's Algorithm SRMDP step by step.
 */
#ifndef SRMDP_ORACLE_H
#define SRMDP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LP0 = 0, ORC_LP1 = 1 };
enum { ORC_GRID_EQUAL_SIZE = 0, ORC_GRID_EQUAL_PROB = 1 };
enum { ORC_DRV_LINEAR = 0, ORC_DRV_LOGISTIC = 1 };
enum { ORC_G_COS_SUM = 0, ORC_G_LOGISTIC = 1 };

/* A problem's own coefficients: b(t, x), sigma(t, x) applied to dW, f(t, x, y, z)
 * and g(x), with parameters p (used by the test-suite through small C plugins;
 * the GPU library takes the same functions as HIP source). */
typedef struct {
    void (*b)(double t, const double *x, const double *p, double *out);                   /* out[d] */
    void (*sigma_dw)(double t, const double *x, const double *dw, const double *p, double *out); /* out[d] */
    double (*f)(double t, const double *x, double y, const double *z, const double *p);
    double (*g)(const double *x, const double *p);
    const double *params;
    double lip_y, lip_z;     /* bounds of |df/dy| and |df/dz_l| (face-flip bound only) */
} orc_model;

typedef struct {
    int32_t d, q;            /* space and Brownian dimensions */
    double T;                /* horizon */
    int32_t N;               /* number of time steps, dt = T/N */
    const double *b;         /* [d] constant drift or NULL (zero) */
    const double *sigma;     /* [d*q] row-major constant diffusion or NULL (identity, q == d) */
    int32_t driver;          /* ORC_DRV_* */
    int32_t terminal;        /* ORC_G_* */
    double r, kappa;         /* linear driver f = -r*y + kappa*sum(z) */
    double clamp_y, clamp_z; /* truncation levels; +inf disables */
    const double *lo, *hi;   /* [d] domain of the stratification */
    const int32_t *cells;    /* [d] cells per dimension, K = prod(cells) */
    double mu;               /* logistic parameter */
    int32_t M;               /* simulations per stratum */
    int32_t basis;           /* ORC_LP0 / ORC_LP1 */
    uint64_t seed;           /* Philox key */
    uint32_t inst;           /* instance tag in the counter */
    /* frozen control-variate network; NULL disables the control variate */
    const double *cv_params; /* MLP parameters, layout of orc_mlp_forward */
    int32_t cv_hidden;
    int32_t cv_bf16;         /* bfloat16 emulation mask of orc_mlp_forward_bf (0: exact) */
    /* diagnostic output: face_flags[i*K + k] = 1 when a simulation of stratum k
     * at step i looked up a fitted row at a point within face_eps cell widths of
     * an interior cell face; NULL disables */
    uint8_t *face_flags;
    double face_eps;
    /* control-variate variants: the network is evaluated at t_j for
     * j - i = 0, cv_stride, 2 cv_stride, ... and its last value weighs dW_j in
     * between (<= 1: every step); z_center subtracts y_{i+1}(X_i) dW_i / dt
     * (g(X_i) when i + 1 = N) from the z response */
    int32_t cv_stride;
    int32_t z_center;
    /* [d] diagonal linear part of the drift, b(t, x)_l = b_l + b_lin_l x_l
     * (Ornstein-Uhlenbeck dynamics), or NULL (zero) */
    const double *b_lin;
    /* ORC_GRID_EQUAL_SIZE: cells of width (hi - lo) / cells inside [lo, hi),
     * the outer ones extended to the nearest boundary cell for evaluation.
     * ORC_GRID_EQUAL_PROB: per dimension the cells' edges are the logistic
     * quantiles F^{-1}(c / cells), c = 0..cells, so that every cube has
     * nu-probability 1/K and the cubes cover R^d (lo and hi are ignored). */
    int32_t grid_kind;
    /* [d] diagonal part of the diffusion linear in the state,
     * sigma(x)_{l,c} = sigma_{l,c} + [l = c] sigma_lin_l x_l (q = d), or NULL */
    const double *sigma_lin;
    /* Test diagnostics.
     * flip_bound [N*K*(1+q)*nb] or NULL: per coefficient of each fitted
     * stratum, a bound on its change if near-face look-ups (those that set
     * face_flags) took the cube across their face, as rounding in another
     * precision may make them do.
     * With a bfloat16 network (cv_bf16 with hidden rounding) the bound also
     * covers hidden activations within 32 binary32 units of a bfloat16
     * rounding midpoint rounded to their other neighbour.
     * face_flip: near-face look-ups take the first cube across their face,
     * and every such ambiguous hidden activation its other neighbour (the
     * run that pins flip_bound).
     * debug_singular: the Gram matrix of stratum debug_singular_stratum at
     * step debug_singular_step is replaced by zero, so that the stratum takes
     * the LP0 fallback of a singular Gram. */
    double *flip_bound;
    int32_t face_flip;
    int32_t debug_singular;
    int32_t debug_singular_step;
    int64_t debug_singular_stratum;
    /* NULL, or the problem's own coefficients: the Euler step is then
     * X_{j+1} = X_j + b(t_j, X_j) dt + sigma(t_j, X_j) dW_j (t_j = j dt), the
     * driver and terminal condition f and g; b, sigma, b_lin, sigma_lin and
     * the built-in driver and terminal are not used. */
    const orc_model *model;
} orc_problem;

/* Threads the OpenMP loops over strata use. */
int orc_max_threads(void);

/* Philox4x32-10 of one counter block. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* First n uniforms of the random stream of simulation (i, k, m). */
void orc_path_uniforms(uint64_t seed, uint32_t inst, int32_t i, uint32_t k, uint32_t m,
                       int32_t n, double *u);

/* Starting point X_i of simulation (i, k, m), drawn from nu_k. */
int orc_start_point(const orc_problem *P, int32_t i, uint32_t k, uint32_t m, double *x);

/* First n standard normals of simulation (i, k, m) (before the sqrt(dt) scale),
 * step by step: out[s q + l] is normal l of path step s. */
int orc_path_normals(const orc_problem *P, int32_t i, uint32_t k, uint32_t m, int32_t n,
                     double *out);

/* Number of coefficients of a table: N * K * (1+q) * nb. */
int64_t orc_table_elems(const orc_problem *P);

/* Runs the backward iteration for i = i_hi down to i_lo (inclusive).  Rows
 * i > i_hi of `table` must already hold the fitted coefficients.  Returns 0 on
 * success, a negative value on invalid input.  `singular` (may be NULL)
 * receives the number of strata whose Gram matrix was singular. */
int orc_solve(const orc_problem *P, double *table, int32_t i_hi, int32_t i_lo,
              int64_t *singular, int32_t threads);

/* Cloud of one stratum at step i, given the fitted rows > i of `table`:
 * Xi [M*d], dWi [M*q], Sp [M] (tail response g(X_N)+sum_{j>i} f_j dt, control
 * variate included), y1 [M] (fitted y_{i+1} at X_{i+1}, g at i+1 = N), and
 * cvi [M] (network term at t_i, zero without control variate). */
int orc_cloud(const orc_problem *P, const double *table, int32_t i, uint32_t k,
              double *Xi, double *dWi, double *Sp, double *y1, double *cvi);

/* Evaluation of the fitted (truncated) y_i and z_i at n points x [n*d]. */
int orc_eval(const orc_problem *P, const double *table, int32_t i, int64_t n,
             const double *x, double *y, double *z);

/* ROOT read-out: LP0 regression on the point x0 at i = 0 with M_root
 * simulations (counter stratum tag 0xFFFFFFFF).  y0 scalar, z0 [q]. */
int orc_root(const orc_problem *P, const double *table, const double *x0, int32_t M_root,
             double *y0, double *z0);

/* Evaluation of the sweep's driver and terminal function (test access). */
double orc_driver(const orc_problem *P, double t, const double *x, double y, const double *z);
double orc_terminal(const orc_problem *P, const double *x);

/* Dense MLP (in -> H -> H -> out, SiLU) forward and parameter gradient of
 * 0.5*|y - target|^2 summed over the batch.  Parameter layout:
 * W1[H][in], b1[H], W2[H][H], b2[H], W3[out][H], b3[out]. */
int64_t orc_mlp_param_count(int32_t in, int32_t H, int32_t out);
void orc_mlp_forward(int32_t in, int32_t H, int32_t out, const double *params,
                     const double *x, int64_t B, double *y);
void orc_mlp_backward(int32_t in, int32_t H, int32_t out, const double *params,
                      const double *x, const double *dy, int64_t B, double *grad);

/* The same with bfloat16 rounding at the points a bfloat16 matrix-instruction
 * implementation rounds (mask: 1 weights, 2 inputs, 4 hidden activations,
 * 8 upstream and hidden-layer gradients (also in the bias gradients), 16 inputs as a pair of bfloat16
 * numbers hi + lo with hi = bf16(x), lo = bf16(x - hi); biases are never
 * rounded). */
void orc_mlp_forward_bf(int32_t in, int32_t H, int32_t out, const double *params,
                        const double *x, int64_t B, double *y, int32_t bf);
void orc_mlp_backward_bf(int32_t in, int32_t H, int32_t out, const double *params,
                         const double *x, const double *dy, int64_t B, double *grad, int32_t bf);

#ifdef __cplusplus
}
#endif
#endif
