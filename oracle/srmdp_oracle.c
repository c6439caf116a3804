/*
 * srmdp_oracle.c -- plain FP64 CPU oracle of the SRMDP backward sweep.
 *
 * TEST INFRASTRUCTURE ONLY (see srmdp_oracle.h).  Slow on purpose: no blocking,
 * no fusion, no reordering beyond what the paper's definitions state.  Each
 * function names the passage of the paper it follows.
 *
 * Readings of the paper taken here (the paper is silent or garbled on them):
 *  - Euler dynamics (Section 2, Algorithm "Euler dynamics") is read with the
 *    time index of the current step j, X_{j+1} = X_j + b(X_j) dt + sigma dW_j,
 *    with the drift b(x)_l = b_l + b_lin_l x_l (constant b, or the
 *    Ornstein-Uhlenbeck drift) and the diffusion sigma(x)_{l,c} = sigma_{l,c}
 *    + [l = c] sigma_lin_l x_l (constant, or with a diagonal part linear in
 *    the state as in geometric Brownian motion; q = d then).
 *  - The z-response of Algorithm SRMDP, eq. (PsiM), uses the tail
 *    g(X_N) + sum_{j=i+1}^{N-1} f_j dt of the same path started at X_i,
 *    multiplied by dW_i / dt, as in the MDP identity eq. (MDP:intro).
 *  - z is fitted before y (the y response contains f_i(., z_i)).
 *  - Truncation T_L (eq. TL) is applied when a fitted function is evaluated;
 *    stored coefficients are untruncated; +inf disables it.
 *  - Only the K bounded cells of the domain are sampled; a point outside the
 *    domain is evaluated with the affine fit of the nearest boundary cell.
 *  - Cells are half-open [x-, x+) as in assumption (A_Strat).
 *  - Uniforms are open, u = (2*(r >> 9) + 1) * 2^-24, exact in binary32 and
 *    binary64, so both precisions of the GPU library see the same number.
 *  - Random inputs: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *    key (seed mod 2^32, seed >> 32) and counter (block, m, k, i | inst << 16);
 *    words 0..d-1 of blocks 0.. give the start point, the following blocks give
 *    the Gaussian increments through Box-Muller (1958) pairs.
 *  - Least squares by the normal equations with a Cholesky factor of the Gram
 *    matrix on the cube-centred, scaled basis (1, xi_1..xi_d),
 *    xi_l = 2 (x_l - c_l) / h_l; same solution as the QR route of Section
 *    "Explicit solutions to OLS".  A pivot <= 1e-12 * trace(G) is treated as
 *    singular and the stratum falls back to the empirical mean (LP0).
 */
#include "srmdp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- Philox -- */

/* Philox4x32-10 as published by Salmon et al. (SC'11): ten rounds of the
 * two-multiplier S-box; the key is bumped by the Weyl constants between
 * rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t p0 = (uint64_t)mult0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)mult1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The random stream of one simulation: uniform number n is word n%4 of the
 * Philox block n/4.  A one-block cache avoids recomputing a block for every
 * word; it changes nothing in the values. */
typedef struct {
    uint32_t key[2];
    uint32_t m, k, tag;
    int64_t cached_block;
    uint32_t words[4];
} path_stream;

static void stream_init(path_stream *s, uint64_t seed, uint32_t inst, int32_t i, uint32_t k,
                        uint32_t m)
{
    s->key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    s->key[1] = (uint32_t)(seed >> 32);
    s->m = m;
    s->k = k;
    s->tag = ((uint32_t)i & 0xFFFFu) | (inst << 16);
    s->cached_block = -1;
}

static uint32_t stream_word(path_stream *s, int64_t n)
{
    int64_t blk = n / 4;
    if (blk != s->cached_block) {
        uint32_t ctr[4] = {(uint32_t)blk, s->m, s->k, s->tag};
        orc_philox4x32_10(ctr, s->key, s->words);
        s->cached_block = blk;
    }
    return s->words[n % 4];
}

/* Open uniform on (0,1): the top 23 bits, made odd, times 2^-24. */
static double word_to_uniform(uint32_t r)
{
    return (2.0 * (double)(r >> 9) + 1.0) * ldexp(1.0, -24);
}

static double stream_uniform(path_stream *s, int64_t n)
{
    return word_to_uniform(stream_word(s, n));
}

void orc_path_uniforms(uint64_t seed, uint32_t inst, int32_t i, uint32_t k, uint32_t m,
                       int32_t n, double *u)
{
    path_stream s;
    stream_init(&s, seed, inst, i, k, m);
    for (int32_t a = 0; a < n; ++a) u[a] = stream_uniform(&s, a);
}

/* Number of Philox blocks used by the start point: ceil(d/4). */
static int start_blocks(int d) { return (d + 3) / 4; }

/* Standard normal l (0 <= l < q) of path step `step` (step j - i of a
 * simulation started at step i).  The q normals of a step are the numbers
 * n = step * Q + l of the path's normal sequence, with Q = q when q divides 4
 * (4/q consecutive steps share a Philox block) and Q = 4 ceil(q/4) otherwise
 * (each step starts on a block of its own, and the last block's unused
 * numbers are skipped).  Number n is Box-Muller on the uniform pair p = n/2
 * that follows the start blocks; even n takes the cosine branch, odd n the
 * sine branch. */
static double stream_normal(path_stream *s, int d, int q, int64_t step, int l)
{
    const double pi = 3.14159265358979323846;
    const int64_t Q = (4 % q == 0) ? q : 4 * ((q + 3) / 4);
    const int64_t n = step * Q + l;
    int64_t p = n / 2;
    int64_t base = 4 * (int64_t)start_blocks(d) + 2 * p;
    double u1 = stream_uniform(s, base);
    double u2 = stream_uniform(s, base + 1);
    double rho = sqrt(-2.0 * log(u1));
    double theta = 2.0 * pi * u2;
    return (n % 2 == 0) ? rho * cos(theta) : rho * sin(theta);
}

/* ------------------------------------------------------------------ grid -- */

typedef struct {
    int d;
    int64_t K;
    int kind;  /* ORC_GRID_* */
    double mu;
    double lo[64], hi[64], h[64];
    int32_t cells[64];
    int64_t stride[64];
} grid_t;

static double logistic_cdf(double mu, double x) { return 1.0 / (1.0 + exp(-mu * x)); }

/* Logistic quantile F^{-1}(p) = log(p / (1 - p)) / mu. */
static double logistic_quantile(double mu, double p) { return log(p / (1.0 - p)) / mu; }

static int grid_init(const orc_problem *P, grid_t *G)
{
    if (P->d < 1 || P->d > 64) return -1;
    if (P->grid_kind != ORC_GRID_EQUAL_SIZE && P->grid_kind != ORC_GRID_EQUAL_PROB) return -1;
    G->d = P->d;
    G->K = 1;
    G->kind = P->grid_kind;
    G->mu = P->mu;
    for (int l = 0; l < P->d; ++l) {
        if (P->cells[l] < 1) return -1;
        if (G->kind == ORC_GRID_EQUAL_SIZE) {
            if (!(P->lo[l] < P->hi[l])) return -1;
            G->lo[l] = P->lo[l];
            G->hi[l] = P->hi[l];
            G->h[l] = (P->hi[l] - P->lo[l]) / (double)P->cells[l];
        }
        G->cells[l] = P->cells[l];
        G->stride[l] = G->K; /* dimension 0 varies fastest */
        G->K *= P->cells[l];
    }
    return 0;
}

/* Position of x along dimension l in cell widths: (x - lo) C / (hi - lo) for
 * equal-size cells; C F(x) for equal-probability cells, whose c-th cell is
 * the set where c <= C F(x) < c + 1. */
static double cell_coord(const grid_t *G, int l, double x)
{
    if (G->kind == ORC_GRID_EQUAL_PROB) return (double)G->cells[l] * logistic_cdf(G->mu, x);
    return (x - G->lo[l]) * ((double)G->cells[l] / (G->hi[l] - G->lo[l]));
}

/* Cell of x along dimension l: floor of its coordinate, clamped to the
 * boundary cells (points outside an equal-size domain belong to the nearest
 * boundary cell for evaluation). */
static int64_t cell_of(const grid_t *G, int l, double x)
{
    double c = floor(cell_coord(G, l, x));
    if (c < 0.0) c = 0.0;
    if (c > (double)(G->cells[l] - 1)) c = (double)(G->cells[l] - 1);
    return (int64_t)c;
}

static int64_t cube_of(const grid_t *G, const double *x)
{
    int64_t k = 0;
    for (int l = 0; l < G->d; ++l) k += cell_of(G, l, x[l]) * G->stride[l];
    return k;
}

static int64_t cube_cell(const grid_t *G, int64_t k, int l)
{
    return (k / G->stride[l]) % G->cells[l];
}

/* Cubes that a look-up at x may take when rounding moves a coordinate lying
 * within eps cell widths of an interior face across it: the cube of x first,
 * then the cubes across each such face, every combination (at most 8, i.e.
 * three faces; a fourth near face in one point is ignored).  Returns the
 * count. */
static int candidate_cubes(const grid_t *G, const double *x, double eps, int64_t *cand)
{
    int n = 1;
    cand[0] = cube_of(G, x);
    for (int l = 0; l < G->d && n <= 4; ++l) {
        double t = cell_coord(G, l, x[l]);
        double c = (double)cell_of(G, l, x[l]);
        double frac = t - c;
        int64_t step = 0;
        if (frac < eps && c > 0.0 && t >= 0.0)
            step = -G->stride[l];
        else if (frac > 1.0 - eps && c < (double)(G->cells[l] - 1))
            step = G->stride[l];
        if (step == 0) continue;
        for (int a = 0; a < n; ++a) cand[n + a] = cand[a] + step;
        n *= 2;
    }
    return n;
}

/* Basis of the local spaces of assumption (A_Strat): LP0 = {1}, LP1 =
 * {1, xi_1..xi_d} with xi an affine coordinate of the cube.  Equal-size
 * cells: xi = 2 (x - centre) / h, in [-1, 1) inside the cube.  Equal-
 * probability cells, unbounded at the ends: xi = mu (x - m) with m the
 * cell's nu-median F^{-1}((c + 1/2) / C).  Only the span enters the fit. */
static int basis_size(const orc_problem *P) { return P->basis == ORC_LP1 ? P->d + 1 : 1; }

static void basis_eval(const orc_problem *P, const grid_t *G, int64_t k, const double *x,
                       double *phi)
{
    phi[0] = 1.0;
    if (P->basis != ORC_LP1) return;
    for (int l = 0; l < G->d; ++l) {
        double c = (double)cube_cell(G, k, l);
        if (G->kind == ORC_GRID_EQUAL_PROB) {
            double m = logistic_quantile(G->mu, (c + 0.5) / (double)G->cells[l]);
            phi[1 + l] = G->mu * (x[l] - m);
        } else {
            double centre = G->lo[l] + (c + 0.5) * G->h[l];
            phi[1 + l] = 2.0 * (x[l] - centre) / G->h[l];
        }
    }
}

/* ------------------------------------------------------- problem data -- */

/* Terminal condition g (Section "Model, stratification, and performance
 * benchmark" for the logistic case; cos of the coordinate sum otherwise). */
double orc_terminal(const orc_problem *P, const double *x)
{
    if (P->model) return P->model->g(x, P->model->params);
    double s = 0.0;
    for (int l = 0; l < P->d; ++l) s += x[l];
    if (P->terminal == ORC_G_LOGISTIC) {
        double w = exp(P->T + s);
        return w / (1.0 + w);
    }
    return cos(s);
}

/* Driver f(t, x, y, z): logistic f = (sum z)(y - (2+q)/(2q)) of the paper's
 * benchmark, or the linear f = -r y + kappa sum z. */
double orc_driver(const orc_problem *P, double t, const double *x, double y, const double *z)
{
    if (P->model) return P->model->f(t, x, y, z, P->model->params);
    double sz = 0.0;
    for (int l = 0; l < P->q; ++l) sz += z[l];
    if (P->driver == ORC_DRV_LOGISTIC)
        return sz * (y - (2.0 + P->q) / (2.0 * P->q));
    return -P->r * y + P->kappa * sz;
}

static double clampv(double v, double L)
{
    if (!(L < INFINITY)) return v;
    if (v < -L) return -L;
    if (v > L) return L;
    return v;
}

/* ---------------------------------------------------------- the MLP ---- */

/* Round a value to bfloat16 (8-bit significand), round to nearest even, as
 * the GPU does when it feeds a value to a bfloat16 matrix instruction.  The
 * value is first rounded to binary32 (the GPU holds it in binary32). */
static double bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return v; /* inf / nan */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* Which values the bfloat16 emulation rounds (bit mask).  ORC_BF_PAIR
 * represents each input by two bfloat16 numbers, hi = bf16(x) and
 * lo = bf16(x - hi) (x taken in binary32, where x - hi is exact), and feeds
 * hi + lo: about 16 significant bits. */
enum { ORC_BF_WEIGHTS = 1, ORC_BF_INPUT = 2, ORC_BF_HIDDEN = 4, ORC_BF_GRADS = 8, ORC_BF_PAIR = 16 };

static double bf16_pair(double v)
{
    const double x = (double)(float)v;
    const double hi = bf16_round(x);
    return hi + bf16_round(x - hi);
}

/* The network's view of input value v under the emulation mask bf. */
static double input_value(double v, int bf)
{
    if (bf & ORC_BF_PAIR) return bf16_pair(v);
    if (bf & ORC_BF_INPUT) return bf16_round(v);
    return v;
}

int64_t orc_mlp_param_count(int32_t in, int32_t H, int32_t out)
{
    return (int64_t)H * in + H + (int64_t)H * H + H + (int64_t)out * H + out;
}

static double silu(double a) { return a / (1.0 + exp(-a)); }
static double silu_grad(double a)
{
    double s = 1.0 / (1.0 + exp(-a));
    return s * (1.0 + a * (1.0 - s));
}

static double maybe_bf16(double v, int on) { return on ? bf16_round(v) : v; }

/* One sample through in -> H -> H -> out with SiLU after both hidden layers;
 * pre-activations a1, a2 and the (possibly rounded) layer inputs h1, h2 are
 * returned.  `bf` selects the values rounded to bfloat16: weights (biases are
 * kept), the input vector, the hidden activations fed to the next layer. */
/* The other bfloat16 neighbour of (float)v: the one round-to-nearest did not
 * pick (the two values bracketing v in the 8-bit significand). */
static double bf16_other(double v)
{
    float f = (float)v, r = (float)bf16_round(v);
    uint32_t u, ur;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return v;
    memcpy(&ur, &r, 4);
    const uint32_t down = u & 0xFFFF0000u, other = ur == down ? down + 0x10000u : down;
    memcpy(&f, &other, 4);
    return (double)f;
}

/* Binary32 units around a bfloat16 rounding midpoint within which the
 * flip-bound diagnostic treats a hidden activation as ambiguous. */
#define ORC_BF16_FLIP_ULPS 32

/* Is (float)v within `ulps` binary32 units of a bfloat16 rounding midpoint
 * (where another rounding of the same value may take the other neighbour)? */
static int bf16_near_midpoint(double v, int ulps)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return 0;
    int low = (int)(u & 0xFFFFu);
    return abs(low - 0x8000) <= ulps;
}

/* One sample through in -> H -> H -> out with SiLU after both hidden layers;
 * pre-activations a1, a2 and the (possibly rounded) layer inputs h1, h2 are
 * returned.  `bf` selects the values rounded to bfloat16: weights (biases are
 * kept), the input vector, the hidden activations fed to the next layer.
 * flip_layer 1 or 2 rounds hidden unit flip_unit of that layer to its other
 * bfloat16 neighbour, 3 rounds every ambiguous hidden activation (within
 * ORC_BF16_FLIP_ULPS of a midpoint) to its other neighbour (the flip-bound
 * diagnostic and its forced run); 0 flips nothing. */
static void mlp_one_flip(int32_t in, int32_t H, int32_t out, const double *p, const double *x,
                         double *y, double *a1, double *a2, double *h1, double *h2, int bf,
                         int flip_layer, int flip_unit)
{
    const double *W1 = p, *b1 = W1 + (int64_t)H * in, *W2 = b1 + H, *b2 = W2 + (int64_t)H * H,
                 *W3 = b2 + H, *b3 = W3 + (int64_t)out * H;
    const int rw = bf & ORC_BF_WEIGHTS, rh = bf & ORC_BF_HIDDEN;
    for (int a = 0; a < H; ++a) {
        double s = b1[a];
        for (int c = 0; c < in; ++c)
            s += maybe_bf16(W1[(int64_t)a * in + c], rw) * input_value(x[c], bf);
        a1[a] = s;
        const int f1 = (flip_layer == 1 && a == flip_unit) ||
                       (flip_layer == 3 && bf16_near_midpoint(silu(s), ORC_BF16_FLIP_ULPS));
        h1[a] = f1 ? bf16_other(silu(s)) : maybe_bf16(silu(s), rh);
    }
    for (int a = 0; a < H; ++a) {
        double s = b2[a];
        for (int c = 0; c < H; ++c) s += maybe_bf16(W2[(int64_t)a * H + c], rw) * h1[c];
        a2[a] = s;
        const int f2 = (flip_layer == 2 && a == flip_unit) ||
                       (flip_layer == 3 && bf16_near_midpoint(silu(s), ORC_BF16_FLIP_ULPS));
        h2[a] = f2 ? bf16_other(silu(s)) : maybe_bf16(silu(s), rh);
    }
    for (int o = 0; o < out; ++o) {
        double s = b3[o];
        for (int c = 0; c < H; ++c) s += maybe_bf16(W3[(int64_t)o * H + c], rw) * h2[c];
        y[o] = s;
    }
}

static void mlp_one_bf(int32_t in, int32_t H, int32_t out, const double *p, const double *x,
                       double *y, double *a1, double *a2, double *h1, double *h2, int bf)
{
    mlp_one_flip(in, H, out, p, x, y, a1, a2, h1, h2, bf, 0, 0);
}

void orc_mlp_forward_bf(int32_t in, int32_t H, int32_t out, const double *params, const double *x,
                        int64_t B, double *y, int32_t bf)
{
    double *buf = (double *)malloc(sizeof(double) * 4 * (size_t)H);
    for (int64_t s = 0; s < B; ++s)
        mlp_one_bf(in, H, out, params, x + s * in, y + s * out, buf, buf + H, buf + 2 * H,
                   buf + 3 * H, bf);
    free(buf);
}

void orc_mlp_forward(int32_t in, int32_t H, int32_t out, const double *params, const double *x,
                     int64_t B, double *y)
{
    orc_mlp_forward_bf(in, H, out, params, x, B, y, 0);
}

/* Gradient of sum_s <dy_s, y_s> with respect to the parameters (dy is the
 * upstream gradient), by the chain rule written layer by layer.  With `bf`,
 * the forward values are the rounded ones of mlp_one_bf, and ORC_BF_GRADS also
 * rounds the upstream gradient and the hidden-layer gradients where they feed a
 * product (the weight-gradient and back-propagation contractions) and in the
 * bias gradients, which sum the same rounded values. */
void orc_mlp_backward_bf(int32_t in, int32_t H, int32_t out, const double *params,
                         const double *x, const double *dy, int64_t B, double *grad, int32_t bf)
{
    const double *W2p = params + (int64_t)H * in + H, *W3p = W2p + (int64_t)H * H + H;
    const int rw = bf & ORC_BF_WEIGHTS, rg = bf & ORC_BF_GRADS;
    double *gW1 = grad, *gb1 = gW1 + (int64_t)H * in, *gW2 = gb1 + H,
           *gb2 = gW2 + (int64_t)H * H, *gW3 = gb2 + H, *gb3 = gW3 + (int64_t)out * H;
    memset(grad, 0, sizeof(double) * (size_t)orc_mlp_param_count(in, H, out));
    double *buf = (double *)malloc(sizeof(double) * (6 * (size_t)H + (size_t)out));
    double *a1 = buf, *a2 = a1 + H, *h1 = a2 + H, *h2 = h1 + H, *d2 = h2 + H, *d1 = d2 + H,
           *yy = d1 + H;
    double *gq = (double *)malloc(sizeof(double) * (size_t)(out + 2 * H));
    double *gr = gq + out, *d2r = gr + H;
    for (int64_t s = 0; s < B; ++s) {
        const double *xs = x + s * in, *g = dy + s * out;
        mlp_one_bf(in, H, out, params, xs, yy, a1, a2, h1, h2, bf);
        for (int o = 0; o < out; ++o) gq[o] = maybe_bf16(g[o], rg);
        for (int o = 0; o < out; ++o) {
            gb3[o] += gq[o];
            for (int c = 0; c < H; ++c) gW3[(int64_t)o * H + c] += gq[o] * h2[c];
        }
        for (int c = 0; c < H; ++c) {
            double acc = 0.0;
            for (int o = 0; o < out; ++o) acc += maybe_bf16(W3p[(int64_t)o * H + c], rw) * gq[o];
            d2[c] = acc * silu_grad(a2[c]);
            d2r[c] = maybe_bf16(d2[c], rg);
        }
        for (int a = 0; a < H; ++a) {
            gb2[a] += d2r[a];
            for (int c = 0; c < H; ++c) gW2[(int64_t)a * H + c] += d2r[a] * h1[c];
        }
        for (int c = 0; c < H; ++c) {
            double acc = 0.0;
            for (int a = 0; a < H; ++a) acc += maybe_bf16(W2p[(int64_t)a * H + c], rw) * d2r[a];
            d1[c] = acc * silu_grad(a1[c]);
            gr[c] = maybe_bf16(d1[c], rg);
        }
        for (int a = 0; a < H; ++a) {
            gb1[a] += gr[a];
            for (int c = 0; c < in; ++c) gW1[(int64_t)a * in + c] += gr[a] * input_value(xs[c], bf);
        }
    }
    free(gq);
    free(buf);
}

void orc_mlp_backward(int32_t in, int32_t H, int32_t out, const double *params, const double *x,
                      const double *dy, int64_t B, double *grad)
{
    orc_mlp_backward_bf(in, H, out, params, x, dy, B, grad, 0);
}

/* The frozen network z_theta(t, x) (q values). */
/* z_theta(t, x).  With dz (non-NULL, bfloat16 hidden activations), dz[l]
 * receives the sum over the ambiguous hidden activations of the change of
 * output l when that activation is rounded to its other neighbour. */
static void cv_net(const orc_problem *P, double t, const double *x, double *z, double *dz)
{
    const int H = P->cv_hidden;
    double inp[65], buf[4 * 256], alt[64], tmp[4 * 256];
    inp[0] = t;
    for (int l = 0; l < P->d; ++l) inp[1 + l] = x[l];
    const int forced = P->face_flip && (P->cv_bf16 & ORC_BF_HIDDEN) ? 3 : 0;
    mlp_one_flip(P->d + 1, H, P->q, P->cv_params, inp, z, buf, buf + H, buf + 2 * H, buf + 3 * H, P->cv_bf16,
                 forced, 0);
    if (!dz) return;
    for (int l = 0; l < P->q; ++l) dz[l] = 0.0;
    if (!(P->cv_bf16 & ORC_BF_HIDDEN)) return;
    for (int layer = 1; layer <= 2; ++layer)
        for (int a = 0; a < H; ++a) {
            double pre = buf[(layer - 1) * H + a];
            if (!bf16_near_midpoint(silu(pre), ORC_BF16_FLIP_ULPS)) continue;
            mlp_one_flip(P->d + 1, H, P->q, P->cv_params, inp, alt, tmp, tmp + H, tmp + 2 * H, tmp + 3 * H,
                         P->cv_bf16, layer, a);
            for (int l = 0; l < P->q; ++l) dz[l] += fabs(alt[l] - z[l]);
        }
}

/* -------------------------------------------------------- validation -- */

static int check_problem(const orc_problem *P, grid_t *G)
{
    if (!P || P->d < 1 || P->d > 64 || P->q < 1 || P->q > 64) return -1;
    if (P->N < 1 || P->N > 65535 || !(P->T > 0.0) || !(P->mu > 0.0)) return -1;
    if (P->basis != ORC_LP0 && P->basis != ORC_LP1) return -1;
    if (!P->sigma && P->q != P->d) return -1;
    if (P->sigma_lin && P->q != P->d) return -1;
    if (P->M < basis_size(P)) return -1; /* M >= dim of the local space */
    if (P->model && (P->q != P->d || !P->model->b || !P->model->sigma_dw || !P->model->f || !P->model->g ||
                     P->b || P->sigma || P->b_lin || P->sigma_lin))
        return -1;
    if (P->cv_params && (P->cv_hidden < 1 || P->cv_hidden > 256 || P->q > 64)) return -1;
    return grid_init(P, G);
}

int64_t orc_table_elems(const orc_problem *P)
{
    grid_t G;
    if (check_problem(P, &G) != 0) return -1;
    return (int64_t)P->N * G.K * (1 + P->q) * basis_size(P);
}

static int64_t rec_size(const orc_problem *P) { return (int64_t)(1 + P->q) * basis_size(P); }

/* ---------------------------------------------------- sampling (nu_k) -- */

/* Algorithm "stratify": inverse CDF of the logistic law restricted to
 * [x-, x+), F(x) = 1 / (1 + exp(-mu x)), given Fm = F(x-) and Fp = F(x+). */
static double stratify_one(double mu, double Fm, double Fp, double U)
{
    return -(1.0 / mu) * log(1.0 / (Fm + U * (Fp - Fm)) - 1.0);
}

static void start_point(const orc_problem *P, const grid_t *G, path_stream *s, int64_t k,
                        double *x)
{
    for (int l = 0; l < P->d; ++l) {
        double c = (double)cube_cell(G, k, l), Fm, Fp;
        if (G->kind == ORC_GRID_EQUAL_PROB) {
            /* F at the quantile edges: c / C and (c + 1) / C */
            Fm = c / (double)G->cells[l];
            Fp = (c + 1.0) / (double)G->cells[l];
        } else {
            double xm = G->lo[l] + c * G->h[l];
            Fm = logistic_cdf(P->mu, xm);
            Fp = logistic_cdf(P->mu, xm + G->h[l]);
        }
        x[l] = stratify_one(P->mu, Fm, Fp, stream_uniform(s, l));
    }
}

int orc_start_point(const orc_problem *P, int32_t i, uint32_t k, uint32_t m, double *x)
{
    grid_t G;
    if (check_problem(P, &G) != 0 || (int64_t)k >= G.K) return -1;
    path_stream s;
    stream_init(&s, P->seed, P->inst, i, k, m);
    start_point(P, &G, &s, k, x);
    return 0;
}

int orc_path_normals(const orc_problem *P, int32_t i, uint32_t k, uint32_t m, int32_t n,
                     double *out)
{
    if (!P || P->d < 1) return -1;
    path_stream s;
    stream_init(&s, P->seed, P->inst, i, k, m);
    for (int32_t a = 0; a < n; ++a) out[a] = stream_normal(&s, P->d, P->q, a / P->q, a % P->q);
    return 0;
}

/* ----------------------------------------------- fitted-table evaluation -- */

/* y-component (c = 0) or z-component c = 1..q of the fitted function at
 * row j, evaluated at x with the record and basis of cube k (fitted: the cell
 * of x, extended past the domain). */
static double fitted_in(const orc_problem *P, const grid_t *G, const double *table, int32_t j,
                        int c, const double *x, int64_t k)
{
    int nb = basis_size(P);
    double phi[65];
    basis_eval(P, G, k, x, phi);
    const double *rec = table + ((int64_t)j * G->K + k) * rec_size(P) + (int64_t)c * nb;
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += rec[b] * phi[b];
    return clampv(v, c == 0 ? P->clamp_y : P->clamp_z);
}

static double fitted(const orc_problem *P, const grid_t *G, const double *table, int32_t j,
                     int c, const double *x)
{
    return fitted_in(P, G, table, j, c, x, cube_of(G, x));
}

static void z_at(const orc_problem *P, const grid_t *G, const double *table, int32_t j,
                 const double *x, double *z)
{
    for (int l = 0; l < P->q; ++l) z[l] = fitted(P, G, table, j, 1 + l, x);
}

int orc_eval(const orc_problem *P, const double *table, int32_t i, int64_t n, const double *x,
             double *y, double *z)
{
    grid_t G;
    if (check_problem(P, &G) != 0 || i < 0 || i >= P->N) return -1;
    for (int64_t a = 0; a < n; ++a) {
        if (y) y[a] = fitted(P, &G, table, i, 0, x + a * P->d);
        if (z) z_at(P, &G, table, i, x + a * P->d, z + a * P->q);
    }
    return 0;
}

/* ------------------------------------------------------- one simulation -- */

/* Largest |f(t, x, y_a, z_b) - f0| over the candidate look-ups y_a, z_b. */
static double driver_spread(const orc_problem *P, double t, const double *x, int ny,
                            const double *yc, int nz, double zc[][64], double f0)
{
    double worst = 0.0;
    for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nz; ++b) {
            double v = fabs(orc_driver(P, t, x, yc[a], zc[b]) - f0);
            if (v > worst) worst = v;
        }
    return worst;
}

/* Simulates one path from X_i (already in x0) to X_N with the Euler scheme and
 * returns what the regressions of step i need:
 *   dWi  -- the increment Delta W_i,
 *   *Sp  -- g(X_N) + sum_{j=i+1}^{N-1} f_j(X_j, y_{j+1}(X_{j+1}), z_j(X_j)) dt
 *           minus the control-variate terms sum_{j=i+1}^{N-1} z_theta(t_j,X_j).dW_j,
 *   *y1  -- y_{i+1}(X_{i+1}) (g(X_N) when i+1 = N),
 *   *cvi -- z_theta(t_i, X_i) . dW_i (zero without control variate).
 * Eq. (MDP:intro) and eq. (PsiM).
 *
 * Diagnostics (test use only).  A point X_{j+1}, j+1 < N, whose coordinate
 * lies within face_eps cell widths of an interior face sets *near; its y and z
 * look-ups may then take the cube across that face in another precision.
 * With flip (non-NULL) the path also returns flip[0] >= |change of S'|,
 * flip[1] >= |change of y1| and flip[2] >= |change of cvi| over every such
 * choice: per step the largest change of f_j dt over the candidate cubes of
 * its two look-ups, plus, with a bfloat16 network, the change of its
 * z_theta . dW_j term when ambiguous hidden roundings go the other way.  With
 * P->face_flip every such point takes the first cube across its face (the
 * forced-flip run that pins the bound). */
static void simulate(const orc_problem *P, const grid_t *G, const double *table, int32_t i,
                     path_stream *s, const double *x0, double *dWi, double *Sp, double *y1,
                     double *cvi, int *near, double *flip)
{
    const int d = P->d, q = P->q;
    const double dt = P->T / P->N, sdt = sqrt(dt);
    const int stride = P->cv_stride > 1 ? P->cv_stride : 1;
    const int track = near || flip || P->face_flip;
    double x[64], xn[64], dW[64], zcv[64], dzcv[64];
    /* z candidates at X_j for row j (zc[zuse] is the look-up the path takes),
     * computed when X_j is reached, i.e. at step j - 1 */
    double zc[8][64], zn[8][64], yc[8];
    int nzc = 0, zuse = 0;
    memcpy(x, x0, sizeof(double) * d);
    double S = 0.0, cv_tail = 0.0, dS = 0.0, dy1 = 0.0, dcvi = 0.0;
    *cvi = 0.0;
    for (int32_t j = i; j < P->N; ++j) {
        for (int l = 0; l < q; ++l)
            dW[l] = sdt * stream_normal(s, d, q, j - i, l);
        if (P->model) {
            /* Algorithm "Euler dynamics" at (t_j, X_j) */
            double bj[64], sj[64];
            P->model->b(j * dt, x, P->model->params, bj);
            P->model->sigma_dw(j * dt, x, dW, P->model->params, sj);
            for (int l = 0; l < d; ++l) xn[l] = x[l] + bj[l] * dt + sj[l];
        } else {
            for (int l = 0; l < d; ++l) {
                double drift = (P->b ? P->b[l] : 0.0) + (P->b_lin ? P->b_lin[l] * x[l] : 0.0);
                double diff = 0.0;
                if (P->sigma)
                    for (int c = 0; c < q; ++c) diff += P->sigma[l * q + c] * dW[c];
                else
                    diff = dW[l];
                if (P->sigma_lin) diff += P->sigma_lin[l] * x[l] * dW[l];
                xn[l] = x[l] + drift * dt + diff;
            }
        }
        double ynext;
        int nyc = 1, use = 0;
        if (j + 1 < P->N) {
            int64_t cand[8];
            if (track) {
                nyc = candidate_cubes(G, xn, P->face_eps, cand);
            } else {
                cand[0] = cube_of(G, xn);
            }
            if (P->face_flip && nyc > 1) use = 1;
            if (near && nyc > 1) *near = 1;
            for (int a = 0; a < nyc; ++a) {
                yc[a] = fitted_in(P, G, table, j + 1, 0, xn, cand[a]);
                for (int l = 0; l < q; ++l) zn[a][l] = fitted_in(P, G, table, j + 1, 1 + l, xn, cand[a]);
            }
            ynext = yc[use];
        } else {
            ynext = yc[0] = orc_terminal(P, xn);
        }
        double cv = 0.0, dcv = 0.0;
        if (P->cv_params) {
            if ((j - i) % stride == 0) cv_net(P, j * dt, x, zcv, flip ? dzcv : NULL);
            for (int l = 0; l < q; ++l) cv += zcv[l] * dW[l];
            if (flip)
                for (int l = 0; l < q; ++l) dcv += dzcv[l] * fabs(dW[l]);
        }
        if (j == i) {
            memcpy(dWi, dW, sizeof(double) * q);
            *y1 = ynext;
            *cvi = cv;
            dcvi = dcv;
            for (int a = 0; a < nyc; ++a)
                if (fabs(yc[a] - ynext) > dy1) dy1 = fabs(yc[a] - ynext);
        } else {
            double f0 = orc_driver(P, j * dt, x, ynext, zc[zuse]);
            S += f0 * dt;
            cv_tail += cv;
            if (flip) dS += driver_spread(P, j * dt, x, nyc, yc, nzc, zc, f0) * dt + dcv;
        }
        if (j + 1 < P->N) {
            memcpy(zc, zn, sizeof(double) * 64 * (size_t)nyc);
            nzc = nyc;
            zuse = use;
        }
        memcpy(x, xn, sizeof(double) * d);
    }
    *Sp = orc_terminal(P, x) + S - cv_tail;
    if (flip) {
        flip[0] = dS;
        flip[1] = dy1;
        flip[2] = dcvi;
    }
}

/* ----------------------------------------------------- least squares -- */

/* Cholesky factor of the n x n SPD matrix A (lower, row-major in L).
 * Returns 0, or 1 if a pivot is <= tol. */
static int cholesky(int n, const double *A, double *L, double tol)
{
    memset(L, 0, sizeof(double) * (size_t)n * n);
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c <= r; ++c) {
            double s = A[r * n + c];
            for (int t = 0; t < c; ++t) s -= L[r * n + t] * L[c * n + t];
            if (r == c) {
                if (!(s > tol)) return 1;
                L[r * n + r] = sqrt(s);
            } else {
                L[r * n + c] = s / L[c * n + c];
            }
        }
    }
    return 0;
}

/* Solves L L^T beta = rhs. */
static void chol_solve(int n, const double *L, const double *rhs, double *beta)
{
    double w[65];
    for (int r = 0; r < n; ++r) {
        double s = rhs[r];
        for (int t = 0; t < r; ++t) s -= L[r * n + t] * w[t];
        w[r] = s / L[r * n + r];
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = w[r];
        for (int t = r + 1; t < n; ++t) s -= L[t * n + r] * beta[t];
        beta[r] = s / L[r * n + r];
    }
}

/* ----------------------------------------------- one stratum at step i -- */

/* The cloud C_{i,k}; flip (NULL or [3M]) receives each simulation's bounds of
 * simulate(). */
static void cloud(const orc_problem *P, const grid_t *G, const double *table, int32_t i, int64_t k,
                  double *Xi, double *dWi, double *Sp, double *y1, double *cvi, double *flip)
{
    int near = 0;
    int *np = P->face_flags ? &near : NULL;
    for (int32_t m = 0; m < P->M; ++m) {
        path_stream s;
        stream_init(&s, P->seed, P->inst, i, (uint32_t)k, (uint32_t)m);
        start_point(P, G, &s, k, Xi + (int64_t)m * P->d);
        simulate(P, G, table, i, &s, Xi + (int64_t)m * P->d, dWi + (int64_t)m * P->q, Sp + m, y1 + m,
                 cvi + m, np, flip ? flip + 3 * (int64_t)m : NULL);
    }
    if (P->face_flags) P->face_flags[(int64_t)i * G->K + k] = (uint8_t)near;
}

int orc_cloud(const orc_problem *P, const double *table, int32_t i, uint32_t k, double *Xi,
              double *dWi, double *Sp, double *y1, double *cvi)
{
    grid_t G;
    if (check_problem(P, &G) != 0 || i < 0 || i >= P->N || (int64_t)k >= G.K) return -1;
    cloud(P, &G, table, i, (int64_t)k, Xi, dWi, Sp, y1, cvi, NULL);
    return 0;
}

/* Bound on |f(t, x, y', z') - f(t, x, y, z)| over |y' - y| <= dy and
 * |z'_l - z_l| <= dz_l (test diagnostic of the face-flip bound). */
static double driver_change_bound(const orc_problem *P, double y, const double *z, double dy,
                                  const double *dz)
{
    double sz = 0.0, sdz = 0.0;
    for (int l = 0; l < P->q; ++l) {
        sz += z[l];
        sdz += dz[l];
    }
    if (P->model) return P->model->lip_y * dy + P->model->lip_z * sdz;
    if (P->driver == ORC_DRV_LOGISTIC) {
        double c = (2.0 + P->q) / (2.0 * P->q);
        return sdz * (fabs(y - c) + dy) + fabs(sz) * dy;
    }
    return fabs(P->r) * dy + fabs(P->kappa) * sdz;
}

/* Algorithm SRMDP, one stratum k at step i: the cloud C_{i,k}, then the z
 * regression of S' dW_i / dt, then the y regression of
 * S_Y = S' + f_i(X_i, y_{i+1}(X_{i+1}), z_i(X_i)) dt, both on the local basis.
 * Writes row i, stratum k of the table; returns 1 if the Gram was singular.
 *
 * Test diagnostics: debug_singular zeroes the Gram of one (step, stratum),
 * which then takes the LP0 fallback; flip_bound receives, per coefficient, a
 * bound on its change when near-face look-ups take the cube across the face
 * (Delta beta = G^-1 sum_m phi_m Delta resp_m, bounded term by term). */
static int fit_stratum(const orc_problem *P, const grid_t *G, double *table, int32_t i, int64_t k,
                       double *work)
{
    const int d = P->d, q = P->q, nb = basis_size(P), M = P->M;
    const double dt = P->T / P->N;
    double *Xi = work, *dWi = Xi + (int64_t)M * d, *Sp = dWi + (int64_t)M * q, *y1 = Sp + M,
           *cvi = y1 + M, *cz = cvi + M, *flip = cz + M, *dcz = flip + 3 * (int64_t)M;
    double *fb = P->flip_bound ? P->flip_bound + ((int64_t)i * G->K + k) * rec_size(P) : NULL;
    cloud(P, G, table, i, k, Xi, dWi, Sp, y1, cvi, fb ? flip : NULL);

    double Gm[65 * 65], L[65 * 65], phi[65], rhs[65], beta[65], zfit[64];
    double *rec = table + ((int64_t)i * G->K + k) * rec_size(P);
    memset(Gm, 0, sizeof(Gm));
    double trace = 0.0;
    for (int m = 0; m < M; ++m) {
        basis_eval(P, G, k, Xi + (int64_t)m * d, phi);
        for (int a = 0; a < nb; ++a)
            for (int c = 0; c < nb; ++c) Gm[a * nb + c] += phi[a] * phi[c];
    }
    if (P->debug_singular && i == P->debug_singular_step && k == P->debug_singular_stratum)
        memset(Gm, 0, sizeof(Gm));
    for (int a = 0; a < nb; ++a) trace += Gm[a * nb + a];
    int singular = cholesky(nb, Gm, L, 1e-12 * trace);

    /* z first: q scalar regressions sharing the Gram matrix.  With z_center the
     * response loses y_{i+1}(X_i) dW_i / dt, whose conditional mean given X_i is
     * zero (y_{i+1} comes from clouds of later steps). */
    for (int m = 0; m < M; ++m) {
        const double *x = Xi + (int64_t)m * d;
        cz[m] = 0.0;
        dcz[m] = 0.0;
        if (!P->z_center) continue;
        if (i + 1 == P->N) {
            cz[m] = orc_terminal(P, x);
            continue;
        }
        int64_t cand[8];
        int nc = candidate_cubes(G, x, P->face_eps, cand);
        if (P->face_flags && nc > 1) P->face_flags[(int64_t)i * G->K + k] = 1;
        cz[m] = fitted_in(P, G, table, i + 1, 0, x, cand[P->face_flip && nc > 1 ? 1 : 0]);
        for (int a = 0; a < nc; ++a) {
            double v = fabs(fitted_in(P, G, table, i + 1, 0, x, cand[a]) - cz[m]);
            if (v > dcz[m]) dcz[m] = v;
        }
    }
    for (int l = 0; l < q; ++l) {
        memset(rhs, 0, sizeof(rhs));
        for (int m = 0; m < M; ++m) {
            double resp = (Sp[m] - cz[m]) * dWi[(int64_t)m * q + l] / dt;
            basis_eval(P, G, k, Xi + (int64_t)m * d, phi);
            for (int a = 0; a < nb; ++a) rhs[a] += phi[a] * resp;
        }
        if (!singular) {
            chol_solve(nb, L, rhs, beta);
        } else {
            memset(beta, 0, sizeof(beta));
            beta[0] = rhs[0] / M;
        }
        for (int a = 0; a < nb; ++a) rec[(1 + l) * nb + a] = beta[a];
    }
    /* y next, with the just-fitted (truncated) z_i at X_i. */
    memset(rhs, 0, sizeof(rhs));
    for (int m = 0; m < M; ++m) {
        const double *x = Xi + (int64_t)m * d;
        basis_eval(P, G, k, x, phi);
        for (int l = 0; l < q; ++l) {
            double v = 0.0;
            for (int a = 0; a < nb; ++a) v += rec[(1 + l) * nb + a] * phi[a];
            zfit[l] = clampv(v, P->clamp_z);
        }
        double SY = Sp[m] + orc_driver(P, i * dt, x, y1[m], zfit) * dt - cvi[m];
        for (int a = 0; a < nb; ++a) rhs[a] += phi[a] * SY;
    }
    if (!singular) {
        chol_solve(nb, L, rhs, beta);
    } else {
        memset(beta, 0, sizeof(beta));
        beta[0] = rhs[0] / M;
    }
    for (int a = 0; a < nb; ++a) rec[a] = beta[a];

    if (fb) {
        /* leverage w_m = G^-1 phi_m of each sample (the LP0 mean when singular) */
        double bz[64][65], dz[64], w[65];
        memset(bz, 0, sizeof(bz));
        memset(fb, 0, sizeof(double) * (size_t)rec_size(P));
        for (int m = 0; m < M; ++m) {
            basis_eval(P, G, k, Xi + (int64_t)m * d, phi);
            if (!singular) {
                chol_solve(nb, L, phi, w);
            } else {
                memset(w, 0, sizeof(w));
                w[0] = 1.0 / M;
            }
            for (int l = 0; l < q; ++l) {
                double dr = (flip[3 * m] + dcz[m]) * fabs(dWi[(int64_t)m * q + l]) / dt;
                for (int a = 0; a < nb; ++a) bz[l][a] += fabs(w[a]) * dr;
            }
        }
        for (int m = 0; m < M; ++m) {
            const double *x = Xi + (int64_t)m * d;
            basis_eval(P, G, k, x, phi);
            for (int l = 0; l < q; ++l) {
                double v = 0.0;
                dz[l] = 0.0;
                for (int a = 0; a < nb; ++a) {
                    v += rec[(1 + l) * nb + a] * phi[a];
                    dz[l] += bz[l][a] * fabs(phi[a]);
                }
                zfit[l] = clampv(v, P->clamp_z);
            }
            double dSY = flip[3 * m] + driver_change_bound(P, y1[m], zfit, flip[3 * m + 1], dz) * dt +
                         flip[3 * m + 2];
            if (!singular) {
                chol_solve(nb, L, phi, w);
            } else {
                memset(w, 0, sizeof(w));
                w[0] = 1.0 / M;
            }
            for (int a = 0; a < nb; ++a) fb[a] += fabs(w[a]) * dSY;
        }
        for (int l = 0; l < q; ++l)
            for (int a = 0; a < nb; ++a) fb[(1 + l) * nb + a] = bz[l][a];
    }
    return singular;
}

int orc_solve(const orc_problem *P, double *table, int32_t i_hi, int32_t i_lo, int64_t *singular,
              int32_t threads)
{
    grid_t G;
    if (check_problem(P, &G) != 0) return -1;
    if (i_hi >= P->N || i_lo < 0 || i_lo > i_hi) return -1;
    if (P->d > 64 || basis_size(P) > 65) return -1;
    int64_t nsing = 0;
    const int64_t wsz = (int64_t)P->M * (P->d + P->q + 8);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    /* Backward iteration; the strata of one step are independent. */
    for (int32_t i = i_hi; i >= i_lo; --i) {
        int64_t step_sing = 0;
#pragma omp parallel reduction(+ : step_sing)
        {
            double *work = (double *)malloc(sizeof(double) * (size_t)wsz);
#pragma omp for schedule(dynamic, 1)
            for (int64_t k = 0; k < G.K; ++k) step_sing += fit_stratum(P, &G, table, i, k, work);
            free(work);
        }
        nsing += step_sing;
    }
    if (singular) *singular = nsing;
    return 0;
}

/* ----------------------------------------------------------- read-out -- */

/* ROOT read-out: the MDP identity with the initial law delta_{x0} (the value
 * functions do not depend on the initial law, Section 2): LP0 regressions on
 * the point x0, z first, then y with the fitted z in the i = 0 driver term. */
int orc_root(const orc_problem *P, const double *table, const double *x0, int32_t M_root,
             double *y0, double *z0)
{
    grid_t G;
    if (check_problem(P, &G) != 0 || M_root < 1) return -1;
    const int q = P->q;
    const double dt = P->T / P->N;
    double *Sp = (double *)malloc(sizeof(double) * (size_t)M_root * (q + 3));
    double *y1 = Sp + M_root, *cvi = y1 + M_root, *dW = cvi + M_root;
    for (int l = 0; l < q; ++l) z0[l] = 0.0;
    for (int32_t m = 0; m < M_root; ++m) {
        path_stream s;
        stream_init(&s, P->seed, P->inst, 0, 0xFFFFFFFFu, (uint32_t)m);
        simulate(P, &G, table, 0, &s, x0, dW + (int64_t)m * q, Sp + m, y1 + m, cvi + m, NULL, NULL);
        for (int l = 0; l < q; ++l) z0[l] += Sp[m] * dW[(int64_t)m * q + l] / dt;
    }
    for (int l = 0; l < q; ++l) z0[l] /= M_root;
    double zc[64];
    for (int l = 0; l < q; ++l) zc[l] = clampv(z0[l], P->clamp_z);
    double acc = 0.0;
    for (int32_t m = 0; m < M_root; ++m)
        acc += Sp[m] + orc_driver(P, 0.0, x0, y1[m], zc) * dt - cvi[m];
    *y0 = acc / M_root;
    for (int l = 0; l < q; ++l) z0[l] = zc[l];
    free(Sp);
    return 0;
}
