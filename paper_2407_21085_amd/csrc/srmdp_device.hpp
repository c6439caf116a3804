// Device building blocks of the SRMDP sweep for gfx950: counter-based random
// inputs, the stratified start sampler, cell location and the problem data.
// Everything here is inlined into the kernels of srmdp_kernels.hip.
#pragma once

#if !defined(__HIPCC_RTC__)  // under hipRTC the runtime is built in; the run-time source declares the integer types
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

namespace srmdp {

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of the two-multiplier S-box on a 128-bit counter, key
// bumped by the Weyl constants between rounds.  Stateless: a simulation's
// stream is addressed by its counter (block, m, k, i | instance << 16).
struct Key {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, Key key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        // three-input XOR in one gfx950 instruction (truth table 0x96)
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
    }
    return c;
}

// Open uniform on (0,1): (2 (w >> 9) + 1) 2^-24, an odd multiple of 2^-24 built
// from the top 23 bits.  Exact in binary32, so both precisions see the same
// real number.  binary32: the bits (w >> 9) | 0x3F800000 are 1 + (w >> 9) 2^-23,
// and subtracting 1 - 2^-24 is exact.
template <typename R>
__device__ __forceinline__ R open_uniform(uint32_t w);

template <>
__device__ __forceinline__ float open_uniform<float>(uint32_t w)
{
    return __uint_as_float((w >> 9) | 0x3F800000u) - 0.99999994039535522461f;  // 1 - 2^-24
}

template <>
__device__ __forceinline__ double open_uniform<double>(uint32_t w)
{
    return (double)(((w >> 9) << 1) | 1u) * 5.9604644775390625e-8;  // 2^-24
}

// Box-Muller (1958): scale * (rho cos(2 pi u2), rho sin(2 pi u2)),
// rho = sqrt(-2 ln u1).  binary32 uses the hardware transcendentals: v_log_f32
// (log2; -2 ln u1 = -2 ln(2) log2 u1, with scale^2 folded into the constant),
// v_sqrt_f32 and v_sin_f32 / v_cos_f32, which take their argument in
// revolutions, so sin(2 pi u2) is v_sin_f32(u2).  binary64 uses the libm
// functions.
__device__ __forceinline__ void box_muller(float u1, float u2, float neg2ln2_s2, float &n0,
                                           float &n1)
{
    const float rho = __builtin_amdgcn_sqrtf(neg2ln2_s2 * __builtin_amdgcn_logf(u1));
    n0 = rho * __builtin_amdgcn_cosf(u2);
    n1 = rho * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ void box_muller(double u1, double u2, double scale, double &n0,
                                           double &n1)
{
    const double rho = scale * sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    n0 = rho * c;
    n1 = rho * s;
}

// Constant handed to box_muller for increments of standard deviation `scale`.
__device__ __forceinline__ float box_muller_constant(float scale)
{
    return -2.0f * 0.69314718055994530942f * scale * scale;
}
__device__ __forceinline__ double box_muller_constant(double scale) { return scale; }

// The Gaussian increments of one simulation.  The D normals of step offset
// s = j - i are the numbers n = s Q + l of the simulation's normal sequence,
// Q = D when D divides 4 (4/D consecutive steps share a Philox block) and
// Q = 4 ceil(D/4) otherwise (each step starts on a block of its own and skips
// the last block's unused numbers), so a step needs no branch on where its
// numbers begin.  Number n is the cosine (n even) or sine (n odd) branch of the
// Box-Muller pair n/2, which takes uniforms 2*(n/2) and 2*(n/2)+1 of the blocks
// that follow the ceil(D/4) start blocks.  One Philox block feeds four normals.
template <typename R, int D>
struct NormalStream {
    uint4 ctr;  // x = block, y = m, z = k, w = tag
    Key key;
    R bm;       // box_muller_constant(scale)
    R buf[4];

    // Normals of standard deviation `scale` (sqrt(dt) gives the increments dW).
    __device__ __forceinline__ void init(Key k, uint32_t m, uint32_t cube, uint32_t tag, R scale)
    {
        key = k;
        ctr = make_uint4(0u, m, cube, tag);
        bm = box_muller_constant(scale);
    }

    __device__ __forceinline__ void fill(uint32_t blk)
    {
        ctr.x = blk;
        const uint4 w = philox4x32_10(ctr, key);
        box_muller(open_uniform<R>(w.x), open_uniform<R>(w.y), bm, buf[0], buf[1]);
        box_muller(open_uniform<R>(w.z), open_uniform<R>(w.w), bm, buf[2], buf[3]);
    }

    // D normals of step offset s = j - i (s is uniform over the wave).
    __device__ __forceinline__ void step(uint32_t s, R *out)
    {
        constexpr uint32_t B0 = (D + 3) / 4;
        if constexpr (4 % D == 0) {
            constexpr uint32_t per = 4 / D;  // steps served by one block
            const uint32_t off = (s % per) * D;
            if (off == 0) fill(B0 + s / per);
#pragma unroll
            for (int l = 0; l < D; ++l) {
                const uint32_t w = off + l;
                out[l] = w == 0 ? buf[0] : w == 1 ? buf[1] : w == 2 ? buf[2] : buf[3];
            }
        } else {
            constexpr uint32_t NBK = (D + 3) / 4;  // blocks per step
#pragma unroll
            for (int b = 0; b < (int)NBK; ++b) {
                fill(B0 + s * NBK + b);
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    if (4 * b + w < D) out[4 * b + w] = buf[w];
            }
        }
    }
};

// Uniform number `idx` of a simulation's stream (start point words).
__device__ __forceinline__ uint32_t stream_word(Key key, uint32_t m, uint32_t cube, uint32_t tag,
                                                uint32_t idx)
{
    const uint4 w = philox4x32_10(make_uint4(idx / 4, m, cube, tag), key);
    const uint32_t r = idx % 4;
    return r == 0 ? w.x : r == 1 ? w.y : r == 2 ? w.z : w.w;
}

// ------------------------------------------------------------ problem data

// Per-dimension constants of one cell [x-, x+) for the restricted logistic
// sampler, F(x) = 1/(1+exp(-mu x)), c the cell centre, delta = F(x+) - F(x-):
//   uc = (F(c) - F(x-)) / delta (the uniform that maps to c),
//   rp = delta / F(c), rs = delta / (1 - F(c)).
template <typename R>
struct alignas(4 * sizeof(R)) CellF {
    R uc, rp, rs, centre;
};

// Algorithm "stratify": x = F^{-1}(p), p = F(x-) + u (F(x+) - F(x-)).  With
// v = u - uc, p - F(c) = delta v, so
//   mu (x - c) = log(p / F(c)) - log((1 - p) / (1 - F(c)))
//              = log1p(rp v) - log1p(-rs v),
// which gives the offset from the centre (hence the centred, scaled basis
// coordinate) to full working precision.
template <typename R>
__device__ __forceinline__ R stratified_offset(const CellF<R> &c, R u, R inv_mu)
{
    const R v = u - c.uc;
    return (log1p(c.rp * v) - log1p(-c.rs * v)) * inv_mu;
}

// log1p(a), a > -1, in binary32 from the hardware log2 (v_log_f32): w = 1 + a
// is rounded, and the factor a / (w - 1) puts back what the rounding dropped
// (Goldberg, "What every computer scientist should know about floating-point
// arithmetic", ACM Computing Surveys 1991, Theorem 4: a few units in the last
// place when the logarithm is); w = 1 means |a| < 2^-24, where log1p(a) = a.
// For a in [-1, -1/2], w is exact (Sterbenz), so the tail keeps the accuracy
// of a itself.
__device__ __forceinline__ float log1p_hw(float a)
{
    const float w = 1.0f + a;
    const float wm1 = w - 1.0f;
    const float l = __builtin_amdgcn_logf(w) * 0.69314718055994530942f;
    return wm1 == 0.0f ? a : l * (a * __builtin_amdgcn_rcpf(wm1));
}

template <>
__device__ __forceinline__ float stratified_offset<float>(const CellF<float> &c, float u,
                                                         float inv_mu)
{
    const float v = u - c.uc;
    return (log1p_hw(c.rp * v) - log1p_hw(-c.rs * v)) * inv_mu;
}

// Terminal condition g.
template <typename R>
__device__ __forceinline__ R terminal_g(int kind, R T, R sum_x)
{
    if (kind == 1) return (R)1 / ((R)1 + exp(-(T + sum_x)));  // omega/(1+omega)
    return cos(sum_x);
}

template <>
__device__ __forceinline__ float terminal_g<float>(int kind, float T, float sum_x)
{
    if (kind == 1) return 1.0f / (1.0f + expf(-(T + sum_x)));
    return cosf(sum_x);
}

// Driver f(t, x, y, z) of the built-in problems; both depend on z only through
// sum_l z_l.  kind 0: -r y + kappa sum z.  kind 1: sum z (y - (2+q)/(2q)).
template <typename R>
__device__ __forceinline__ R driver_f(int kind, R r, R kappa, R c_logistic, R y, R zsum)
{
    if (kind == 1) return zsum * (y - c_logistic);
    return kappa * zsum - r * y;
}

template <typename R>
__device__ __forceinline__ R clamp_level(R v, R L)
{
    return fmin(fmax(v, -L), L);
}

template <>
__device__ __forceinline__ float clamp_level<float>(float v, float L)
{
    return fminf(fmaxf(v, -L), L);
}

}  // namespace srmdp
