// The control-variate network z_theta(t, x): in -> 64 -> 64 -> out with SiLU
// after both hidden layers, bfloat16 weights and layer inputs, binary32
// accumulation and biases, on v_mfma_f32_32x32x16_bf16.  One wavefront
// evaluates 64 samples, one per lane.
//
// The layers are computed transposed, Z^T = W H^T, so that the samples are the
// N dimension of the matrix instruction.  Lane layout of the instruction
// (M x N x K = 32 x 32 x 16), l = lane, h = l / 32:
//   A: lane l holds row l % 32, k = 8 h + c (c = 0..7)
//   B: lane l holds column l % 32, k = 8 h + c
//   C: lane l holds column l % 32; element r is row 8 (r / 4) + 4 h + r % 4.
// Elements 8 s .. 8 s + 7 of a C tile, taken as the next layer's B operand of
// K step 2 mt + s, put hidden unit 16 ks + 8 (c / 4) + 4 h + c % 4 at K position
// 16 ks + 8 h + c: the next layer's K order is the unit order with bits 2 and 3
// swapped inside each block of 16.  The packed weights carry that permutation,
// so activations never leave registers between layers.
//
// Each input enters as a pair of bf16 numbers, hi = bf16(x) and
// lo = bf16(x - hi), in two K steps of the first layer that share the weight
// fragment: about 16 significant bits, so that the network's view of a point
// does not jump by a bf16 ulp (2^-8 relative) when x moves by a rounding error.
//
// Parameters (binary32 master copy) are laid out as W1 [64 x in], b1 [64],
// W2 [64 x 64], b2 [64], W3 [out x 64], b3 [out], row-major.
#pragma once

#if !defined(__HIPCC_RTC__)  // under hipRTC the runtime is built in; the run-time source declares the integer types
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

namespace srmdp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

constexpr int kMlpH = 64;       // hidden width
constexpr int kMlpMaxIn = 16;   // input width bound (one K step)
constexpr int kMlpMaxOut = 16;  // output width bound (rows 0..15 of one tile)

// Fragments of the packed weights, 64 lanes x 8 bf16 each (1 KiB).
//   forward:  W1 [mt] 0..1, W2 [mt][ks] 2..9, W3 [ks] 10..13
//   backward: W3^T [mt] 14..15 (K = outputs), W2^T [mt][ks] 16..23
constexpr int kFragW1 = 0, kFragW2 = 2, kFragW3 = 10, kFragW3T = 14, kFragW2T = 16;
constexpr int kFrags = 24, kFwdFrags = 14;
constexpr int kFragElems = 64 * 8;
// Packed buffer: biases first (b1 [64] | b2 [64] | b3 [32], zero-padded), then
// the fragments, so that the forward part is one contiguous prefix.
constexpr int kBiasB1 = 0, kBiasB2 = 64, kBiasB3 = 128, kBiasFloats = 160;
constexpr size_t kPackedBiasBytes = kBiasFloats * sizeof(float);
constexpr size_t kPackedBytes = kPackedBiasBytes + (size_t)kFrags * kFragElems * 2;
constexpr size_t kPackedFwdBytes = kPackedBiasBytes + (size_t)kFwdFrags * kFragElems * 2;

struct MlpShape {
    int in, out;
    __host__ __device__ int oW1() const { return 0; }
    __host__ __device__ int oB1() const { return kMlpH * in; }
    __host__ __device__ int oW2() const { return oB1() + kMlpH; }
    __host__ __device__ int oB2() const { return oW2() + kMlpH * kMlpH; }
    __host__ __device__ int oW3() const { return oB2() + kMlpH; }
    __host__ __device__ int oB3() const { return oW3() + out * kMlpH; }
    __host__ __device__ int count() const { return oB3() + out; }
};

// Hidden unit fed at K position p of layers 2 and 3 (and output row fed at K
// position p of the back-propagation through layer 3).
__host__ __device__ __forceinline__ int mlp_perm(int p)
{
    return (p & ~0xC) | ((p & 4) << 1) | ((p & 8) >> 1);
}

// Row of element r of a C tile held by a lane of half h.
__host__ __device__ __forceinline__ int c_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Parameter index that element c of fragment f in lane `lane` holds, or -1 (zero).
__host__ __device__ inline int pack_source(const MlpShape &s, int f, int lane, int c)
{
    const int h = lane >> 5, r = lane & 31;
    if (f < kFragW2) {  // W1 [mt]: row j, K = input 8 h + c
        const int j = 32 * f + r, k = 8 * h + c;
        return k < s.in ? s.oW1() + j * s.in + k : -1;
    }
    if (f < kFragW3) {  // W2 [mt][ks]: row a, K = unit perm(16 ks + 8 h + c)
        const int g = f - kFragW2, mt = g >> 2, ks = g & 3;
        return s.oW2() + (32 * mt + r) * kMlpH + mlp_perm(16 * ks + 8 * h + c);
    }
    if (f < kFragW3T) {  // W3 [ks]: row o
        const int ks = f - kFragW3;
        return r < s.out ? s.oW3() + r * kMlpH + mlp_perm(16 * ks + 8 * h + c) : -1;
    }
    if (f < kFragW2T) {  // W3^T [mt]: row j, K = output perm(8 h + c)
        const int mt = f - kFragW3T, o = mlp_perm(8 * h + c);
        return o < s.out ? s.oW3() + o * kMlpH + 32 * mt + r : -1;
    }
    {  // W2^T [mt][ks]: row j, K = unit a = perm(16 ks + 8 h + c)
        const int g = f - kFragW2T, mt = g >> 2, ks = g & 3;
        return s.oW2() + mlp_perm(16 * ks + 8 * h + c) * kMlpH + 32 * mt + r;
    }
}

__host__ __device__ inline int bias_source(const MlpShape &s, int i)
{
    if (i < kBiasB2) return s.oB1() + i;
    if (i < kBiasB3) return s.oB2() + i - kBiasB2;
    return i - kBiasB3 < s.out ? s.oB3() + i - kBiasB3 : -1;
}

// ------------------------------------------------------------ arithmetic

__device__ __forceinline__ f32x16 mfma_bf16(const bf16x8 &a, const bf16x8 &b, const f32x16 &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero_tile()
{
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = 0.0f;
    return c;
}

// Logistic sigmoid 1 / (1 + e^{-a}) from the hardware exp2 and reciprocal.
__device__ __forceinline__ float sigmoid_hw(float a)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * a));
}
__device__ __forceinline__ float silu_hw(float a) { return a * sigmoid_hw(a); }
// d/da [a sigma(a)] = sigma(a) (1 + a (1 - sigma(a)))
__device__ __forceinline__ float silu_grad_hw(float a)
{
    const float s = sigmoid_hw(a);
    return s * (1.0f + a * (1.0f - s));
}

// Swaps lanes 32..63 of x with lanes 0..31 of y (v_permlane32_swap): after
// the call x holds (x_lo, y_lo) and y holds (x_hi, y_hi).
__device__ __forceinline__ void swap_halves(uint32_t &x, uint32_t &y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
}
__device__ __forceinline__ void swap_halves(float &x, float &y)
{
    uint32_t a = __float_as_uint(x), b = __float_as_uint(y);
    swap_halves(a, b);
    x = __uint_as_float(a);
    y = __uint_as_float(b);
}

// ------------------------------------------------------------ forward

// Weights as seen by one wavefront: fragments (LDS or global) and biases.
struct MlpWeights {
    const bf16x8 *frag;  // [kFrags][64]
    const float *bias;   // [kBiasFloats]
    __device__ __forceinline__ bf16x8 a(int f, int lane) const { return frag[f * 64 + lane]; }
    // C tile initialised with the biases of rows 32 mt + c_row(r, h)
    __device__ __forceinline__ f32x16 bias_tile(int off, int mt, int h) const
    {
        f32x16 c;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 v = *reinterpret_cast<const float4 *>(bias + off + 32 * mt + 8 * g + 4 * h);
            c[4 * g] = v.x;
            c[4 * g + 1] = v.y;
            c[4 * g + 2] = v.z;
            c[4 * g + 3] = v.w;
        }
        return c;
    }
};

// SiLU of elements 8 s .. 8 s + 7 of a C tile, as a bf16 B operand.
__device__ __forceinline__ bf16x8 silu_operand(const f32x16 &c, int s)
{
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = (__bf16)silu_hw(c[8 * s + e]);
    return b;
}

// What a tile's forward pass keeps for back-propagation.
struct MlpTile {
    f32x16 c1[2], c2[2];  // pre-activations (rows = hidden units)
    bf16x8 h1[4], h2[4];  // SiLU outputs, bf16, as B operands of layers 2 and 3
};

// Layer-1 B operands of one N tile: the hi and lo parts of the inputs.
struct TileInput {
    bf16x8 hi, lo;
};

// Forward pass of one N tile (32 samples) from its layer-1 B operands; returns
// the output tile (rows = outputs, zero beyond `out`).
template <bool KEEP>
__device__ __forceinline__ f32x16 mlp_tile_forward(const MlpWeights &w, int lane, const TileInput &b1,
                                                   MlpTile *keep)
{
    const int h = lane >> 5;
    f32x16 c1[2], c2[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const bf16x8 a = w.a(kFragW1 + mt, lane);
        c1[mt] = mfma_bf16(a, b1.lo, mfma_bf16(a, b1.hi, w.bias_tile(kBiasB1, mt, h)));
    }
    bf16x8 h1[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) h1[ks] = silu_operand(c1[ks >> 1], ks & 1);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        c2[mt] = w.bias_tile(kBiasB2, mt, h);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) c2[mt] = mfma_bf16(w.a(kFragW2 + 4 * mt + ks, lane), h1[ks], c2[mt]);
    }
    bf16x8 h2[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) h2[ks] = silu_operand(c2[ks >> 1], ks & 1);
    f32x16 c3 = w.bias_tile(kBiasB3, 0, h);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) c3 = mfma_bf16(w.a(kFragW3 + ks, lane), h2[ks], c3);
    if constexpr (KEEP) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            keep->c1[mt] = c1[mt];
            keep->c2[mt] = c2[mt];
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            keep->h1[ks] = h1[ks];
            keep->h2[ks] = h2[ks];
        }
    }
    return c3;
}

// Inputs 0..7 (first) and 8..15 (second) of a lane's own sample, as the two
// layer-1 B operands of the tiles: tile 0 holds the samples of lanes 0..31,
// tile 1 those of lanes 32..63, and lane l supplies inputs 8 h .. 8 h + 7 of
// sample 32 nt + l % 32, so half of each operand comes from the other half-wave.
__device__ __forceinline__ void split_tiles(const bf16x8 &first, const bf16x8 &second, bf16x8 &t0, bf16x8 &t1)
{
    u32x4 a = __builtin_bit_cast(u32x4, first), b = __builtin_bit_cast(u32x4, second);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t x = a[e], y = b[e];
        swap_halves(x, y);  // x = (own first | partner's second), y = (partner's first | own second)
        a[e] = x;
        b[e] = y;
    }
    t0 = __builtin_bit_cast(bf16x8, a);
    t1 = __builtin_bit_cast(bf16x8, b);
}

// Layer-1 operands of both tiles from a lane's input vector (16 floats,
// zero-padded): hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in binary32).
__device__ __forceinline__ void input_operands(const float *in16, TileInput &t0, TileInput &t1)
{
    bf16x8 hf, hs, lf, ls;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        hf[e] = (__bf16)in16[e];
        hs[e] = (__bf16)in16[8 + e];
        lf[e] = (__bf16)(in16[e] - (float)hf[e]);
        ls[e] = (__bf16)(in16[8 + e] - (float)hs[e]);
    }
    split_tiles(hf, hs, t0.hi, t1.hi);
    split_tiles(lf, ls, t0.lo, t1.lo);
}

// z_theta(t, x) of this lane's sample (Q <= 16 values); every lane of the
// wavefront must call it (D inputs after t).
template <int D, int Q>
__device__ __forceinline__ void mlp_eval_z(const MlpWeights &w, int lane, float t, const float *x, float *z)
{
    static_assert(D + 1 <= kMlpMaxIn && Q <= kMlpMaxOut, "network shape");
    float in16[16];
    in16[0] = t;
#pragma unroll
    for (int e = 1; e < 16; ++e) in16[e] = e <= D ? x[e - 1] : 0.0f;
    TileInput b0, b1;
    input_operands(in16, b0, b1);
    // The two tiles one after the other, so that only one tile's activations
    // occupy registers.
    constexpr int R = Q <= 8 ? 4 : 8;  // output elements r < R hold outputs < Q
    float y0[R], y1[R];
    {
        const f32x16 c = mlp_tile_forward<false>(w, lane, b0, nullptr);
#pragma unroll
        for (int r = 0; r < R; ++r) y0[r] = c[r];
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        const f32x16 c = mlp_tile_forward<false>(w, lane, b1, nullptr);
#pragma unroll
        for (int r = 0; r < R; ++r) y1[r] = c[r];
    }
    // Element r of tile nt is output c_row(r, h) of sample 32 nt + l % 32; after
    // swapping halves, y0[r] is output c_row(r, 0) and y1[r] output c_row(r, 1)
    // of this lane's own sample.
#pragma unroll
    for (int r = 0; r < R; ++r) {
        swap_halves(y0[r], y1[r]);
        if (c_row(r, 0) < Q) z[c_row(r, 0)] = y0[r];
        if (c_row(r, 1) < Q) z[c_row(r, 1)] = y1[r];
    }
}

// ------------------------------------------------------------ backward

// Per-wavefront gradient accumulators.  The bias gradients sum the bf16
// deltas that the weight-gradient products read: lane (h, c) adds the eight
// samples 8 h .. 8 h + 7 of row c (of each 16-sample K step) of its A operand,
// and the two half-waves are added when flushed.
struct MlpGrad {
    f32x16 w3[2];     // dW3 [rows o][cols j = 32 nt + l % 32]
    f32x16 w2[2][2];  // dW2 [rows a, tile mt][cols j, tile nt]
    f32x16 w1[2];     // dW1 [rows j, tile mt][cols: inputs, hi parts 0..15, lo parts 16..31]
    float b1[2], b2[2], b3;  // rows 32 mt + l % 32 (b3: row l % 32)
    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            w3[t] = zero_tile();
            w1[t] = zero_tile();
            w2[t][0] = zero_tile();
            w2[t][1] = zero_tile();
            b1[t] = 0.0f;
            b2[t] = 0.0f;
        }
        b3 = 0.0f;
    }
};

__device__ __forceinline__ float sum8(const bf16x8 &v)
{
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) s += (float)v[e];
    return s;
}

// Row stride (bf16) of the per-wavefront transpose buffers: 32 samples + 8 pad.
constexpr int kXpStride = 40;
constexpr int kXpRows = 64;
constexpr size_t kXpBytesPerWave = 2 * (size_t)kXpRows * kXpStride * 2;

__device__ __forceinline__ void lds_order() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ bf16x8 xp_read(const __bf16 *buf, int row, int col0)
{
    return *reinterpret_cast<const bf16x8 *>(buf + row * kXpStride + col0);
}

// Back-propagation of one tile: g[r] (r < 8) is the upstream gradient of output
// c_row(r, h) of this lane's column sample, b1 the tile's layer-1 B operands,
// t the tile's forward state.  Weight gradients contract over the tile's 32
// samples, which needs the activations with samples along K: they go through
// two per-wavefront LDS buffers A and B ([64 rows][kXpStride] bf16 each).
__device__ __forceinline__ void mlp_tile_backward(const MlpWeights &w, int lane, const MlpTile &t,
                                                  const TileInput &b1, const float *g, __bf16 *bufA,
                                                  __bf16 *bufB, MlpGrad &acc)
{
    const int h = lane >> 5, col = lane & 31;
    // layer 3: dW3 += G H2^T, db3 += G
    bf16x8 gop;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        gop[r] = (__bf16)g[r];
        bufB[c_row(r, h) * kXpStride + col] = gop[r];
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int c = 0; c < 8; ++c) bufA[(32 * (ks >> 1) + c_row(8 * (ks & 1) + c, h)) * kXpStride + col] = t.h2[ks][c];
    lds_order();
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const bf16x8 a = xp_read(bufB, col, 16 * kk + 8 * h);
        acc.b3 += sum8(a);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc.w3[nt] = mfma_bf16(a, xp_read(bufA, 32 * nt + col, 16 * kk + 8 * h), acc.w3[nt]);
    }
    // D2 = (W3^T G) * SiLU'(c2)
    f32x16 d2[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        d2[mt] = mfma_bf16(w.a(kFragW3T + mt, lane), gop, zero_tile());
#pragma unroll
        for (int r = 0; r < 16; ++r) d2[mt][r] *= silu_grad_hw(t.c2[mt][r]);
    }
    bf16x8 d2op[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int c = 0; c < 8; ++c) d2op[ks][c] = (__bf16)d2[ks >> 1][8 * (ks & 1) + c];
    lds_order();
    // layer 2: dW2 += D2 H1^T
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int u = (32 * (ks >> 1) + c_row(8 * (ks & 1) + c, h)) * kXpStride + col;
            bufA[u] = d2op[ks][c];
            bufB[u] = t.h1[ks][c];
        }
    lds_order();
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        bf16x8 bo[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) bo[nt] = xp_read(bufB, 32 * nt + col, 16 * kk + 8 * h);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const bf16x8 a = xp_read(bufA, 32 * mt + col, 16 * kk + 8 * h);
            acc.b2[mt] += sum8(a);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc.w2[mt][nt] = mfma_bf16(a, bo[nt], acc.w2[mt][nt]);
        }
    }
    // D1 = (W2^T D2) * SiLU'(c1)
    f32x16 d1[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        d1[mt] = zero_tile();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) d1[mt] = mfma_bf16(w.a(kFragW2T + 4 * mt + ks, lane), d2op[ks], d1[mt]);
#pragma unroll
        for (int r = 0; r < 16; ++r) d1[mt][r] *= silu_grad_hw(t.c1[mt][r]);
    }
    lds_order();
    // layer 1: dW1 += D1 X, with the hi parts of the inputs in columns 0..15
    // and the lo parts in columns 16..31 (summed when flushed)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) bufA[(32 * mt + c_row(r, h)) * kXpStride + col] = (__bf16)d1[mt][r];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        bufB[(8 * h + c) * kXpStride + col] = b1.hi[c];
        bufB[(16 + 8 * h + c) * kXpStride + col] = b1.lo[c];
    }
    lds_order();
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const bf16x8 bo = xp_read(bufB, col, 16 * kk + 8 * h);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const bf16x8 a = xp_read(bufA, 32 * mt + col, 16 * kk + 8 * h);
            acc.b1[mt] += sum8(a);
            acc.w1[mt] = mfma_bf16(a, bo, acc.w1[mt]);
        }
    }
    lds_order();
}

// Adds (or stores, add = false) a wavefront's accumulators into a gradient in
// the parameter layout.  Waves of a workgroup must take turns.
__device__ __forceinline__ void mlp_grad_flush(const MlpShape &s, int lane, MlpGrad &acc, float *grad,
                                               bool add)
{
    const int h = lane >> 5, col = lane & 31;
    auto put = [&](int idx, float v) {
        if (add) grad[idx] += v;
        else grad[idx] = v;
    };
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int o = c_row(r, h);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            if (o < s.out) put(s.oW3() + o * kMlpH + 32 * nt + col, acc.w3[nt][r]);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) put(s.oW2() + (32 * mt + o) * kMlpH + 32 * nt + col, acc.w2[mt][nt][r]);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const float v = acc.w1[mt][r] + __shfl_xor(acc.w1[mt][r], 16, 64);  // hi + lo columns
            if (col < s.in) put(s.oW1() + (32 * mt + o) * s.in + col, v);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const float v1 = acc.b1[mt] + __shfl_xor(acc.b1[mt], 32, 64);
        const float v2 = acc.b2[mt] + __shfl_xor(acc.b2[mt], 32, 64);
        if (h == 0) {
            put(s.oB1() + 32 * mt + col, v1);
            put(s.oB2() + 32 * mt + col, v2);
        }
    }
    const float v3 = acc.b3 + __shfl_xor(acc.b3, 32, 64);
    if (h == 0 && col < s.out) put(s.oB3() + col, v3);
}

}  // namespace srmdp
