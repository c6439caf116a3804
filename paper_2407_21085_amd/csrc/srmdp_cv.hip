// The learned control variate on gfx950: the network z_theta(t, x) of
// srmdp_mlp.hpp, its packing, batched forward and backward passes, the Adam
// training kernel, the training pairs a backward step produces, and the
// sweep-step kernels that subtract sum_j z_theta(t_j, X_j) . dW_j from the
// responses.
//
// The control variate keeps eq. (PsiM)'s regressions unbiased: for j > i the
// increment dW_j is independent of (X_i, ..., X_j) and of the network, which is
// frozen before step i and trained only on pairs of steps > i, so every
// subtracted term has conditional mean zero given X_i; z_theta(t_i, X_i) . dW_i
// is removed from the y response only (the z response S' dW_i / dt would see
// its conditional mean z_theta(t_i, X_i)).
#include "srmdp_sweep.hpp"

namespace srmdp {

constexpr int kMaxParams = kMlpH * kMlpMaxIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpMaxOut * kMlpH + kMlpMaxOut;
constexpr uint32_t kCvPairStratum = 0xFFFFFFFEu;  // counter stratum of the training-pair draws
constexpr uint32_t kInitStratum = 0xFFFFFFFDu;    // counter stratum of the initial weights
constexpr int kBackwardChunk = 1024;              // samples per workgroup of mlp_backward_kernel

// Fragments and biases of the parameters theta (binary32, parameter layout).
__device__ __forceinline__ void pack_weights(const MlpShape &s, const float *theta, __bf16 *frag,
                                             float *bias, int tid, int nthreads)
{
    for (int e = tid; e < kFrags * kFragElems; e += nthreads) {
        const int f = e / kFragElems, rem = e % kFragElems;
        const int src = pack_source(s, f, rem / 8, rem % 8);
        frag[e] = (__bf16)(src >= 0 ? theta[src] : 0.0f);
    }
    for (int i = tid; i < kBiasFloats; i += nthreads) {
        const int src = bias_source(s, i);
        bias[i] = src >= 0 ? theta[src] : 0.0f;
    }
}

// The bf16 slots (indices into the fragment array) that hold parameter p, the
// inverse of pack_source: one for W1, two for W2 (W2 and W2^T) and W3 (W3 and
// W3^T), none for the biases (bias slot in *bias_slot, else -1).
__device__ __forceinline__ int param_slots(const MlpShape &s, int p, int *slot, int *bias_slot)
{
    auto at = [](int f, int h, int r, int c) { return (f * 64 + 32 * h + r) * 8 + c; };
    *bias_slot = -1;
    if (p < s.oB1()) {
        const int j = p / s.in, k = p % s.in;
        slot[0] = at(kFragW1 + (j >> 5), k >> 3, j & 31, k & 7);
        return 1;
    }
    if (p < s.oW2()) {
        *bias_slot = kBiasB1 + p - s.oB1();
        return 0;
    }
    if (p < s.oB2()) {
        const int a = (p - s.oW2()) / kMlpH, u = (p - s.oW2()) % kMlpH;
        const int pu = mlp_perm(u), pa = mlp_perm(a);
        slot[0] = at(kFragW2 + 4 * (a >> 5) + (pu >> 4), (pu >> 3) & 1, a & 31, pu & 7);
        slot[1] = at(kFragW2T + 4 * (u >> 5) + (pa >> 4), (pa >> 3) & 1, u & 31, pa & 7);
        return 2;
    }
    if (p < s.oW3()) {
        *bias_slot = kBiasB2 + p - s.oB2();
        return 0;
    }
    if (p < s.oB3()) {
        const int o = (p - s.oW3()) / kMlpH, u = (p - s.oW3()) % kMlpH;
        const int pu = mlp_perm(u), po = mlp_perm(o);
        slot[0] = at(kFragW3 + (pu >> 4), (pu >> 3) & 1, o, pu & 7);
        slot[1] = at(kFragW3T + (u >> 5), po >> 3, u & 31, po & 7);
        return 2;
    }
    *bias_slot = kBiasB3 + p - s.oB3();
    return 0;
}

__global__ void mlp_pack_kernel(MlpShape s, const float *__restrict__ theta, unsigned char *__restrict__ packed)
{
    pack_weights(s, theta, reinterpret_cast<__bf16 *>(packed + kPackedBiasBytes),
                 reinterpret_cast<float *>(packed), blockIdx.x * blockDim.x + threadIdx.x,
                 gridDim.x * blockDim.x);
}

// Glorot-uniform weights from Philox4x32-10 (key = seed), zero biases; the
// output layer optionally zero, so that the first backward step runs with a
// vanishing control variate.
__global__ void mlp_init_kernel(MlpShape s, uint32_t k0, uint32_t k1, int zero_output_layer,
                                float *__restrict__ theta)
{
    const int P = s.count();
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        float fan = 0.0f;
        if (p < s.oB1()) fan = (float)(s.in + kMlpH);
        else if (p >= s.oW2() && p < s.oB2()) fan = (float)(2 * kMlpH);
        else if (p >= s.oW3() && p < s.oB3() && !zero_output_layer) fan = (float)(kMlpH + s.out);
        float v = 0.0f;
        if (fan > 0.0f) {
            const uint4 w = philox4x32_10(make_uint4((uint32_t)p / 4u, 0u, kInitStratum, 0u), Key{k0, k1});
            const uint32_t r = p % 4 == 0 ? w.x : p % 4 == 1 ? w.y : p % 4 == 2 ? w.z : w.w;
            v = (2.0f * open_uniform<float>(r) - 1.0f) * sqrtf(6.0f / fan);
        }
        theta[p] = v;
    }
}

__global__ void zero_f32_kernel(float *p, int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0.0f;
}

// Copies `bytes` (multiple of 16) of packed weights to LDS.
__device__ __forceinline__ void stage_weights(const unsigned char *packed, unsigned char *lds, size_t bytes)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(packed);
    uint4 *dst = reinterpret_cast<uint4 *>(lds);
    for (int v = threadIdx.x; v < (int)(bytes / 16); v += blockDim.x) dst[v] = src[v];
}

__device__ __forceinline__ void load_input(const float *x, int in, int64_t s, int64_t B, float *in16)
{
#pragma unroll
    for (int c = 0; c < 16; ++c) in16[c] = (c < in && s < B) ? x[s * in + c] : 0.0f;
}

// y [B][out] = z_theta(x [B][in]); one wavefront per 64 samples.
__global__ void __launch_bounds__(256) mlp_forward_kernel(MlpShape s, const unsigned char *__restrict__ packed,
                                                         const float *__restrict__ x, int64_t B,
                                                         float *__restrict__ y)
{
    __shared__ __align__(16) unsigned char wl[kPackedFwdBytes];
    stage_weights(packed, wl, kPackedFwdBytes);
    __syncthreads();
    const MlpWeights w{reinterpret_cast<const bf16x8 *>(wl + kPackedBiasBytes), reinterpret_cast<const float *>(wl)};
    const int lane = threadIdx.x & 63, h = lane >> 5, wave = threadIdx.x >> 6;
    for (int64_t g = (int64_t)blockIdx.x * 4 + wave; g * 64 < B; g += (int64_t)gridDim.x * 4) {
        float in16[16];
        load_input(x, s.in, g * 64 + lane, B, in16);
        TileInput op[2];
        input_operands(in16, op[0], op[1]);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const f32x16 out = mlp_tile_forward<false>(w, lane, op[nt], nullptr);
            const int64_t sm = g * 64 + 32 * nt + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = c_row(r, h);
                if (o < s.out && sm < B) y[sm * s.out + o] = out[r];
            }
        }
    }
}

// The transpose buffers of the four wavefronts share their LDS with the four
// per-wavefront gradients, which are written only after the last tile.
union GradScratch {
    __bf16 xp[4][2][kXpRows * kXpStride];
    float part[4][kMaxParams];
};

struct GradLds {
    bf16x8 frag[kFrags * 64];
    float bias[kBiasFloats];
    GradScratch u;
};

// Partial gradients of sum_s <dy_s, y_s> over chunks of kBackwardChunk samples:
// partial [block][P].
__global__ void __launch_bounds__(256) mlp_backward_kernel(MlpShape s, const unsigned char *__restrict__ packed,
                                                          const float *__restrict__ x,
                                                          const float *__restrict__ dy, int64_t B,
                                                          float *__restrict__ partial)
{
    __shared__ __align__(16) GradLds L;
    stage_weights(packed, reinterpret_cast<unsigned char *>(L.bias), kPackedBiasBytes);
    stage_weights(packed + kPackedBiasBytes, reinterpret_cast<unsigned char *>(L.frag), kPackedBytes - kPackedBiasBytes);
    __syncthreads();
    const MlpWeights w{L.frag, L.bias};
    const int lane = threadIdx.x & 63, h = lane >> 5, wave = threadIdx.x >> 6;
    MlpGrad acc;
    acc.clear();
    const int64_t start = (int64_t)blockIdx.x * kBackwardChunk;
    for (int g = wave; g < kBackwardChunk / 64; g += 4) {
        const int64_t base = start + 64 * g;
        if (base >= B) break;  // wave-uniform
        float in16[16];
        load_input(x, s.in, base + lane, B, in16);
        TileInput op[2];
        input_operands(in16, op[0], op[1]);
#pragma unroll 1
        for (int nt = 0; nt < 2; ++nt) {
            MlpTile keep;
            mlp_tile_forward<true>(w, lane, op[nt], &keep);
            const int64_t sm = base + 32 * nt + (lane & 31);
            float gr[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int o = c_row(r, h);
                gr[r] = (o < s.out && sm < B) ? dy[sm * s.out + o] : 0.0f;
            }
            mlp_tile_backward(w, lane, keep, op[nt], gr, L.u.xp[wave][0], L.u.xp[wave][1], acc);
        }
    }
    __syncthreads();  // every wavefront is done with the transpose buffers
    mlp_grad_flush(s, lane, acc, L.u.part[wave], false);
    __syncthreads();
    const int P = s.count();
    for (int p = threadIdx.x; p < P; p += blockDim.x)
        partial[(size_t)blockIdx.x * P + p] = ((L.u.part[0][p] + L.u.part[1][p]) + L.u.part[2][p]) + L.u.part[3][p];
}

// grad = sum over blocks of partial, in block order.
__global__ void grad_reduce_kernel(const float *__restrict__ partial, int nblocks, int P, float *__restrict__ grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float acc = 0.0f;
    for (int b = 0; b < nblocks; ++b) acc += partial[(size_t)b * P + p];
    grad[p] = acc;
}

struct TrainLds {
    bf16x8 frag[kFrags * 64];
    float bias[kBiasFloats];
    GradScratch u;
    float loss[4];
};

// Gradient of Adam update u, spread over batch / 256 workgroups.  Workgroup b
// takes the 256 pairs from (u batch + 256 b) mod S of x16 / z16, 64 per
// wavefront: forward and backward passes on the matrix cores with the packed
// network of packed_out, the loss gradient 2 (z_theta - z) / batch, the
// wavefronts' gradients summed in wavefront order.  partial [b][pstride]
// receives the gradient (P values) and the sum of squared errors (entry P).
__global__ void __launch_bounds__(256) mlp_train_grad_kernel(MlpTrainArgs A, int u, float *__restrict__ partial,
                                                            int pstride)
{
    __shared__ __align__(16) TrainLds L;
    stage_weights(A.packed_out, reinterpret_cast<unsigned char *>(L.bias), kPackedBiasBytes);
    stage_weights(A.packed_out + kPackedBiasBytes, reinterpret_cast<unsigned char *>(L.frag),
                  kPackedBytes - kPackedBiasBytes);
    __syncthreads();
    const MlpShape s{A.in, A.out};
    const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5, wave = tid >> 6;
    const MlpWeights w{L.frag, L.bias};
    const float gscale = 2.0f / (float)A.batch;
    MlpGrad acc;
    acc.clear();
    float lsum = 0.0f;
    const int64_t base = ((int64_t)u * A.batch + (int64_t)(4 * blockIdx.x + wave) * 64) % A.S;
    const float4 *xs = reinterpret_cast<const float4 *>(A.x16 + (base + lane) * 16);
    float in16[16];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float4 q = xs[v];
        in16[4 * v] = q.x;
        in16[4 * v + 1] = q.y;
        in16[4 * v + 2] = q.z;
        in16[4 * v + 3] = q.w;
    }
    TileInput op[2];
    input_operands(in16, op[0], op[1]);
#pragma unroll 1
    for (int nt = 0; nt < 2; ++nt) {
        MlpTile keep;
        const f32x16 yv = mlp_tile_forward<true>(w, lane, op[nt], &keep);
        const int64_t sm = base + 32 * nt + (lane & 31);
        const float4 za = *reinterpret_cast<const float4 *>(A.z16 + sm * 16 + 4 * h);
        const float4 zb = *reinterpret_cast<const float4 *>(A.z16 + sm * 16 + 8 + 4 * h);
        const float zz[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
        float gr[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const float diff = c_row(r, h) < s.out ? yv[r] - zz[r] : 0.0f;
            lsum += diff * diff;
            gr[r] = gscale * diff;
        }
        mlp_tile_backward(w, lane, keep, op[nt], gr, L.u.xp[wave][0], L.u.xp[wave][1], acc);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m, 64);
    if (lane == 0) L.loss[wave] = lsum;
    __syncthreads();  // every wavefront is done with the transpose buffers
    mlp_grad_flush(s, lane, acc, L.u.part[wave], false);
    __syncthreads();
    const int P = s.count();
    float *out = partial + (size_t)blockIdx.x * pstride;
    for (int p = tid; p < P; p += 256)
        out[p] = ((L.u.part[0][p] + L.u.part[1][p]) + L.u.part[2][p]) + L.u.part[3][p];
    if (tid == 0) out[P] = ((L.loss[0] + L.loss[1]) + L.loss[2]) + L.loss[3];
}

// Adam step of update u: the gradient of each parameter is the sum of the
// nblk workgroup partials in workgroup order; theta (binary32 master weights)
// and the moments are updated in place, and the parameter's bf16 slots (or
// its bias entry) are rewritten in the packed network.  Every other byte of
// packed_out keeps what the packing of theta put there.
__global__ void __launch_bounds__(256) mlp_adam_kernel(MlpTrainArgs A, int u, const float *__restrict__ partial,
                                                      int nblk, int pstride)
{
    const MlpShape s{A.in, A.out};
    const int P = s.count();
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < P) {
        // in workgroup order; the loads go out eight at a time
        float gp = 0.0f;
        int b = 0;
        for (; b + 8 <= nblk; b += 8) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = partial[(size_t)(b + e) * pstride + p];
#pragma unroll
            for (int e = 0; e < 8; ++e) gp += v[e];
        }
        for (; b < nblk; ++b) gp += partial[(size_t)b * pstride + p];
        const float t = (float)(A.adam_t0 + u + 1);
        const float bc1 = 1.0f - powf(A.beta1, t), bc2 = 1.0f - powf(A.beta2, t);
        const float m = A.beta1 * A.adam_m[p] + (1.0f - A.beta1) * gp;
        const float v = A.beta2 * A.adam_v[p] + (1.0f - A.beta2) * gp * gp;
        A.adam_m[p] = m;
        A.adam_v[p] = v;
        const float th = A.theta[p] - A.lr * (m / bc1) / (sqrtf(v / bc2) + A.eps);
        A.theta[p] = th;
        int slot[2], bslot;
        const int n = param_slots(s, p, slot, &bslot);
        __bf16 *frag16 = reinterpret_cast<__bf16 *>(A.packed_out + kPackedBiasBytes);
        for (int e = 0; e < n; ++e) frag16[slot[e]] = (__bf16)th;
        if (bslot >= 0) reinterpret_cast<float *>(A.packed_out)[bslot] = th;
    }
    if (p == 0 && A.loss) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += partial[(size_t)b * pstride + P];
        A.loss[u] = l / (float)A.batch;
    }
}

// The training pairs of step i: pair s draws a stratum k and a simulation m
// from Philox4x32-10 counter (0, s, kCvPairStratum, tag), rebuilds that
// simulation's start X_i^(m) of the sweep (the same draw), and takes the
// fitted, truncated z_i of stratum k there as the target.  x16 [S][16] holds
// (t_i, X_i, 0...), z16 [S][16] holds (z_i, 0...).
template <int D, int NB>
__global__ void cv_pairs_kernel(const StepArgs<float> a, const CellF<float> *__restrict__ cellF,
                                const float *__restrict__ table, int64_t S, float *__restrict__ x16,
                                float *__restrict__ z16)
{
    constexpr int REC = (1 + D) * NB;
    const Key key{a.key0, a.key1};
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const uint4 w = philox4x32_10(make_uint4(0u, (uint32_t)s, kCvPairStratum, a.tag), key);
        const uint32_t k = __umulhi(w.x, a.K), m = __umulhi(w.y, (uint32_t)a.M);
        float x[D], phi[NB];
        sample_start<float, D, NB>(a, cellF, k, m, x, phi);
        float *xo = x16 + s * 16, *zo = z16 + s * 16;
        xo[0] = (float)a.i * a.dt;
#pragma unroll
        for (int e = 1; e < 16; ++e) xo[e] = e <= D ? x[e - 1] : 0.0f;
        const float *rec = table + ((size_t)a.i * a.K + k) * REC;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            float v = 0.0f;
            if (e < D) {
#pragma unroll
                for (int b = 0; b < NB; ++b) v += rec[(1 + e) * NB + b] * phi[b];
                v = clamp_level<float>(v, a.clamp_z);
            }
            zo[e] = v;
        }
    }
}

// ------------------------------------------------------------- launchers

hipError_t launch_mlp_pack(int in, int out, const float *theta, void *packed, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((kFrags * kFragElems + 255) / 256), dim3(256), 0, st,
                       MlpShape{in, out}, theta, (unsigned char *)packed);
    return hipGetLastError();
}

hipError_t launch_mlp_init(int in, int out, uint64_t seed, int zero_output_layer, float *theta, hipStream_t st)
{
    const MlpShape s{in, out};
    hipLaunchKernelGGL(mlp_init_kernel, dim3((s.count() + 255) / 256), dim3(256), 0, st, s,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), zero_output_layer, theta);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)),
                       dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int in, int out, const void *packed, const float *x, int64_t B, float *y,
                              hipStream_t st)
{
    const int64_t groups = (B + 63) / 64;
    const int64_t blocks = (groups + 3) / 4;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192)),
                       dim3(256), 0, st, MlpShape{in, out}, (const unsigned char *)packed, x, B, y);
    return hipGetLastError();
}

size_t mlp_backward_partials(int64_t B) { return (size_t)((B + kBackwardChunk - 1) / kBackwardChunk); }

hipError_t launch_mlp_backward(int in, int out, const void *packed, const float *x, const float *dy,
                               int64_t B, float *partial, float *grad, hipStream_t st)
{
    const MlpShape s{in, out};
    const int nb = (int)mlp_backward_partials(B);
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(nb), dim3(256), 0, st, s, (const unsigned char *)packed, x,
                       dy, B, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((s.count() + 255) / 256), dim3(256), 0, st, partial, nb,
                       s.count(), grad);
    return hipGetLastError();
}

int mlp_train_partial_stride(int in, int out) { return (MlpShape{in, out}.count() + 1 + 63) & ~63; }

size_t mlp_train_partial_bytes(int in, int out, int batch)
{
    return (size_t)(batch / 256) * mlp_train_partial_stride(in, out) * sizeof(float);
}

hipError_t launch_mlp_train(const MlpTrainArgs &t, float *partial, hipStream_t st)
{
    const int nblk = t.batch / 256, pstride = mlp_train_partial_stride(t.in, t.out);
    const int P = MlpShape{t.in, t.out}.count();
    for (int u = 0; u < t.updates; ++u) {
        hipLaunchKernelGGL(mlp_train_grad_kernel, dim3(nblk), dim3(256), 0, st, t, u, partial, pstride);
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((P + 255) / 256), dim3(256), 0, st, t, u,
                           (const float *)partial, nblk, pstride);
    }
    return hipGetLastError();
}

// The control-variate step kernel asks for three wavefronts per SIMD: the
// network's tiles would otherwise take the register budget down to two.
template <int D, int NB, int LK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
sweep_step_cv_kernel(const StepArgs<float> a, const CellF<float> *__restrict__ cellF, const float *__restrict__ bsig,
                     float *__restrict__ lk, float *__restrict__ table, unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<float, D, NB, LK, true>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF, bsig, lk, table,
                                        counters, smem);
}

// The same on equal-probability cells (look-up modes Y and YZ).
template <int D, int NB, int LK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
sweep_step_cv_ep_kernel(const StepArgs<float> a, const CellF<float> *__restrict__ cellF,
                        const float *__restrict__ bsig, float *__restrict__ lk, float *__restrict__ table,
                        unsigned long long *__restrict__ counters)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_group<float, D, NB, LK, true, false, true>(a, xcd_block_order(blockIdx.x, gridDim.x), cellF, bsig, lk,
                                                     table, counters, smem);
}

template <int D, int NB, int LK>
static hipError_t launch_step_cv_impl(const StepArgs<float> &a, const LaunchShape &s, const void *cellF,
                                      const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    if (a.equal_prob) {
        if constexpr (LK == kLookupFull) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((sweep_step_cv_ep_kernel<D, NB, LK>), dim3(s.blocks), dim3(s.threads), s.lds_bytes,
                               st, a, (const CellF<float> *)cellF, (const float *)bsig, (float *)lk, (float *)table,
                               (unsigned long long *)counters);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((sweep_step_cv_kernel<D, NB, LK>), dim3(s.blocks), dim3(s.threads), s.lds_bytes, st, a,
                       (const CellF<float> *)cellF, (const float *)bsig, (float *)lk, (float *)table,
                       (unsigned long long *)counters);
    return hipGetLastError();
}

template <int D, int NB>
static hipError_t launch_cv_pairs_impl(const StepArgs<float> &a, const void *cellF, const void *table,
                                       int64_t S, float *x16, float *z16, hipStream_t st)
{
    const int64_t blocks = (S + 255) / 256;
    hipLaunchKernelGGL((cv_pairs_kernel<D, NB>), dim3((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)),
                       dim3(256), 0, st, a, (const CellF<float> *)cellF, (const float *)table, S, x16, z16);
    return hipGetLastError();
}

#define SRMDP_CV_FOR_EACH_D(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8)

template <int D>
static hipError_t dispatch_step_cv_d(const StepArgs<float> &a, const LaunchShape &s, int basis, int lkmode,
                                     const void *cf, const void *bs, void *lk, void *tab, void *ctr, hipStream_t st)
{
    if (basis == 0) {
        if (lkmode == kLookupY) return launch_step_cv_impl<D, 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
        if (lkmode == kLookupYZ) return launch_step_cv_impl<D, 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
        return launch_step_cv_impl<D, 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
    }
    if (lkmode == kLookupY) return launch_step_cv_impl<D, D + 1, kLookupY>(a, s, cf, bs, lk, tab, ctr, st);
    if (lkmode == kLookupYZ) return launch_step_cv_impl<D, D + 1, kLookupYZ>(a, s, cf, bs, lk, tab, ctr, st);
    return launch_step_cv_impl<D, D + 1, kLookupFull>(a, s, cf, bs, lk, tab, ctr, st);
}

hipError_t launch_step_cv(int d, const StepArgs<float> &a, const LaunchShape &s, int basis, int lkmode,
                          const void *cellF, const void *bsig, void *lk, void *table, void *counters,
                          hipStream_t st)
{
    switch (d) {
#define X(DD) \
    case DD: return dispatch_step_cv_d<DD>(a, s, basis, lkmode, cellF, bsig, lk, table, counters, st);
        SRMDP_CV_FOR_EACH_D(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cv_pairs(int d, int basis, const StepArgs<float> &a, const void *cellF, const void *table,
                           int64_t S, float *x16, float *z16, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                              \
    case DD:                                                                               \
        if (basis == 0) return launch_cv_pairs_impl<DD, 1>(a, cellF, table, S, x16, z16, st); \
        return launch_cv_pairs_impl<DD, DD + 1>(a, cellF, table, S, x16, z16, st);
        SRMDP_CV_FOR_EACH_D(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

bool cv_dimension_compiled(int d)
{
    switch (d) {
#define X(DD) case DD: return true;
        SRMDP_CV_FOR_EACH_D(X)
#undef X
    default: return false;
    }
}

}  // namespace srmdp
