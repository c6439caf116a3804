// Ragged batches of SRMDP instances (same d, basis, precision, look-up mode
// and grid kind; any K, M, N, seeds and driver parameters): one launch per global
// backward step runs the stratum groups of every active instance, in a
// grid-stride loop over the flattened list of groups.  Each group is computed
// exactly as in the per-instance sweep (Algorithm SRMDP, Section 3.1,
// eq. (PsiM)), so a batched table equals the one srmdp_solve returns.
#include "srmdp_sweep.hpp"

namespace srmdp {

template <typename R, int D, int NB, int LK, bool EP>
__global__ void __launch_bounds__(256) sweep_batch_kernel(const BatchInstance<R> *__restrict__ inst, int n_active,
                                                         uint32_t total_items, int g)
{
    extern __shared__ __align__(16) unsigned char smem[];
    for (uint32_t item = blockIdx.x; item < total_items; item += gridDim.x) {
        int lo = 0, hi = n_active - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].first_item <= item) lo = mid;
            else hi = mid - 1;
        }
        const int b = __builtin_amdgcn_readfirstlane(lo);
        const BatchInstance<R> &I = inst[b];
        StepArgs<R> a = I.a;
        a.i = a.N - 1 - g;
        a.tag = ((uint32_t)a.i & 0xFFFFu) | (I.instance << 16);
        sweep_group<R, D, NB, LK, false, false, EP>(a, item - I.first_item, (const CellF<R> *)I.cellF, (const R *)I.bsig,
                                         (R *)I.lk, (R *)I.table, (unsigned long long *)I.counters, smem);
        __syncthreads();  // the next group reuses the LDS
    }
}

template <typename R, int D, int NB, int LK, bool EP>
static hipError_t launch_batch_impl(const void *inst, int n_active, uint32_t total, int g, unsigned threads,
                                    size_t lds, hipStream_t st)
{
    const unsigned blocks = total < 8192u ? (total > 0 ? total : 1u) : 8192u;
    hipLaunchKernelGGL((sweep_batch_kernel<R, D, NB, LK, EP>), dim3(blocks), dim3(threads), lds, st,
                       (const BatchInstance<R> *)inst, n_active, total, g);
    return hipGetLastError();
}

template <typename R, int D, bool EP>
static hipError_t dispatch_batch_d(int basis, int lkmode, const void *inst, int n, uint32_t total, int g,
                                   unsigned threads, size_t lds, hipStream_t st)
{
    if (basis == 0) {
        if (lkmode == kLookupY) return launch_batch_impl<R, D, 1, kLookupY, EP>(inst, n, total, g, threads, lds, st);
        if (lkmode == kLookupYZ) return launch_batch_impl<R, D, 1, kLookupYZ, EP>(inst, n, total, g, threads, lds, st);
        return launch_batch_impl<R, D, 1, kLookupFull, EP>(inst, n, total, g, threads, lds, st);
    }
    if (lkmode == kLookupY) return launch_batch_impl<R, D, D + 1, kLookupY, EP>(inst, n, total, g, threads, lds, st);
    if (lkmode == kLookupYZ) return launch_batch_impl<R, D, D + 1, kLookupYZ, EP>(inst, n, total, g, threads, lds, st);
    return launch_batch_impl<R, D, D + 1, kLookupFull, EP>(inst, n, total, g, threads, lds, st);
}

#define SRMDP_BATCH_FOR_EACH_D(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8)

template <typename R>
hipError_t launch_batch_step(int d, int basis, int lkmode, bool equal_prob, const void *inst, int n_active,
                             uint32_t total_items, int g, unsigned threads, size_t lds_bytes, hipStream_t st)
{
    switch (d) {
#define X(DD)                                                                                                      \
    case DD:                                                                                                       \
        return equal_prob ? dispatch_batch_d<R, DD, true>(basis, lkmode, inst, n_active, total_items, g, threads, \
                                                          lds_bytes, st)                                          \
                          : dispatch_batch_d<R, DD, false>(basis, lkmode, inst, n_active, total_items, g, threads, \
                                                           lds_bytes, st);
        SRMDP_BATCH_FOR_EACH_D(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_batch_step<float>(int, int, int, bool, const void *, int, uint32_t, int, unsigned, size_t,
                                             hipStream_t);
template hipError_t launch_batch_step<double>(int, int, int, bool, const void *, int, uint32_t, int, unsigned,
                                              size_t, hipStream_t);

// Host-to-device copy through kernel arguments, in chunks below the 4 KiB
// argument limit.
struct UploadChunk {
    unsigned char bytes[3072];
};

__global__ void upload_kernel(UploadChunk c, uint32_t n, unsigned char *__restrict__ dst)
{
    for (uint32_t v = threadIdx.x; v < n; v += blockDim.x) dst[v] = c.bytes[v];
}

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const unsigned char *s = (const unsigned char *)src;
    unsigned char *d = (unsigned char *)dst;
    for (size_t off = 0; off < bytes; off += sizeof(UploadChunk)) {
        UploadChunk c;
        const size_t n = bytes - off < sizeof c.bytes ? bytes - off : sizeof c.bytes;
        for (size_t v = 0; v < n; ++v) c.bytes[v] = s[off + v];
        hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, st, c, (uint32_t)n, d + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace srmdp
