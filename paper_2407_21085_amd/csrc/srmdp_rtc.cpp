// Problems with their own coefficients (srmdp_model): the sweep-step kernel
// and its near-face diagnostic specialised with the caller's drift, diffusion,
// driver and terminal condition, compiled at run time with hipRTC for the
// current device and kept for the process.
//
// The device code is the library's own (srmdp_sweep.hpp and the headers it
// includes, embedded at build time); the model enters as the policy `Model`
// of sweep_group / face_flags_kernel, whose look-ups read whole records.  One
// program per model, dimension, basis, precision, grid kind and cloud storage
// (in LDS, or streamed through it for large M).
// hipRTC is opened with dlopen on the first model, so problems without one
// never load it.
#include "../../include/srmdp.h"

#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "srmdp_internal.hpp"
#include "srmdp_rtc_sources.inc"  // kRtcHeaderCount, kRtcHeaderNames, kRtcHeaderBodies (generated)

namespace srmdp {
namespace {

struct RtcApi {
    decltype(&hiprtcCreateProgram) create = nullptr;
    decltype(&hiprtcAddNameExpression) add_name = nullptr;
    decltype(&hiprtcCompileProgram) compile = nullptr;
    decltype(&hiprtcGetLoweredName) lowered = nullptr;
    decltype(&hiprtcGetProgramLogSize) log_size = nullptr;
    decltype(&hiprtcGetProgramLog) log = nullptr;
    decltype(&hiprtcGetCodeSize) code_size = nullptr;
    decltype(&hiprtcGetCode) code = nullptr;
    decltype(&hiprtcDestroyProgram) destroy = nullptr;
    std::string error;
};

const RtcApi &rtc_api()
{
    static const RtcApi api = [] {
        RtcApi r;
        void *h = nullptr;
        for (const char *name : {"libhiprtc.so.7", "libhiprtc.so"}) {
            h = dlopen(name, RTLD_NOW | RTLD_LOCAL);
            if (h) break;
        }
        if (!h) {
            const char *e = dlerror();
            r.error = std::string("cannot load hipRTC: ") + (e ? e : "libhiprtc.so not found");
            return r;
        }
        bool ok = true;
        auto sym = [&](auto &fn, const char *name) {
            fn = reinterpret_cast<std::remove_reference_t<decltype(fn)>>(dlsym(h, name));
            if (!fn) ok = false;
        };
        sym(r.create, "hiprtcCreateProgram");
        sym(r.add_name, "hiprtcAddNameExpression");
        sym(r.compile, "hiprtcCompileProgram");
        sym(r.lowered, "hiprtcGetLoweredName");
        sym(r.log_size, "hiprtcGetProgramLogSize");
        sym(r.log, "hiprtcGetProgramLog");
        sym(r.code_size, "hiprtcGetCodeSize");
        sym(r.code, "hiprtcGetCode");
        sym(r.destroy, "hiprtcDestroyProgram");
        if (!ok) r.error = "hipRTC library lacks an entry point";
        return r;
    }();
    return api;
}

// The run-time translation unit: the integer types (hipRTC keeps them in a
// namespace of its own), the sweep device code, the caller's source, the
// policy that calls it, and the step kernel.
std::string kernel_source(const srmdp_model *m, int d, int nb, bool is_float, bool ep, bool gr)
{
    std::string s;
    s += "using __hip_internal::uint8_t; using __hip_internal::uint16_t; using __hip_internal::uint32_t;\n"
         "using __hip_internal::uint64_t; using __hip_internal::int8_t; using __hip_internal::int16_t;\n"
         "using __hip_internal::int32_t; using __hip_internal::int64_t;\n"
         "#include \"srmdp_sweep.hpp\"\n";
    s += std::string("typedef ") + (is_float ? "float" : "double") + " srmdp_real;\n";
    s += "#define SRMDP_D " + std::to_string(d) + "\n#define SRMDP_Q " + std::to_string(d) + "\n";
    s += "#line 1 \"model\"\n";
    s += m->source;
    s += "\n#line 1 \"srmdp_model_glue\"\n"
         "namespace srmdp_model_glue {\n"
         "struct Model {\n"
         "    static constexpr bool kUser = true;\n"
         "    template <typename R, int D>\n"
         "    static __device__ __forceinline__ void step(const srmdp::StepArgs<R> &a, const R *p, R t, const R *x,\n"
         "                                                const R *dW, R *xn)\n"
         "    {\n"
         "        R b[D], s[D];\n"
         "        srmdp_b(t, x, p, b);\n"
         "        srmdp_sigma_dw(t, x, dW, p, s);\n"
         "#pragma unroll\n"
         "        for (int l = 0; l < D; ++l) xn[l] = x[l] + b[l] * a.dt + s[l];\n"
         "    }\n"
         "    template <typename R, int D>\n"
         "    static __device__ __forceinline__ R driver(const srmdp::StepArgs<R> &, const R *p, R t, const R *x, R y,\n"
         "                                               const R *z)\n"
         "    {\n"
         "        return srmdp_f(t, x, y, z, p);\n"
         "    }\n"
         "    template <typename R, int D>\n"
         "    static __device__ __forceinline__ R terminal(const srmdp::StepArgs<R> &, const R *p, const R *x)\n"
         "    {\n"
         "        return srmdp_g(x, p);\n"
         "    }\n"
         "};\n"
         "}  // namespace srmdp_model_glue\n";
    const std::string D = std::to_string(d), NB = std::to_string(nb);
    s += "extern \"C\" __global__ void __launch_bounds__(256)\n"
         "srmdp_model_step(const srmdp::StepArgs<srmdp_real> a, const srmdp::CellF<srmdp_real> *__restrict__ cellF,\n"
         "                 const srmdp_real *__restrict__ bsig, srmdp_real *__restrict__ lk,\n"
         "                 srmdp_real *__restrict__ table, unsigned long long *__restrict__ counters)\n"
         "{\n"
         "    extern __shared__ __align__(16) unsigned char smem[];\n"
         "    srmdp::sweep_group<srmdp_real, " + D + ", " + NB + ", srmdp::kLookupFull, false, " +
         (gr ? "true" : "false") + ", " + (ep ? "true" : "false") + ", srmdp_model_glue::Model>(\n"
         "        a, srmdp::xcd_block_order(blockIdx.x, gridDim.x), cellF, bsig, lk, table, counters, smem);\n"
         "}\n";
    return s;
}

std::string face_flags_name(int d, int nb, bool is_float, bool ep)
{
    return std::string("srmdp::face_flags_kernel<") + (is_float ? "float" : "double") + ", " + std::to_string(d) +
           ", " + std::to_string(nb) + (ep ? ", true" : ", false") + ", srmdp_model_glue::Model>";
}

struct Entry {
    hipModule_t module = nullptr;
    hipFunction_t step = nullptr, face_flags = nullptr;
};
std::mutex g_rtc_mu;
std::unordered_map<std::string, Entry> g_rtc;

}  // namespace

srmdp_status model_kernels(const srmdp_model *m, int d, int nb, int is_float, bool equal_prob, bool streamed,
                           ModelKernels &out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(SRMDP_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::string key = std::to_string(dev) + "|" + std::to_string(d) + "|" + std::to_string(nb) + "|" +
                      std::to_string(is_float) + "|" + (equal_prob ? "ep|" : "es|") + (streamed ? "gr|" : "lds|") +
                      m->source;
    std::lock_guard<std::mutex> lock(g_rtc_mu);
    auto it = g_rtc.find(key);
    if (it == g_rtc.end()) {
        const RtcApi &api = rtc_api();
        if (!api.error.empty()) return set_error(SRMDP_E_UNSUPPORTED, "%s", api.error.c_str());
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return set_error(SRMDP_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        std::string arch = prop.gcnArchName;
        arch = "--offload-arch=" + arch.substr(0, arch.find(':'));
        const std::string src = kernel_source(m, d, nb, is_float != 0, equal_prob, streamed);
        hiprtcProgram prog;
        if (api.create(&prog, src.c_str(), "srmdp_model.hip", kRtcHeaderCount, kRtcHeaderBodies,
                       kRtcHeaderNames) != HIPRTC_SUCCESS)
            return set_error(SRMDP_E_HIP, "hiprtcCreateProgram failed");
        const std::string ff = face_flags_name(d, nb, is_float != 0, equal_prob);
        api.add_name(prog, ff.c_str());
        // packed binary32 instructions are kept out, as in the compiled kernels
        const char *opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                              "-packed-fp32-ops"};
        const hiprtcResult rc = api.compile(prog, 7, opts);
        if (rc != HIPRTC_SUCCESS) {
            size_t n = 0;
            api.log_size(prog, &n);
            std::string log(n, '\0');
            if (n) api.log(prog, &log[0]);
            api.destroy(&prog);
            return set_error(SRMDP_E_INVALID, "the model does not compile: %.400s", log.c_str());
        }
        const char *lowered = nullptr;
        api.lowered(prog, ff.c_str(), &lowered);
        const std::string ff_lowered = lowered ? lowered : "";
        size_t n = 0;
        api.code_size(prog, &n);
        std::vector<char> code(n);
        api.code(prog, code.data());
        api.destroy(&prog);
        Entry ent;
        e = hipModuleLoadData(&ent.module, code.data());
        if (e != hipSuccess) return set_error(SRMDP_E_HIP, "hipModuleLoadData: %s", hipGetErrorString(e));
        e = hipModuleGetFunction(&ent.step, ent.module, "srmdp_model_step");
        if (e == hipSuccess) e = hipModuleGetFunction(&ent.face_flags, ent.module, ff_lowered.c_str());
        if (e != hipSuccess) {
            (void)hipModuleUnload(ent.module);
            return set_error(SRMDP_E_HIP, "hipModuleGetFunction: %s", hipGetErrorString(e));
        }
        it = g_rtc.emplace(key, ent).first;
    }
    out.step = it->second.step;
    out.face_flags = it->second.face_flags;
    return SRMDP_OK;
}

template <typename R>
hipError_t launch_model_step(const ModelKernels &k, const StepArgs<R> &a, const LaunchShape &s, const void *cellF,
                             const void *bsig, void *lk, void *table, void *counters, hipStream_t st)
{
    void *args[] = {(void *)&a, (void *)&cellF, (void *)&bsig, (void *)&lk, (void *)&table, (void *)&counters};
    return hipModuleLaunchKernel((hipFunction_t)k.step, s.blocks, 1, 1, s.threads, 1, 1, (unsigned)s.lds_bytes, st,
                                 args, nullptr);
}

template <typename R>
hipError_t launch_model_face_flags(const ModelKernels &k, const StepArgs<R> &a, const void *cellF, const void *bsig,
                                   void *counters, hipStream_t st)
{
    void *args[] = {(void *)&a, (void *)&cellF, (void *)&bsig, (void *)&counters};
    return hipModuleLaunchKernel((hipFunction_t)k.face_flags, a.K, 1, 1, 64, 1, 1, 0, st, args, nullptr);
}

template hipError_t launch_model_step<float>(const ModelKernels &, const StepArgs<float> &, const LaunchShape &,
                                             const void *, const void *, void *, void *, void *, hipStream_t);
template hipError_t launch_model_step<double>(const ModelKernels &, const StepArgs<double> &, const LaunchShape &,
                                              const void *, const void *, void *, void *, void *, hipStream_t);
template hipError_t launch_model_face_flags<float>(const ModelKernels &, const StepArgs<float> &, const void *,
                                                   const void *, void *, hipStream_t);
template hipError_t launch_model_face_flags<double>(const ModelKernels &, const StepArgs<double> &, const void *,
                                                    const void *, void *, hipStream_t);

}  // namespace srmdp
