// srmdp_solve_noalloc: the backward sweep for callers that cannot allocate
// device memory.  It runs srmdp_solve's kernels with the workspace taken from a
// file-scope device array instead of a caller's buffer.
//
// The array is a device symbol: in host code its name is only a stand-in, so
// the host never passes `scratch` itself to a kernel or a copy.  Its device
// address is resolved once per device with hipGetSymbolAddress (that device
// current) and kept in g_scratch; every use goes through that address.
#include "../../include/srmdp.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "srmdp_internal.hpp"

static __device__ __align__(256) unsigned char scratch[SRMDP_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch;  // device address of `scratch`, per device (nullptr = not resolved)

// Address of this device's copy of `scratch`; resolved on the first call on
// each device, with that device current.
srmdp_status scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return srmdp::set_error(SRMDP_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch.size()) g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return srmdp::set_error(SRMDP_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                    hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SRMDP_OK;
}

}  // namespace

extern "C" srmdp_status srmdp_solve_noalloc(const srmdp_problem *problem, const srmdp_grid *grid,
                                            const srmdp_options *opts, void *table, void *stream)
{
    if (!opts) return srmdp::set_error(SRMDP_E_INVALID, "opts must be non-NULL");
    if (problem && problem->model)
        return srmdp::set_error(SRMDP_E_INVALID,
                                "srmdp_solve_noalloc does not take a problem with a model (compiling and loading "
                                "its kernels allocates)");
    if (opts->flags & SRMDP_F_GRAPH)
        return srmdp::set_error(SRMDP_E_INVALID,
                                "srmdp_solve_noalloc does not take SRMDP_F_GRAPH (instantiating a graph allocates)");
    if (opts->flags & SRMDP_F_CHECK_FINITE)
        return srmdp::set_error(SRMDP_E_INVALID,
                                "srmdp_solve_noalloc does not take SRMDP_F_CHECK_FINITE (it copies counters to "
                                "the host and synchronises)");
    if ((opts->flags & SRMDP_F_AUTOTUNE) && opts->lanes_per_cube == 0)
        return srmdp::set_error(SRMDP_E_INVALID,
                                "srmdp_solve_noalloc does not autotune (timing launches creates events and "
                                "synchronises); give lanes_per_cube or drop SRMDP_F_AUTOTUNE");
    const size_t need = srmdp_workspace_bytes(problem, grid, opts);
    if (need > SRMDP_NOALLOC_SCRATCH_BYTES)
        return srmdp::set_error(SRMDP_E_WORKSPACE,
                                "the sweep needs %zu bytes of workspace; srmdp_solve_noalloc serves at most %zu "
                                "(SRMDP_NOALLOC_SCRATCH_BYTES): use srmdp_solve with a caller workspace",
                                need, (size_t)SRMDP_NOALLOC_SCRATCH_BYTES);
    // need == 0 means invalid arguments: srmdp_solve reports which, before
    // anything is enqueued.
    void *ws = nullptr;
    const srmdp_status rc = scratch_address(&ws);
    if (rc != SRMDP_OK) return rc;
    return srmdp_solve(problem, grid, opts, table, ws, SRMDP_NOALLOC_SCRATCH_BYTES, nullptr, stream);
}
