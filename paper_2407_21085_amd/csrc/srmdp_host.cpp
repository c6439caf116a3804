// Host runtime of the SRMDP library: argument checks, workspace layout,
// launch shapes, the backward driver (one kernel per step, optionally replayed
// from a cached hipGraph) and the read-outs.  Implements include/srmdp.h.
#include "../../include/srmdp.h"

#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <map>
#include <numeric>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "srmdp_internal.hpp"
#include "srmdp_mlp.hpp"

using namespace srmdp;

static thread_local std::string g_error;

namespace {

// Annotation ranges for profilers (roctx of rocprofiler-sdk, shown by
// `rocprofv3 --marker-trace`): one per backward step, per training update and
// per batched global step, pushed on the host when the work is enqueued.  The
// roctx library is opened on first use; without it a range costs a null check.
struct RoctxApi {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
};

const RoctxApi &roctx_api()
{
    static const RoctxApi api = [] {
        RoctxApi r;
        for (const char *name : {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"}) {
            void *h = dlopen(name, RTLD_NOW | RTLD_LOCAL);
            if (!h) continue;
            r.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
            r.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
            if (!r.push || !r.pop) r.push = nullptr, r.pop = nullptr;
            break;
        }
        return r;
    }();
    return api;
}

class TraceRange {
  public:
    TraceRange(const char *what, int index)
    {
        const RoctxApi &api = roctx_api();
        if (!api.push) return;
        char name[64];
        std::snprintf(name, sizeof name, "%s %d", what, index);
        active_ = api.push(name) >= 0;
    }
    ~TraceRange()
    {
        if (active_) roctx_api().pop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;

  private:
    bool active_ = false;
};

srmdp_status fail(srmdp_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
srmdp_status fail(srmdp_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

}  // namespace

srmdp_status srmdp::set_error(srmdp_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

namespace {

srmdp_status hip_fail(hipError_t e, const char *what)
{
    return fail(SRMDP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int kMaxModelParams = 64;  // srmdp_model.n_params

// Timing events of one call, destroyed on every return path.
struct EventSet {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    EventSet() = default;
    EventSet(const EventSet &) = delete;
    EventSet &operator=(const EventSet &) = delete;
    ~EventSet()
    {
        for (hipEvent_t &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    hipError_t create(int n)
    {
        for (int j = 0; j < n; ++j) {
            const hipError_t err = hipEventCreate(&e[j]);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }
};

// ------------------------------------------------------------- validation
struct Shape {
    int d, q, N, nb, cmax;
    uint64_t K;
    bool equal_prob;  // SRMDP_GRID_EQUAL_PROB
};

srmdp_status check_problem(const srmdp_problem *p, const srmdp_grid *g, Shape &s)
{
    if (!p || !g) return fail(SRMDP_E_INVALID, "problem and grid must be non-NULL");
    if (p->d < 1 || p->d > SRMDP_MAX_D)
        return fail(SRMDP_E_INVALID, "d = %d outside 1..%d", p->d, SRMDP_MAX_D);
    if (p->q != p->d)
        return fail(SRMDP_E_INVALID, "the built-in driver and terminal need q == d (q = %d, d = %d)",
                    p->q, p->d);
    if (p->model) {
        const srmdp_model *m = p->model;
        if (!m->source || !m->source[0]) return fail(SRMDP_E_INVALID, "model source must be non-empty");
        if (m->n_params < 0 || m->n_params > kMaxModelParams)
            return fail(SRMDP_E_INVALID, "model n_params = %d outside 0..%d", m->n_params, kMaxModelParams);
        if (m->n_params > 0 && !m->params) return fail(SRMDP_E_INVALID, "model params NULL with n_params > 0");
        for (int v = 0; v < m->n_params; ++v)
            if (!std::isfinite(m->params[v])) return fail(SRMDP_E_INVALID, "model parameter %d is not finite", v);
        if (p->b || p->sigma || p->b_lin || p->sigma_lin || p->r != 0.0 || p->kappa != 0.0 || p->driver != 0 ||
            p->terminal != 0)
            return fail(SRMDP_E_INVALID, "a problem with a model takes no built-in coefficients");
    }
    if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(SRMDP_E_INVALID, "T must be finite and > 0");
    if (p->N < 1 || p->N > 65535) return fail(SRMDP_E_INVALID, "N = %d outside 1..65535", p->N);
    if (p->driver != SRMDP_DRV_LINEAR && p->driver != SRMDP_DRV_LOGISTIC)
        return fail(SRMDP_E_INVALID, "unknown driver %d", p->driver);
    if (p->terminal != SRMDP_G_COS_SUM && p->terminal != SRMDP_G_LOGISTIC)
        return fail(SRMDP_E_INVALID, "unknown terminal %d", p->terminal);
    if (!(p->clamp_y > 0.0) || !(p->clamp_z > 0.0))
        return fail(SRMDP_E_INVALID, "truncation levels must be > 0 (INFINITY = off)");
    if (!std::isfinite(p->r) || !std::isfinite(p->kappa))
        return fail(SRMDP_E_INVALID, "driver parameters must be finite");
    if (g->kind != SRMDP_GRID_EQUAL_SIZE && g->kind != SRMDP_GRID_EQUAL_PROB)
        return fail(SRMDP_E_INVALID, "unknown grid kind %d", (int)g->kind);
    const bool equal_size = g->kind == SRMDP_GRID_EQUAL_SIZE;
    if (!g->cells || (equal_size && (!g->lo || !g->hi)))
        return fail(SRMDP_E_INVALID, "grid arrays must be non-NULL");
    if (!(g->mu > 0.0) || !std::isfinite(g->mu)) return fail(SRMDP_E_INVALID, "mu must be > 0");
    s.d = p->d;
    s.q = p->q;
    s.N = p->N;
    s.equal_prob = !equal_size;
    s.K = 1;
    s.cmax = 1;
    for (int l = 0; l < p->d; ++l) {
        if (equal_size && (!(g->lo[l] < g->hi[l]) || !std::isfinite(g->lo[l]) || !std::isfinite(g->hi[l])))
            return fail(SRMDP_E_INVALID, "grid dimension %d: need finite lo < hi", l);
        if (g->cells[l] < 1) return fail(SRMDP_E_INVALID, "grid dimension %d: cells < 1", l);
        s.K *= (uint64_t)g->cells[l];
        if (s.K > (1ull << 24)) return fail(SRMDP_E_INVALID, "K exceeds 2^24 strata");
        s.cmax = std::max(s.cmax, (int)g->cells[l]);
    }
    if (p->b)
        for (int l = 0; l < p->d; ++l)
            if (!std::isfinite(p->b[l])) return fail(SRMDP_E_INVALID, "drift must be finite");
    if (p->sigma)
        for (int l = 0; l < p->d * p->q; ++l)
            if (!std::isfinite(p->sigma[l])) return fail(SRMDP_E_INVALID, "sigma must be finite");
    if (p->b_lin)
        for (int l = 0; l < p->d; ++l)
            if (!std::isfinite(p->b_lin[l])) return fail(SRMDP_E_INVALID, "b_lin must be finite");
    if (p->sigma_lin)
        for (int l = 0; l < p->d; ++l)
            if (!std::isfinite(p->sigma_lin[l])) return fail(SRMDP_E_INVALID, "sigma_lin must be finite");
    return SRMDP_OK;
}

srmdp_status check_options(const srmdp_options *o, const Shape &s, int &nb)
{
    if (!o) return fail(SRMDP_E_INVALID, "options must be non-NULL");
    if (o->basis != SRMDP_LP0 && o->basis != SRMDP_LP1)
        return fail(SRMDP_E_INVALID, "unknown basis %d", o->basis);
    if (o->prec != SRMDP_FP64 && o->prec != SRMDP_FP32)
        return fail(SRMDP_E_INVALID, "unknown precision %d", o->prec);
    nb = o->basis == SRMDP_LP1 ? s.d + 1 : 1;
    if (o->M < nb)
        return fail(SRMDP_E_INVALID, "M = %d is below the dimension %d of the local space", o->M, nb);
    if (o->instance >= 65536u) return fail(SRMDP_E_INVALID, "instance must be < 65536");
    const int hi = o->step_hi < 0 ? s.N - 1 : o->step_hi;
    const int lo = o->step_lo < 0 ? 0 : o->step_lo;
    if (hi >= s.N || lo > hi) return fail(SRMDP_E_INVALID, "steps %d..%d outside 0..%d", hi, lo, s.N - 1);
    const int L = o->lanes_per_cube;
    if (L != 0 && L != 8 && L != 16 && L != 32 && L != 64 && L != 128 && L != 256)
        return fail(SRMDP_E_INVALID, "lanes_per_cube must be 0, 8, 16, 32, 64, 128 or 256");
    if (o->flags & ~(uint32_t)(SRMDP_F_GRAPH | SRMDP_F_CHECK_FINITE | SRMDP_F_CV_CENTER_Z | SRMDP_F_AUTOTUNE |
                               SRMDP_F_GLOBAL_ROWS | SRMDP_F_DEBUG_SINGULAR))
        return fail(SRMDP_E_INVALID, "unknown flag bits");
    if ((o->flags & SRMDP_F_DEBUG_SINGULAR) &&
        (o->debug_step < 0 || o->debug_step >= s.N || (uint64_t)o->debug_stratum >= s.K))
        return fail(SRMDP_E_INVALID, "SRMDP_F_DEBUG_SINGULAR: step %d or stratum %u outside the grid", o->debug_step,
                    o->debug_stratum);
    if (o->global_rows_strata < 0) return fail(SRMDP_E_INVALID, "global_rows_strata < 0");
    if ((o->flags & SRMDP_F_GLOBAL_ROWS) && o->cv != SRMDP_CV_NONE)
        return fail(SRMDP_E_UNSUPPORTED, "global cloud rows run without the control variate");

    if ((o->flags & SRMDP_F_CV_CENTER_Z) && o->cv == SRMDP_CV_NONE)
        return fail(SRMDP_E_INVALID, "SRMDP_F_CV_CENTER_Z needs a control variate");
    if (o->cv_stride > 65535) return fail(SRMDP_E_INVALID, "cv_stride above 65535");
    if (!(o->face_eps < 0.5) || std::isnan(o->face_eps))
        return fail(SRMDP_E_INVALID, "face_eps must be < 0.5 cell widths");
    if (o->cv != SRMDP_CV_NONE && o->cv != SRMDP_CV_FROZEN && o->cv != SRMDP_CV_ONLINE)
        return fail(SRMDP_E_INVALID, "unknown control variate %d", o->cv);
    if (o->cv != SRMDP_CV_NONE) {
        if (!o->cv_params) return fail(SRMDP_E_INVALID, "the control variate needs cv_params");
        if (s.d + 1 > kMlpMaxIn || s.q > kMlpMaxOut)
            return fail(SRMDP_E_UNSUPPORTED, "the control variate takes d + 1 <= %d inputs", kMlpMaxIn);
        if (o->prec != SRMDP_FP32)
            return fail(SRMDP_E_UNSUPPORTED, "the control variate runs in binary32 sweeps only");
        if (o->cv == SRMDP_CV_ONLINE) {
            const srmdp_mlp_train_config &c = o->cv_train;
            if (c.updates_per_step < 1 || c.updates_per_step > 4096)
                return fail(SRMDP_E_INVALID, "cv_train.updates_per_step outside 1..4096");
            if (c.batch < 256 || c.batch > 65536 || c.batch % 256 != 0)
                return fail(SRMDP_E_INVALID, "cv_train.batch must be a multiple of 256 up to 65536");
            if (!(c.lr > 0.0f) || !(c.beta1 >= 0.0f && c.beta1 < 1.0f) || !(c.beta2 >= 0.0f && c.beta2 < 1.0f) ||
                !(c.eps > 0.0f) || !std::isfinite(c.lr))
                return fail(SRMDP_E_INVALID, "Adam needs lr > 0, betas in [0, 1) and eps > 0");
        }
    }
    return SRMDP_OK;
}

int lookup_mode(const srmdp_problem *p)
{
    if (p->model || std::isfinite(p->clamp_z)) return kLookupFull;  // a model's driver reads every z_c
    if (p->driver == SRMDP_DRV_LINEAR && p->kappa == 0.0) return kLookupY;
    return kLookupYZ;
}

// ------------------------------------------------------------- workspace
constexpr int kRootBlocks = 512;

bool make_shape(const Shape &s, int nb, int is_float, int M, int L, LaunchShape &ls, size_t &per_cube,
                bool cv = false, const srmdp_options *o = nullptr);
int lanes_for(const srmdp_options *o);

struct Layout {
    size_t counters, cellF, bsig, lookup, root_partial, root_out;
    size_t cv_packed, cv_m, cv_v, cv_x, cv_z, cv_loss, cv_part;  // control variate (0 = absent)
    size_t grows;                                                 // global cloud rows (0 = absent)
    int64_t cv_pairs;                                    // training pairs per step
    size_t total;
};

Layout layout(const Shape &s, int nb, int is_float, int lk, const srmdp_options *o = nullptr)
{
    const size_t rsz = is_float ? 4 : 8;
    Layout L{};
    size_t off = 0;
    L.counters = off;
    off = align_up(off + kCounterCount * sizeof(unsigned long long), 256);
    L.cellF = off;
    off = align_up(off + (size_t)s.d * s.cmax * 4 * rsz, 256);
    L.bsig = off;
    // b | sigma | b_lin | sigma_lin, or a model's parameters
    off = align_up(off + (size_t)std::max(3 * s.d + s.d * s.q, kMaxModelParams) * rsz, 256);
    L.root_partial = off;
    off = align_up(off + (size_t)kRootBlocks * (s.d + 2) * sizeof(double), 256);
    L.root_out = off;
    off = align_up(off + (size_t)(s.d + 1) * sizeof(double), 256);
    L.lookup = off;
    off = align_up(off + (size_t)s.N * s.K * lookup_width(is_float, s.d, nb, lk) * rsz, 256);
    if (o && o->cv != SRMDP_CV_NONE) {
        L.cv_packed = off;
        off = align_up(off + kPackedBytes, 256);
        if (o->cv == SRMDP_CV_ONLINE) {
            const size_t P = (size_t)MlpShape{s.d + 1, s.q}.count();
            L.cv_pairs = (int64_t)o->cv_train.updates_per_step * o->cv_train.batch;
            L.cv_m = off;
            off = align_up(off + P * sizeof(float), 256);
            L.cv_v = off;
            off = align_up(off + P * sizeof(float), 256);
            L.cv_x = off;
            off = align_up(off + (size_t)L.cv_pairs * 16 * sizeof(float), 256);
            L.cv_z = off;
            off = align_up(off + (size_t)L.cv_pairs * 16 * sizeof(float), 256);
            L.cv_loss = off;
            off = align_up(off + (size_t)s.N * o->cv_train.updates_per_step * sizeof(float), 256);
            L.cv_part = off;
            off = align_up(off + mlp_train_partial_bytes(s.d + 1, s.q, o->cv_train.batch), 256);
        }
    }
    if (o && o->cv == SRMDP_CV_NONE && o->M >= 1) {
        LaunchShape ls;
        size_t per_cube;
        if (make_shape(s, nb, is_float, o->M, lanes_for(o), ls, per_cube, false, o) && ls.grows) {
            L.grows = off;
            off = align_up(off + (size_t)ls.kc * ls.grow_bytes, 256);
        }
    }
    L.total = off;
    return L;
}

// ------------------------------------------------------------- arguments
template <typename R>
void fill_step_args(StepArgs<R> &a, const srmdp_problem *p, const srmdp_grid *g, const Shape &s,
                    const srmdp_options *o)
{
    std::memset(&a, 0, sizeof a);
    a.debug_singular = 0xFFFFFFFFu;
    uint32_t stride = 1;
    for (int l = 0; l < s.d; ++l) {
        if (g->kind == SRMDP_GRID_EQUAL_PROB) {
            a.lo[l] = (R)0;
            a.scale[l] = (R)(0.5 * g->mu);
        } else {
            a.lo[l] = (R)g->lo[l];
            a.scale[l] = (R)((double)g->cells[l] / (g->hi[l] - g->lo[l]));
        }
        a.cmax_f[l] = (R)(g->cells[l] - 1);
        a.stride[l] = stride;
        a.stride_f[l] = (R)stride;
        a.cells[l] = (uint32_t)g->cells[l];
        stride *= (uint32_t)g->cells[l];
    }
    a.cmax = s.cmax;
    a.K = (uint32_t)s.K;
    a.N = s.N;
    a.dt_d = p->T / p->N;
    a.inv_dt = 1.0 / a.dt_d;
    a.dt = (R)a.dt_d;
    a.sqrt_dt = (R)std::sqrt(a.dt_d);
    a.T = (R)p->T;
    a.inv_mu = (R)(1.0 / g->mu);
    a.equal_prob = g->kind == SRMDP_GRID_EQUAL_PROB ? 1 : 0;
    a.driver = p->driver;
    a.terminal = p->terminal;
    a.r = (R)p->r;
    a.kappa = (R)p->kappa;
    a.c_logistic = (R)((2.0 + p->q) / (2.0 * p->q));
    a.clamp_y = (R)p->clamp_y;
    a.clamp_z = (R)p->clamp_z;
    bool ident = true;
    if (p->sigma)
        for (int l = 0; l < s.d; ++l)
            for (int c = 0; c < s.q; ++c)
                if (p->sigma[l * s.q + c] != (l == c ? 1.0 : 0.0)) ident = false;
    a.identity_sigma = ident ? 1 : 0;
    bool drift = false;
    if (p->b)
        for (int l = 0; l < s.d; ++l)
            if (p->b[l] != 0.0) drift = true;
    a.has_drift = drift ? 1 : 0;
    bool lin = false;
    if (p->b_lin)
        for (int l = 0; l < s.d; ++l)
            if (p->b_lin[l] != 0.0) lin = true;
    a.has_lin_drift = lin ? 1 : 0;
    bool lin_sigma = false;
    if (p->sigma_lin)
        for (int l = 0; l < s.d; ++l)
            if (p->sigma_lin[l] != 0.0) lin_sigma = true;
    a.has_lin_sigma = lin_sigma ? 1 : 0;
    if (o) {
        a.M = o->M;
        a.key0 = (uint32_t)(o->seed & 0xFFFFFFFFull);
        a.key1 = (uint32_t)(o->seed >> 32);
        a.check_finite = (o->flags & SRMDP_F_CHECK_FINITE) ? 1 : 0;
        a.face_flags = o->face_flags;
        a.face_eps = (R)(o->face_eps > 0.0 ? o->face_eps : 1e-5);
        a.cv_stride = o->cv_stride > 1 ? o->cv_stride : 1;
        a.z_center = (o->flags & SRMDP_F_CV_CENTER_Z) ? 1 : 0;
    } else {
        a.cv_stride = 1;
    }
}

// The d x q diffusion matrix of the set-up (identity when the problem gives none).
struct SigmaHost {
    double v[kMaxDim * kMaxDim];
};

void fill_setup_args(SetupArgs &sa, SigmaHost &sg, const srmdp_problem *p, const srmdp_grid *g, const Shape &s)
{
    std::memset(&sa, 0, sizeof sa);
    for (int l = 0; l < s.d; ++l) {
        sa.lo[l] = g->kind == SRMDP_GRID_EQUAL_SIZE ? g->lo[l] : 0.0;
        sa.hi[l] = g->kind == SRMDP_GRID_EQUAL_SIZE ? g->hi[l] : 0.0;
        sa.cells[l] = g->cells[l];
        sa.b[l] = p->b ? p->b[l] : 0.0;
        sa.b_lin[l] = p->b_lin ? p->b_lin[l] : 0.0;
        sa.sigma_lin[l] = p->sigma_lin ? p->sigma_lin[l] : 0.0;
    }
    for (int t = 0; t < s.d * s.q; ++t)
        sg.v[t] = p->sigma ? p->sigma[t] : ((t / s.q) == (t % s.q) ? 1.0 : 0.0);
    sa.d = s.d;
    sa.q = s.q;
    sa.cmax = s.cmax;
    sa.mu = g->mu;
    sa.equal_prob = g->kind == SRMDP_GRID_EQUAL_PROB ? 1 : 0;
}

// Lanes per stratum: enough to give every lane one path up to a wavefront.
// With the control variate every lane of a wavefront must run the same number
// of paths: the largest power of two up to 64 that divides M.
// Default lanes per stratum: the next power of two >= M (one simulation per
// lane), at most 256.  Larger M then spreads over more wavefronts of one
// workgroup instead of more trips of one wavefront: at d = 8, M = 512 takes a
// third of the time it takes with 64 lanes.
int auto_lanes(int M)
{
    int L = 8;
    while (L < M && L < 256) L *= 2;
    return L;
}

int lanes_for(const srmdp_options *o)
{
    return o->lanes_per_cube ? o->lanes_per_cube : auto_lanes(o->M);
}

constexpr size_t kGlobalRowsBudget = (size_t)2 << 30;  // bytes of global cloud rows per launch

// Strata per global-rows launch: what the budget holds (or the caller's
// choice), a multiple of 8 so that every lanes setting divides it.
uint32_t grows_strata(const Shape &s, size_t grow_bytes, const srmdp_options *o)
{
    uint64_t kc = (o && o->global_rows_strata > 0) ? (uint64_t)o->global_rows_strata : kGlobalRowsBudget / grow_bytes;
    kc = std::max<uint64_t>(8, (kc + 7) / 8 * 8);
    return (uint32_t)std::min<uint64_t>(kc, ((uint64_t)s.K + 7) / 8 * 8);
}

// One wavefront per workgroup when a stratum fits in one (several strata share
// it when M is small): the regression's barriers are then wave-local, and the
// wavefronts of a CU drift apart, so one wave's latency-bound regression
// overlaps other waves' path arithmetic instead of the whole CU stalling at
// the same barrier.
// With the control variate a workgroup of up to four wavefronts shares one LDS
// copy of the network's forward weights.
// Without it, a stratum whose cloud does not fit in a workgroup's 64 KB of LDS
// (or any stratum, with SRMDP_F_GLOBAL_ROWS) streams its cloud through an LDS
// window in rounds, keeping S' and y_{i+1} per sample in global memory, and
// each step runs in launches of ls.kc strata.
bool make_shape(const Shape &s, int nb, int is_float, int M, int L, LaunchShape &ls, size_t &per_cube, bool cv,
                const srmdp_options *o)
{
    ls.grows = false;
    ls.kc = 0;
    ls.grow_bytes = 0;
    ls.stage_chunks = 0;
    per_cube = align_up(cube_lds_bytes(is_float, s.d, nb, M, cv), 16);
    if (cv) {
        const size_t cap = 64 * 1024 - kPackedFwdBytes;
        int cpw = 256 / L;
        while (cpw * L > 64 && (size_t)cpw * per_cube > cap) cpw /= 2;
        if ((size_t)cpw * per_cube > cap) return false;
        ls.threads = (unsigned)(cpw * L);
        ls.blocks = (unsigned)((s.K + cpw - 1) / cpw);
        ls.lds_bytes = kPackedFwdBytes + (size_t)cpw * per_cube;
        return true;
    }
    const size_t lds_cap = 64 * 1024;
    const bool force = (o && (o->flags & SRMDP_F_GLOBAL_ROWS)) || !lds_dimension_compiled(s.d);
    if (force || per_cube > lds_cap) {
        ls.grows = true;
        const int pb = cube_stream_chunks(is_float, s.d, nb, L, lds_cap);
        if (pb < 1) return false;
        per_cube = align_up(cube_stream_lds_bytes(is_float, s.d, nb, L, pb), 16);
        ls.grow_bytes = cube_global_bytes(is_float, M);
        ls.kc = grows_strata(s, ls.grow_bytes, o);
        ls.stage_chunks = pb;
    }
    int cpw = std::max(1, 64 / L);
    while (cpw > 1 && (size_t)cpw * per_cube > lds_cap) cpw /= 2;
    if ((size_t)cpw * per_cube > lds_cap) return false;
    ls.threads = (unsigned)(cpw * L);
    ls.blocks = (unsigned)((s.K + cpw - 1) / cpw);
    ls.lds_bytes = (size_t)cpw * per_cube;
    return true;
}

// One backward step without the control variate: one launch, or with global
// rows one launch per ls.kc strata.
// mk: the problem's own model kernels (compiled for this shape's grid kind and
// cloud storage), or nullptr for the built-in problems.
template <typename R>
hipError_t launch_plain_step(const Shape &s, StepArgs<R> &a, const LaunchShape &ls, int basis, int lk,
                             unsigned char *ws, size_t off_cellF, size_t off_bsig, size_t off_lookup,
                             size_t off_counters, size_t off_grows, void *table, hipStream_t st,
                             const ModelKernels *mk = nullptr)
{
    a.cell_table = ws + off_cellF;
    if (!ls.grows && mk)
        return launch_model_step<R>(*mk, a, ls, ws + off_cellF, ws + off_bsig, ws + off_lookup, table,
                                    ws + off_counters, st);
    if (!ls.grows && a.equal_prob)
        return launch_step_ep_lds<R>(s.d, a, ls, basis, lk, ws + off_cellF, ws + off_bsig, ws + off_lookup, table,
                                     ws + off_counters, st);
    if (!ls.grows)
        return launch_step<R>(s.d, a, ls, basis, lk, ws + off_cellF, ws + off_bsig, ws + off_lookup, table,
                              ws + off_counters, st);
    const uint32_t cpw = ls.threads / (uint32_t)a.lanes;
    for (uint32_t k0 = 0; k0 < s.K; k0 += ls.kc) {
        a.k0 = k0;
        a.k_end = std::min<uint32_t>(s.K, k0 + ls.kc);
        a.grows = ws + off_grows;
        a.grow_bytes = ls.grow_bytes;
        a.stage_chunks = ls.stage_chunks;
        LaunchShape sub = ls;
        sub.blocks = (a.k_end - k0 + cpw - 1) / cpw;
        const hipError_t e =
            mk ? launch_model_step<R>(*mk, a, sub, ws + off_cellF, ws + off_bsig, ws + off_lookup, table,
                                      ws + off_counters, st)
               : launch_step_gr<R>(s.d, a, sub, basis, lk, ws + off_cellF, ws + off_bsig, ws + off_lookup, table,
                                   ws + off_counters, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The sweep kernels compiled for the shape: every compiled dimension has the
// global-rows kernel in binary32 with look-up modes Y and YZ; the LDS kernel
// (both precisions, every mode) exists for the dimensions of the main file.
srmdp_status sweep_supported(const Shape &s, const srmdp_options *o, int lk)
{
    if (s.equal_prob && o->cv != SRMDP_CV_NONE && lk == kLookupFull)
        return fail(SRMDP_E_UNSUPPORTED, "the control variate on equal-probability cells takes no z truncation");
    if (!dimension_compiled(s.d)) return fail(SRMDP_E_UNSUPPORTED, "d = %d is not compiled", s.d);
    if (!lds_dimension_compiled(s.d) &&
        (o->prec != SRMDP_FP32 || (lk != kLookupY && lk != kLookupYZ) || o->cv != SRMDP_CV_NONE))
        return fail(SRMDP_E_UNSUPPORTED,
                    "d = %d runs binary32 sweeps without z truncation or control variate only", s.d);
    return SRMDP_OK;
}

// What a problem with its own model runs: d = 1..8 (its look-ups read whole
// records, (d + 1)^2 coefficients for LP1), either grid kind, clouds in LDS or
// streamed through it (large M, or SRMDP_F_GLOBAL_ROWS), without the control
// variate or the autotuner.  *streamed tells which cloud storage the shape
// takes, for which the model's kernel is compiled.
srmdp_status model_supported(const Shape &s, int nb, const srmdp_options *o, bool *streamed)
{
    if (s.d > 8) return fail(SRMDP_E_UNSUPPORTED, "a model runs for d = 1..8");
    if (o->cv != SRMDP_CV_NONE) return fail(SRMDP_E_UNSUPPORTED, "a model runs without the control variate");
    if (o->flags & SRMDP_F_AUTOTUNE) return fail(SRMDP_E_UNSUPPORTED, "a model runs without the autotuner");
    LaunchShape ls;
    size_t per_cube;
    if (!make_shape(s, nb, o->prec == SRMDP_FP32, o->M, lanes_for(o), ls, per_cube, false, o))
        return fail(SRMDP_E_UNSUPPORTED, "no launch shape fits M = %d", o->M);
    *streamed = ls.grows;
    return SRMDP_OK;
}

// Backward-step launches per step.
uint32_t launches_per_step(const Shape &s, const LaunchShape &ls)
{
    return ls.grows ? (uint32_t)((s.K + ls.kc - 1) / ls.kc) : 1u;
}

// ------------------------------------------------------------- graph cache
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::unordered_map<std::string, GraphEntry> g_graphs;

std::string graph_key(const void *args, size_t n, hipStream_t st)
{
    std::string k((const char *)args, n);
    k.append((const char *)&st, sizeof st);
    return k;
}

template <typename R>
srmdp_status enqueue_sweep(const srmdp_problem *p, const srmdp_grid *g, const srmdp_options *o,
                           const Shape &s, int nb, int lk, void *table, unsigned char *ws,
                           const Layout &lay, hipStream_t st, const ModelKernels *mk,
                           hipEvent_t steps0 = nullptr, hipEvent_t steps1 = nullptr)
{
    const int is_float = sizeof(R) == 4;
    const int L = lanes_for(o);
    const bool cv = o->cv != SRMDP_CV_NONE;
    LaunchShape ls;
    size_t per_cube;
    if (!make_shape(s, nb, is_float, o->M, L, ls, per_cube, cv, o))
        return fail(SRMDP_E_UNSUPPORTED, "M = %d does not fit the per-workgroup LDS budget", o->M);
    StepArgs<R> a;
    fill_step_args<R>(a, p, g, s, o);
    a.lanes = L;
    a.lds_per_cube = per_cube;
    SetupArgs sa;
    SigmaHost sg;
    fill_setup_args(sa, sg, p, g, s);
    const int hi = o->step_hi < 0 ? s.N - 1 : o->step_hi;
    const int lo = o->step_lo < 0 ? 0 : o->step_lo;

    HIP_TRY(launch_zero_u64((unsigned long long *)(ws + lay.counters), kCounterCount, st), "zero counters");
    HIP_TRY(launch_setup<R>(sa, sg.v, ws + lay.cellF, ws + lay.bsig, st), "setup kernel");
    if (mk && p->model->n_params > 0) {  // a model reads its parameters where bsig was
        std::vector<R> pv(p->model->params, p->model->params + p->model->n_params);
        HIP_TRY(launch_upload(ws + lay.bsig, pv.data(), pv.size() * sizeof(R), st), "model parameters");
    }
    const MlpShape net{s.d + 1, s.q};
    if (cv) {
        a.cv_packed = ws + lay.cv_packed;
        HIP_TRY(launch_mlp_pack(net.in, net.out, o->cv_params, ws + lay.cv_packed, st), "network pack");
        if (o->cv == SRMDP_CV_ONLINE) {
            HIP_TRY(launch_zero_f32((float *)(ws + lay.cv_m), net.count(), st), "Adam state");
            HIP_TRY(launch_zero_f32((float *)(ws + lay.cv_v), net.count(), st), "Adam state");
        }
    }
    if (hi < s.N - 1)
        HIP_TRY(launch_lookup_rows<R>(s.d, o->basis, lk, table, ws + lay.lookup, (uint32_t)s.K, hi + 1,
                                      s.N - 1, st),
                "look-up rows");
    if (steps0) HIP_TRY(hipEventRecord(steps0, st), "hipEventRecord");
    a.cell_table = ws + lay.cellF;
    for (int i = hi; i >= lo; --i) {
        TraceRange range("srmdp backward step", i);
        a.i = i;
        a.tag = ((uint32_t)i & 0xFFFFu) | (o->instance << 16);
        a.debug_singular =
            (o->flags & SRMDP_F_DEBUG_SINGULAR) && i == o->debug_step ? o->debug_stratum : 0xFFFFFFFFu;
        bool launched = false;
        if constexpr (std::is_same<R, float>::value) {
            if (cv) {
                HIP_TRY(launch_step_cv(s.d, a, ls, o->basis, lk, ws + lay.cellF, ws + lay.bsig, ws + lay.lookup,
                                       table, ws + lay.counters, st),
                        "sweep step");
                if (o->cv == SRMDP_CV_ONLINE) {
                    float *x16 = (float *)(ws + lay.cv_x), *z16 = (float *)(ws + lay.cv_z);
                    HIP_TRY(launch_cv_pairs(s.d, o->basis, a, ws + lay.cellF, table, lay.cv_pairs, x16, z16, st),
                            "training pairs");
                    const int U = o->cv_train.updates_per_step;
                    MlpTrainArgs t{};
                    t.in = net.in;
                    t.out = net.out;
                    t.theta = o->cv_params;
                    t.adam_m = (float *)(ws + lay.cv_m);
                    t.adam_v = (float *)(ws + lay.cv_v);
                    t.adam_t0 = (int64_t)(hi - i) * U;
                    t.x16 = x16;
                    t.z16 = z16;
                    t.S = lay.cv_pairs;
                    t.updates = U;
                    t.batch = o->cv_train.batch;
                    t.lr = o->cv_train.lr;
                    t.beta1 = o->cv_train.beta1;
                    t.beta2 = o->cv_train.beta2;
                    t.eps = o->cv_train.eps;
                    t.packed_out = ws + lay.cv_packed;
                    t.loss = (float *)(ws + lay.cv_loss) + (size_t)(hi - i) * U;
                    TraceRange train_range("srmdp network training after step", i);
                    HIP_TRY(launch_mlp_train(t, (float *)(ws + lay.cv_part), st), "network training");
                }
                launched = true;
            }
        }
        if (mk) {
            HIP_TRY(launch_plain_step<R>(s, a, ls, o->basis, lk, ws, lay.cellF, lay.bsig, lay.lookup, lay.counters,
                                         lay.grows, table, st, mk),
                    "sweep step (model)");
            launched = true;
        }
        if (!launched)
            HIP_TRY(launch_plain_step<R>(s, a, ls, o->basis, lk, ws, lay.cellF, lay.bsig, lay.lookup, lay.counters,
                                         lay.grows, table, st),
                    "sweep step");
        if (a.face_flags && mk)
            HIP_TRY(launch_model_face_flags<R>(*mk, a, ws + lay.cellF, ws + lay.bsig, ws + lay.counters, st),
                    "near-face flags (model)");
        else if (a.face_flags)
            HIP_TRY(launch_face_flags<R>(s.d, o->basis, a, ws + lay.cellF, ws + lay.bsig,
                                         ws + lay.counters, st),
                    "near-face flags");
    }
    if (steps1) HIP_TRY(hipEventRecord(steps1, st), "hipEventRecord");
    return SRMDP_OK;
}

template <typename R>
srmdp_status solve_impl(const srmdp_problem *p, const srmdp_grid *g, const srmdp_options *o,
                        const Shape &s, int nb, void *table, void *workspace, srmdp_stats *stats,
                        hipStream_t st, const ModelKernels *mk)
{
    const int lk = lookup_mode(p);
    const Layout lay = layout(s, nb, sizeof(R) == 4, lk, o);
    unsigned char *ws = (unsigned char *)workspace;
    EventSet ev;
    hipEvent_t &e0 = ev.e[0], &e1 = ev.e[1], &s0 = ev.e[2], &s1 = ev.e[3];
    bool graph_used = false;
    if (stats) {
        HIP_TRY(ev.create(4), "hipEventCreate");
        HIP_TRY(hipEventRecord(e0, st), "hipEventRecord");
    }
    srmdp_status rc = SRMDP_OK;
    if ((o->flags & SRMDP_F_GRAPH) && st != nullptr) {
        // key: every scalar argument and pointer that the captured launches bake in
        std::vector<unsigned char> key;
        auto put = [&](const void *v, size_t n) {
            key.insert(key.end(), (const unsigned char *)v, (const unsigned char *)v + n);
        };
        put(p, sizeof *p);
        if (p->b) put(p->b, sizeof(double) * s.d);
        if (p->sigma) put(p->sigma, sizeof(double) * s.d * s.q);
        if (p->b_lin) put(p->b_lin, sizeof(double) * s.d);
        if (p->sigma_lin) put(p->sigma_lin, sizeof(double) * s.d);
        if (p->model) {
            put(p->model->source, std::strlen(p->model->source));
            if (p->model->n_params > 0) put(p->model->params, sizeof(double) * p->model->n_params);
        }
        put(&g->kind, sizeof g->kind);
        if (g->kind == SRMDP_GRID_EQUAL_SIZE) {
            put(g->lo, sizeof(double) * s.d);
            put(g->hi, sizeof(double) * s.d);
        }
        put(g->cells, sizeof(int32_t) * s.d);
        put(&g->mu, sizeof g->mu);
        put(o, sizeof *o);
        put(&table, sizeof table);
        put(&workspace, sizeof workspace);
        const std::string k = graph_key(key.data(), key.size(), st);
        std::lock_guard<std::mutex> lock(g_graph_mu);
        auto it = g_graphs.find(k);
        if (it == g_graphs.end()) {
            GraphEntry ent;
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            rc = enqueue_sweep<R>(p, g, o, s, nb, lk, table, ws, lay, st, mk);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &graph);
            if (rc != SRMDP_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
            ent.graph = graph;
            HIP_TRY(hipGraphInstantiate(&ent.exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            it = g_graphs.emplace(k, ent).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.exec, st), "hipGraphLaunch");
        graph_used = true;
    } else {
        rc = enqueue_sweep<R>(p, g, o, s, nb, lk, table, ws, lay, st, mk, s0, s1);
        if (rc != SRMDP_OK) return rc;
    }
    const bool need_sync = stats || (o->flags & SRMDP_F_CHECK_FINITE);
    if (need_sync) {
        unsigned long long ctr[kCounterCount] = {0, 0, 0, 0};
        if (stats) HIP_TRY(hipEventRecord(e1, st), "hipEventRecord");
        HIP_TRY(hipMemcpyAsync(ctr, ws + lay.counters, sizeof ctr, hipMemcpyDeviceToHost, st), "counters");
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (stats) {
            std::memset(stats, 0, sizeof *stats);
            stats->singular_cubes = ctr[kCounterSingular];
            const int hi = o->step_hi < 0 ? s.N - 1 : o->step_hi;
            const int lo = o->step_lo < 0 ? 0 : o->step_lo;
            uint64_t steps = 0;
            for (int i = lo; i <= hi; ++i) steps += (uint64_t)(s.N - i);
            stats->path_steps = steps * s.K * (uint64_t)o->M;
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            stats->ms_total = ms;
            stats->ms_steps = -1.f;
            if (!graph_used) {
                HIP_TRY(hipEventElapsedTime(&ms, s0, s1), "hipEventElapsedTime");
                stats->ms_steps = ms;
            }
            uint32_t per_step = 1;
            if (o->cv == SRMDP_CV_NONE) {
                LaunchShape ls;
                size_t per_cube;
                if (make_shape(s, nb, sizeof(R) == 4, o->M, lanes_for(o), ls, per_cube, false, o))
                    per_step = launches_per_step(s, ls);
            }
            stats->step_launches = (hi - lo + 1) * (int32_t)per_step;
            stats->near_face_paths = ctr[kCounterNearFace];
            stats->lanes_per_cube = lanes_for(o);
            if (o->cv == SRMDP_CV_ONLINE) {
                const int U = o->cv_train.updates_per_step;
                std::vector<float> loss((size_t)(hi - lo + 1) * U);
                HIP_TRY(hipMemcpy(loss.data(), ws + lay.cv_loss, loss.size() * sizeof(float),
                                  hipMemcpyDeviceToHost),
                        "loss copy");
                double first = 0.0, last = 0.0;
                for (int u = 0; u < U; ++u) {
                    first += loss[u];
                    last += loss[(size_t)(hi - lo) * U + u];
                }
                stats->cv_loss_first = (float)(first / U);
                stats->cv_loss_last = (float)(last / U);
            }
        }
        if ((o->flags & SRMDP_F_CHECK_FINITE) && ctr[kCounterNonFinite] != 0)
            return fail(SRMDP_E_NUMERIC, "%llu non-finite coefficients", ctr[kCounterNonFinite]);
    }
    return SRMDP_OK;
}

}  // namespace

namespace {
template <typename R>
srmdp_status root_impl(const srmdp_problem *p, const srmdp_grid *g, const srmdp_options *o,
                       const Shape &s, int nb, const void *table, const double *x0, int M_root,
                       double *y0, double *z0, unsigned char *ws, hipStream_t st)
{
    const int lk = lookup_mode(p);
    const Layout lay = layout(s, nb, sizeof(R) == 4, lk);
    StepArgs<R> a;
    fill_step_args<R>(a, p, g, s, o);
    a.i = 0;
    a.tag = (o->instance << 16);
    a.face_flags = nullptr;
    SetupArgs sa;
    SigmaHost sg;
    fill_setup_args(sa, sg, p, g, s);
    RootPoint rp{};
    for (int l = 0; l < s.d; ++l) rp.x[l] = x0[l];
    HIP_TRY(launch_setup<R>(sa, sg.v, ws + lay.cellF, ws + lay.bsig, st), "setup kernel");
    if (s.N > 1)
        HIP_TRY(launch_lookup_rows<R>(s.d, o->basis, lk, table, ws + lay.lookup, (uint32_t)s.K, 1, s.N - 1, st),
                "look-up rows");
    const int blocks = std::min(kRootBlocks, std::max(1, (M_root + 255) / 256));
    a.cell_table = ws + lay.cellF;
    HIP_TRY(launch_root<R>(s.d, o->basis, lk, a, ws + lay.bsig, ws + lay.lookup, rp, M_root, blocks,
                           (double *)(ws + lay.root_partial), (double *)(ws + lay.root_out), st),
            "root kernels");
    double out[SRMDP_MAX_D + 1];
    HIP_TRY(hipMemcpyAsync(out, ws + lay.root_out, sizeof(double) * (s.d + 1), hipMemcpyDeviceToHost, st),
            "root copy");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    *y0 = out[0];
    for (int l = 0; l < s.q; ++l) z0[l] = out[1 + l];
    return SRMDP_OK;
}

// ------------------------------------------------------------- autotuner
// Lanes per stratum, chosen by timing one backward step (the middle of the
// requested range, so that paths have the average length) with each
// candidate; results are cached per shape for the life of the process.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, int> g_tuned;

std::vector<int64_t> tune_key(const Shape &s, int nb, const srmdp_options *o, int lk)
{
    return {s.d, s.q, nb, o->prec, lk, o->M, (int64_t)s.K, s.N, o->cv != SRMDP_CV_NONE ? 1 : 0,
            o->cv_stride, o->basis};
}

bool lanes_valid(const srmdp_options *o, int L)
{
    int cap = 8;
    while (cap < o->M && cap < 256) cap *= 2;
    return L <= cap;
}

template <typename R>
srmdp_status tune_impl(const srmdp_problem *p, const srmdp_grid *g, const srmdp_options *o, const Shape &s, int nb,
                       void *table, unsigned char *ws, hipStream_t st, int *best, float *ms_out)
{
    const int lk = lookup_mode(p);
    const bool cv = o->cv != SRMDP_CV_NONE;
    const Layout lay = layout(s, nb, sizeof(R) == 4, lk, o);
    const int hi = o->step_hi < 0 ? s.N - 1 : o->step_hi;
    const int lo = o->step_lo < 0 ? 0 : o->step_lo;
    const int it = (hi + lo) / 2;
    StepArgs<R> a;
    fill_step_args<R>(a, p, g, s, o);
    a.i = it;
    a.tag = ((uint32_t)it & 0xFFFFu) | (o->instance << 16);
    a.face_flags = nullptr;
    SetupArgs sa;
    SigmaHost sg;
    fill_setup_args(sa, sg, p, g, s);
    HIP_TRY(launch_zero_u64((unsigned long long *)(ws + lay.counters), kCounterCount, st), "zero counters");
    HIP_TRY(launch_setup<R>(sa, sg.v, ws + lay.cellF, ws + lay.bsig, st), "setup kernel");
    if (it < s.N - 1)
        HIP_TRY(launch_lookup_rows<R>(s.d, o->basis, lk, table, ws + lay.lookup, (uint32_t)s.K, it + 1, s.N - 1, st),
                "look-up rows");
    if (cv) {
        a.cv_packed = ws + lay.cv_packed;
        HIP_TRY(launch_mlp_pack(s.d + 1, s.q, o->cv_params, ws + lay.cv_packed, st), "network pack");
    }
    EventSet ev;
    hipEvent_t &e0 = ev.e[0], &e1 = ev.e[1];
    HIP_TRY(ev.create(2), "hipEventCreate");
    const int cand[6] = {8, 16, 32, 64, 128, 256};
    float best_ms = 0.f;
    *best = 0;
    srmdp_status rc = SRMDP_OK;
    for (int c = 0; c < 6 && rc == SRMDP_OK; ++c) {
        if (ms_out) ms_out[c] = -1.f;
        const int L = cand[c];
        if (!lanes_valid(o, L)) continue;
        LaunchShape ls;
        size_t per_cube;
        if (!make_shape(s, nb, sizeof(R) == 4, o->M, L, ls, per_cube, cv, o)) continue;
        a.lanes = L;
        a.lds_per_cube = per_cube;
        auto launch = [&]() -> hipError_t {
            if constexpr (std::is_same<R, float>::value) {
                if (cv) {
                    a.cell_table = ws + lay.cellF;
                    return launch_step_cv(s.d, a, ls, o->basis, lk, ws + lay.cellF, ws + lay.bsig, ws + lay.lookup,
                                          table, ws + lay.counters, st);
                }
            }
            return launch_plain_step<R>(s, a, ls, o->basis, lk, ws, lay.cellF, lay.bsig, lay.lookup, lay.counters,
                                        lay.grows, table, st);
        };
        hipError_t e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune launch");
            break;
        }
        ms /= 3.f;
        if (ms_out) ms_out[c] = ms;
        if (*best == 0 || ms < best_ms) {
            *best = L;
            best_ms = ms;
        }
    }
    if (rc == SRMDP_OK && *best == 0) rc = fail(SRMDP_E_UNSUPPORTED, "no lanes-per-stratum candidate fits");
    return rc;
}

srmdp_status tune_cached(const srmdp_problem *p, const srmdp_grid *g, const srmdp_options *o, const Shape &s, int nb,
                         void *table, unsigned char *ws, hipStream_t st, int *best, float *ms_out, bool force)
{
    const auto key = tune_key(s, nb, o, lookup_mode(p));
    if (!force) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *best = it->second;
            return SRMDP_OK;
        }
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) return fail(SRMDP_E_INVALID, "the autotuner cannot run during capture");
    srmdp_status rc = o->prec == SRMDP_FP32 ? tune_impl<float>(p, g, o, s, nb, table, ws, st, best, ms_out)
                                            : tune_impl<double>(p, g, o, s, nb, table, ws, st, best, ms_out);
    if (rc == SRMDP_OK) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key] = *best;
    }
    return rc;
}

// ---------------------------------------------------------- batched sweep
struct BatchPlan {
    std::vector<int> order;      // instances sorted by N, descending
    std::vector<int> lanes;      // per instance
    std::vector<size_t> ws_off;  // per instance sub-workspace offset
    std::vector<Shape> shapes;
    size_t inst_bytes = 0, total = 0;
    int nb = 0, lk = 0, gmax = 0;
};

template <typename R>
size_t batch_inst_size() { return sizeof(BatchInstance<R>); }

srmdp_status plan_batch(int n, const srmdp_problem *P, const srmdp_grid *G, const srmdp_options *O, BatchPlan &bp)
{
    if (n < 1) return fail(SRMDP_E_INVALID, "a batch needs at least one instance");
    if (!P || !G || !O) return fail(SRMDP_E_INVALID, "problems, grids and options must be non-NULL");
    bp.shapes.resize(n);
    bp.lanes.resize(n);
    bp.ws_off.resize(n);
    for (int b = 0; b < n; ++b) {
        int nb;
        srmdp_status rc = check_problem(&P[b], &G[b], bp.shapes[b]);
        if (rc == SRMDP_OK) rc = check_options(&O[b], bp.shapes[b], nb);
        if (rc != SRMDP_OK) return fail(rc, "instance %d: %s", b, g_error.c_str());
        if (P[b].model) return fail(SRMDP_E_UNSUPPORTED, "instance %d: batches do not take a problem with a model", b);
        const int lk = lookup_mode(&P[b]);
        if (b == 0) {
            bp.nb = nb;
            bp.lk = lk;
        } else if (P[b].d != P[0].d || O[b].basis != O[0].basis || O[b].prec != O[0].prec || lk != bp.lk ||
                   bp.shapes[b].equal_prob != bp.shapes[0].equal_prob) {
            return fail(SRMDP_E_INVALID, "instance %d: a batch shares d, basis, precision, look-up mode and grid kind",
                        b);
        }
        if (O[b].cv != SRMDP_CV_NONE || O[b].face_flags || O[b].step_hi >= 0 || O[b].step_lo >= 0 ||
            (O[b].flags & SRMDP_F_DEBUG_SINGULAR))
            return fail(SRMDP_E_UNSUPPORTED, "instance %d: batches run plain full sweeps", b);
        bp.gmax = std::max(bp.gmax, P[b].N);
    }
    if (!lds_dimension_compiled(P[0].d))
        return fail(SRMDP_E_UNSUPPORTED, "d = %d is not compiled for batches", P[0].d);
    bp.order.resize(n);
    std::iota(bp.order.begin(), bp.order.end(), 0);
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](int x, int y) { return P[x].N > P[y].N; });
    const int is_float = O[0].prec == SRMDP_FP32;
    bp.inst_bytes = align_up((size_t)n * (is_float ? batch_inst_size<float>() : batch_inst_size<double>()), 256);
    size_t off = bp.inst_bytes;
    for (int b = 0; b < n; ++b) {
        bp.ws_off[b] = off;
        off += align_up(layout(bp.shapes[b], bp.nb, is_float, bp.lk, &O[b]).total, 256);
    }
    bp.total = off;
    return SRMDP_OK;
}

// Lanes per instance: explicit, tuned (cached per shape) or one lane per
// simulation up to 256.  A batch runs workgroups of 256 threads, each holding
// 256 / L strata, so that the LDS of a workgroup, about 256 (M / L) rows, stays
// similar across instances of very different M (the workgroup's LDS is the
// largest any instance needs).  Tuning runs kernels and synchronises, so it
// happens before any capture.
srmdp_status resolve_batch_lanes(int n, const srmdp_problem *P, const srmdp_grid *G, const srmdp_options *O,
                                 void *const *tables, unsigned char *ws, BatchPlan &bp, hipStream_t st)
{
    for (int b = 0; b < n; ++b) {
        int L = O[b].lanes_per_cube;
        if (L == 0 && (O[b].flags & SRMDP_F_AUTOTUNE)) {
            srmdp_options o = O[b];
            o.lanes_per_cube = 0;
            srmdp_status rc = tune_cached(&P[b], &G[b], &o, bp.shapes[b], bp.nb, tables[b], ws + bp.ws_off[b], st,
                                          &L, nullptr, false);
            if (rc != SRMDP_OK) return rc;
        }
        if (L == 0) {
            L = 8;
            while (L < O[b].M && L < 256) L *= 2;
        }
        bp.lanes[b] = L;
    }
    return SRMDP_OK;
}

template <typename R>
srmdp_status enqueue_batch(int n, const srmdp_problem *P, const srmdp_grid *G, const srmdp_options *O,
                           void *const *tables, unsigned char *ws, const BatchPlan &bp, hipStream_t st)
{
    const int is_float = sizeof(R) == 4;
    const unsigned threads = 256;
    std::vector<BatchInstance<R>> inst(n);
    size_t lds = 0;
    uint32_t first = 0;
    std::vector<uint32_t> prefix(n + 1, 0);
    for (int r = 0; r < n; ++r) {
        const int b = bp.order[r];
        const Shape &s = bp.shapes[b];
        const int L = bp.lanes[b];
        const int cpw = (int)threads / L;
        const size_t per_cube = align_up(cube_lds_bytes(is_float, s.d, bp.nb, O[b].M, false), 16);
        lds = std::max(lds, (size_t)cpw * per_cube);
        const Layout lay = layout(s, bp.nb, is_float, bp.lk, &O[b]);
        unsigned char *w = ws + bp.ws_off[b];
        BatchInstance<R> &I = inst[r];
        std::memset(&I, 0, sizeof I);
        fill_step_args<R>(I.a, &P[b], &G[b], s, &O[b]);
        I.a.lanes = L;
        I.a.lds_per_cube = per_cube;
        I.a.face_flags = nullptr;
        I.cellF = w + lay.cellF;
        I.a.cell_table = I.cellF;
        I.bsig = w + lay.bsig;
        I.lk = w + lay.lookup;
        I.table = tables[b];
        I.counters = w + lay.counters;
        I.first_item = first;
        I.items = (uint32_t)((s.K + cpw - 1) / cpw);
        I.instance = O[b].instance;
        first += I.items;
        prefix[r + 1] = first;
    }
    if (lds > 64 * 1024) return fail(SRMDP_E_UNSUPPORTED, "a batch instance does not fit the LDS budget");
    for (int b = 0; b < n; ++b) {
        const Layout lay = layout(bp.shapes[b], bp.nb, is_float, bp.lk, &O[b]);
        unsigned char *w = ws + bp.ws_off[b];
        SetupArgs sa;
        SigmaHost sg;
        fill_setup_args(sa, sg, &P[b], &G[b], bp.shapes[b]);
        HIP_TRY(launch_zero_u64((unsigned long long *)(w + lay.counters), kCounterCount, st), "zero counters");
        HIP_TRY(launch_setup<R>(sa, sg.v, w + lay.cellF, w + lay.bsig, st), "setup kernel");
    }
    HIP_TRY(launch_upload(ws, inst.data(), sizeof(BatchInstance<R>) * n, st), "instance upload");
    int active = n;
    for (int g = 0; g < bp.gmax; ++g) {
        TraceRange range("srmdp batched global step", g);
        while (active > 0 && P[bp.order[active - 1]].N <= g) --active;
        HIP_TRY(launch_batch_step<R>(P[0].d, O[0].basis, bp.lk, bp.shapes[0].equal_prob, ws, active, prefix[active], g,
                                     threads, lds, st),
                "batched step");
    }
    return SRMDP_OK;
}

template <typename R>
srmdp_status batch_impl(int n, const srmdp_problem *P, const srmdp_grid *G, const srmdp_options *O,
                        void *const *tables, unsigned char *ws, BatchPlan &bp, srmdp_stats *stats, hipStream_t st)
{
    srmdp_status rc = resolve_batch_lanes(n, P, G, O, tables, ws, bp, st);
    if (rc != SRMDP_OK) return rc;
    EventSet ev;
    hipEvent_t &e0 = ev.e[0], &e1 = ev.e[1];
    if (stats) {
        HIP_TRY(ev.create(2), "hipEventCreate");
        HIP_TRY(hipEventRecord(e0, st), "hipEventRecord");
    }
    if ((O[0].flags & SRMDP_F_GRAPH) && st != nullptr) {
        std::vector<unsigned char> key;
        auto put = [&](const void *v, size_t sz) {
            key.insert(key.end(), (const unsigned char *)v, (const unsigned char *)v + sz);
        };
        const char tagb[] = "batch";
        put(tagb, sizeof tagb);
        for (int b = 0; b < n; ++b) {
            put(&P[b], sizeof P[b]);
            if (P[b].b) put(P[b].b, sizeof(double) * P[b].d);
            if (P[b].sigma) put(P[b].sigma, sizeof(double) * P[b].d * P[b].q);
            if (P[b].b_lin) put(P[b].b_lin, sizeof(double) * P[b].d);
            if (P[b].sigma_lin) put(P[b].sigma_lin, sizeof(double) * P[b].d);
            put(&G[b].kind, sizeof G[b].kind);
            if (G[b].kind == SRMDP_GRID_EQUAL_SIZE) {
                put(G[b].lo, sizeof(double) * P[b].d);
                put(G[b].hi, sizeof(double) * P[b].d);
            }
            put(G[b].cells, sizeof(int32_t) * P[b].d);
            put(&G[b].mu, sizeof G[b].mu);
            put(&O[b], sizeof O[b]);
            put(&tables[b], sizeof tables[b]);
            put(&bp.lanes[b], sizeof bp.lanes[b]);
        }
        put(&ws, sizeof ws);
        const std::string k = graph_key(key.data(), key.size(), st);
        std::lock_guard<std::mutex> lock(g_graph_mu);
        auto it = g_graphs.find(k);
        if (it == g_graphs.end()) {
            GraphEntry ent;
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            rc = enqueue_batch<R>(n, P, G, O, tables, ws, bp, st);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &graph);
            if (rc != SRMDP_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
            ent.graph = graph;
            HIP_TRY(hipGraphInstantiate(&ent.exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            it = g_graphs.emplace(k, ent).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.exec, st), "hipGraphLaunch");
    } else {
        rc = enqueue_batch<R>(n, P, G, O, tables, ws, bp, st);
        if (rc != SRMDP_OK) return rc;
    }
    if (stats) {
        HIP_TRY(hipEventRecord(e1, st), "hipEventRecord");
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        const int is_float = sizeof(R) == 4;
        for (int b = 0; b < n; ++b) {
            const Layout lay = layout(bp.shapes[b], bp.nb, is_float, bp.lk, &O[b]);
            unsigned long long ctr[kCounterCount] = {0, 0, 0, 0};
            HIP_TRY(hipMemcpy(ctr, ws + bp.ws_off[b] + lay.counters, sizeof ctr, hipMemcpyDeviceToHost), "counters");
            std::memset(&stats[b], 0, sizeof stats[b]);
            stats[b].singular_cubes = ctr[kCounterSingular];
            stats[b].path_steps = (uint64_t)bp.shapes[b].N * (bp.shapes[b].N + 1) / 2 * bp.shapes[b].K * (uint64_t)O[b].M;
            stats[b].ms_total = ms;
            stats[b].ms_steps = -1.f;
            stats[b].step_launches = bp.gmax;
            stats[b].lanes_per_cube = bp.lanes[b];
        }
    }
    return SRMDP_OK;
}

}  // namespace

// ===================================================================== ABI

extern "C" {

int32_t srmdp_abi_version(void) { return 108; }

const char *srmdp_last_error(void) { return g_error.c_str(); }

size_t srmdp_table_elems(const srmdp_problem *problem, const srmdp_grid *grid, int32_t basis)
{
    Shape s;
    if (check_problem(problem, grid, s) != SRMDP_OK) return 0;
    if (basis != SRMDP_LP0 && basis != SRMDP_LP1) return 0;
    const int nb = basis == SRMDP_LP1 ? s.d + 1 : 1;
    return (size_t)s.N * s.K * (1 + s.q) * nb;
}

size_t srmdp_workspace_bytes(const srmdp_problem *problem, const srmdp_grid *grid,
                             const srmdp_options *opts)
{
    Shape s;
    int nb;
    if (check_problem(problem, grid, s) != SRMDP_OK) return 0;
    if (check_options(opts, s, nb) != SRMDP_OK) return 0;
    return layout(s, nb, opts->prec == SRMDP_FP32, lookup_mode(problem), opts).total;
}

srmdp_status srmdp_solve(const srmdp_problem *problem, const srmdp_grid *grid,
                         const srmdp_options *opts, void *table, void *workspace, size_t ws_bytes,
                         srmdp_stats *stats, void *stream)
{
    g_error.clear();
    Shape s;
    int nb;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    rc = check_options(opts, s, nb);
    if (rc != SRMDP_OK) return rc;
    if (!table || !workspace) return fail(SRMDP_E_INVALID, "table and workspace must be non-NULL");
    const size_t need = layout(s, nb, opts->prec == SRMDP_FP32, lookup_mode(problem), opts).total;
    if (ws_bytes < need)
        return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!problem->model) {  // a model's kernels are compiled for it (model_supported below)
        rc = sweep_supported(s, opts, lookup_mode(problem));
        if (rc != SRMDP_OK) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    srmdp_options o = *opts;
    ModelKernels mk;
    const ModelKernels *mkp = nullptr;
    if (problem->model) {
        bool streamed = false;
        rc = model_supported(s, nb, opts, &streamed);
        if (rc != SRMDP_OK) return rc;
        rc = model_kernels(problem->model, s.d, nb, opts->prec == SRMDP_FP32, s.equal_prob, streamed, mk);
        if (rc != SRMDP_OK) return rc;
        mkp = &mk;
    }
    if ((o.flags & SRMDP_F_AUTOTUNE) && o.lanes_per_cube == 0) {
        int L = 0;
        rc = tune_cached(problem, grid, &o, s, nb, table, (unsigned char *)workspace, st, &L, nullptr, false);
        if (rc != SRMDP_OK) return rc;
        o.lanes_per_cube = L;
    }
    if (o.prec == SRMDP_FP32) return solve_impl<float>(problem, grid, &o, s, nb, table, workspace, stats, st, mkp);
    return solve_impl<double>(problem, grid, &o, s, nb, table, workspace, stats, st, mkp);
}

srmdp_status srmdp_tune_lanes(const srmdp_problem *problem, const srmdp_grid *grid, const srmdp_options *opts,
                              void *table, void *workspace, size_t ws_bytes, int32_t *lanes, float *ms,
                              void *stream)
{
    g_error.clear();
    Shape s;
    int nb;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    if (problem->model) return fail(SRMDP_E_UNSUPPORTED, "srmdp_tune_lanes does not take a problem with a model");
    rc = check_options(opts, s, nb);
    if (rc != SRMDP_OK) return rc;
    if (!table || !workspace || !lanes) return fail(SRMDP_E_INVALID, "table, workspace and lanes are required");
    const size_t need = layout(s, nb, opts->prec == SRMDP_FP32, lookup_mode(problem), opts).total;
    if (ws_bytes < need) return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    rc = sweep_supported(s, opts, lookup_mode(problem));
    if (rc != SRMDP_OK) return rc;
    int L = 0;
    rc = tune_cached(problem, grid, opts, s, nb, table, (unsigned char *)workspace, (hipStream_t)stream, &L, ms,
                     true);
    if (rc != SRMDP_OK) return rc;
    *lanes = L;
    return SRMDP_OK;
}

size_t srmdp_workspace_bytes_batch(int32_t n, const srmdp_problem *problems, const srmdp_grid *grids,
                                   const srmdp_options *opts)
{
    BatchPlan bp;
    if (plan_batch(n, problems, grids, opts, bp) != SRMDP_OK) return 0;
    return bp.total;
}

srmdp_status srmdp_solve_batch(int32_t n, const srmdp_problem *problems, const srmdp_grid *grids,
                               const srmdp_options *opts, void *const *tables, void *workspace, size_t ws_bytes,
                               srmdp_stats *stats, void *stream)
{
    g_error.clear();
    BatchPlan bp;
    srmdp_status rc = plan_batch(n, problems, grids, opts, bp);
    if (rc != SRMDP_OK) return rc;
    if (!tables || !workspace) return fail(SRMDP_E_INVALID, "tables and workspace must be non-NULL");
    for (int b = 0; b < n; ++b)
        if (!tables[b]) return fail(SRMDP_E_INVALID, "table %d is NULL", b);
    if (ws_bytes < bp.total) return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, bp.total);
    hipStream_t st = (hipStream_t)stream;
    unsigned char *ws = (unsigned char *)workspace;
    if (opts[0].prec == SRMDP_FP32) return batch_impl<float>(n, problems, grids, opts, tables, ws, bp, stats, st);
    return batch_impl<double>(n, problems, grids, opts, tables, ws, bp, stats, st);
}

srmdp_status srmdp_eval(const srmdp_problem *problem, const srmdp_grid *grid, int32_t basis,
                        int32_t prec, const void *table, int32_t i, const double *x, int64_t n,
                        double *y, double *z, void *stream)
{
    g_error.clear();
    Shape s;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    if (basis != SRMDP_LP0 && basis != SRMDP_LP1) return fail(SRMDP_E_INVALID, "unknown basis");
    if (prec != SRMDP_FP64 && prec != SRMDP_FP32) return fail(SRMDP_E_INVALID, "unknown precision");
    if (i < 0 || i >= s.N) return fail(SRMDP_E_INVALID, "row %d outside 0..%d", i, s.N - 1);
    if (n < 0) return fail(SRMDP_E_INVALID, "n < 0");
    if (n == 0) return SRMDP_OK;
    if (!table || !x || (!y && !z)) return fail(SRMDP_E_INVALID, "table, x and one output are required");
    if (!dimension_compiled(s.d)) return fail(SRMDP_E_UNSUPPORTED, "d = %d is not compiled", s.d);
    hipStream_t st = (hipStream_t)stream;
    if (prec == SRMDP_FP32) {
        StepArgs<float> a;
        fill_step_args<float>(a, problem, grid, s, nullptr);
        a.i = i;
        HIP_TRY(launch_eval<float>(s.d, basis, a, table, x, n, y, z, st), "eval kernel");
    } else {
        StepArgs<double> a;
        fill_step_args<double>(a, problem, grid, s, nullptr);
        a.i = i;
        HIP_TRY(launch_eval<double>(s.d, basis, a, table, x, n, y, z, st), "eval kernel");
    }
    return SRMDP_OK;
}


srmdp_status srmdp_to_raw_basis(const srmdp_problem *problem, const srmdp_grid *grid, int32_t basis,
                                int32_t prec, const void *table, void *raw, void *stream)
{
    g_error.clear();
    Shape s;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    if (basis != SRMDP_LP0 && basis != SRMDP_LP1) return fail(SRMDP_E_INVALID, "unknown basis");
    if (prec != SRMDP_FP64 && prec != SRMDP_FP32) return fail(SRMDP_E_INVALID, "unknown precision");
    if (!table || !raw) return fail(SRMDP_E_INVALID, "table and raw are required");
    hipStream_t st = (hipStream_t)stream;
    const size_t rsz = prec == SRMDP_FP32 ? 4 : 8;
    if (basis == SRMDP_LP0) {  // (1) is its own raw basis
        if (raw != table)
            HIP_TRY(hipMemcpyAsync(raw, table, (size_t)s.N * s.K * (1 + s.q) * rsz, hipMemcpyDeviceToDevice, st),
                    "hipMemcpyAsync");
        return SRMDP_OK;
    }
    if (prec == SRMDP_FP32) {
        StepArgs<float> a;
        fill_step_args<float>(a, problem, grid, s, nullptr);
        HIP_TRY(launch_raw_basis<float>(s.d, s.q, a, table, raw, st), "raw-basis kernel");
    } else {
        StepArgs<double> a;
        fill_step_args<double>(a, problem, grid, s, nullptr);
        HIP_TRY(launch_raw_basis<double>(s.d, s.q, a, table, raw, st), "raw-basis kernel");
    }
    return SRMDP_OK;
}

srmdp_status srmdp_root(const srmdp_problem *problem, const srmdp_grid *grid, const srmdp_options *opts,
                        const void *table, const double *x0, int32_t M_root, double *y0, double *z0,
                        void *workspace, size_t ws_bytes, void *stream)
{
    g_error.clear();
    Shape s;
    int nb;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    if (problem->model) return fail(SRMDP_E_UNSUPPORTED, "srmdp_root does not take a problem with a model");
    rc = check_options(opts, s, nb);
    if (rc != SRMDP_OK) return rc;
    if (!table || !x0 || !y0 || !z0 || !workspace)
        return fail(SRMDP_E_INVALID, "table, x0, y0, z0 and workspace are required");
    if (M_root < 1) return fail(SRMDP_E_INVALID, "M_root must be >= 1");
    for (int l = 0; l < s.d; ++l)
        if (!std::isfinite(x0[l])) return fail(SRMDP_E_INVALID, "x0 must be finite");
    const size_t need = layout(s, nb, opts->prec == SRMDP_FP32, lookup_mode(problem), opts).total;
    if (ws_bytes < need) return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!dimension_compiled(s.d)) return fail(SRMDP_E_UNSUPPORTED, "d = %d is not compiled", s.d);
    hipStream_t st = (hipStream_t)stream;
    if (opts->prec == SRMDP_FP32)
        return root_impl<float>(problem, grid, opts, s, nb, table, x0, M_root, y0, z0,
                                (unsigned char *)workspace, st);
    return root_impl<double>(problem, grid, opts, s, nb, table, x0, M_root, y0, z0,
                             (unsigned char *)workspace, st);
}

srmdp_status srmdp_cv_pairs(const srmdp_problem *problem, const srmdp_grid *grid, const srmdp_options *opts,
                            const void *table, int32_t i, int64_t n, float *x16, float *z16, void *workspace,
                            size_t ws_bytes, void *stream)
{
    g_error.clear();
    Shape s;
    int nb;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    if (problem->model) return fail(SRMDP_E_UNSUPPORTED, "srmdp_cv_pairs does not take a problem with a model");
    rc = check_options(opts, s, nb);
    if (rc != SRMDP_OK) return rc;
    if (opts->prec != SRMDP_FP32) return fail(SRMDP_E_UNSUPPORTED, "training pairs come from binary32 tables");
    if (i < 0 || i >= s.N) return fail(SRMDP_E_INVALID, "step %d outside 0..%d", i, s.N - 1);
    if (n < 0 || n > 0xFFFFFFFFll) return fail(SRMDP_E_INVALID, "n outside 0..2^32-1");
    if (s.d + 1 > kMlpMaxIn || s.q > kMlpMaxOut) return fail(SRMDP_E_UNSUPPORTED, "d + 1 > %d", kMlpMaxIn);
    if (!table || !x16 || !z16 || !workspace) return fail(SRMDP_E_INVALID, "table, x16, z16 and workspace are required");
    const size_t need = layout(s, nb, 1, lookup_mode(problem), opts).total;
    if (ws_bytes < need) return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!cv_dimension_compiled(s.d)) return fail(SRMDP_E_UNSUPPORTED, "d = %d is not compiled", s.d);
    if (n == 0) return SRMDP_OK;
    hipStream_t st = (hipStream_t)stream;
    const Layout lay = layout(s, nb, 1, lookup_mode(problem), opts);
    unsigned char *ws = (unsigned char *)workspace;
    SetupArgs sa;
    SigmaHost sg;
    fill_setup_args(sa, sg, problem, grid, s);
    StepArgs<float> a;
    fill_step_args<float>(a, problem, grid, s, opts);
    a.i = i;
    a.tag = ((uint32_t)i & 0xFFFFu) | (opts->instance << 16);
    HIP_TRY(launch_setup<float>(sa, sg.v, ws + lay.cellF, ws + lay.bsig, st), "setup kernel");
    HIP_TRY(launch_cv_pairs(s.d, opts->basis, a, ws + lay.cellF, table, n, x16, z16, st), "training pairs");
    return SRMDP_OK;
}

int64_t srmdp_mlp_param_count(int32_t in, int32_t out)
{
    if (in < 1 || in > kMlpMaxIn || out < 1 || out > kMlpMaxOut) return 0;
    return MlpShape{in, out}.count();
}

size_t srmdp_mlp_packed_bytes(void) { return kPackedBytes; }

static srmdp_status check_net(int32_t in, int32_t out)
{
    if (in < 1 || in > kMlpMaxIn || out < 1 || out > kMlpMaxOut)
        return fail(SRMDP_E_INVALID, "network shape %d -> %d outside 1..%d -> 1..%d", in, out, kMlpMaxIn,
                    kMlpMaxOut);
    return SRMDP_OK;
}

srmdp_status srmdp_mlp_init(int32_t in, int32_t out, uint64_t seed, int32_t zero_output_layer, float *params,
                            void *stream)
{
    g_error.clear();
    srmdp_status rc = check_net(in, out);
    if (rc != SRMDP_OK) return rc;
    if (!params) return fail(SRMDP_E_INVALID, "params must be non-NULL");
    HIP_TRY(launch_mlp_init(in, out, seed, zero_output_layer, params, (hipStream_t)stream), "network init");
    return SRMDP_OK;
}

srmdp_status srmdp_mlp_pack(int32_t in, int32_t out, const float *params, void *packed, void *stream)
{
    g_error.clear();
    srmdp_status rc = check_net(in, out);
    if (rc != SRMDP_OK) return rc;
    if (!params || !packed) return fail(SRMDP_E_INVALID, "params and packed must be non-NULL");
    HIP_TRY(launch_mlp_pack(in, out, params, packed, (hipStream_t)stream), "network pack");
    return SRMDP_OK;
}

srmdp_status srmdp_mlp_forward(int32_t in, int32_t out, const void *packed, const float *x, int64_t n, float *y,
                               void *stream)
{
    g_error.clear();
    srmdp_status rc = check_net(in, out);
    if (rc != SRMDP_OK) return rc;
    if (n < 0) return fail(SRMDP_E_INVALID, "n < 0");
    if (n == 0) return SRMDP_OK;
    if (!packed || !x || !y) return fail(SRMDP_E_INVALID, "packed, x and y must be non-NULL");
    HIP_TRY(launch_mlp_forward(in, out, packed, x, n, y, (hipStream_t)stream), "network forward");
    return SRMDP_OK;
}

size_t srmdp_mlp_backward_workspace(int32_t in, int32_t out, int64_t n)
{
    if (check_net(in, out) != SRMDP_OK || n < 0) return 0;
    return std::max<size_t>(1, mlp_backward_partials(n)) * (size_t)MlpShape{in, out}.count() * sizeof(float);
}

srmdp_status srmdp_mlp_backward(int32_t in, int32_t out, const void *packed, const float *x, const float *dy,
                                int64_t n, float *grad, void *workspace, size_t ws_bytes, void *stream)
{
    g_error.clear();
    srmdp_status rc = check_net(in, out);
    if (rc != SRMDP_OK) return rc;
    if (n < 0) return fail(SRMDP_E_INVALID, "n < 0");
    if (!packed || !grad || (n > 0 && (!x || !dy)) || !workspace)
        return fail(SRMDP_E_INVALID, "packed, x, dy, grad and workspace must be non-NULL");
    const size_t need = srmdp_mlp_backward_workspace(in, out, n);
    if (ws_bytes < need) return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        HIP_TRY(launch_zero_f32(grad, MlpShape{in, out}.count(), st), "zero gradient");
        return SRMDP_OK;
    }
    HIP_TRY(launch_mlp_backward(in, out, packed, x, dy, n, (float *)workspace, grad, st), "network backward");
    return SRMDP_OK;
}

size_t srmdp_mlp_train_workspace_bytes(int32_t in, int32_t out, const srmdp_mlp_train_config *cfg)
{
    if (check_net(in, out) != SRMDP_OK || !cfg || cfg->batch < 256 || cfg->batch > 65536 || cfg->batch % 256 != 0)
        return 0;
    return mlp_train_partial_bytes(in, out, cfg->batch);
}

srmdp_status srmdp_mlp_train(int32_t in, int32_t out, float *params, float *adam_m, float *adam_v, int64_t adam_t0,
                             const float *x16, const float *z16, int64_t n, const srmdp_mlp_train_config *cfg,
                             void *packed_out, float *loss, void *workspace, size_t ws_bytes, void *stream)
{
    g_error.clear();
    srmdp_status rc = check_net(in, out);
    if (rc != SRMDP_OK) return rc;
    if (!params || !adam_m || !adam_v || !x16 || !z16 || !cfg || !packed_out || !workspace)
        return fail(SRMDP_E_INVALID, "params, adam_m, adam_v, x16, z16, cfg, packed_out and workspace are required");
    if (n < 64 || n % 64 != 0) return fail(SRMDP_E_INVALID, "n must be a positive multiple of 64");
    if (adam_t0 < 0) return fail(SRMDP_E_INVALID, "adam_t0 < 0");
    if (((uintptr_t)x16 | (uintptr_t)z16) % 16 != 0) return fail(SRMDP_E_INVALID, "x16 and z16 must be 16-byte aligned");
    if (cfg->updates_per_step < 1 || cfg->updates_per_step > 4096)
        return fail(SRMDP_E_INVALID, "updates_per_step outside 1..4096");
    if (cfg->batch < 256 || cfg->batch > 65536 || cfg->batch % 256 != 0)
        return fail(SRMDP_E_INVALID, "batch must be a multiple of 256 up to 65536");
    if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f))
        return fail(SRMDP_E_INVALID, "Adam needs lr > 0, betas in [0, 1) and eps > 0");
    if (ws_bytes < mlp_train_partial_bytes(in, out, cfg->batch))
        return fail(SRMDP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes,
                    mlp_train_partial_bytes(in, out, cfg->batch));
    MlpTrainArgs t{};
    t.in = in;
    t.out = out;
    t.theta = params;
    t.adam_m = adam_m;
    t.adam_v = adam_v;
    t.adam_t0 = adam_t0;
    t.x16 = x16;
    t.z16 = z16;
    t.S = n;
    t.updates = cfg->updates_per_step;
    t.batch = cfg->batch;
    t.lr = cfg->lr;
    t.beta1 = cfg->beta1;
    t.beta2 = cfg->beta2;
    t.eps = cfg->eps;
    t.packed_out = (unsigned char *)packed_out;
    t.loss = loss;
    const hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_mlp_pack(in, out, params, packed_out, st), "network pack");
    HIP_TRY(launch_mlp_train(t, (float *)workspace, st), "network training");
    return SRMDP_OK;
}

srmdp_status srmdp_draw(const srmdp_problem *problem, const srmdp_grid *grid, const srmdp_options *opts,
                        int32_t kind, int32_t i, uint32_t k0, uint32_t nk, uint32_t m0, uint32_t nm,
                        int32_t count, double *out, void *stream)
{
    g_error.clear();
    Shape s;
    int nb;
    srmdp_status rc = check_problem(problem, grid, s);
    if (rc != SRMDP_OK) return rc;
    rc = check_options(opts, s, nb);
    if (rc != SRMDP_OK) return rc;
    if (kind < 0 || kind > 2) return fail(SRMDP_E_INVALID, "kind must be 0, 1 or 2");
    if (i < 0 || i >= s.N) return fail(SRMDP_E_INVALID, "step %d outside 0..%d", i, s.N - 1);
    if (count < 1 || (kind == 2 && count != s.d)) return fail(SRMDP_E_INVALID, "bad count");
    if (kind == 2 && ((uint64_t)k0 + nk > s.K)) return fail(SRMDP_E_INVALID, "strata outside the grid");
    if (!out) return fail(SRMDP_E_INVALID, "out must be non-NULL");
    if ((uint64_t)nk * nm == 0) return SRMDP_OK;
    if (!dimension_compiled(s.d)) return fail(SRMDP_E_UNSUPPORTED, "d = %d is not compiled", s.d);
    hipStream_t st = (hipStream_t)stream;
    SetupArgs sa;
    SigmaHost sg;
    fill_setup_args(sa, sg, problem, grid, s);
    if (opts->prec == SRMDP_FP32) {
        StepArgs<float> a;
        fill_step_args<float>(a, problem, grid, s, opts);
        a.i = i;
        a.tag = ((uint32_t)i & 0xFFFFu) | (opts->instance << 16);
        HIP_TRY(launch_draw<float>(s.d, a, sa, kind, k0, nk, m0, nm, count, out, st), "draw kernel");
    } else {
        StepArgs<double> a;
        fill_step_args<double>(a, problem, grid, s, opts);
        a.i = i;
        a.tag = ((uint32_t)i & 0xFFFFu) | (opts->instance << 16);
        HIP_TRY(launch_draw<double>(s.d, a, sa, kind, k0, nk, m0, nm, count, out, st), "draw kernel");
    }
    return SRMDP_OK;
}

void srmdp_release_graphs(void)
{
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto &kv : g_graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
}

}  // extern "C"
