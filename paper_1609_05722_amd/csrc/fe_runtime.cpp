// Host runtime behind include/fe.h: argument validation, workspace layout,
// filter-bank upload and the launch sequence of the denoising scheme
// (eq. 3.7: Anscombe transform, iPiano iterations, closed-form inverse).
#include "fe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "fe_internal.h"
#include "fe_plan.h"

struct fe_ctx {
    int device = 0;
    int m = 0, nf = 0;
    std::vector<float> taps, alpha;  // host copies
    fe::FusedBank fused;             // matrix-core operand tables
    mutable fe::TuneTable tune;      // measured tile shapes (internally locked)
};

namespace {

thread_local std::string g_error;

fe_status fail(fe_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

fe_status hip_fail(hipError_t e, const char *what)
{
    return fail(FE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Keeps the caller's current device across a call.
struct DeviceGuard {
    int saved = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&saved) != hipSuccess) saved = -1;
        if (saved != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (saved >= 0 && hipGetDevice(&cur) == hipSuccess && cur != saved)
            (void)hipSetDevice(saved);
    }
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int radius(const fe_ctx *c) { return (c->m - 1) / 2; }

fe_status check_job(const fe_ctx *c, const fe_job &j, int idx)
{
    const int r = radius(c);
    if (j.height < 1 || j.width < 1 || j.height < r || j.width < r)
        return fail(FE_ERR_INVALID, "job %d: image %dx%d smaller than the filter radius %d",
                    idx, j.height, j.width, r);
    if ((long long)j.height * j.width > (1LL << 31) - 1)
        return fail(FE_ERR_INVALID, "job %d: image too large", idx);
    if (!j.counts) return fail(FE_ERR_INVALID, "job %d: counts is NULL", idx);
    if (!(j.lambda > 0.0f) || !std::isfinite(j.lambda))
        return fail(FE_ERR_INVALID, "job %d: lambda must be finite and > 0", idx);
    if (!(j.tau > 0.0f) || !std::isfinite(j.tau))
        return fail(FE_ERR_INVALID, "job %d: tau must be finite and > 0", idx);
    if (!(j.gamma >= 0.0f && j.gamma < 1.0f))
        return fail(FE_ERR_INVALID, "job %d: gamma must be in [0, 1)", idx);
    if (j.iterations < 0) return fail(FE_ERR_INVALID, "job %d: negative iteration count", idx);
    if (j.data_term != FE_DATA_AUTO && j.data_term != FE_DATA_QUADRATIC &&
        j.data_term != FE_DATA_IDIV)
        return fail(FE_ERR_INVALID, "job %d: unknown data term %d", idx, j.data_term);
    if (j.data_term == FE_DATA_AUTO && !std::isfinite(j.peak))
        return fail(FE_ERR_INVALID, "job %d: peak must be finite with FE_DATA_AUTO", idx);
    if (j.precision != FE_PREC_FP32 && j.precision != FE_PREC_BF16 &&
        j.precision != FE_PREC_FP16)
        return fail(FE_ERR_INVALID, "job %d: unknown precision %d", idx, j.precision);
    return FE_OK;
}

fe_status check_batch(const fe_ctx *c, const fe_job *jobs, int32_t n)
{
    if (!c) return fail(FE_ERR_INVALID, "ctx is NULL");
    if (n < 0) return fail(FE_ERR_INVALID, "negative job count");
    if (n > 0 && !jobs) return fail(FE_ERR_INVALID, "jobs is NULL");
    for (int i = 0; i < n; ++i) {
        fe_status st = check_job(c, jobs[i], i);
        if (st != FE_OK) return st;
    }
    return FE_OK;
}

size_t state_bytes(int H, int W) { return 2 * (size_t)H * W * sizeof(float); }

// Workspace of fe_denoise: [job table][state of job 0][state of job 1]...
struct DenoiseLayout {
    size_t table_bytes = 0;
    std::vector<size_t> state_off;
    size_t total = 0;
};

DenoiseLayout layout_for(const fe_job *jobs, int32_t n)
{
    DenoiseLayout L;
    L.table_bytes = align256(fe::fused_table_bytes(n));
    size_t off = L.table_bytes;
    L.state_off.resize(n);
    for (int i = 0; i < n; ++i) {
        L.state_off[i] = off;
        off += align256(state_bytes(jobs[i].height, jobs[i].width));
    }
    L.total = std::max<size_t>(off, 256);
    return L;
}

fe_status check_workspace(void *ws, size_t ws_bytes, size_t need)
{
    if (!ws) return fail(FE_ERR_INVALID, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(FE_ERR_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(FE_ERR_INVALID, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    return FE_OK;
}

fe_status check_states(const fe_job *jobs, float *const *states, int32_t n)
{
    if (n > 0 && !states) return fail(FE_ERR_INVALID, "states is NULL");
    for (int i = 0; i < n; ++i)
        if (!states[i]) return fail(FE_ERR_INVALID, "state %d is NULL", i);
    (void)jobs;
    return FE_OK;
}

// v = f_A(y) into both planes of every state (u^0 = u^{-1} = v).
fe_status enqueue_begin(const fe_job *jobs, float *const *states, int32_t n, hipStream_t s)
{
    for (int i = 0; i < n; ++i) {
        const long plane = (long)jobs[i].height * jobs[i].width;
        hipError_t e = fe::launch_anscombe_init(jobs[i].counts, states[i], states[i] + plane,
                                                plane, s);
        if (e != hipSuccess) return hip_fail(e, "anscombe init");
    }
    return FE_OK;
}

fe_status enqueue_end(const fe_job *jobs, float *const *states, const int32_t *done, int32_t n,
                      hipStream_t s)
{
    for (int i = 0; i < n; ++i) {
        const long plane = (long)jobs[i].height * jobs[i].width;
        const float *u = states[i] + ((done[i] & 1) ? plane : 0);
        hipError_t e = fe::launch_inverse_anscombe(u, jobs[i].out, jobs[i].out_anscombe, plane, s);
        if (e != hipSuccess) return hip_fail(e, "inverse anscombe");
    }
    return FE_OK;
}

// Debug mode (environment FE_VALIDATE=1): before the counts are used, a
// device pass rejects negative, NaN or infinite values.  It allocates a few
// flags, synchronises the stream and is skipped while the stream is being
// captured into a graph.
bool validation_enabled()
{
    const char *v = std::getenv("FE_VALIDATE");
    return v && v[0] == '1' && v[1] == 0;
}

fe_status validate_counts(const float *const *planes, const long *sizes, int n, hipStream_t s)
{
    if (!validation_enabled() || n <= 0) return FE_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return FE_OK;
    int *flags = nullptr;
    hipError_t e = hipMalloc((void **)&flags, sizeof(int) * n);
    if (e != hipSuccess) return hip_fail(e, "validation flags");
    std::vector<int> h(n, 0);
    e = fe::launch_zero_ints(flags, n, s);
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = fe::launch_check_counts(planes[i], sizes[i], flags + i, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), flags, sizeof(int) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(flags);
    if (e != hipSuccess) return hip_fail(e, "validation");
    for (int i = 0; i < n; ++i)
        if (h[i]) return fail(FE_ERR_INVALID, "job %d: counts hold a negative, NaN or infinite value", i);
    return FE_OK;
}

fe_status validate_jobs(const fe_job *jobs, int n, hipStream_t s)
{
    if (!validation_enabled()) return FE_OK;
    std::vector<const float *> planes(n);
    std::vector<long> sizes(n);
    for (int i = 0; i < n; ++i) {
        planes[i] = jobs[i].counts;
        sizes[i] = (long)jobs[i].height * jobs[i].width;
    }
    return validate_counts(planes.data(), sizes.data(), n, s);
}

fe_status enqueue_advance(const fe_ctx *c, const fe_job *jobs, float *const *states,
                          const int32_t *done, const int32_t *count, int32_t n, void *table,
                          hipStream_t s)
{
    std::vector<fe::AdvanceItem> items(n);
    for (int i = 0; i < n; ++i) items[i] = {&jobs[i], states[i], done[i], count[i]};
    hipError_t e = fe::run_fused(c->fused, items.data(), n, table, s, &c->tune);
    if (e != hipSuccess) return hip_fail(e, "fused step");
    return FE_OK;
}

}  // namespace

fe_status fe::validate_job_counts(int device, const fe_job *jobs, int n)
{
    if (!validation_enabled() || n <= 0) return FE_OK;
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return validate_jobs(jobs, n, nullptr);
}

extern "C" {

const char *fe_last_error(void) { return g_error.c_str(); }

fe_status fe_create(const fe_prior *prior, int device, fe_ctx **out)
{
    if (!out) return fail(FE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!prior || !prior->filters || !prior->weights)
        return fail(FE_ERR_INVALID, "prior, filters and weights must be non-NULL");
    const int m = prior->m, nf = prior->n_filters;
    if (m != 3 && m != 5 && m != 7)
        return fail(FE_ERR_UNSUPPORTED, "filter side %d not built (3, 5, 7)", m);
    if (nf < 1 || nf > fe::kMaxFilters)
        return fail(FE_ERR_UNSUPPORTED, "filter count %d outside 1..%d", nf, fe::kMaxFilters);
    for (int i = 0; i < nf; ++i)
        if (!(prior->weights[i] >= 0.0f) || !std::isfinite(prior->weights[i]))
            return fail(FE_ERR_INVALID, "weight %d must be finite and >= 0", i);
    for (int i = 0; i < nf * m * m; ++i)
        if (!std::isfinite(prior->filters[i]))
            return fail(FE_ERR_INVALID, "filter tap %d is not finite", i);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(FE_ERR_INVALID, "device %d not available", device);

    fe_ctx *c = new (std::nothrow) fe_ctx;
    if (!c) return fail(FE_ERR_NOMEM, "host allocation failed");
    c->device = device;
    c->m = m;
    c->nf = nf;
    c->taps.assign(prior->filters, prior->filters + (size_t)nf * m * m);
    c->alpha.assign(prior->weights, prior->weights + nf);

    DeviceGuard g(device);
    if (g.err != hipSuccess) {
        delete c;
        return hip_fail(g.err, "hipSetDevice");
    }
    hipError_t e = fe::fused_upload(c->taps.data(), c->alpha.data(), m, nf, &c->fused);
    // the device address of fe_advance_noalloc's static job table (once
    // per device, with the device current)
    if (e == hipSuccess) e = fe::noalloc_setup(device);
    if (e != hipSuccess) {
        fe_status st = e == hipErrorOutOfMemory ? fail(FE_ERR_NOMEM, "device allocation failed")
                                                : hip_fail(e, "fe_create upload");
        fe_destroy(c);
        return st;
    }
    *out = c;
    return FE_OK;
}

void fe_destroy(fe_ctx *c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    fe::fused_release(&c->fused);
    delete c;
}

fe_status fe_workspace_size(const fe_ctx *c, const fe_job *jobs, int32_t n, size_t *bytes)
{
    if (!bytes) return fail(FE_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    fe_status st = check_batch(c, jobs, n);
    if (st != FE_OK) return st;
    *bytes = layout_for(jobs, n).total;
    return FE_OK;
}

fe_status fe_denoise(const fe_ctx *c, const fe_job *jobs, int32_t n,
                     void *workspace, size_t ws_bytes, void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st != FE_OK) return st;
    if (n == 0) return FE_OK;
    DenoiseLayout L = layout_for(jobs, n);
    st = check_workspace(workspace, ws_bytes, L.total);
    if (st != FE_OK) return st;
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    st = validate_jobs(jobs, n, s);
    if (st != FE_OK) return st;
    char *ws = (char *)workspace;
    std::vector<float *> states(n);
    std::vector<int32_t> zero(n, 0), iters(n);
    for (int i = 0; i < n; ++i) {
        states[i] = (float *)(ws + L.state_off[i]);
        iters[i] = jobs[i].iterations;
    }
    st = enqueue_begin(jobs, states.data(), n, s);
    if (st == FE_OK)
        st = enqueue_advance(c, jobs, states.data(), zero.data(), iters.data(), n, ws, s);
    if (st == FE_OK) st = enqueue_end(jobs, states.data(), iters.data(), n, s);
    return st;
}

fe_status fe_state_bytes(const fe_ctx *c, int32_t height, int32_t width, size_t *bytes)
{
    if (!bytes) return fail(FE_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    if (!c) return fail(FE_ERR_INVALID, "ctx is NULL");
    const int r = radius(c);
    if (height < 1 || width < 1 || height < r || width < r)
        return fail(FE_ERR_INVALID, "image %dx%d smaller than the filter radius %d", height,
                    width, r);
    *bytes = state_bytes(height, width);
    return FE_OK;
}

fe_status fe_begin(const fe_ctx *c, const fe_job *jobs, float *const *states, int32_t n,
                   void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st == FE_OK) st = check_states(jobs, states, n);
    if (st != FE_OK || n == 0) return st;
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    st = validate_jobs(jobs, n, (hipStream_t)hip_stream);
    if (st != FE_OK) return st;
    return enqueue_begin(jobs, states, n, (hipStream_t)hip_stream);
}

fe_status fe_advance_workspace_size(const fe_ctx *c, int32_t n, size_t *bytes)
{
    if (!bytes) return fail(FE_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    if (!c) return fail(FE_ERR_INVALID, "ctx is NULL");
    if (n < 0) return fail(FE_ERR_INVALID, "negative job count");
    *bytes = align256(fe::fused_table_bytes(n));
    return FE_OK;
}

fe_status fe_advance(const fe_ctx *c, const fe_job *jobs, float *const *states,
                     const int32_t *done, const int32_t *count, int32_t n, void *workspace,
                     size_t ws_bytes, void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st == FE_OK) st = check_states(jobs, states, n);
    if (st != FE_OK || n == 0) return st;
    if (!done || !count) return fail(FE_ERR_INVALID, "done and count must be non-NULL");
    for (int i = 0; i < n; ++i)
        if (done[i] < 0 || count[i] < 0)
            return fail(FE_ERR_INVALID, "job %d: negative done or count", i);
    size_t need = 0;
    fe_advance_workspace_size(c, n, &need);
    st = check_workspace(workspace, ws_bytes, need);
    if (st != FE_OK) return st;
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return enqueue_advance(c, jobs, states, done, count, n, workspace, (hipStream_t)hip_stream);
}

fe_status fe_advance_noalloc(const fe_ctx *c, const fe_job *jobs, float *const *states,
                             const int32_t *done, const int32_t *count, int32_t n,
                             void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st == FE_OK) st = check_states(jobs, states, n);
    if (st != FE_OK || n == 0) return st;
    if (!done || !count) return fail(FE_ERR_INVALID, "done and count must be non-NULL");
    for (int i = 0; i < n; ++i)
        if (done[i] < 0 || count[i] < 0)
            return fail(FE_ERR_INVALID, "job %d: negative done or count", i);
    if (n > FE_NOALLOC_MAX_JOBS || fe::fused_table_bytes(n) > fe::kNoallocScratchBytes)
        return fail(FE_ERR_INVALID, "fe_advance_noalloc: %d jobs exceed the static job table "
                                    "(at most %d jobs)", n, FE_NOALLOC_MAX_JOBS);
    void *table = fe::noalloc_scratch(c->device);
    if (!table) return fail(FE_ERR_DEVICE, "static job table not set up on device %d", c->device);
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return enqueue_advance(c, jobs, states, done, count, n, table, (hipStream_t)hip_stream);
}

fe_status fe_end(const fe_ctx *c, const fe_job *jobs, float *const *states,
                 const int32_t *done, int32_t n, void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st == FE_OK) st = check_states(jobs, states, n);
    if (st != FE_OK || n == 0) return st;
    if (!done) return fail(FE_ERR_INVALID, "done is NULL");
    for (int i = 0; i < n; ++i)
        if (done[i] < 0) return fail(FE_ERR_INVALID, "job %d: negative done", i);
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return enqueue_end(jobs, states, done, n, (hipStream_t)hip_stream);
}

// ---- binning variant ----------------------------------------------------
namespace {
struct BinnedLayout {
    std::vector<fe_job> bjobs;          // the jobs on the binned images
    std::vector<size_t> yb_off, xb_off; // binned counts and estimates
    size_t inner_off = 0, inner_bytes = 0, total = 0;
};

fe_status binned_layout(const fe_ctx *c, const fe_job *jobs, int32_t n, BinnedLayout *L)
{
    const int r = radius(c);
    size_t off = 0;
    L->bjobs.assign(jobs, jobs + n);
    L->yb_off.resize(n);
    L->xb_off.resize(n);
    for (int i = 0; i < n; ++i) {
        const int Hb = (jobs[i].height + 2) / 3, Wb = (jobs[i].width + 2) / 3;
        if (Hb < r || Wb < r || jobs[i].height < 2 || jobs[i].width < 2)
            return fail(FE_ERR_INVALID, "job %d: binned image %dx%d smaller than the filter radius",
                        i, Hb, Wb);
        const size_t b = align256((size_t)Hb * Wb * sizeof(float));
        L->yb_off[i] = off;
        off += b;
        L->xb_off[i] = off;
        off += b;
        fe_job &bj = L->bjobs[i];
        bj.height = Hb;
        bj.width = Wb;
        bj.peak = 9.0f * jobs[i].peak;  // the binned image's peak picks the data term
    }
    L->inner_off = off;
    L->inner_bytes = layout_for(L->bjobs.data(), n).total;
    L->total = off + L->inner_bytes;
    return FE_OK;
}
}  // namespace

fe_status fe_binned_workspace_size(const fe_ctx *c, const fe_job *jobs, int32_t n, size_t *bytes)
{
    if (!bytes) return fail(FE_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    fe_status st = check_batch(c, jobs, n);
    if (st != FE_OK) return st;
    BinnedLayout L;
    st = binned_layout(c, jobs, n, &L);
    if (st != FE_OK) return st;
    *bytes = std::max<size_t>(L.total, 256);
    return FE_OK;
}

fe_status fe_denoise_binned(const fe_ctx *c, const fe_job *jobs, int32_t n, void *workspace,
                            size_t ws_bytes, void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st != FE_OK || n == 0) return st;
    BinnedLayout L;
    st = binned_layout(c, jobs, n, &L);
    if (st != FE_OK) return st;
    st = check_workspace(workspace, ws_bytes, L.total);
    if (st != FE_OK) return st;
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    st = validate_jobs(jobs, n, s);
    if (st != FE_OK) return st;
    char *ws = (char *)workspace;
    for (int i = 0; i < n; ++i) {
        float *yb = (float *)(ws + L.yb_off[i]);
        hipError_t e = fe::launch_bin3(jobs[i].counts, jobs[i].height, jobs[i].width, yb, s);
        if (e != hipSuccess) return hip_fail(e, "bin3");
        L.bjobs[i].counts = yb;
        L.bjobs[i].out = (float *)(ws + L.xb_off[i]);
        // out_anscombe (if given) receives the binned u_hat, Hb * Wb values
    }
    st = fe_denoise(c, L.bjobs.data(), n, ws + L.inner_off, L.inner_bytes, hip_stream);
    if (st != FE_OK) return st;
    for (int i = 0; i < n; ++i) {
        if (!jobs[i].out) continue;
        hipError_t e = fe::launch_upsample3(L.bjobs[i].out, L.bjobs[i].height, L.bjobs[i].width,
                                            jobs[i].out, jobs[i].height, jobs[i].width, s);
        if (e != hipSuccess) return hip_fail(e, "upsample3");
    }
    return FE_OK;
}

// ---- autotuning of the tile height ---------------------------------------
fe_status fe_autotune(const fe_ctx *c, const fe_job *jobs, int32_t n, int32_t trial_iterations,
                      void *hip_stream)
{
    fe_status st = check_batch(c, jobs, n);
    if (st != FE_OK || n == 0) return st;
    if (trial_iterations < 2 || (trial_iterations & 1))
        return fail(FE_ERR_INVALID, "trial_iterations must be even and >= 2");
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    // scratch states and job table, allocated for the measurement only
    size_t total = align256(fe::fused_table_bytes(n));
    std::vector<size_t> off(n);
    for (int i = 0; i < n; ++i) {
        off[i] = total;
        total += align256(state_bytes(jobs[i].height, jobs[i].width));
    }
    char *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&buf, total);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    std::vector<float *> states(n);
    std::vector<fe::AdvanceItem> items(n);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        states[i] = (float *)(buf + off[i]);
        items[i] = {&jobs[i], states[i], 0, trial_iterations};
    }
    if (e == hipSuccess && enqueue_begin(jobs, states.data(), n, s) != FE_OK) e = hipErrorUnknown;
    for (int prec = FE_PREC_FP32; prec <= FE_PREC_FP16 && e == hipSuccess; ++prec) {
        std::vector<fe::AdvanceItem> grp;
        for (auto &it : items)
            if (it.job->precision == prec) grp.push_back(it);
        if (grp.empty()) continue;
        const int gn = (int)grp.size();
        fe::TileChoice best;
        float best_ms = 1e30f;
        for (int nw : fe::wave_options(prec)) {
            const std::vector<int> cand = fe::tile_candidates(c->fused, prec, grp.data(), gn, nw, 6);
            for (int ty : cand) {
                const fe::TileChoice tc{nw, ty};
                // one untimed pass, then the timed one (even counts keep parity)
                e = fe::run_fused(c->fused, grp.data(), gn, buf, s, nullptr, prec, tc);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                if (e == hipSuccess) e = fe::run_fused(c->fused, grp.data(), gn, buf, s, nullptr, prec, tc);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = tc;
                }
            }
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess && best.ty > 0)
            c->tune.store(fe::batch_key(prec, grp.data(), gn), best);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    return FE_OK;
}

fe_status fe_tuning_save(const fe_ctx *c, const char *path)
{
    if (!c || !path) return fail(FE_ERR_INVALID, "ctx and path must be non-NULL");
    std::ofstream f(path);
    if (!f) return fail(FE_ERR_INVALID, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(c->tune.mu);
    f << "# fe tuning table: m=" << c->m << " n_filters=" << c->nf
      << "; lines: waves tile_height key\n";
    for (auto &kv : c->tune.tab) f << kv.second.waves << " " << kv.second.ty << " " << kv.first << "\n";
    return f ? FE_OK : fail(FE_ERR_INVALID, "write to %s failed", path);
}

fe_status fe_tuning_load(const fe_ctx *c, const char *path)
{
    if (!c || !path) return fail(FE_ERR_INVALID, "ctx and path must be non-NULL");
    std::ifstream f(path);
    if (!f) return fail(FE_ERR_INVALID, "cannot read %s", path);
    // parse the whole file first: a malformed file changes nothing
    std::string line;
    std::vector<std::pair<std::string, fe::TileChoice>> entries;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ls(line);
        int nw = 0, ty = 0;
        std::string key;
        if (!(ls >> nw >> ty >> key) || key.size() < 3 || key[0] != 'p')
            return fail(FE_ERR_INVALID, "malformed tuning line: %s", line.c_str());
        const int prec = key[1] - '0';
        const int hi = (prec >= FE_PREC_FP32 && prec <= FE_PREC_FP16)
                           ? fe::max_tile_rows(c->fused, prec, nw) : 0;
        if (hi <= 0 || ty < fe::kMinTileRows || ty > hi)
            return fail(FE_ERR_INVALID, "tuning line out of range (waves %d, height %d): %s",
                        nw, ty, line.c_str());
        entries.emplace_back(key, fe::TileChoice{nw, ty});
    }
    for (auto &kv : entries) c->tune.store(kv.first, kv.second);
    return FE_OK;
}

// ---- captured step sequence ---------------------------------------------
struct fe_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

fe_status fe_advance_graph_create(const fe_ctx *c, const fe_job *jobs, float *const *states,
                                  const int32_t *done, const int32_t *count, int32_t n,
                                  void *workspace, size_t ws_bytes, fe_graph **out)
{
    if (!out) return fail(FE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    fe_status st = check_batch(c, jobs, n);
    if (st == FE_OK) st = check_states(jobs, states, n);
    if (st != FE_OK) return st;
    if (n == 0 || !done || !count) return fail(FE_ERR_INVALID, "empty batch or NULL counts");
    for (int i = 0; i < n; ++i)
        if (done[i] < 0 || count[i] < 0 || (count[i] & 1))
            return fail(FE_ERR_INVALID, "job %d: counts must be even and >= 0 so that "
                                        "replays keep the state parity", i);
    size_t need = 0;
    fe_advance_workspace_size(c, n, &need);
    st = check_workspace(workspace, ws_bytes, need);
    if (st != FE_OK) return st;
    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    fe_graph *gr = new (std::nothrow) fe_graph;
    if (!gr) return fail(FE_ERR_NOMEM, "host allocation failed");
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue_advance(c, jobs, states, done, count, n, workspace, cap);
        hipError_t e2 = hipStreamEndCapture(cap, &gr->graph);
        if (st != FE_OK) e = hipErrorUnknown;
        else e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        fe_graph_destroy(gr);
        return st != FE_OK ? st : hip_fail(e, "graph capture");
    }
    *out = gr;
    return FE_OK;
}

fe_status fe_graph_launch(const fe_graph *gr, void *hip_stream)
{
    if (!gr || !gr->exec) return fail(FE_ERR_INVALID, "graph is NULL");
    hipError_t e = hipGraphLaunch(gr->exec, (hipStream_t)hip_stream);
    return e == hipSuccess ? FE_OK : hip_fail(e, "graph launch");
}

void fe_graph_destroy(fe_graph *gr)
{
    if (!gr) return;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
}

}  // extern "C"

namespace {

fe_status check_grad_jobs(const fe_ctx *c, const fe_grad_job *jobs, int32_t n)
{
    if (!c) return fail(FE_ERR_INVALID, "ctx is NULL");
    if (n < 0) return fail(FE_ERR_INVALID, "negative job count");
    if (n > 0 && !jobs) return fail(FE_ERR_INVALID, "jobs is NULL");
    const int r = radius(c);
    for (int i = 0; i < n; ++i) {
        const fe_grad_job &j = jobs[i];
        if (j.height < 1 || j.width < 1 || j.height < r || j.width < r)
            return fail(FE_ERR_INVALID, "job %d: image %dx%d smaller than the filter radius %d",
                        i, j.height, j.width, r);
        if ((long long)j.height * j.width > (1LL << 31) - 1)
            return fail(FE_ERR_INVALID, "job %d: image too large", i);
        if (!j.counts || !j.u) return fail(FE_ERR_INVALID, "job %d: counts and u must be non-NULL", i);
        if (!(j.lambda > 0.0f) || !std::isfinite(j.lambda))
            return fail(FE_ERR_INVALID, "job %d: lambda must be finite and > 0", i);
        if (j.data_term != FE_DATA_QUADRATIC && j.data_term != FE_DATA_IDIV)
            return fail(FE_ERR_INVALID, "job %d: data term must be FE_DATA_QUADRATIC or "
                                        "FE_DATA_IDIV", i);
    }
    return FE_OK;
}

std::vector<fe::GradItem> grad_items(const fe_grad_job *jobs, int32_t n)
{
    std::vector<fe::GradItem> it(n);
    for (int i = 0; i < n; ++i)
        it[i] = {jobs[i].height, jobs[i].width, jobs[i].counts, jobs[i].u, jobs[i].grad,
                 jobs[i].lambda, jobs[i].data_term};
    return it;
}

}  // namespace

extern "C" {

fe_status fe_energy_grad_batch_workspace_size(const fe_ctx *c, const fe_grad_job *jobs,
                                              int32_t n, size_t *bytes)
{
    if (!bytes) return fail(FE_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    fe_status st = check_grad_jobs(c, jobs, n);
    if (st != FE_OK) return st;
    std::vector<fe::GradItem> it = grad_items(jobs, n);
    *bytes = fe::grad_workspace_bytes(c->fused, it.data(), n);
    return FE_OK;
}

fe_status fe_energy_grad_batch(const fe_ctx *c, const fe_grad_job *jobs, int32_t n,
                               int32_t precision, double *energies, void *workspace,
                               size_t ws_bytes, void *hip_stream)
{
    fe_status st = check_grad_jobs(c, jobs, n);
    if (st != FE_OK) return st;
    if (precision < FE_PREC_FP32 || precision > FE_PREC_FP16)
        return fail(FE_ERR_INVALID, "precision %d is not an FE_PREC_* value", precision);
    std::vector<fe::GradItem> it = grad_items(jobs, n);
    st = check_workspace(workspace, ws_bytes, fe::grad_workspace_bytes(c->fused, it.data(), n));
    if (st != FE_OK) return st;
    bool any_grad = false;
    for (int i = 0; i < n; ++i) any_grad = any_grad || jobs[i].grad;
    if (n == 0 || (!energies && !any_grad)) return FE_OK;

    DeviceGuard g(c->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    {
        std::vector<const float *> planes(n);
        std::vector<long> sizes(n);
        for (int i = 0; i < n; ++i) {
            planes[i] = jobs[i].counts;
            sizes[i] = (long)jobs[i].height * jobs[i].width;
        }
        st = validate_counts(planes.data(), sizes.data(), n, s);
        if (st != FE_OK) return st;
    }
    double *edev = nullptr;
    hipError_t e = fe::run_grad(c->fused, it.data(), n, precision, energies != nullptr,
                                workspace, &edev, s);
    if (e != hipSuccess) return hip_fail(e, "energy / gradient launch");
    if (energies) {
        e = hipMemcpyAsync(energies, edev, sizeof(double) * n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "energy readback");
    }
    return FE_OK;
}

fe_status fe_energy_grad_workspace_size(const fe_ctx *c, int32_t H, int32_t W, size_t *bytes)
{
    if (!bytes) return fail(FE_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    if (!c) return fail(FE_ERR_INVALID, "ctx is NULL");
    const int r = radius(c);
    if (H < 1 || W < 1 || H < r || W < r)
        return fail(FE_ERR_INVALID, "image %dx%d smaller than the filter radius %d", H, W, r);
    if ((long long)H * W > (1LL << 31) - 1) return fail(FE_ERR_INVALID, "image too large");
    fe::GradItem it{H, W, nullptr, nullptr, nullptr, 1.0f, FE_DATA_QUADRATIC};
    *bytes = fe::grad_workspace_bytes(c->fused, &it, 1);
    return FE_OK;
}

fe_status fe_energy_grad(const fe_ctx *c, int32_t H, int32_t W, const float *counts,
                         const float *u, float lambda, int32_t data_term, int32_t precision,
                         double *energy, float *grad, void *workspace, size_t ws_bytes,
                         void *hip_stream)
{
    const fe_grad_job j{H, W, counts, u, grad, lambda, data_term};
    return fe_energy_grad_batch(c, &j, 1, precision, energy, workspace, ws_bytes, hip_stream);
}

}  // extern "C"
