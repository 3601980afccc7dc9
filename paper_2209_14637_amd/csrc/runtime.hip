// Host runtime of libtsk: context, validation, workspace, timing and the C
// entry points declared in include/tsk.h.
#include <cstdio>
#include <cstring>
#include <new>

#include "tsk_common.hpp"

tsk_status tsk_gram_enqueue(tsk_ctx c, const tsk_stack *s, int compute, double *G);
tsk_status tsk_stage_enqueue(tsk_ctx c, const tsk_stack *s, int dtype, void *dst, int64_t ldd, int64_t strided,
                             float *scale, double *norm2);
tsk_status tsk_stage_mx_enqueue(tsk_ctx c, const tsk_stack *s, void *dst, int64_t ldd, int64_t strided,
                                uint8_t *bscale);
tsk_status tsk_eig_enqueue(tsk_ctx c, const double *G, int64_t m, int k, float *S, double *lambda,
                           int32_t *iters_out, double tol_default);
tsk_status tsk_apply_enqueue(tsk_ctx c, const float *S, int k, const tsk_stack *s, int r, float *L, float *R,
                             float *sigma, double *relerr, int32_t *flags);
tsk_status tsk_apply_noalloc_enqueue(tsk_ctx c, const float *S, int k, const tsk_stack *s, int r, float *L,
                                     float *R, float *sigma, double *relerr, int32_t *flags);
tsk_status tsk_scratch_init(tsk_ctx c, int device);
tsk_status tsk_random_sketch_enqueue(tsk_ctx c, int kind, int64_t k, int64_t m, uint64_t seed, float *S);
tsk_status tsk_opt_tail_enqueue(tsk_ctx c, const tsk_stack *s, int r, double *tail, double *fro);
tsk_status tsk_apply2_enqueue(tsk_ctx c, const float *S, int k, const float *W, int l, const tsk_stack *s, int r,
                              float *L, float *R, float *sigma, double *relerr, int32_t *flags);
tsk_status tsk_train2_enqueue(tsk_ctx c, const tsk_stack *s, int k, int l, int max_sweeps, double tol, float *S,
                              float *W, double *core2, int32_t *sweeps_out);
tsk_status tsk_error_enqueue(tsk_ctx c, const tsk_stack *s, const float *L, const float *R, int r,
                             double *relerr);
tsk_status tsk_apply_multi_enqueue(tsk_ctx c, const tsk_problem *pr, int np, int compute);
tsk_status tsk_plan_create_enqueue(tsk_ctx c, const tsk_problem *pr, int np, int compute, tsk_plan *out);
tsk_status tsk_plan_launch_enqueue(tsk_ctx c, const tsk_plan *plans, int n);
void tsk_plan_destroy_impl(tsk_plan p);

tsk_status tsk_fail(tsk_ctx c, tsk_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

tsk_status tsk_hip(tsk_ctx c, hipError_t e, const char *what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
    return tsk_fail(c, TSK_E_DEVICE, buf);
}

tsk_status tsk_grow(tsk_ctx c, TskBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return TSK_OK;
    // work already queued may still use the old buffer
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "workspace sync");
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    const size_t nb = (bytes + (1 << 20) - 1) & ~(size_t)((1 << 20) - 1);
    if (getenv("TSK_FAULT_NOMEM") || hipMalloc(&b.p, nb) != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        char buf[128];
        snprintf(buf, sizeof buf, "workspace allocation of %zu bytes failed", nb);
        return tsk_fail(c, TSK_E_NOMEM, buf);
    }
    b.bytes = nb;
    return TSK_OK;
}

// The context's two pipeline streams and their fork / join events (created
// on first use, on the context's device, default priority).
// TSK_PIPELINE_STREAMS (diagnostic, read when the streams are created): their
// number, 2..TSK_MAX_PIPE (default TSK_DEFAULT_PIPE).
tsk_status tsk_pipeline_streams(tsk_ctx c) {
    if (c->pl[0]) return TSK_OK;
    int np = TSK_DEFAULT_PIPE;
    if (const char *v = getenv("TSK_PIPELINE_STREAMS")) np = atoi(v);
    np = np < 2 ? 2 : (np > TSK_MAX_PIPE ? TSK_MAX_PIPE : np);
    hipError_t e = hipSuccess;
    for (int i = 0; i < np && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&c->pl[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->pl_fork, hipEventDisableTiming);
    for (int i = 0; i < np && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->pl_join[i], hipEventDisableTiming);
    c->npl = np;
    if (e != hipSuccess) {
        c->npl = 0;
        for (int i = 0; i < TSK_MAX_PIPE; ++i) {
            if (c->pl[i]) (void)hipStreamDestroy(c->pl[i]);
            if (c->pl_join[i]) (void)hipEventDestroy(c->pl_join[i]);
            c->pl[i] = nullptr;
            c->pl_join[i] = nullptr;
        }
        if (c->pl_fork) (void)hipEventDestroy(c->pl_fork);
        c->pl_fork = nullptr;
        return tsk_hip(c, e, "pipeline streams");
    }
    return TSK_OK;
}

TskTune tsk_tuning(tsk_ctx c, int64_t m, int64_t n, int kp, int dtype) {
    const auto it = c->tune.find(std::make_tuple(m, n, kp, dtype));
    return it == c->tune.end() ? TskTune{} : it->second;
}

// The pointer must lie in a device allocation that holds [p, p + bytes).
tsk_status tsk_check_dev(tsk_ctx c, const void *p, size_t bytes, const char *name) {
    if (!p) return tsk_fail(c, TSK_E_ARG, std::string(name) + ": null pointer");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        return tsk_fail(c, TSK_E_ARG, std::string(name) + ": not a device allocation");
    }
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) == hipSuccess) {
        if (attr.type == hipMemoryTypeDevice && attr.device != c->device)
            return tsk_fail(c, TSK_E_ARG, std::string(name) + ": memory of another device");
    } else {
        (void)hipGetLastError();
    }
    const char *lo = (const char *)base, *hi = lo + size, *q = (const char *)p;
    if (q < lo || q + bytes > hi) {
        char buf[200];
        snprintf(buf, sizeof buf, "%s: needs %zu bytes, allocation holds %zu from that address", name, bytes,
                 (size_t)(hi - q));
        return tsk_fail(c, TSK_E_SHAPE, buf);
    }
    return TSK_OK;
}

static size_t dtype_size(int32_t dt) {
    switch (dt) {
        case TSK_F64: return 8;
        case TSK_F32: return 4;
        case TSK_BF16: return 2;
        case TSK_F8E4M3: return 1;
        case TSK_MXE4M3: return 1;
        default: return 0;
    }
}

tsk_status tsk_check_stack(tsk_ctx c, const tsk_stack *s, const char *name) {
    std::string nm(name);
    if (!s) return tsk_fail(c, TSK_E_ARG, nm + ": null stack");
    if (!s->A) return tsk_fail(c, TSK_E_ARG, nm + ": null data pointer");
    const size_t es = dtype_size(s->dtype);
    const bool scaled = s->dtype == TSK_F8E4M3 || s->dtype == TSK_MXE4M3;
    if (s->dtype != TSK_F32 && s->dtype != TSK_BF16 && !scaled)
        return tsk_fail(c, TSK_E_ARG, nm + ": dtype must be TSK_F32, TSK_BF16, TSK_F8E4M3 or TSK_MXE4M3");
    if (scaled && !s->scale) return tsk_fail(c, TSK_E_ARG, nm + ": e4m3 stacks need scale");
    if (!scaled && s->scale) return tsk_fail(c, TSK_E_ARG, nm + ": scale must be NULL");
    if (s->m < 1 || s->n < 1 || s->count < 1) return tsk_fail(c, TSK_E_SHAPE, nm + ": m, n, count must be >= 1");
    if (s->ld < s->n) return tsk_fail(c, TSK_E_SHAPE, nm + ": ld < n");
    if (s->stride < s->m * s->ld) return tsk_fail(c, TSK_E_SHAPE, nm + ": stride < m*ld");
    const int64_t q = (int64_t)(16 / es);  // elements per 16 bytes
    if (((uintptr_t)s->A & 15) || (s->ld % q) || (s->stride % q))
        return tsk_fail(c, TSK_E_SHAPE, nm + ": data must be 16-byte aligned with ld, stride multiples of 16 bytes");
    if (s->m > (1 << 20) || s->n > (1 << 20) || s->count > (1 << 24))
        return tsk_fail(c, TSK_E_SHAPE, nm + ": dimension too large");
    const size_t need = ((size_t)(s->count - 1) * s->stride + (size_t)(s->m - 1) * s->ld + s->n) * es;
    TSK_TRY(tsk_check_dev(c, s->A, need, (nm + ".A").c_str()));
    if (s->dtype == TSK_F8E4M3)
        TSK_TRY(tsk_check_dev(c, s->scale, sizeof(float) * s->count, (nm + ".scale").c_str()));
    if (s->dtype == TSK_MXE4M3)
        TSK_TRY(tsk_check_dev(c, s->scale, (size_t)(s->count * s->m * ((s->n + 31) / 32)),
                              (nm + ".scale").c_str()));
    return TSK_OK;
}

// Gram compute rules shared by tsk_gram and tsk_train.
static tsk_status check_gram_compute(tsk_ctx c, const tsk_stack *s, int32_t compute, const char *who) {
    std::string w(who);
    if (compute == TSK_F32) {
        if (s->dtype != TSK_F32) return tsk_fail(c, TSK_E_ARG, w + ": compute TSK_F32 needs an FP32 stack");
        return TSK_OK;
    }
    if (compute == TSK_BF16) {
        if (s->dtype != TSK_F32 && s->dtype != TSK_BF16)
            return tsk_fail(c, TSK_E_ARG, w + ": compute TSK_BF16 needs an FP32 or bf16 stack");
        return TSK_OK;
    }
    if (compute == TSK_F8E4M3) {
        if (s->dtype != TSK_F8E4M3) return tsk_fail(c, TSK_E_ARG, w + ": compute TSK_F8E4M3 needs an e4m3 stack");
        return TSK_OK;
    }
    if (compute == TSK_MXE4M3) {
        if (s->dtype != TSK_MXE4M3)
            return tsk_fail(c, TSK_E_ARG, w + ": compute TSK_MXE4M3 needs a block-scaled e4m3 stack");
        return TSK_OK;
    }
    return tsk_fail(c, TSK_E_ARG, w + ": compute must be TSK_F32, TSK_BF16, TSK_F8E4M3 or TSK_MXE4M3");
}

void tsk_ev_begin(tsk_ctx c, int cls, hipEvent_t *a) {
    *a = nullptr;
    if (!(c->timing >> cls & 1u)) return;
    if (c->pool.empty()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->pool.push_back(e);
    }
    *a = c->pool.back();
    c->pool.pop_back();
    (void)hipEventRecord(*a, c->stream);
}

void tsk_ev_end(tsk_ctx c, int cls, hipEvent_t a) {
    if (!a) return;
    hipEvent_t b;
    if (c->pool.empty()) {
        if (hipEventCreate(&b) != hipSuccess) return;
    } else {
        b = c->pool.back();
        c->pool.pop_back();
    }
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({cls, a, b});
}

static void drain_events(tsk_ctx c) {
    for (auto &ev : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
            c->launches[ev.cls] += 1;
            c->ms[ev.cls] += ms;
        }
        c->pool.push_back(ev.a);
        c->pool.push_back(ev.b);
    }
    c->pending.clear();
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

extern "C" {

tsk_status tsk_create(tsk_ctx *out, int device, void *hip_stream) {
    if (!out) return TSK_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return TSK_E_DEVICE;
    }
    if (device < 0 || device >= ndev) return TSK_E_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TSK_E_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TSK_E_DEVICE;
    tsk_ctx c = new (std::nothrow) tsk_ctx_s();
    if (!c) return TSK_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    {
        DeviceGuard g(device);
        const tsk_status st = tsk_scratch_init(c, device);
        if (st != TSK_OK) {
            delete c;
            return st;
        }
    }
    *out = c;
    return TSK_OK;
}

void tsk_destroy(tsk_ctx c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    drain_events(c);
    TskBuf *bufs[] = {&c->gram_part, &c->gram_G,  &c->eig_Y0,   &c->eig_Y1, &c->eig_Rinv, &c->eig_part,
                      &c->eig_C,     &c->eig_X,   &c->eig_GX,   &c->eig_small, &c->eig_U, &c->counters,
                      &c->ap_ws,     &c->er_part, &c->st_part,  &c->mp_ws,  &c->mp_tab, &c->mt_ws, &c->ap2_ws, &c->t2_ws};
    for (TskBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->mp_pin) (void)hipHostFree(c->mp_pin);
    if (c->mp_ev) (void)hipEventDestroy(c->mp_ev);
    if (c->switch_ev) (void)hipEventDestroy(c->switch_ev);
    for (int i = 0; i < TSK_MAX_PIPE; ++i) {
        if (c->pl[i]) (void)hipStreamDestroy(c->pl[i]);
        if (c->pl_join[i]) (void)hipEventDestroy(c->pl_join[i]);
    }
    if (c->pl_fork) (void)hipEventDestroy(c->pl_fork);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

tsk_status tsk_set_stream(tsk_ctx c, void *hip_stream) {
    if (!c) return TSK_E_ARG;
    if ((hipStream_t)hip_stream == c->stream) return TSK_OK;
    // The workspace is shared by every call of the context: work enqueued
    // later on the new stream waits for everything enqueued on the old one.
    DeviceGuard g(c->device);
    if (!c->switch_ev) {
        hipError_t e = hipEventCreateWithFlags(&c->switch_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            c->switch_ev = nullptr;
            return tsk_hip(c, e, "stream switch event");
        }
    }
    hipError_t e = hipEventRecord(c->switch_ev, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)hip_stream, c->switch_ev, 0);
    if (e != hipSuccess) return tsk_hip(c, e, "stream switch");
    c->stream = (hipStream_t)hip_stream;
    return TSK_OK;
}

const char *tsk_last_error(tsk_ctx c) { return c ? c->err.c_str() : "null context"; }

tsk_status tsk_gram(tsk_ctx c, const tsk_stack *train, int32_t compute, double *G) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, train, "train"));
    TSK_TRY(check_gram_compute(c, train, compute, "tsk_gram"));
    TSK_TRY(tsk_check_dev(c, G, sizeof(double) * train->m * train->m, "G"));
    return tsk_gram_enqueue(c, train, compute, G);
}

tsk_status tsk_stage(tsk_ctx c, const tsk_stack *src, int32_t dtype, void *dst, int64_t ld, int64_t stride,
                     float *scale, double *norm2) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, src, "src"));
    if (src->dtype != TSK_F32) return tsk_fail(c, TSK_E_ARG, "tsk_stage: src must be an FP32 stack");
    if (dtype != TSK_BF16 && dtype != TSK_F8E4M3)
        return tsk_fail(c, TSK_E_ARG, "tsk_stage: dtype must be TSK_BF16 or TSK_F8E4M3 (block scales: tsk_stage_mx)");
    if (dtype == TSK_F8E4M3 && !scale) return tsk_fail(c, TSK_E_ARG, "tsk_stage: TSK_F8E4M3 needs scale");
    if (dtype == TSK_BF16 && scale) return tsk_fail(c, TSK_E_ARG, "tsk_stage: scale must be NULL for TSK_BF16");
    tsk_stack d = *src;
    d.A = dst;
    d.dtype = dtype;
    d.scale = scale;
    d.ld = ld;
    d.stride = stride;
    TSK_TRY(tsk_check_stack(c, &d, "dst"));
    if (norm2) TSK_TRY(tsk_check_dev(c, norm2, sizeof(double) * src->count, "norm2"));
    return tsk_stage_enqueue(c, src, dtype, dst, ld, stride, scale, norm2);
}

tsk_status tsk_stage_mx(tsk_ctx c, const tsk_stack *src, void *dst, int64_t ld, int64_t stride, uint8_t *bscale) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, src, "src"));
    if (src->dtype != TSK_F32) return tsk_fail(c, TSK_E_ARG, "tsk_stage_mx: src must be an FP32 stack");
    if (!bscale) return tsk_fail(c, TSK_E_ARG, "tsk_stage_mx: bscale is required");
    tsk_stack d = *src;
    d.A = dst;
    d.dtype = TSK_MXE4M3;
    d.scale = reinterpret_cast<const float *>(bscale);
    d.ld = ld;
    d.stride = stride;
    TSK_TRY(tsk_check_stack(c, &d, "dst"));
    return tsk_stage_mx_enqueue(c, src, dst, ld, stride, bscale);
}

tsk_status tsk_eig_topk(tsk_ctx c, const double *G, int64_t m, int32_t k, float *S, double *lambda,
                        int32_t *iters) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    if (m < 2 || m > (1 << 16)) return tsk_fail(c, TSK_E_SHAPE, "tsk_eig_topk: need 2 <= m <= 65536");
    if (k < 1 || k >= m) return tsk_fail(c, TSK_E_ARG, "tsk_eig_topk: need 1 <= k < m");
    if (k > 52) return tsk_fail(c, TSK_E_ARG, "tsk_eig_topk: k > 52 not supported");
    if (!lambda) return tsk_fail(c, TSK_E_ARG, "tsk_eig_topk: lambda is required");
    TSK_TRY(tsk_check_dev(c, G, sizeof(double) * m * m, "G"));
    TSK_TRY(tsk_check_dev(c, S, sizeof(float) * k * m, "S"));
    tsk_status st = tsk_eig_enqueue(c, G, m, k, S, lambda, iters, TSK_EIG_TOL_F32);
    return st;
}

tsk_status tsk_train(tsk_ctx c, const tsk_stack *train, int32_t k, int32_t compute, float *S, double *lambda,
                     int32_t *iters) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, train, "train"));
    TSK_TRY(check_gram_compute(c, train, compute, "tsk_train"));
    const int64_t m = train->m;
    if (k < 1 || k >= m) return tsk_fail(c, TSK_E_ARG, "tsk_train: need 1 <= k < m");
    if (k > 52) return tsk_fail(c, TSK_E_ARG, "tsk_train: k > 52 not supported");
    if (!lambda) return tsk_fail(c, TSK_E_ARG, "tsk_train: lambda is required");
    TSK_TRY(tsk_check_dev(c, S, sizeof(float) * k * m, "S"));
    TSK_TRY(tsk_grow(c, c->gram_G, sizeof(double) * m * m));
    double *G = (double *)c->gram_G.p;
    TSK_TRY(tsk_gram_enqueue(c, train, compute, G));
    const double tol = compute == TSK_F8E4M3 || compute == TSK_MXE4M3 ? TSK_EIG_TOL_F8
                       : compute == TSK_BF16                          ? TSK_EIG_TOL_BF16
                                                                      : TSK_EIG_TOL_F32;
    return tsk_eig_enqueue(c, G, m, k, S, lambda, iters, tol);
}

// Arguments of one SCW problem (tsk_apply, or one problem of tsk_apply_multi).
static tsk_status check_apply(tsk_ctx c, const float *S, int32_t k, const tsk_stack *test, int32_t r,
                              int32_t compute, float *L, float *R, float *sigma, double *relerr, int32_t *flags) {
    TSK_TRY(tsk_check_stack(c, test, "test"));
    if (compute != TSK_F32 && compute != TSK_BF16 && compute != TSK_F8E4M3)
        return tsk_fail(c, TSK_E_ARG, "tsk_apply: compute must be TSK_F32, TSK_BF16 or TSK_F8E4M3");
    if (test->dtype != compute) return tsk_fail(c, TSK_E_ARG, "tsk_apply: compute must match the stack's dtype");
    const int64_t m = test->m, n = test->n, cnt = test->count;
    if (r < 1 || r >= k) return tsk_fail(c, TSK_E_ARG, "tsk_apply: need 1 <= r < k");
    if (k > m || k > n) return tsk_fail(c, TSK_E_ARG, "tsk_apply: need k <= min(m, n)");
    if (k > 64) return tsk_fail(c, TSK_E_ARG, "tsk_apply: k > 64 not supported");
    TSK_TRY(tsk_check_dev(c, S, sizeof(float) * k * m, "S"));
    TSK_TRY(tsk_check_dev(c, L, sizeof(float) * cnt * m * r, "L"));
    TSK_TRY(tsk_check_dev(c, R, sizeof(float) * cnt * n * r, "R"));
    TSK_TRY(tsk_check_dev(c, sigma, sizeof(float) * cnt * r, "sigma"));
    if (relerr) TSK_TRY(tsk_check_dev(c, relerr, sizeof(double) * cnt, "relerr"));
    if (flags) TSK_TRY(tsk_check_dev(c, flags, sizeof(int32_t) * cnt, "flags"));
    return TSK_OK;
}

static tsk_status check_multi(tsk_ctx c, const tsk_problem *probs, int32_t nprobs, int32_t compute);

tsk_status tsk_apply_multi_plan(tsk_ctx c, const tsk_problem *probs, int32_t nprobs, int32_t compute,
                                tsk_plan *plan) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    if (!plan) return tsk_fail(c, TSK_E_ARG, "tsk_apply_multi_plan: null plan pointer");
    *plan = nullptr;
    TSK_TRY(check_multi(c, probs, nprobs, compute));
    return tsk_plan_create_enqueue(c, probs, nprobs, compute, plan);
}

tsk_status tsk_plan_launch(tsk_ctx c, const tsk_plan *plans, int32_t nplans) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    if (!plans || nplans < 1) return tsk_fail(c, TSK_E_ARG, "tsk_plan_launch: need nplans >= 1");
    return tsk_plan_launch_enqueue(c, plans, nplans);
}

void tsk_plan_destroy(tsk_plan plan) { tsk_plan_destroy_impl(plan); }

tsk_status tsk_apply_multi(tsk_ctx c, const tsk_problem *probs, int32_t nprobs, int32_t compute) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(check_multi(c, probs, nprobs, compute));
    return tsk_apply_multi_enqueue(c, probs, nprobs, compute);
}

static tsk_status check_multi(tsk_ctx c, const tsk_problem *probs, int32_t nprobs, int32_t compute) {
    if (!probs || nprobs < 1 || nprobs > (1 << 20))
        return tsk_fail(c, TSK_E_ARG, "tsk_apply_multi: need 1 <= nprobs <= 2^20 problems");
    int64_t items = 0;
    for (int i = 0; i < nprobs; ++i) {
        const tsk_problem &p = probs[i];
        tsk_status st = check_apply(c, p.S, p.k, &p.A, p.r, compute, p.L, p.R, p.sigma, p.relerr, p.flags);
        if (st != TSK_OK) {
            c->err = "problem " + std::to_string(i) + ": " + c->err;
            return st;
        }
        items += p.A.count * (p.A.n / 64 + 2 * (p.A.m / 64) + 6);
    }
    if (items > ((int64_t)1 << 31) - 1) return tsk_fail(c, TSK_E_SHAPE, "tsk_apply_multi: batch too large");
    return TSK_OK;
}

tsk_status tsk_apply(tsk_ctx c, const float *S, int32_t k, const tsk_stack *test, int32_t r, int32_t compute,
                     float *L, float *R, float *sigma, double *relerr, int32_t *flags) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(check_apply(c, S, k, test, r, compute, L, R, sigma, relerr, flags));
    return tsk_apply_enqueue(c, S, k, test, r, L, R, sigma, relerr, flags);
}

tsk_status tsk_apply_noalloc(tsk_ctx c, const float *S, int32_t k, const tsk_stack *test, int32_t r,
                             int32_t compute, float *L, float *R, float *sigma, double *relerr, int32_t *flags) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(check_apply(c, S, k, test, r, compute, L, R, sigma, relerr, flags));
    return tsk_apply_noalloc_enqueue(c, S, k, test, r, L, R, sigma, relerr, flags);
}

tsk_status tsk_random_sketch(tsk_ctx c, int32_t kind, int32_t k, int64_t m, uint64_t seed, float *S) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    if (kind != TSK_SKETCH_GAUSSIAN && kind != TSK_SKETCH_SIGN && kind != TSK_SKETCH_SPARSE)
        return tsk_fail(c, TSK_E_ARG, "tsk_random_sketch: unknown kind");
    if (k < 1 || m < k || m > (1 << 24)) return tsk_fail(c, TSK_E_ARG, "tsk_random_sketch: need 1 <= k <= m <= 2^24");
    TSK_TRY(tsk_check_dev(c, S, sizeof(float) * (size_t)k * m, "S"));
    return tsk_random_sketch_enqueue(c, kind, k, m, seed, S);
}

tsk_status tsk_train2(tsk_ctx c, const tsk_stack *train, int32_t k, int32_t l, int32_t max_sweeps, double tol,
                      float *S, float *W, double *core2, int32_t *sweeps) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, train, "train"));
    if (train->dtype != TSK_F32) return tsk_fail(c, TSK_E_ARG, "tsk_train2: the training stack must be FP32");
    const int64_t m = train->m, n = train->n;
    if (k < 1 || k >= m || l < 1 || l >= n) return tsk_fail(c, TSK_E_ARG, "tsk_train2: need 1 <= k < m, 1 <= l < n");
    if (k > 52 || l > 52) return tsk_fail(c, TSK_E_ARG, "tsk_train2: k, l <= 52");
    if (m > (1 << 16) || n > (1 << 16)) return tsk_fail(c, TSK_E_SHAPE, "tsk_train2: need m, n <= 65536");
    if (max_sweeps < 0 || max_sweeps > 1000) return tsk_fail(c, TSK_E_ARG, "tsk_train2: need 0 <= max_sweeps <= 1000");
    TSK_TRY(tsk_check_dev(c, S, sizeof(float) * k * m, "S"));
    TSK_TRY(tsk_check_dev(c, W, sizeof(float) * l * n, "W"));
    return tsk_train2_enqueue(c, train, k, l, max_sweeps, tol > 0 ? tol : 1e-10, S, W, core2, sweeps);
}

tsk_status tsk_apply2(tsk_ctx c, const float *S, int32_t k, const float *W, int32_t l, const tsk_stack *test,
                      int32_t r, int32_t compute, float *L, float *R, float *sigma, double *relerr, int32_t *flags) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(check_apply(c, S, k, test, r, compute, L, R, sigma, relerr, flags));
    if (l < 1 || r >= l) return tsk_fail(c, TSK_E_ARG, "tsk_apply2: need 1 <= r < l");
    if (l > test->m || l > test->n || l > 64) return tsk_fail(c, TSK_E_ARG, "tsk_apply2: need l <= min(m, n), l <= 64");
    TSK_TRY(tsk_check_dev(c, W, sizeof(float) * l * test->n, "W"));
    return tsk_apply2_enqueue(c, S, k, W, l, test, r, L, R, sigma, relerr, flags);
}

tsk_status tsk_opt_tail(tsk_ctx c, const tsk_stack *A, int32_t r, double *tail, double *fro) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, A, "A"));
    if (!tail || !fro) return tsk_fail(c, TSK_E_ARG, "tsk_opt_tail: tail and fro are required (host)");
    if (r < 1 || r >= A->m || r > 52) return tsk_fail(c, TSK_E_ARG, "tsk_opt_tail: need 1 <= r < m, r <= 52");
    if (A->m > (1 << 16)) return tsk_fail(c, TSK_E_SHAPE, "tsk_opt_tail: need m <= 65536");
    return tsk_opt_tail_enqueue(c, A, r, tail, fro);
}

tsk_status tsk_error(tsk_ctx c, const tsk_stack *A, const float *L, const float *R, int32_t r, double *relerr) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    TSK_TRY(tsk_check_stack(c, A, "A"));
    if (A->dtype != TSK_F32) return tsk_fail(c, TSK_E_ARG, "tsk_error: A must be an FP32 stack");
    if (r < 1 || r > 64) return tsk_fail(c, TSK_E_ARG, "tsk_error: need 1 <= r <= 64");
    const int64_t m = A->m, n = A->n, cnt = A->count;
    TSK_TRY(tsk_check_dev(c, L, sizeof(float) * cnt * m * r, "L"));
    TSK_TRY(tsk_check_dev(c, R, sizeof(float) * cnt * n * r, "R"));
    TSK_TRY(tsk_check_dev(c, relerr, sizeof(double) * cnt, "relerr"));
    return tsk_error_enqueue(c, A, L, R, r, relerr);
}

tsk_status tsk_set_eig_params(tsk_ctx c, int32_t block, int32_t max_iter, double tol, int32_t check) {
    if (!c) return TSK_E_ARG;
    c->eig_block = block > 0 ? block : 0;
    c->eig_max_iter = max_iter > 0 ? max_iter : 300;
    c->eig_tol = tol > 0 ? tol : 0.0;  // 0: the default for the Gram's precision
    c->eig_check = check > 0 ? check : 6;
    return TSK_OK;
}

tsk_status tsk_set_tuning(tsk_ctx c, int64_t m, int64_t n, int32_t k, int32_t dtype, int32_t groups,
                          int32_t pj_cols) {
    if (!c) return TSK_E_ARG;
    c->err.clear();
    if (m < 1 || n < 1 || k < 1 || k > 64) return tsk_fail(c, TSK_E_ARG, "tsk_set_tuning: need m, n >= 1, 1 <= k <= 64");
    if (dtype != TSK_F32 && dtype != TSK_BF16 && dtype != TSK_F8E4M3)
        return tsk_fail(c, TSK_E_ARG, "tsk_set_tuning: dtype must be TSK_F32, TSK_BF16 or TSK_F8E4M3");
    if (groups < 0 || groups > 64) return tsk_fail(c, TSK_E_ARG, "tsk_set_tuning: need 0 <= groups <= 64");
    if (pj_cols != 0 && !(dtype == TSK_BF16 && (pj_cols == 64 || pj_cols == 128)))
        return tsk_fail(c, TSK_E_ARG, "tsk_set_tuning: pj_cols must be 0, or 64 or 128 for TSK_BF16");
    const auto key = std::make_tuple(m, n, (k + 15) / 16 * 16, (int)dtype);
    if (groups == 0 && pj_cols == 0)
        c->tune.erase(key);
    else
        c->tune[key] = TskTune{groups, pj_cols};
    return TSK_OK;
}

tsk_status tsk_timing_enable(tsk_ctx c, int32_t mask) {
    if (!c) return TSK_E_ARG;
    c->timing = (uint32_t)mask & ((1u << TSK_KERNEL_COUNT) - 1u);
    return TSK_OK;
}

tsk_status tsk_timing_read(tsk_ctx c, int32_t reset, int64_t *launches, double *ms) {
    if (!c) return TSK_E_ARG;
    DeviceGuard g(c->device);
    drain_events(c);
    for (int i = 0; i < TSK_KERNEL_COUNT; ++i) {
        if (launches) launches[i] = c->launches[i];
        if (ms) ms[i] = c->ms[i];
    }
    if (reset) {
        memset(c->launches, 0, sizeof c->launches);
        memset(c->ms, 0, sizeof c->ms);
    }
    return TSK_OK;
}

}  // extern "C"
