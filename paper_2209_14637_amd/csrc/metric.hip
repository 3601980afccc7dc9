// Metric (4.1) of the paper's Section 4 compares each SCW output with the
// best rank-r approximation of the same matrix (Eckart-Young, Section 1):
//     ||A_d - [A_d]_r||_F^2 = sum_{i > r} sigma_i(A_d)^2
//                          = trace(G_d) - sum_{i <= r} lambda_i(G_d),
// G_d = A_d A_d^T.  Here G_d is formed by the Gram kernels on the single
// slice (FP32 accumulation of exact products, FP64 across chunks), its top-r
// eigenvalues by the filtered subspace iteration of tsk_eig_topk, and its
// trace by a fixed-order FP64 sum of the diagonal.  One slice after another.
#include "tsk_common.hpp"

tsk_status tsk_gram_enqueue(tsk_ctx c, const tsk_stack *s, int compute, double *G);
tsk_status tsk_eig_enqueue(tsk_ctx c, const double *G, int64_t m, int k, float *S, double *lambda,
                           int32_t *iters_out, double tol_default);

namespace {

// trace of the m x m matrix G into *out (one workgroup, fixed order).
__global__ void trace_kernel(const double *__restrict__ G, int64_t m, double *__restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) s += G[i * m + i];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

tsk_status tsk_opt_tail_enqueue(tsk_ctx c, const tsk_stack *s, int r, double *tail, double *fro) {
    const int64_t m = s->m;
    const int compute = s->dtype == TSK_F32 ? TSK_F32 : s->dtype == TSK_BF16 ? TSK_BF16 : s->dtype;
    TSK_TRY(tsk_grow(c, c->gram_G, sizeof(double) * m * m));
    TSK_TRY(tsk_grow(c, c->mt_ws, sizeof(float) * (size_t)r * m + 256));
    double *G = (double *)c->gram_G.p;
    float *S = (float *)c->mt_ws.p;
    double *tr = (double *)((char *)c->mt_ws.p + ((sizeof(float) * (size_t)r * m + 255) & ~(size_t)255));
    const size_t es = s->dtype == TSK_F32 ? 4 : s->dtype == TSK_BF16 ? 2 : 1;
    double lam[64 + 1];
    for (int64_t d = 0; d < s->count; ++d) {
        tsk_stack one = *s;
        one.count = 1;
        one.A = (const char *)s->A + (size_t)d * s->stride * es;
        if (s->dtype == TSK_F8E4M3) one.scale = s->scale + d;
        if (s->dtype == TSK_MXE4M3)  // the slice's block exponents
            one.scale = reinterpret_cast<const float *>(reinterpret_cast<const uint8_t *>(s->scale) +
                                                        (size_t)d * s->m * ((s->n + 31) / 32));
        TSK_TRY(tsk_gram_enqueue(c, &one, compute, G));
        TSK_LAUNCH(c, TSK_KERNEL_ERROR, hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, c->stream,
                                                           (const double *)G, m, tr));
        double t = 0.0;
        hipError_t e = hipMemcpyAsync(&t, tr, sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return tsk_hip(c, e, "trace copy");
        const tsk_status st = tsk_eig_enqueue(c, G, m, r, S, lam, nullptr, TSK_EIG_TOL_F32);  // synchronises
        if (st != TSK_OK) return st;
        double top = 0.0;
        for (int i = 0; i < r; ++i) top += lam[i] > 0.0 ? lam[i] : 0.0;
        tail[d] = t > top ? sqrt(t - top) : 0.0;
        fro[d] = sqrt(t > 0.0 ? t : 0.0);
    }
    return TSK_OK;
}
