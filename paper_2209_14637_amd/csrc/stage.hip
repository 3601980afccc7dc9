// Staging of FP32 slices into the storage format of a reduced-precision
// form (the paper fixes no precision; these formats are this library's
// production forms):
//   bf16 : round to nearest even, one pass;
//   e4m3 : per-slice power-of-two scale s_d = 2^floor(log2(448 / amax_d))
//          (so |x s_d| <= 448 and nothing saturates), then x s_d rounded to
//          nearest even; two passes (amax first).
// Both also give ||A_d||_F^2 of the FP32 source in FP64 (summed in a fixed
// order, so it is reproducible).  Every kernel is a coalesced stream:
// thread work item = 8 consecutive elements of one row.
#include "tsk_common.hpp"

namespace {

constexpr int ST_ROWS = 16;  // rows per workgroup

__device__ __forceinline__ void load8(const float *__restrict__ p, int64_t c, int64_t n, float (&x)[8]) {
    if (c + 7 < n) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        const float4 b = *reinterpret_cast<const float4 *>(p + 4);
        x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
        x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = c + e < n ? p[e] : 0.f;
    }
}

// bf16: dst = RNE(src); part[d * gridDim.x + block] = FP64 sum of squares.
__global__ __launch_bounds__(256) void stage_bf16_kernel(const float *__restrict__ src, int64_t m, int64_t n,
                                                         int64_t ld, int64_t stride, uint16_t *__restrict__ dst,
                                                         int64_t ldd, int64_t strided, double *__restrict__ part) {
    __shared__ double red[4];
    const int64_t d = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * ST_ROWS;
    const int gpr = (int)((n + 7) / 8);
    const int rows = (int)(m - r0 < ST_ROWS ? m - r0 : ST_ROWS);
    const float *S = src + d * stride;
    uint16_t *D = dst + d * strided;
    double ss = 0.0;
    for (int e = threadIdx.x; e < rows * gpr; e += 256) {
        const int64_t row = r0 + e / gpr;
        const int64_t c = (int64_t)(e % gpr) * 8;
        float x[8];
        load8(S + row * ld + c, c, n, x);
#pragma unroll
        for (int u = 0; u < 8; ++u) ss += (double)x[u] * (double)x[u];
        const v4u w = v4u{pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]), pack_bf16(x[4], x[5]), pack_bf16(x[6], x[7])};
        uint16_t *q = D + row * ldd + c;
        if (c + 7 < n) {
            *reinterpret_cast<v4u *>(q) = w;
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (c + u < n) q[u] = (uint16_t)(w[u >> 1] >> (16 * (u & 1)));
        }
    }
    ss = block_sum_f64(ss, red);
    if (threadIdx.x == 0 && part) part[d * gridDim.x + blockIdx.x] = ss;
}

// e4m3 pass 1: per-block amax and FP64 sum of squares.
__global__ __launch_bounds__(256) void stage_amax_kernel(const float *__restrict__ src, int64_t m, int64_t n,
                                                         int64_t ld, int64_t stride, double *__restrict__ part,
                                                         float *__restrict__ amax_part) {
    __shared__ double red[4];
    __shared__ float redm[4];
    const int64_t d = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * ST_ROWS;
    const int gpr = (int)((n + 7) / 8);
    const int rows = (int)(m - r0 < ST_ROWS ? m - r0 : ST_ROWS);
    const float *S = src + d * stride;
    double ss = 0.0;
    float mx = 0.f;
    for (int e = threadIdx.x; e < rows * gpr; e += 256) {
        const int64_t row = r0 + e / gpr;
        const int64_t c = (int64_t)(e % gpr) * 8;
        float x[8];
        load8(S + row * ld + c, c, n, x);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            ss += (double)x[u] * (double)x[u];
            mx = fmaxf(mx, fabsf(x[u]));
        }
    }
    ss = block_sum_f64(ss, red);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[d * gridDim.x + blockIdx.x] = ss;
        amax_part[d * gridDim.x + blockIdx.x] = fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3]));
    }
}

// Per slice: norm2 = ordered sum of the block partials; for e4m3 also the
// scale 2^j, j = floor(log2(448 / amax)) from amax = fa 2^ea (1/2 <= fa < 1):
// 448 / amax = (0.875 / fa) 2^(9 - ea) and 0.875 / fa lies in (0.875, 1.75],
// so j = 9 - ea when fa <= 0.875 and 8 - ea otherwise; clamped to
// [-126, 127]; amax 0 (or non-finite) gives 1.
__global__ void stage_final_kernel(const double *__restrict__ part, const float *__restrict__ amax_part, int nblk,
                                   int64_t count, double *__restrict__ norm2, float *__restrict__ scale) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= count) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[d * nblk + b];
    if (norm2) norm2[d] = s;
    if (scale) {
        float amax = 0.f;
        for (int b = 0; b < nblk; ++b) amax = fmaxf(amax, amax_part[d * nblk + b]);
        float sc = 1.f;
        if (amax > 0.f && isfinite(amax)) {
            int ea;
            const float fa = frexpf(amax, &ea);
            int j = fa <= 0.875f ? 9 - ea : 8 - ea;
            j = j > 127 ? 127 : (j < -126 ? -126 : j);
            sc = ldexpf(1.f, j);
        }
        scale[d] = sc;
    }
}

// e4m3 pass 2: dst = RNE(src * scale_d) (exact product: power-of-two scale).
__global__ __launch_bounds__(256) void stage_e4m3_kernel(const float *__restrict__ src, int64_t m, int64_t n,
                                                         int64_t ld, int64_t stride, const float *__restrict__ scale,
                                                         uint8_t *__restrict__ dst, int64_t ldd, int64_t strided) {
    const int64_t d = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * ST_ROWS;
    const int gpr = (int)((n + 7) / 8);
    const int rows = (int)(m - r0 < ST_ROWS ? m - r0 : ST_ROWS);
    const float *S = src + d * stride;
    uint8_t *D = dst + d * strided;
    const float sc = scale[d];
    for (int e = threadIdx.x; e < rows * gpr; e += 256) {
        const int64_t row = r0 + e / gpr;
        const int64_t c = (int64_t)(e % gpr) * 8;
        float x[8];
        load8(S + row * ld + c, c, n, x);
        unsigned w0 = 0u, w1 = 0u;
        w0 = __builtin_amdgcn_cvt_pk_fp8_f32(x[0] * sc, x[1] * sc, w0, false);
        w0 = __builtin_amdgcn_cvt_pk_fp8_f32(x[2] * sc, x[3] * sc, w0, true);
        w1 = __builtin_amdgcn_cvt_pk_fp8_f32(x[4] * sc, x[5] * sc, w1, false);
        w1 = __builtin_amdgcn_cvt_pk_fp8_f32(x[6] * sc, x[7] * sc, w1, true);
        uint8_t *q = D + row * ldd + c;
        if (c + 7 < n) {
            *reinterpret_cast<uint2 *>(q) = uint2{w0, w1};
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (c + u < n) q[u] = (uint8_t)((u < 4 ? w0 : w1) >> (8 * (u & 3)));
        }
    }
}

// Block-scaled e4m3 (the MX layout: one power of two per 32 consecutive
// elements of a row).  A group of 8 lanes takes one block, 4 values per
// lane; the block's amax by a 3-step exchange within the group; its
// exponent j as in stage_final_kernel (0 for an all-zero block); the values
// times 2^j (exact) rounded to nearest even; bscale[block] = 127 - j.
// Blocks are numbered (slice, row, block) in row-major order.
__global__ __launch_bounds__(256) void stage_mx_kernel(const float *__restrict__ src, int64_t m, int64_t n,
                                                       int64_t ld, int64_t stride, int64_t count,
                                                       uint8_t *__restrict__ dst, int64_t ldd, int64_t strided,
                                                       uint8_t *__restrict__ bscale, int64_t nbk) {
    const int64_t g = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 3;
    const int l = threadIdx.x & 7;
    const bool live = g < count * m * nbk;
    const int64_t b = live ? g % nbk : 0, row = live ? (g / nbk) % m : 0, d = live ? g / (nbk * m) : 0;
    const int64_t c = b * 32 + 4 * l;
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    if (live && c < n) {
        const float *p = src + d * stride + row * ld + c;
        if (c + 3 < n) {
            const float4 v = *reinterpret_cast<const float4 *>(p);
            x[0] = v.x;
            x[1] = v.y;
            x[2] = v.z;
            x[3] = v.w;
        } else {
            for (int e = 0; c + e < n; ++e) x[e] = p[e];
        }
    }
    float amax = fmaxf(fmaxf(fabsf(x[0]), fabsf(x[1])), fmaxf(fabsf(x[2]), fabsf(x[3])));
    amax = fmaxf(amax, __shfl_xor(amax, 1));
    amax = fmaxf(amax, __shfl_xor(amax, 2));
    amax = fmaxf(amax, __shfl_xor(amax, 4));
    int j = 0;
    if (amax > 0.f && isfinite(amax)) {
        int ea;
        const float fa = frexpf(amax, &ea);
        j = fa <= 0.875f ? 9 - ea : 8 - ea;
        j = j > 127 ? 127 : (j < -126 ? -126 : j);
    }
    const float sc = ldexpf(1.f, j);
    unsigned w = __builtin_amdgcn_cvt_pk_fp8_f32(x[0] * sc, x[1] * sc, 0u, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(x[2] * sc, x[3] * sc, w, true);
    if (!live) return;
    if (c < n) {
        uint8_t *q = dst + d * strided + row * ldd + c;
        if (c + 3 < n) {
            *reinterpret_cast<unsigned *>(q) = w;
        } else {
            for (int e = 0; c + e < n; ++e) q[e] = (uint8_t)(w >> (8 * e));
        }
    }
    if (l == 0) bscale[g] = (uint8_t)(127 - j);
}

}  // namespace

tsk_status tsk_stage_mx_enqueue(tsk_ctx c, const tsk_stack *s, void *dst, int64_t ldd, int64_t strided,
                                uint8_t *bscale) {
    const int64_t nbk = (s->n + 31) / 32;
    const int64_t groups = s->count * s->m * nbk;
    const int64_t blocks = (groups * 8 + 255) / 256;
    TSK_LAUNCH(c, TSK_KERNEL_STAGE,
               hipLaunchKernelGGL(stage_mx_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                                  (const float *)s->A, s->m, s->n, s->ld, s->stride, s->count, (uint8_t *)dst, ldd,
                                  strided, bscale, nbk));
    return TSK_OK;
}

tsk_status tsk_stage_enqueue(tsk_ctx c, const tsk_stack *s, int dtype, void *dst, int64_t ldd, int64_t strided,
                             float *scale, double *norm2) {
    const int64_t m = s->m, n = s->n, count = s->count;
    const int nblk = (int)((m + ST_ROWS - 1) / ST_ROWS);
    const bool e4m3 = dtype == TSK_F8E4M3;
    const size_t np = (size_t)nblk * count;
    TSK_TRY(tsk_grow(c, c->st_part, np * (sizeof(double) + sizeof(float))));
    double *part = (double *)c->st_part.p;
    float *amax_part = (float *)(part + np);
    const dim3 g((unsigned)nblk, (unsigned)count);
    const float *A = (const float *)s->A;
    if (!e4m3) {
        TSK_LAUNCH(c, TSK_KERNEL_STAGE,
                   hipLaunchKernelGGL(stage_bf16_kernel, g, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride,
                                      (uint16_t *)dst, ldd, strided, norm2 ? part : nullptr));
        if (norm2)
            TSK_LAUNCH(c, TSK_KERNEL_STAGE,
                       hipLaunchKernelGGL(stage_final_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                                          c->stream, (const double *)part, (const float *)nullptr, nblk, count,
                                          norm2, (float *)nullptr));
        return TSK_OK;
    }
    TSK_LAUNCH(c, TSK_KERNEL_STAGE,
               hipLaunchKernelGGL(stage_amax_kernel, g, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, part,
                                  amax_part));
    TSK_LAUNCH(c, TSK_KERNEL_STAGE,
               hipLaunchKernelGGL(stage_final_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream,
                                  (const double *)part, (const float *)amax_part, nblk, count, norm2, scale));
    TSK_LAUNCH(c, TSK_KERNEL_STAGE,
               hipLaunchKernelGGL(stage_e4m3_kernel, g, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride,
                                  (const float *)scale, (uint8_t *)dst, ldd, strided));
    return TSK_OK;
}
