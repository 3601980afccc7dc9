// Mode-1 Gram of the training tensor, G = A_(1) A_(1)^T = sum_d A_d A_d^T
// (Section 3.1, eqs. 3.2-3.3).  FP32 MFMA products, FP32 accumulation inside
// a chunk of slices, ordered FP64 reduction across chunks.
//
// Work decomposition
//  * G's lower triangle is cut into 128x128 tiles (bi >= bj), T tiles.
//  * The slices are cut into nchunks = 8 * per_xcd contiguous chunks.
//  * One workgroup = (tile, chunk).  Workgroup w runs on XCD w % 8, so the
//    id is laid out as w = 8 * (T * sub + t) + xcd with chunk = xcd * per_xcd
//    + sub: all tiles of a chunk run on the same XCD at about the same time
//    and share that chunk's rows through its L2.
//  * Each of the 4 waves owns a 64x64 quarter of the tile: 4x4 MFMA
//    16x16x4 f32 tiles accumulated in registers.
//  * The contraction index (slice, column) can be visited in any order as
//    long as both operands use the same order, so each lane loads 2 float4
//    (columns c0+4q..+3 and c0+16+4q..+3 of one row) and feeds component u
//    of them to MFMA number u: row reads are 128 contiguous bytes per row.
#include "tsk_common.hpp"

namespace {

constexpr int GT = 128;

__device__ __forceinline__ void tile_coords(int t, int &bi, int &bj) {
    int b = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((b + 1) * (b + 2) / 2 <= t) ++b;
    while (b > 0 && b * (b + 1) / 2 > t) --b;
    bi = b;
    bj = t - b * (b + 1) / 2;
}

__device__ __forceinline__ void load_row8(const float *__restrict__ row, int64_t c0, int q, int64_t n,
                                          bool fast, bool valid, float (&v)[8]) {
    if (!valid) {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = 0.f;
        return;
    }
    if (fast) {
        const float4 x = *reinterpret_cast<const float4 *>(row + c0 + 4 * q);
        const float4 y = *reinterpret_cast<const float4 *>(row + c0 + 16 + 4 * q);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ca = c0 + 4 * q + u, cb = c0 + 16 + 4 * q + u;
            v[u] = ca < n ? row[ca] : 0.f;
            v[4 + u] = cb < n ? row[cb] : 0.f;
        }
    }
}

__global__ __launch_bounds__(256) void gram_f32_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                       int64_t ld, int64_t stride, int64_t count, int T,
                                                       int nchunks, int per_xcd, float *__restrict__ part) {
    const int w = blockIdx.x;
    const int xcd = w & 7, local = w >> 3;
    const int t = local % T, sub = local / T;
    const int chunk = xcd * per_xcd + sub;
    const int64_t d0 = (int64_t)chunk * count / nchunks;
    const int64_t d1 = (int64_t)(chunk + 1) * count / nchunks;
    if (d0 >= d1) return;
    int bi, bj;
    tile_coords(t, bi, bj);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, ii = lane & 15;
    const int64_t rbase = (int64_t)bi * GT + (wv >> 1) * 64;
    const int64_t cbase = (int64_t)bj * GT + (wv & 1) * 64;
    const bool same = (rbase == cbase);

    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int64_t d = d0; d < d1; ++d) {
        const float *Ad = A + d * stride;
        const float *ra[4], *rb[4];
        bool va[4], vb[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int64_t r = rbase + x * 16 + ii, c = cbase + x * 16 + ii;
            va[x] = r < m;
            vb[x] = c < m;
            ra[x] = Ad + (va[x] ? r : 0) * ld;
            rb[x] = Ad + (vb[x] ? c : 0) * ld;
        }
        for (int64_t c0 = 0; c0 < n; c0 += 32) {
            const bool fast = (c0 + 32 <= n);
            float a[4][8], b[4][8];
#pragma unroll
            for (int x = 0; x < 4; ++x) load_row8(ra[x], c0, q, n, fast, va[x], a[x]);
            if (same) {
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int u = 0; u < 8; ++u) b[x][u] = a[x][u];
            } else {
#pragma unroll
                for (int x = 0; x < 4; ++x) load_row8(rb[x], c0, q, n, fast, vb[x], b[x]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x4_f32(a[x][u], b[y][u], acc[x][y]);
        }
    }
    float *P = part + ((int64_t)chunk * T + t) * (GT * GT);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int lr = (wv >> 1) * 64 + x * 16 + 4 * q + r;
                const int lc = (wv & 1) * 64 + y * 16 + ii;
                P[lr * GT + lc] = acc[x][y][r];
            }
}

// G[i][j] = sum over non-empty chunks (in chunk order) of the partial tiles,
// in FP64; diagonal tiles use their lower entry for both (i,j) and (j,i).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const float *__restrict__ part, int64_t m,
                                                          int64_t count, int T, int nchunks,
                                                          double *__restrict__ G) {
    const int t = blockIdx.x / (GT * GT / 256);
    const int e = (blockIdx.x % (GT * GT / 256)) * 256 + threadIdx.x;
    const int lr = e / GT, lc = e % GT;
    int bi, bj;
    tile_coords(t, bi, bj);
    const int64_t i = (int64_t)bi * GT + lr, j = (int64_t)bj * GT + lc;
    if (i >= m || j >= m) return;
    if (bi == bj && lr < lc) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const int64_t d0 = (int64_t)c * count / nchunks, d1 = (int64_t)(c + 1) * count / nchunks;
        if (d0 >= d1) continue;
        s += (double)part[((int64_t)c * T + t) * (GT * GT) + e];
    }
    G[i * m + j] = s;
    G[j * m + i] = s;
}

}  // namespace

// Enqueue the Gram of a validated FP32 stack into device G (m x m FP64).
tsk_status tsk_gram_enqueue(tsk_ctx c, const tsk_stack *s, double *G) {
    const int64_t m = s->m, count = s->count;
    const int nb = (int)((m + GT - 1) / GT);
    const int T = nb * (nb + 1) / 2;
    int per_xcd = (2048 + 8 * T - 1) / (8 * T);
    const int64_t cap = count / 8;
    if (per_xcd > cap) per_xcd = (int)(cap > 1 ? cap : 1);
    if (per_xcd < 1) per_xcd = 1;
    const int nchunks = 8 * per_xcd;
    const size_t part_bytes = (size_t)nchunks * T * GT * GT * sizeof(float);
    TSK_TRY(tsk_grow(c, c->gram_part, part_bytes));
    float *part = (float *)c->gram_part.p;
    const unsigned grid = (unsigned)(8 * per_xcd * T);
    TSK_LAUNCH(c, TSK_KERNEL_GRAM,
               hipLaunchKernelGGL(gram_f32_kernel, dim3(grid), dim3(256), 0, c->stream,
                                  (const float *)s->A, m, s->n, s->ld, s->stride, count, T, nchunks,
                                  per_xcd, part));
    TSK_LAUNCH(c, TSK_KERNEL_GRAM_REDUCE,
               hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)(T * (GT * GT / 256))), dim3(256), 0,
                                  c->stream, (const float *)part, m, count, T, nchunks, G));
    return TSK_OK;
}
