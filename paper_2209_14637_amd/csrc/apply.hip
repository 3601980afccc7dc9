// SCW (Algorithm 1) on a stack of test matrices, FP32 path.
//
//  sketch  : B_d = S A_d (k x n), the 1-mode product of Section 2 slice by
//            slice, FP32 MFMA; also ||A_d||_F^2 in FP64.
//  cholqr2 : V_d^T = orthonormal basis of the row space of B_d (k x n) by
//            CholeskyQR2 in FP64 -- Section 3.2 allows QR in place of the SVD
//            of line 1 because only the orthogonalisation is used.
//  project : C_d = A_d V_d (m x k), FP32 MFMA (second pass over A_d).
//  finish  : C_d^T C_d = Y diag(sigma^2) Y^T (FP64 Jacobi), rank-r truncation,
//            L_d = C_d Y_r, R_d = V_d Y_r, sigma, and the error from the
//            Pythagorean identity of the proof of Theorem 1.
//  error   : explicit ||A_d - L_d R_d^T||_F / ||A_d||_F (tsk_error).
//
// MFMA operand layout: see tsk_common.hpp.  kp = k rounded up to 16; the
// padded rows of S / columns of V are zero so no masking is needed on them.
#include "tsk_common.hpp"

namespace {

// One wave per workgroup: 400 matrices x 12 panels is 4800 equal work units,
// a little over the machine's resident-wave count, and single waves let the
// last units run at full speed on otherwise idle SIMDs.
constexpr int SK_PANEL = 64;   // columns of A_d per sketch workgroup (one wave)
constexpr int PJ_ROWS = 64;    // rows of A_d per project workgroup (one wave)
constexpr int MAXK = 64;
constexpr int NTRI_PER_THREAD = (MAXK * (MAXK + 1) / 2 + 255) / 256;  // upper-triangle entries per thread

// St (m x kp) = S^T with zero columns k..kp-1
__global__ void transpose_sketch_kernel(const float *__restrict__ S, int k, int kp, int64_t m,
                                        float *__restrict__ St) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * kp) return;
    const int64_t i = e / kp;
    const int s = (int)(e % kp);
    St[e] = s < k ? S[(int64_t)s * m + i] : 0.f;
}

template <int MT>
__global__ __launch_bounds__(64) void sketch_f32_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                         int64_t ld, int64_t stride, const float *__restrict__ St,
                                                         float *__restrict__ B, int64_t ldb,
                                                         double *__restrict__ fro_part, int npanel) {
    constexpr int kp = MT * 16;
    const int64_t d = blockIdx.y;
    const int panel = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, jj = lane & 15;
    const int64_t col4 = (int64_t)panel * SK_PANEL + 4 * jj;  // this lane's 4 columns
    const bool full = col4 + 3 < n;
    const bool any = col4 < n;
    const float *Ad = A + d * stride;
    v4f acc[MT][4];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[a][t] = v4f{0.f, 0.f, 0.f, 0.f};
    double fro = 0.0;
    constexpr int U = 8;  // row groups of 4 in flight
    for (int64_t i0 = 0; i0 < m; i0 += 4 * U) {
        float4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = i0 + 4 * u + q;
            x[u] = float4{0.f, 0.f, 0.f, 0.f};
            if (row < m && any) {
                const float *p = Ad + row * ld + col4;
                if (full) {
                    x[u] = *reinterpret_cast<const float4 *>(p);
                } else {
                    x[u].x = p[0];
                    if (col4 + 1 < n) x[u].y = p[1];
                    if (col4 + 2 < n) x[u].z = p[2];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = i0 + 4 * u + q;
            fro += (double)x[u].x * x[u].x + (double)x[u].y * x[u].y + (double)x[u].z * x[u].z +
                   (double)x[u].w * x[u].w;
            float s[MT];
#pragma unroll
            for (int a = 0; a < MT; ++a) s[a] = row < m ? St[row * kp + a * 16 + jj] : 0.f;
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                acc[a][0] = mfma16x16x4_f32(s[a], x[u].x, acc[a][0]);
                acc[a][1] = mfma16x16x4_f32(s[a], x[u].y, acc[a][1]);
                acc[a][2] = mfma16x16x4_f32(s[a], x[u].z, acc[a][2]);
                acc[a][3] = mfma16x16x4_f32(s[a], x[u].w, acc[a][3]);
            }
        }
    }
    // lane holds B[a*16 + 4q + r][col4 + t] in acc[a][t][r]
    if (any) {
        float *Bd = B + d * kp * ldb;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int srow = a * 16 + 4 * q + r;
                float4 v = float4{acc[a][0][r], acc[a][1][r], acc[a][2][r], acc[a][3][r]};
                *reinterpret_cast<float4 *>(Bd + srow * ldb + col4) = v;
            }
    }
    const double tot = wave_sum_f64(fro);
    if (threadIdx.x == 0) fro_part[d * npanel + panel] = tot;
}

// ---------------------------------------------------------------------------
// Small dense helpers, one workgroup (256 threads) per matrix.
// ---------------------------------------------------------------------------

// Gram of k vectors stored as the ROWS of X (k x n, row stride ldx, FP32):
// C[a][b] = sum_c X[a][c] X[b][c] in FP64 (full symmetric, LDS stride ld).
// Work: 4x4 register blocks of C (a-block <= b-block) x column slices, float4
// loads over 4 consecutive columns; slices summed through LDS (scratch:
// 256*16 doubles).  Columns in [n, round4(n)) must hold zeros.
__device__ inline void row_gram(const float *__restrict__ X, int64_t ldx, int k, int64_t n, double *C, int ld,
                                double *scratch) {
    const int nb = (k + 3) / 4;
    const int nblk = nb * (nb + 1) / 2;
    const int ns = 256 / nblk;
    const int tid = threadIdx.x;
    const int sl = tid / nblk, blk = tid % nblk;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    int ta = 0, tb = 0;
    if (sl < ns) {
        int e = blk, rr = 0, len = nb;
        while (e >= len) {
            e -= len;
            ++rr;
            --len;
        }
        ta = rr;
        tb = rr + e;
        const float *xa[4], *xb[4];
        bool va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            va[u] = 4 * ta + u < k;
            vb[u] = 4 * tb + u < k;
            xa[u] = X + (va[u] ? 4 * ta + u : 0) * ldx;
            xb[u] = X + (vb[u] ? 4 * tb + u : 0) * ldx;
        }
        for (int64_t c4 = 4 * (int64_t)sl; c4 < n; c4 += 4 * ns) {
            float4 fa[4], fb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                fa[u] = va[u] ? *reinterpret_cast<const float4 *>(xa[u] + c4) : float4{0.f, 0.f, 0.f, 0.f};
                fb[u] = vb[u] ? *reinterpret_cast<const float4 *>(xb[u] + c4) : float4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[u * 4 + v] += (double)fa[u].x * fb[v].x + (double)fa[u].y * fb[v].y +
                                      (double)fa[u].z * fb[v].z + (double)fa[u].w * fb[v].w;
        }
    }
    __syncthreads();
    if (sl < ns) {
#pragma unroll
        for (int u = 0; u < 16; ++u) scratch[(sl * nblk + blk) * 16 + u] = acc[u];
    }
    __syncthreads();
    for (int e = tid; e < nblk * 16; e += 256) {
        const int bk = e / 16, u = e % 16;
        double sum = 0.0;
        for (int z = 0; z < ns; ++z) sum += scratch[(z * nblk + bk) * 16 + u];
        int ee = bk, rr = 0, len = nb;
        while (ee >= len) {
            ee -= len;
            ++rr;
            --len;
        }
        const int a = 4 * rr + u / 4, b = 4 * (rr + ee) + u % 4;
        if (a < k && b < k) {
            C[a * ld + b] = sum;
            C[b * ld + a] = sum;
        }
    }
    __syncthreads();
}

// dst (KP x ldv) = Rinv^T src for the first k rows, FP32; rows k..KP-1 and
// columns n..ldv-1 are written as zero.  Rf: Rinv (KP x KP, FP32, LDS).
template <int KP>
__device__ inline void apply_rinv_t(const float *__restrict__ src, float *__restrict__ dst, int64_t ldv, int k,
                                    int64_t n, const float *Rf, uint16_t *__restrict__ vb = nullptr) {
    for (int64_t c = threadIdx.x; c < ldv; c += blockDim.x) {
        float col[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) col[t] = (t < k && c < n) ? src[t * ldv + c] : 0.f;
        // Rf is upper triangular (zero below the diagonal): full-length dot
        // products keep col[] statically indexed, i.e. in registers
#pragma nounroll
        for (int i = 0; i < KP; ++i) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < KP; ++t) s += Rf[t * KP + i] * col[t];
            dst[i * ldv + c] = s;
            if (vb) {
                // bf16 pair: hi = RNE(s), lo = RNE(s - hi) (s - hi is exact)
                const unsigned h = pack_bf16(s, 0.f) & 0xffffu;
                const unsigned l = pack_bf16(s - bf16_lo(h), 0.f) & 0xffffu;
                vb[i * ldv + c] = (uint16_t)h;
                vb[(KP + i) * ldv + c] = (uint16_t)l;
            }
        }
    }
}

// CholeskyQR2 of B_d^T: V_d^T (k x n, rows orthonormal) spans the row space
// of B_d.  Grams in FP64 from FP32 data, Cholesky and inverse in FP64, the
// triangular application in FP32 (the span does not depend on the accuracy
// of R; the second pass restores orthogonality).  Dead pivots in the first
// pass (singular-value ratio below 1e-6, the FP32 rounding level of B) flag
// the matrix as rank deficient and leave zero rows in V^T.
template <int KP>
__global__ __launch_bounds__(256) void cholqr2_kernel(const float *__restrict__ B, int64_t ldv,
                                                      float *__restrict__ Vt, int k, int64_t n,
                                                      int *__restrict__ qflag, uint16_t *__restrict__ Vb) {
    // C | R | X (KP*KP doubles each); the Gram's slice scratch (4096 doubles)
    // sits after C and is dead once C is assembled
    constexpr int SCR = (3 * KP * KP > KP * KP + 4096) ? 3 * KP * KP : KP * KP + 4096;
    __shared__ double lds[SCR];
    __shared__ float Rf[KP * KP];
    __shared__ int dead[KP];
    double *C = lds, *R = lds + KP * KP, *X = lds + 2 * KP * KP;
    const int64_t d = blockIdx.x;
    const float *Bd = B + d * KP * ldv;
    float *Vd = Vt + d * KP * ldv;
    int nd1 = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const float *src = pass == 0 ? Bd : Vd;
        for (int e = threadIdx.x; e < KP * KP; e += 256) lds[e] = 0.0;
        __syncthreads();
        row_gram(src, ldv, k, n, C, KP, lds + KP * KP);
        const int nd = chol_factor_inverse(C, KP, KP, 1e-12, R, X, dead, k);
        if (pass == 0) nd1 = nd;
        for (int e = threadIdx.x; e < KP * KP; e += 256) Rf[e] = (float)X[e];
        __syncthreads();
        apply_rinv_t<KP>(src, Vd, ldv, k, n, Rf, (pass == 1 && Vb) ? Vb + d * 2 * KP * ldv : nullptr);
        __syncthreads();
    }
    if (threadIdx.x == 0) qflag[d] = nd1 > 0 ? TSK_FLAG_RANKDEF : 0;
}

// ---------------------------------------------------------------------------
// C_d = A_d V_d
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(64) void project_f32_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                          int64_t ld, int64_t stride, const float *__restrict__ Vt,
                                                          int64_t ldv, float *__restrict__ C) {
    constexpr int kp = NT * 16;
    const int64_t d = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, ii = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * PJ_ROWS;
    const float *Ad = A + d * stride;
    const float *Vd = Vt + d * kp * ldv;
    const float *arow[4];
    bool av[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t row = r0 + a * 16 + ii;
        av[a] = row < m;
        arow[a] = Ad + (av[a] ? row : 0) * ld;
    }
    v4f acc[4][NT];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int64_t c0 = 0; c0 < n; c0 += 16) {
        const int64_t cc = c0 + 4 * q;
        const bool full = cc + 3 < n;
        float4 xa[4], xb[NT];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            xa[a] = float4{0.f, 0.f, 0.f, 0.f};
            if (av[a] && cc < n) {
                if (full) {
                    xa[a] = *reinterpret_cast<const float4 *>(arow[a] + cc);
                } else {
                    xa[a].x = arow[a][cc];
                    if (cc + 1 < n) xa[a].y = arow[a][cc + 1];
                    if (cc + 2 < n) xa[a].z = arow[a][cc + 2];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NT; ++b) xb[b] = *reinterpret_cast<const float4 *>(Vd + (b * 16 + ii) * ldv + cc);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                acc[a][b] = mfma16x16x4_f32(xa[a].x, xb[b].x, acc[a][b]);
                acc[a][b] = mfma16x16x4_f32(xa[a].y, xb[b].y, acc[a][b]);
                acc[a][b] = mfma16x16x4_f32(xa[a].z, xb[b].z, acc[a][b]);
                acc[a][b] = mfma16x16x4_f32(xa[a].w, xb[b].w, acc[a][b]);
            }
    }
    float *Cd = C + d * m * kp;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + a * 16 + 4 * q + r;
            if (row < m) {
#pragma unroll
                for (int b = 0; b < NT; ++b) Cd[row * kp + b * 16 + ii] = acc[a][b][r];
            }
        }
}

// ---------------------------------------------------------------------------
// bf16 form.  A_d is stored in bf16; S and V_d are each split into a bf16
// pair (hi + lo), two MFMAs per product, so the products carry about 16
// significant bits of S and V and the only extra rounding is that of A_d.
// ---------------------------------------------------------------------------
constexpr int SKB_PANEL = 128;  // columns per sketch wave (16 lanes x 8)
constexpr int PJB_ROWS = 128;   // rows per project wave (8 row tiles)

// Sb = [S_hi; S_lo], each kp x mp bf16 with zero padding (rows >= k,
// columns >= m).
__global__ void prep_sketch_bf16_kernel(const float *__restrict__ S, int k, int kp, int64_t m, int64_t mp,
                                        uint16_t *__restrict__ Sb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)kp * mp) return;
    const int s = (int)(e / mp);
    const int64_t i = e % mp;
    const float x = (s < k && i < m) ? S[(int64_t)s * m + i] : 0.f;
    const unsigned h = pack_bf16(x, 0.f) & 0xffffu;
    const unsigned l = pack_bf16(x - bf16_lo(h), 0.f) & 0xffffu;
    Sb[e] = (uint16_t)h;
    Sb[(int64_t)kp * mp + e] = (uint16_t)l;
}

__device__ __forceinline__ v4u load_bf16x8(const uint16_t *p, int64_t c, int64_t n) {
    if (c + 7 < n) return *reinterpret_cast<const v4u *>(p);
    unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (c + e < n) w[e >> 1] |= (unsigned)p[e] << (16 * (e & 1));
    return v4u{w[0], w[1], w[2], w[3]};
}

// B_d = S A_d.  The contraction runs over the rows of A_d, but an MFMA lane
// needs 8 consecutive contraction indices: lane (q, i) loads 16 bytes (8
// columns) from each of the 8 rows r0 + 8q + e and transposes the 8 x 8
// block in registers, so that MFMA u (u = 0..7) takes column c0 + 8i + u
// of those 8 rows.  One wave covers 128 columns, 32 rows per step; the next
// step's rows are in flight during the MFMAs.  ||A_d||^2 is accumulated from
// the same registers (FP32 per step, FP64 across steps).
template <int MT>
__global__ __launch_bounds__(64) void sketch_bf16_kernel(const uint16_t *__restrict__ A, int64_t m, int64_t n,
                                                          int64_t ld, int64_t stride, const uint16_t *__restrict__ Sb,
                                                          int64_t mp, float *__restrict__ B, int64_t ldb,
                                                          double *__restrict__ fro_part, int npanel) {
    constexpr int kp = MT * 16;
    const int64_t d = blockIdx.y;
    const int panel = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, ii = lane & 15;
    const int64_t c8 = (int64_t)panel * SKB_PANEL + 8 * ii;
    const bool any = c8 < n;
    const uint16_t *Ad = A + d * stride + (any ? c8 : 0);
    const uint16_t *Sh = Sb + (int64_t)ii * mp + 8 * q;
    const uint16_t *Sl = Sh + (int64_t)kp * mp;
    v4f acc[MT][8];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[a][u] = v4f{0.f, 0.f, 0.f, 0.f};
    double fro = 0.0;
    v4u x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t row = 8 * q + e;
        x[e] = (any && row < m) ? load_bf16x8(Ad + row * ld, c8, n) : v4u{0u, 0u, 0u, 0u};
    }
    for (int64_t r0 = 0; r0 < m; r0 += 32) {
        const bool more = r0 + 32 < m;
        v4u nx[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t row = r0 + 32 + 8 * q + e;
            nx[e] = (more && any && row < m) ? load_bf16x8(Ad + row * ld, c8, n) : v4u{0u, 0u, 0u, 0u};
        }
        v4u sh[MT], sl[MT];
#pragma unroll
        for (int a = 0; a < MT; ++a) {
            sh[a] = *reinterpret_cast<const v4u *>(Sh + (int64_t)a * 16 * mp + r0);
            sl[a] = *reinterpret_cast<const v4u *>(Sl + (int64_t)a * 16 * mp + r0);
        }
        float f = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) f += sumsq_bf16x8(x[e]);
        fro += (double)f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = u >> 1;
            v4u bt;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const unsigned lo = x[2 * t][j], hi = x[2 * t + 1][j];
                bt[t] = (u & 1) ? ((lo >> 16) | (hi & 0xffff0000u)) : ((lo & 0xffffu) | (hi << 16));
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                acc[a][u] = mfma16x16x32_bf16(sh[a], bt, acc[a][u]);
                acc[a][u] = mfma16x16x32_bf16(sl[a], bt, acc[a][u]);
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = nx[e];
    }
    // lane holds B[a*16 + 4q + r][c8 + u] in acc[a][u][r]
    if (any) {
        float *Bd = B + d * kp * ldb + c8;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float *o = Bd + (int64_t)(a * 16 + 4 * q + r) * ldb;
                *reinterpret_cast<float4 *>(o) = float4{acc[a][0][r], acc[a][1][r], acc[a][2][r], acc[a][3][r]};
                *reinterpret_cast<float4 *>(o + 4) = float4{acc[a][4][r], acc[a][5][r], acc[a][6][r], acc[a][7][r]};
            }
    }
    const double tot = wave_sum_f64(fro);
    if (threadIdx.x == 0) fro_part[d * npanel + panel] = tot;
}

// C_d = A_d V_d: contraction over the columns of A_d (contiguous), so lane
// (q, i) reads 8 consecutive columns of row i of each of 8 row tiles; V_d^T
// rows give the other operand directly.  One wave covers 128 rows.
template <int NT>
__global__ __launch_bounds__(64) void project_bf16_kernel(const uint16_t *__restrict__ A, int64_t m, int64_t n,
                                                           int64_t ld, int64_t stride, const uint16_t *__restrict__ Vb,
                                                           int64_t ldv, float *__restrict__ C) {
    constexpr int kp = NT * 16;
    const int64_t d = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, ii = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * PJB_ROWS;
    const uint16_t *Ad = A + d * stride;
    const uint16_t *arow[8];
    bool av[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int64_t row = r0 + a * 16 + ii;
        av[a] = row < m;
        arow[a] = Ad + (av[a] ? row : 0) * ld + 8 * q;
    }
    const uint16_t *Vh = Vb + d * 2 * kp * ldv + (int64_t)ii * ldv + 8 * q;
    const uint16_t *Vl = Vh + (int64_t)kp * ldv;
    v4f acc[8][NT];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    v4u xa[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) xa[a] = (av[a] && 8 * q < n) ? load_bf16x8(arow[a], 8 * q, n) : v4u{0u, 0u, 0u, 0u};
    for (int64_t c0 = 0; c0 < n; c0 += 32) {
        const int64_t cn = c0 + 32 + 8 * q;  // this lane's columns in the next step
        v4u nxa[8];
#pragma unroll
        for (int a = 0; a < 8; ++a)
            nxa[a] = (av[a] && cn < n) ? load_bf16x8(arow[a] + c0 + 32, cn, n) : v4u{0u, 0u, 0u, 0u};
        v4u vh[NT], vl[NT];
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            vh[b] = *reinterpret_cast<const v4u *>(Vh + (int64_t)b * 16 * ldv + c0);
            vl[b] = *reinterpret_cast<const v4u *>(Vl + (int64_t)b * 16 * ldv + c0);
        }
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                acc[a][b] = mfma16x16x32_bf16(xa[a], vh[b], acc[a][b]);
                acc[a][b] = mfma16x16x32_bf16(xa[a], vl[b], acc[a][b]);
            }
#pragma unroll
        for (int a = 0; a < 8; ++a) xa[a] = nxa[a];
    }
    float *Cd = C + d * m * kp;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + a * 16 + 4 * q + r;
            if (row < m) {
#pragma unroll
                for (int b = 0; b < NT; ++b) Cd[row * kp + b * 16 + ii] = acc[a][b][r];
            }
        }
}

// ---------------------------------------------------------------------------
// Rank-r truncation, outputs and the fused error.  One workgroup per matrix.
//   H = C^T C (FP64), Jacobi -> Y, sigma^2 (descending); L = C Y_r,
//   R = V Y_r; relerr from ||A||^2 - sum_{i<=r} sigma_i^2.
// ---------------------------------------------------------------------------

// Gram of the KP columns of C (m x KP row-major FP32): H[a][b] = sum_i
// C[i][a] C[i][b], FP64, 4x4 register blocks x row slices (scratch: 4096).
__device__ inline void col_gram(const float *__restrict__ Cm, int KP, int k, int64_t m, double *H, int ld,
                                double *scratch) {
    const int nb = (k + 3) / 4;
    const int nblk = nb * (nb + 1) / 2;
    const int ns = 256 / nblk;
    const int tid = threadIdx.x;
    const int sl = tid / nblk, blk = tid % nblk;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    int ta = 0, tb = 0;
    {
        int e = blk, rr = 0, len = nb;
        while (e >= len) {
            e -= len;
            ++rr;
            --len;
        }
        ta = rr;
        tb = rr + e;
    }
    if (sl < ns) {
        for (int64_t i = sl; i < m; i += ns) {
            const float4 fa = *reinterpret_cast<const float4 *>(Cm + i * KP + 4 * ta);
            const float4 fb = *reinterpret_cast<const float4 *>(Cm + i * KP + 4 * tb);
            const float av[4] = {fa.x, fa.y, fa.z, fa.w}, bv[4] = {fb.x, fb.y, fb.z, fb.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u * 4 + v] += (double)av[u] * (double)bv[v];
        }
    }
    __syncthreads();
    if (sl < ns) {
#pragma unroll
        for (int u = 0; u < 16; ++u) scratch[(sl * nblk + blk) * 16 + u] = acc[u];
    }
    __syncthreads();
    for (int e = tid; e < nblk * 16; e += 256) {
        const int bk = e / 16, u = e % 16;
        double sum = 0.0;
        for (int z = 0; z < ns; ++z) sum += scratch[(z * nblk + bk) * 16 + u];
        int ee = bk, rr = 0, len = nb;
        while (ee >= len) {
            ee -= len;
            ++rr;
            --len;
        }
        const int a = 4 * rr + u / 4, b = 4 * (rr + ee) + u % 4;
        if (a < k && b < k) {
            H[a * ld + b] = sum;
            H[b * ld + a] = sum;
        }
    }
    __syncthreads();
}

template <int KP>
__global__ __launch_bounds__(256) void finish_kernel(const float *__restrict__ C, int64_t m, int k, int r,
                                                     const float *__restrict__ Vt, int64_t ldv, int64_t n,
                                                     const double *__restrict__ fro_part, int npanel,
                                                     const int *__restrict__ qflag, float *__restrict__ L,
                                                     float *__restrict__ R, float *__restrict__ sigma,
                                                     double *__restrict__ relerr, int *__restrict__ flags) {
    // H | W | Hn (KP*KP each); the Gram scratch (4096) overlaps W and Hn
    constexpr int SCR = (3 * KP * KP > KP * KP + 4096) ? 3 * KP * KP : KP * KP + 4096;
    __shared__ double lds[SCR];
    __shared__ float Yr[KP * KP];  // first r eigenvector columns, descending
    __shared__ double rot[KP];
    __shared__ int pairs[(KP - 1) * (KP / 2)];
    __shared__ int perm[KP];
    __shared__ double red4[4];
    __shared__ double s_lam[KP];
    const int64_t d = blockIdx.x;
    const int tid = threadIdx.x;
    const float *Cd = C + d * m * KP;
    double *H = lds, *W = lds + KP * KP, *Hn = lds + 2 * KP * KP;
    for (int e = tid; e < KP * KP; e += 256) H[e] = 0.0;
    __syncthreads();
    col_gram(Cd, KP, k, m, H, KP, lds + KP * KP);
    const int kk = k + (k & 1);  // even size for the parallel ordering
    H = jacobi_eig_lds(H, Hn, W, kk, KP, rot, pairs, 40, red4);
    if (tid == 0) sort_diag_desc(H, kk, KP, perm);
    __syncthreads();
    for (int t = tid; t < kk; t += 256) s_lam[t] = H[perm[t] * KP + perm[t]];
    for (int e = tid; e < KP * KP; e += 256) {
        const int u = e / KP, t = e % KP;
        Yr[e] = (u < k && t < r) ? (float)W[u * KP + perm[t]] : 0.f;
    }
    __syncthreads();
    double fro2 = 0.0;
    for (int p = 0; p < npanel; ++p) fro2 += fro_part[d * npanel + p];
    const bool finite = isfinite(fro2);
    const float qnan = __builtin_nanf("");
    if (tid < r) sigma[d * r + tid] = finite ? (float)sqrt(fmax(s_lam[tid], 0.0)) : qnan;
    if (tid == 0) {
        double cap = 0.0;
        for (int t = 0; t < r; ++t) cap += fmax(s_lam[t], 0.0);
        int fl = qflag[d];
        if (!finite) fl |= TSK_FLAG_NONFIN;
        const double sr = sqrt(fmax(s_lam[r - 1], 0.0)), sr1 = sqrt(fmax(s_lam[r], 0.0));
        const double s1 = sqrt(fmax(s_lam[0], 0.0));
        if (sr - sr1 <= 1e-6 * s1) fl |= TSK_FLAG_TIE;
        if (flags) flags[d] = fl;
        if (relerr) relerr[d] = !finite ? (double)qnan : (fro2 > 0.0 ? sqrt(fmax(fro2 - cap, 0.0) / fro2) : 0.0);
    }
    // L = C Y_r: one row of C per thread
    float *Ld = L + d * m * r;
    for (int64_t i = tid; i < m; i += 256) {
        float cv[KP];
#pragma unroll
        for (int u = 0; u < KP; u += 4) {
            const float4 f = *reinterpret_cast<const float4 *>(Cd + i * KP + u);
            cv[u] = f.x;
            cv[u + 1] = f.y;
            cv[u + 2] = f.z;
            cv[u + 3] = f.w;
        }
        for (int t = 0; t < r; ++t) {
            float s = 0.f;
#pragma unroll
            for (int u = 0; u < KP; ++u) s += cv[u] * Yr[u * KP + t];
            Ld[i * r + t] = finite ? s : qnan;
        }
    }
    // R = V Y_r with V[j][u] = Vt[u][j]: one column of V^T per thread
    const float *Vd = Vt + d * KP * ldv;
    float *Rd = R + d * n * r;
    for (int64_t j = tid; j < n; j += 256) {
        float vv[KP];
#pragma unroll
        for (int u = 0; u < KP; ++u) vv[u] = u < k ? Vd[u * ldv + j] : 0.f;
        for (int t = 0; t < r; ++t) {
            float s = 0.f;
#pragma unroll
            for (int u = 0; u < KP; ++u) s += vv[u] * Yr[u * KP + t];
            Rd[j * r + t] = finite ? s : qnan;
        }
    }
}

// ---------------------------------------------------------------------------
// Explicit residual: per (16-row block, matrix) partial sums of
// (A - L R^T)^2 and A^2, then a per-matrix finalisation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void error_part_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                         int64_t ld, int64_t stride, const float *__restrict__ L,
                                                         const float *__restrict__ R, int r,
                                                         double *__restrict__ part) {
    __shared__ double Ls[16 * MAXK];
    __shared__ double red[4];
    const int64_t d = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    const float *Ad = A + d * stride;
    const float *Ld = L + d * m * r;
    const float *Rd = R + d * n * r;
    for (int e = threadIdx.x; e < 16 * r; e += 256) {
        const int64_t i = i0 + e / r;
        Ls[e] = i < m ? (double)Ld[i0 * r + e] : 0.0;
    }
    __syncthreads();
    double res2 = 0.0, fro2 = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        double rj[MAXK];
        for (int t = 0; t < r; ++t) rj[t] = (double)Rd[j * r + t];
        for (int i = 0; i < 16; ++i) {
            if (i0 + i >= m) break;
            double ah = 0.0;
            for (int t = 0; t < r; ++t) ah += Ls[i * r + t] * rj[t];
            const double a = (double)Ad[(i0 + i) * ld + j];
            res2 += (a - ah) * (a - ah);
            fro2 += a * a;
        }
    }
    res2 = block_sum_f64(res2, red);
    fro2 = block_sum_f64(fro2, red);
    if (threadIdx.x == 0) {
        double *o = part + (d * gridDim.x + blockIdx.x) * 2;
        o[0] = res2;
        o[1] = fro2;
    }
}

__global__ void error_final_kernel(const double *__restrict__ part, int nblk, int64_t count,
                                   double *__restrict__ relerr) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= count) return;
    double r2 = 0.0, f2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        r2 += part[(d * nblk + b) * 2];
        f2 += part[(d * nblk + b) * 2 + 1];
    }
    relerr[d] = f2 > 0.0 ? sqrt(r2 / f2) : 0.0;
}

}  // namespace

tsk_status tsk_apply_enqueue(tsk_ctx c, const float *S, int k, const tsk_stack *s, int r, float *L, float *R,
                             float *sigma, double *relerr, int32_t *flags) {
    const int64_t m = s->m, n = s->n, count = s->count;
    const int kp = (k + 15) / 16 * 16;
    const int64_t ldv = (n + 63) / 64 * 64;
    const int npanel = (int)((n + SK_PANEL - 1) / SK_PANEL);
    TSK_TRY(tsk_grow(c, c->ap_St, sizeof(float) * m * kp));
    TSK_TRY(tsk_grow(c, c->ap_B, sizeof(float) * count * kp * ldv));
    TSK_TRY(tsk_grow(c, c->ap_Vt, sizeof(float) * count * kp * ldv));
    TSK_TRY(tsk_grow(c, c->ap_C, sizeof(float) * count * m * kp));
    TSK_TRY(tsk_grow(c, c->ap_fro, sizeof(double) * count * npanel));
    TSK_TRY(tsk_grow(c, c->ap_qflag, sizeof(int) * count));
    float *St = (float *)c->ap_St.p, *B = (float *)c->ap_B.p, *Vt = (float *)c->ap_Vt.p, *Cm = (float *)c->ap_C.p;
    double *fro = (double *)c->ap_fro.p;
    int *qflag = (int *)c->ap_qflag.p;
    const float *A = (const float *)s->A;
    TSK_LAUNCH(c, TSK_KERNEL_SKETCH,
               hipLaunchKernelGGL(transpose_sketch_kernel, dim3((unsigned)((m * kp + 255) / 256)), dim3(256), 0,
                                  c->stream, S, k, kp, m, St));
    const dim3 gs((unsigned)npanel, (unsigned)count);
    switch (kp / 16) {
        case 1: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<1>, gs, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        case 2: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<2>, gs, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        case 3: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<3>, gs, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        case 4: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<4>, gs, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        default: return tsk_fail(c, TSK_E_ARG, "k > 64");
    }
    const dim3 gq((unsigned)count);
    switch (kp / 16) {
        case 1: TSK_LAUNCH(c, TSK_KERNEL_QR, hipLaunchKernelGGL(cholqr2_kernel<16>, gq, dim3(256), 0, c->stream, (const float *)B, ldv, Vt, k, n, qflag, (uint16_t *)nullptr)); break;
        case 2: TSK_LAUNCH(c, TSK_KERNEL_QR, hipLaunchKernelGGL(cholqr2_kernel<32>, gq, dim3(256), 0, c->stream, (const float *)B, ldv, Vt, k, n, qflag, (uint16_t *)nullptr)); break;
        case 3: TSK_LAUNCH(c, TSK_KERNEL_QR, hipLaunchKernelGGL(cholqr2_kernel<48>, gq, dim3(256), 0, c->stream, (const float *)B, ldv, Vt, k, n, qflag, (uint16_t *)nullptr)); break;
        case 4: TSK_LAUNCH(c, TSK_KERNEL_QR, hipLaunchKernelGGL(cholqr2_kernel<64>, gq, dim3(256), 0, c->stream, (const float *)B, ldv, Vt, k, n, qflag, (uint16_t *)nullptr)); break;
    }
    const dim3 gp((unsigned)((m + PJ_ROWS - 1) / PJ_ROWS), (unsigned)count);
    switch (kp / 16) {
        case 1: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<1>, gp, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
        case 2: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<2>, gp, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
        case 3: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<3>, gp, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
        case 4: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<4>, gp, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
    }
#define TSK_FINISH(KPV)                                                                                        \
    TSK_LAUNCH(c, TSK_KERNEL_FINISH,                                                                           \
               hipLaunchKernelGGL(finish_kernel<KPV>, dim3((unsigned)count), dim3(256), 0, c->stream,          \
                                  (const float *)Cm, m, k, r, (const float *)Vt, ldv, n, (const double *)fro, \
                                  npanel, (const int *)qflag, L, R, sigma, relerr, flags))
    switch (kp / 16) {
        case 1: TSK_FINISH(16); break;
        case 2: TSK_FINISH(32); break;
        case 3: TSK_FINISH(48); break;
        case 4: TSK_FINISH(64); break;
    }
#undef TSK_FINISH
    return TSK_OK;
}

tsk_status tsk_apply_bf16_enqueue(tsk_ctx c, const float *S, int k, const tsk_stack *s, int r, float *L, float *R,
                                  float *sigma, double *relerr, int32_t *flags) {
    const int64_t m = s->m, n = s->n, count = s->count;
    const int kp = (k + 15) / 16 * 16;
    const int64_t mp = (m + 31) / 32 * 32;
    const int64_t ldv = (n + 63) / 64 * 64;
    const int npanel = (int)((n + SKB_PANEL - 1) / SKB_PANEL);
    TSK_TRY(tsk_grow(c, c->ap_Sb, sizeof(uint16_t) * 2 * kp * mp));
    TSK_TRY(tsk_grow(c, c->ap_B, sizeof(float) * count * kp * ldv));
    TSK_TRY(tsk_grow(c, c->ap_Vt, sizeof(float) * count * kp * ldv));
    TSK_TRY(tsk_grow(c, c->ap_Vb, sizeof(uint16_t) * count * 2 * kp * ldv));
    TSK_TRY(tsk_grow(c, c->ap_C, sizeof(float) * count * m * kp));
    TSK_TRY(tsk_grow(c, c->ap_fro, sizeof(double) * count * npanel));
    TSK_TRY(tsk_grow(c, c->ap_qflag, sizeof(int) * count));
    uint16_t *Sb = (uint16_t *)c->ap_Sb.p, *Vb = (uint16_t *)c->ap_Vb.p;
    float *B = (float *)c->ap_B.p, *Vt = (float *)c->ap_Vt.p, *Cm = (float *)c->ap_C.p;
    double *fro = (double *)c->ap_fro.p;
    int *qflag = (int *)c->ap_qflag.p;
    const uint16_t *A = (const uint16_t *)s->A;
    TSK_LAUNCH(c, TSK_KERNEL_SKETCH,
               hipLaunchKernelGGL(prep_sketch_bf16_kernel, dim3((unsigned)((kp * mp + 255) / 256)), dim3(256), 0,
                                  c->stream, S, k, kp, m, mp, Sb));
    const dim3 gs((unsigned)npanel, (unsigned)count);
#define TSK_SKB(MTV)                                                                                              \
    TSK_LAUNCH(c, TSK_KERNEL_SKETCH,                                                                              \
               hipLaunchKernelGGL(sketch_bf16_kernel<MTV>, gs, dim3(64), 0, c->stream, A, m, n, s->ld, s->stride, \
                                  (const uint16_t *)Sb, mp, B, ldv, fro, npanel))
    switch (kp / 16) {
        case 1: TSK_SKB(1); break;
        case 2: TSK_SKB(2); break;
        case 3: TSK_SKB(3); break;
        case 4: TSK_SKB(4); break;
        default: return tsk_fail(c, TSK_E_ARG, "k > 64");
    }
#undef TSK_SKB
    const dim3 gq((unsigned)count);
#define TSK_QRB(KPV)                                                                                  \
    TSK_LAUNCH(c, TSK_KERNEL_QR, hipLaunchKernelGGL(cholqr2_kernel<KPV>, gq, dim3(256), 0, c->stream, \
                                                    (const float *)B, ldv, Vt, k, n, qflag, Vb))
    switch (kp / 16) {
        case 1: TSK_QRB(16); break;
        case 2: TSK_QRB(32); break;
        case 3: TSK_QRB(48); break;
        case 4: TSK_QRB(64); break;
    }
#undef TSK_QRB
    const dim3 gp((unsigned)((m + PJB_ROWS - 1) / PJB_ROWS), (unsigned)count);
#define TSK_PJB(NTV)                                                                                     \
    TSK_LAUNCH(c, TSK_KERNEL_PROJECT,                                                                    \
               hipLaunchKernelGGL(project_bf16_kernel<NTV>, gp, dim3(64), 0, c->stream, A, m, n, s->ld, \
                                  s->stride, (const uint16_t *)Vb, ldv, Cm))
    switch (kp / 16) {
        case 1: TSK_PJB(1); break;
        case 2: TSK_PJB(2); break;
        case 3: TSK_PJB(3); break;
        case 4: TSK_PJB(4); break;
    }
#undef TSK_PJB
#define TSK_FINISH(KPV)                                                                                        \
    TSK_LAUNCH(c, TSK_KERNEL_FINISH,                                                                           \
               hipLaunchKernelGGL(finish_kernel<KPV>, dim3((unsigned)count), dim3(256), 0, c->stream,          \
                                  (const float *)Cm, m, k, r, (const float *)Vt, ldv, n, (const double *)fro, \
                                  npanel, (const int *)qflag, L, R, sigma, relerr, flags))
    switch (kp / 16) {
        case 1: TSK_FINISH(16); break;
        case 2: TSK_FINISH(32); break;
        case 3: TSK_FINISH(48); break;
        case 4: TSK_FINISH(64); break;
    }
#undef TSK_FINISH
    return TSK_OK;
}

tsk_status tsk_error_enqueue(tsk_ctx c, const tsk_stack *s, const float *L, const float *R, int r, double *relerr) {
    const int64_t m = s->m, n = s->n, count = s->count;
    const int nblk = (int)((m + 15) / 16);
    TSK_TRY(tsk_grow(c, c->er_part, sizeof(double) * 2 * nblk * count));
    double *part = (double *)c->er_part.p;
    TSK_LAUNCH(c, TSK_KERNEL_ERROR,
               hipLaunchKernelGGL(error_part_kernel, dim3((unsigned)nblk, (unsigned)count), dim3(256), 0, c->stream,
                                  (const float *)s->A, m, n, s->ld, s->stride, L, R, r, part));
    TSK_LAUNCH(c, TSK_KERNEL_ERROR,
               hipLaunchKernelGGL(error_final_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream,
                                  (const double *)part, nblk, count, relerr));
    return TSK_OK;
}
