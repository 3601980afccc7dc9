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

constexpr int SK_PANEL = 256;  // columns of A_d per sketch workgroup (64 per wave)
constexpr int PJ_ROWS = 256;   // rows of A_d per project workgroup (64 per wave)
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
__global__ __launch_bounds__(256) void sketch_f32_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                         int64_t ld, int64_t stride, const float *__restrict__ St,
                                                         float *__restrict__ B, int64_t ldb,
                                                         double *__restrict__ fro_part, int npanel) {
    constexpr int kp = MT * 16;
    const int64_t d = blockIdx.y;
    const int panel = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, jj = lane & 15;
    const int64_t col4 = (int64_t)panel * SK_PANEL + wv * 64 + 4 * jj;  // this lane's 4 columns
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
    __shared__ double red[4];
    const double tot = block_sum_f64(fro, red);
    if (threadIdx.x == 0) fro_part[d * npanel + panel] = tot;
}

// ---------------------------------------------------------------------------
// CholeskyQR2 of B_d^T, one workgroup per matrix.
// ---------------------------------------------------------------------------

// C (k x k, upper triangle, LDS) = src src^T, src k x n rows with stride lds_src.
__device__ inline void gram_rows(const float *__restrict__ src, int k, int64_t n, int64_t ldsrc, double *C,
                                 float *stage /* k x 256 */) {
    const int tid = threadIdx.x;
    const int ntri = k * (k + 1) / 2;
    double acc[NTRI_PER_THREAD];
    int ea[NTRI_PER_THREAD], eb[NTRI_PER_THREAD];
#pragma unroll
    for (int u = 0; u < NTRI_PER_THREAD; ++u) {
        acc[u] = 0.0;
        int e = tid + u * 256, a = 0, rowlen = k;
        if (e < ntri) {
            while (e >= rowlen) {
                e -= rowlen;
                ++a;
                --rowlen;
            }
            ea[u] = a;
            eb[u] = a + e;
        } else {
            ea[u] = eb[u] = -1;
        }
    }
    for (int64_t c0 = 0; c0 < n; c0 += 256) {
        __syncthreads();
        for (int e = tid; e < k * 256; e += 256) {
            const int a = e / 256;
            const int64_t cc = c0 + (e % 256);
            stage[e] = cc < n ? src[a * ldsrc + cc] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NTRI_PER_THREAD; ++u) {
            if (ea[u] < 0) continue;
            const float *ra = stage + ea[u] * 256, *rb = stage + eb[u] * 256;
            double s = 0.0;
            for (int c = 0; c < 256; ++c) s += (double)ra[c] * (double)rb[c];
            acc[u] += s;
        }
    }
#pragma unroll
    for (int u = 0; u < NTRI_PER_THREAD; ++u)
        if (ea[u] >= 0) {
            C[ea[u] * MAXK + eb[u]] = acc[u];
            C[eb[u] * MAXK + ea[u]] = acc[u];
        }
    __syncthreads();
}

// In-LDS Cholesky (ld = MAXK) with dead pivots, then Rinv by column-parallel
// back substitution (k <= 64).  Returns the number of dead indices.
__device__ inline int chol_inv_small(double *C, double *Rinv, int k, double tol_rel, int *dead) {
    const int tid = threadIdx.x;
    __shared__ double s_maxd;
    __shared__ int s_nd;
    if (tid == 0) {
        double mx = 0.0;
        for (int j = 0; j < k; ++j) mx = fmax(mx, C[j * MAXK + j]);
        s_maxd = mx;
        s_nd = 0;
    }
    __syncthreads();
    const double thr = tol_rel * s_maxd;
    for (int j = 0; j < k; ++j) {
        const double piv = C[j * MAXK + j];
        const bool dj = !(piv > thr) || !(piv > 0.0);
        if (tid == 0) {
            dead[j] = dj;
            if (dj) ++s_nd;
        }
        if (!dj) {
            const int L = k - j - 1;
            const double inv = 1.0 / piv;
            for (int e = tid; e < L * L; e += blockDim.x) {
                const int a = j + 1 + e / L, b = j + 1 + e % L;
                if (a <= b) C[a * MAXK + b] -= C[j * MAXK + a] * C[j * MAXK + b] * inv;
            }
        }
        __syncthreads();
    }
    // R[a][b] = C[a][b]/sqrt(C[a][a]) (rows of dead a are zero); invert by
    // back substitution, one thread per column, R read straight from C.
    if (tid < k) {
        const int j = tid;
        for (int i = j; i >= 0; --i) {
            double v = 0.0;
            if (!dead[i]) {
                const double di = sqrt(C[i * MAXK + i]);
                double s = (i == j) ? 1.0 : 0.0;
                for (int t = i + 1; t <= j; ++t) s -= (C[i * MAXK + t] / di) * Rinv[t * MAXK + j];
                v = s / di;
            }
            Rinv[i * MAXK + j] = v;
        }
        for (int i = j + 1; i < k; ++i) Rinv[i * MAXK + j] = 0.0;
    }
    __syncthreads();
    return s_nd;
}

// dst (k x ldv) = Rinv^T src, columns >= n and rows k..kp-1 set to zero.
__device__ inline void apply_rinv_t(const float *__restrict__ src, int64_t ldsrc, float *__restrict__ dst,
                                    int64_t lddst, int k, int kp, int64_t n, int64_t ldv, const double *Rinv) {
    for (int64_t c = threadIdx.x; c < ldv; c += blockDim.x) {
        double col[MAXK];
        if (c < n) {
            for (int t = 0; t < k; ++t) col[t] = (double)src[t * ldsrc + c];
        }
        for (int i = 0; i < kp; ++i) {
            double s = 0.0;
            if (c < n && i < k) {
                for (int t = 0; t <= i; ++t) s += Rinv[t * MAXK + i] * col[t];
            }
            dst[i * lddst + c] = (float)s;
        }
    }
}

__global__ __launch_bounds__(256) void cholqr2_kernel(const float *__restrict__ B, int64_t ldb, float *__restrict__ Vt,
                                                      int k, int kp, int64_t n, int *__restrict__ qflag) {
    __shared__ double C[MAXK * MAXK];
    __shared__ double Rinv[MAXK * MAXK];
    __shared__ float stage[MAXK * 256];
    __shared__ int dead[MAXK];
    const int64_t d = blockIdx.x;
    const float *Bd = B + d * kp * ldb;
    float *Vd = Vt + d * kp * ldb;
    // pass 1: threshold 1e-12 on the pivot ratio (singular-value ratio 1e-6,
    // the FP32 rounding level of B)
    gram_rows(Bd, k, n, ldb, C, stage);
    const int nd1 = chol_inv_small(C, Rinv, k, 1e-12, dead);
    apply_rinv_t(Bd, ldb, Vd, ldb, k, kp, n, ldb, Rinv);
    __syncthreads();
    // pass 2 on the (nearly orthonormal) first pass
    gram_rows(Vd, k, n, ldb, C, stage);
    chol_inv_small(C, Rinv, k, 1e-12, dead);
    __syncthreads();
    apply_rinv_t(Vd, ldb, Vd, ldb, k, kp, n, ldb, Rinv);
    if (threadIdx.x == 0) qflag[d] = nd1 > 0 ? TSK_FLAG_RANKDEF : 0;
}

// ---------------------------------------------------------------------------
// C_d = A_d V_d
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256) void project_f32_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                          int64_t ld, int64_t stride, const float *__restrict__ Vt,
                                                          int64_t ldv, float *__restrict__ C) {
    constexpr int kp = NT * 16;
    const int64_t d = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, ii = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * PJ_ROWS + wv * 64;
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
// Rank-r truncation, outputs and the fused error.  One workgroup per matrix.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finish_kernel(const float *__restrict__ C, int64_t m, int k, int kp, int r,
                                                     const float *__restrict__ Vt, int64_t ldv, int64_t n,
                                                     const double *__restrict__ fro_part, int npanel,
                                                     const int *__restrict__ qflag, float *__restrict__ L,
                                                     float *__restrict__ R, float *__restrict__ sigma,
                                                     double *__restrict__ relerr, int *__restrict__ flags) {
    __shared__ double H[MAXK * MAXK];
    __shared__ double W[MAXK * MAXK];
    __shared__ double Yr[MAXK * MAXK];  // first r eigenvector columns, descending
    __shared__ float stage[64 * MAXK];
    __shared__ double rot[MAXK];
    __shared__ int pairs[MAXK];
    __shared__ int perm[MAXK];
    __shared__ double red4[4];
    __shared__ double s_lam[MAXK];
    const int64_t d = blockIdx.x;
    const int tid = threadIdx.x;
    const float *Cd = C + d * m * kp;
    const int kk = k + (k & 1);  // even size for the parallel Jacobi ordering
    // H = C^T C (k x k), FP64
    const int ntri = k * (k + 1) / 2;
    double acc[NTRI_PER_THREAD];
    int ea[NTRI_PER_THREAD], eb[NTRI_PER_THREAD];
#pragma unroll
    for (int u = 0; u < NTRI_PER_THREAD; ++u) {
        int e = tid + u * 256, a = 0, rowlen = k;
        acc[u] = 0.0;
        if (e < ntri) {
            while (e >= rowlen) {
                e -= rowlen;
                ++a;
                --rowlen;
            }
            ea[u] = a;
            eb[u] = a + e;
        } else {
            ea[u] = eb[u] = -1;
        }
    }
    for (int64_t i0 = 0; i0 < m; i0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * kp; e += 256) {
            const int64_t row = i0 + e / kp;
            stage[e] = row < m ? Cd[i0 * kp + e] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NTRI_PER_THREAD; ++u) {
            if (ea[u] < 0) continue;
            double s = 0.0;
            for (int i = 0; i < 64; ++i) s += (double)stage[i * kp + ea[u]] * (double)stage[i * kp + eb[u]];
            acc[u] += s;
        }
    }
    for (int e = tid; e < MAXK * MAXK; e += 256) H[e] = 0.0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NTRI_PER_THREAD; ++u)
        if (ea[u] >= 0) {
            H[ea[u] * MAXK + eb[u]] = acc[u];
            H[eb[u] * MAXK + ea[u]] = acc[u];
        }
    __syncthreads();
    jacobi_eig_lds(H, W, kk, MAXK, rot, pairs, 40, red4);
    if (tid == 0) sort_diag_desc(H, kk, MAXK, perm);
    __syncthreads();
    for (int t = tid; t < kk; t += 256) s_lam[t] = H[perm[t] * MAXK + perm[t]];
    for (int e = tid; e < k * r; e += 256) {
        const int s = e / r, t = e % r;
        Yr[s * MAXK + t] = W[s * MAXK + perm[t]];
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
    // L = C Y_r (m x r)
    float *Ld = L + d * m * r;
    for (int64_t e = tid; e < m * r; e += 256) {
        const int64_t i = e / r;
        const int t = (int)(e % r);
        double s = 0.0;
        for (int u = 0; u < k; ++u) s += (double)Cd[i * kp + u] * Yr[u * MAXK + t];
        Ld[e] = finite ? (float)s : qnan;
    }
    // R = V Y_r (n x r), V[j][u] = Vt[u][j]
    const float *Vd = Vt + d * kp * ldv;
    float *Rd = R + d * n * r;
    for (int64_t e = tid; e < n * r; e += 256) {
        const int64_t j = e / r;
        const int t = (int)(e % r);
        double s = 0.0;
        for (int u = 0; u < k; ++u) s += (double)Vd[u * ldv + j] * Yr[u * MAXK + t];
        Rd[e] = finite ? (float)s : qnan;
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
        case 1: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<1>, gs, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        case 2: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<2>, gs, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        case 3: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<3>, gs, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        case 4: TSK_LAUNCH(c, TSK_KERNEL_SKETCH, hipLaunchKernelGGL(sketch_f32_kernel<4>, gs, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)St, B, ldv, fro, npanel)); break;
        default: return tsk_fail(c, TSK_E_ARG, "k > 64");
    }
    TSK_LAUNCH(c, TSK_KERNEL_QR,
               hipLaunchKernelGGL(cholqr2_kernel, dim3((unsigned)count), dim3(256), 0, c->stream, (const float *)B,
                                  ldv, Vt, k, kp, n, qflag));
    const dim3 gp((unsigned)((m + PJ_ROWS - 1) / PJ_ROWS), (unsigned)count);
    switch (kp / 16) {
        case 1: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<1>, gp, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
        case 2: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<2>, gp, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
        case 3: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<3>, gp, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
        case 4: TSK_LAUNCH(c, TSK_KERNEL_PROJECT, hipLaunchKernelGGL(project_f32_kernel<4>, gp, dim3(256), 0, c->stream, A, m, n, s->ld, s->stride, (const float *)Vt, ldv, Cm)); break;
    }
    TSK_LAUNCH(c, TSK_KERNEL_FINISH,
               hipLaunchKernelGGL(finish_kernel, dim3((unsigned)count), dim3(256), 0, c->stream, (const float *)Cm, m, k,
                                  kp, r, (const float *)Vt, ldv, n, (const double *)fro, npanel, (const int *)qflag, L,
                                  R, sigma, relerr, flags));
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
