// Leading-k eigenvectors of the symmetric mode-1 Gram: the Tucker1 factor
// S* = (U^(1))_k^T of Section 3.1 (the first k left singular vectors of
// A_(1) are the top-k eigenvectors of G = A_(1) A_(1)^T).
//
// Method: block subspace iteration in FP64 with a block of p >= k columns
// (padded to pp, a multiple of 16; padding columns are kept at zero).
//   Y_{t+1} = (G Y_t) Rinv_t,  C = Y_{t+1}^T Y_{t+1} = R^T R,  Rinv_{t+1} = R^-1
// so X_t = Y_t Rinv_t is the orthonormal basis of iteration t (Cholesky QR;
// the span is all that subspace iteration needs).  Every `check` iterations a
// Rayleigh-Ritz step on X forms H = X^T G X, diagonalises it (Jacobi), and
// tests the residuals ||G u_i - theta_i u_i|| <= tol * theta_1 for i < k.
//
// Kernels
//  eig_iter   : one workgroup per 16 rows; FP64 MFMA 16x16x4 for G Y (the
//               four waves split the contraction), Rinv epilogue, partial
//               upper triangle of Y^T Y.
//  eig_chol   : 16 workgroups sum the partials in a fixed order; the last one
//               (ticket counter) runs Cholesky with dead-pivot detection and
//               a blocked upper-triangular inverse, all in LDS.
//  eig_x / eig_gx / eig_rr / eig_res / eig_conv / eig_emit: Rayleigh-Ritz,
//               residuals, sign canonicalisation and the FP32 output S.
#include "tsk_common.hpp"

namespace {

constexpr int EIG_RB = 16;       // rows per workgroup in the row-block kernels
constexpr int EIG_MAXPP = 80;    // largest padded block
constexpr int EIG_NRED = 16;     // workgroups of the partial reductions

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Start block: uniform(-1,1) entries from a counter-based hash, zero padding.
__global__ void eig_init_kernel(double *Y, int64_t m, int pp, int p, double *Rinv, uint64_t seed) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m * pp) {
        const int64_t i = e / pp;
        const int j = (int)(e % pp);
        double v = 0.0;
        if (j < p) {
            uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)i * 131071ull + (uint64_t)j));
            v = ((double)(h >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
        }
        Y[e] = v;
    }
    if (e < (int64_t)pp * pp) {
        const int i = (int)(e / pp), j = (int)(e % pp);
        Rinv[e] = (i == j && i < p) ? 1.0 : 0.0;
    }
}

// Z[16][pp] = G[r0:r0+16, :] * Yin (m x pp) with FP64 MFMA; the 4 waves split
// the contraction and their partial tiles are summed into Zs (LDS, 16 x pp).
__device__ inline void rowblock_gemm(const double *__restrict__ G, int64_t m, int pp,
                                     const double *__restrict__ Yin, int64_t r0, double *Zs,
                                     double *wpart /* 4 x 16 x pp LDS */) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, ii = lane & 15;
    const int nt = pp / 16;
    const int64_t row = r0 + ii;
    const bool rv = row < m;
    const double *grow = G + (rv ? row : 0) * m;
    // contraction range of this wave, multiples of 16
    const int64_t kq = ((m + 63) / 64) * 16;
    const int64_t kb = wv * kq, ke = (kb + kq < m) ? kb + kq : m;
    v4d acc[EIG_MAXPP / 16];
#pragma unroll
    for (int x = 0; x < EIG_MAXPP / 16; ++x) acc[x] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = kb; k0 < ke; k0 += 16) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t kk = k0 + 4 * q + u;
            a[u] = (rv && kk < m) ? grow[kk] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t kk = k0 + 4 * q + u;
            const bool kv = kk < m;
            const double *yr = Yin + (kv ? kk : 0) * pp + ii;
#pragma unroll
            for (int x = 0; x < EIG_MAXPP / 16; ++x) {
                if (x < nt) {
                    const double b = kv ? yr[x * 16] : 0.0;
                    acc[x] = mfma16x16x4_f64(a[u], b, acc[x]);
                }
            }
        }
    }
#pragma unroll
    for (int x = 0; x < EIG_MAXPP / 16; ++x) {
        if (x < nt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) wpart[(wv * 16 + q + 4 * r) * pp + x * 16 + ii] = acc[x][r];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * pp; e += blockDim.x)
        Zs[e] = wpart[e] + wpart[16 * pp + e] + wpart[32 * pp + e] + wpart[48 * pp + e];
    __syncthreads();
}

__device__ __forceinline__ void tri_index(int e, int pp, int &a, int &b) {
    // e-th entry of the upper triangle (a <= b), row-major
    int r = 0, rowlen = pp;
    while (e >= rowlen) {
        e -= rowlen;
        ++r;
        --rowlen;
    }
    a = r;
    b = r + e;
}

__global__ __launch_bounds__(256) void eig_iter_kernel(const double *__restrict__ G, int64_t m, int pp,
                                                       const double *__restrict__ Yp,
                                                       const double *__restrict__ Rinv,
                                                       double *__restrict__ Yn, double *__restrict__ partC) {
    extern __shared__ double lds[];
    double *wpart = lds;                       // 4*16*pp
    double *Zs = wpart + 64 * pp;              // 16*pp
    double *Rs = Zs + 16 * pp;                 // pp*pp
    double *Ys = Rs + pp * pp;                 // 16*pp
    const int64_t r0 = (int64_t)blockIdx.x * EIG_RB;
    for (int e = threadIdx.x; e < pp * pp; e += blockDim.x) Rs[e] = Rinv[e];
    rowblock_gemm(G, m, pp, Yp, r0, Zs, wpart);
    for (int e = threadIdx.x; e < 16 * pp; e += blockDim.x) {
        const int i = e / pp, j = e % pp;
        double s = 0.0;
        for (int t = 0; t <= j; ++t) s += Zs[i * pp + t] * Rs[t * pp + j];
        const bool valid = (r0 + i) < m;
        Ys[e] = valid ? s : 0.0;
        if (valid) Yn[(r0 + i) * pp + j] = s;
    }
    __syncthreads();
    const int ntri = pp * (pp + 1) / 2;
    double *out = partC + (int64_t)blockIdx.x * ntri;
    for (int e = threadIdx.x; e < ntri; e += blockDim.x) {
        int a, b;
        tri_index(e, pp, a, b);
        double s = 0.0;
#pragma unroll 4
        for (int i = 0; i < 16; ++i) s += Ys[i * pp + a] * Ys[i * pp + b];
        out[e] = s;
    }
}

// Blocked inverse of an upper-triangular pp x pp matrix R (LDS) into X (LDS):
// 8x8 diagonal blocks inverted by one thread each, then neighbouring blocks
// merged level by level with X12 = -X11 R12 X22.  Zero diagonal entries
// (dead pivots) give zero rows/columns in X.  T: LDS scratch (pp*pp/4).
__device__ inline void upper_tri_inverse(const double *R, double *X, int pp, double *T) {
    const int tid = threadIdx.x;
    for (int e = tid; e < pp * pp; e += blockDim.x) X[e] = 0.0;
    __syncthreads();
    const int nblk = pp / 8;
    if (tid < nblk) {
        const int o = tid * 8;
        for (int j = 7; j >= 0; --j) {
            // column j of the block inverse by back substitution
            for (int i = j; i >= 0; --i) {
                const double rii = R[(o + i) * pp + (o + i)];
                if (rii == 0.0) { X[(o + i) * pp + (o + j)] = 0.0; continue; }
                double s = (i == j) ? 1.0 : 0.0;
                for (int t = i + 1; t <= j; ++t) s -= R[(o + i) * pp + (o + t)] * X[(o + t) * pp + (o + j)];
                X[(o + i) * pp + (o + j)] = s / rii;
            }
        }
    }
    __syncthreads();
    for (int s = 8; s < pp; s *= 2) {
        const int ngroups = (pp + 2 * s - 1) / (2 * s);
        // T_g = R12 * X22  (s1 x s2 per group, stored at offset g*s*s)
        for (int e = tid; e < ngroups * s * s; e += blockDim.x) {
            const int g = e / (s * s), a = (e / s) % s, b = e % s;
            const int o = g * 2 * s, s2 = (pp - o - s < s) ? pp - o - s : s;
            if (s2 <= 0 || b >= s2) continue;
            double acc = 0.0;
            for (int cidx = 0; cidx <= b; ++cidx)
                acc += R[(o + a) * pp + (o + s + cidx)] * X[(o + s + cidx) * pp + (o + s + b)];
            T[e] = acc;
        }
        __syncthreads();
        for (int e = tid; e < ngroups * s * s; e += blockDim.x) {
            const int g = e / (s * s), a = (e / s) % s, b = e % s;
            const int o = g * 2 * s, s2 = (pp - o - s < s) ? pp - o - s : s;
            if (s2 <= 0 || b >= s2) continue;
            double acc = 0.0;
            for (int cidx = a; cidx < s; ++cidx) acc += X[(o + a) * pp + (o + cidx)] * T[g * s * s + cidx * s + b];
            X[(o + a) * pp + (o + s + b)] = -acc;
        }
        __syncthreads();
    }
}

// Cholesky C = R^T R of a symmetric positive semi-definite pp x pp matrix in
// LDS (upper triangle used, overwritten).  A pivot <= tol_rel * max(diag)
// marks the index dead: its row of R is zero.  On exit R (LDS) holds the
// factor.  Returns (in every thread) the number of dead indices among the
// first `live` ones.
__device__ inline int cholesky_lds(double *C, double *R, int pp, int live, double tol_rel, int *dead) {
    const int tid = threadIdx.x;
    __shared__ double s_maxd;
    __shared__ int s_ndead;
    if (tid == 0) {
        double mx = 0.0;
        for (int j = 0; j < pp; ++j) mx = fmax(mx, C[j * pp + j]);
        s_maxd = mx;
        s_ndead = 0;
    }
    __syncthreads();
    const double thr = tol_rel * s_maxd;
    for (int j = 0; j < pp; ++j) {
        const double piv = C[j * pp + j];
        const bool dj = !(piv > thr) || !(piv > 0.0);
        if (tid == 0) {
            dead[j] = dj;
            if (dj && j < live) ++s_ndead;
        }
        if (!dj) {
            const int L = pp - j - 1;
            const double inv = 1.0 / piv;
            for (int e = tid; e < L * L; e += blockDim.x) {
                const int a = j + 1 + e / L, b = j + 1 + e % L;
                if (a <= b) C[a * pp + b] -= C[j * pp + a] * C[j * pp + b] * inv;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < pp * pp; e += blockDim.x) {
        const int a = e / pp, b = e % pp;
        double v = 0.0;
        if (b >= a && !dead[a]) v = C[a * pp + b] / sqrt(C[a * pp + a]);
        R[e] = v;
    }
    __syncthreads();
    return s_ndead;
}

// Sum the per-workgroup upper-triangle partials (fixed order) and, in the
// last workgroup, factor and invert.
__global__ __launch_bounds__(256) void eig_chol_kernel(const double *__restrict__ partC, int nparts, int pp,
                                                       int live, double *__restrict__ Cg,
                                                       double *__restrict__ Rinv, unsigned *counter,
                                                       double tol_rel, int *ndead_out) {
    extern __shared__ double lds[];
    const int ntri = pp * (pp + 1) / 2;
    const int per = (ntri + gridDim.x - 1) / gridDim.x;
    const int e0 = blockIdx.x * per, e1 = (e0 + per < ntri) ? e0 + per : ntri;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nparts; ++w) s += partC[(int64_t)w * ntri + e];
        Cg[e] = s;
    }
    __threadfence();
    __syncthreads();
    __shared__ unsigned ticket;
    if (threadIdx.x == 0) ticket = atomicAdd(counter, 1u);
    __syncthreads();
    if (ticket != gridDim.x - 1) return;
    __threadfence();
    // T (inverse scratch, up to pp*pp entries) reuses C once the factor is out
    double *C = lds, *R = C + pp * pp, *X = R + pp * pp, *T = C;
    __shared__ int dead[EIG_MAXPP];
    for (int e = threadIdx.x; e < ntri; e += blockDim.x) {
        int a, b;
        tri_index(e, pp, a, b);
        const double v = Cg[e];
        C[a * pp + b] = v;
        C[b * pp + a] = v;
    }
    __syncthreads();
    const int nd = cholesky_lds(C, R, pp, live, tol_rel, dead);
    upper_tri_inverse(R, X, pp, T);
    for (int e = threadIdx.x; e < pp * pp; e += blockDim.x) Rinv[e] = X[e];
    if (threadIdx.x == 0) {
        *ndead_out = nd;
        *counter = 0u;
    }
}

// X = Y Rinv (orthonormal basis), one row block per workgroup.
__global__ __launch_bounds__(256) void eig_x_kernel(const double *__restrict__ Y, const double *__restrict__ Rinv,
                                                    int64_t m, int pp, double *__restrict__ X) {
    const int64_t r0 = (int64_t)blockIdx.x * EIG_RB;
    for (int e = threadIdx.x; e < EIG_RB * pp; e += blockDim.x) {
        const int i = e / pp, j = e % pp;
        if (r0 + i >= m) continue;
        const double *yr = Y + (r0 + i) * pp;
        double s = 0.0;
        for (int t = 0; t <= j; ++t) s += yr[t] * Rinv[t * pp + j];
        X[(r0 + i) * pp + j] = s;
    }
}

// GX = G X and the partial upper triangle of X^T G X per row block.
__global__ __launch_bounds__(256) void eig_gx_kernel(const double *__restrict__ G, int64_t m, int pp,
                                                     const double *__restrict__ X, double *__restrict__ GX,
                                                     double *__restrict__ partH) {
    extern __shared__ double lds[];
    double *wpart = lds, *Zs = wpart + 64 * pp, *Xs = Zs + 16 * pp;
    const int64_t r0 = (int64_t)blockIdx.x * EIG_RB;
    rowblock_gemm(G, m, pp, X, r0, Zs, wpart);
    for (int e = threadIdx.x; e < 16 * pp; e += blockDim.x) {
        const int i = e / pp;
        const bool valid = (r0 + i) < m;
        Xs[e] = valid ? X[(r0 + i) * pp + (e % pp)] : 0.0;
        if (valid) GX[(r0 + i) * pp + (e % pp)] = Zs[e];
        else Zs[e] = 0.0;
    }
    __syncthreads();
    const int ntri = pp * (pp + 1) / 2;
    for (int e = threadIdx.x; e < ntri; e += blockDim.x) {
        int a, b;
        tri_index(e, pp, a, b);
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += Xs[i * pp + a] * Zs[i * pp + b];
        partH[(int64_t)blockIdx.x * ntri + e] = s;
    }
}

// Sum partial H (symmetrised) and, in the last workgroup, diagonalise it:
// W (pp x pp, eigenvector columns in descending eigenvalue order), theta.
__global__ __launch_bounds__(256) void eig_rr_kernel(const double *__restrict__ partH, int nparts, int pp,
                                                     double *__restrict__ Hg, double *__restrict__ Wout,
                                                     double *__restrict__ theta, unsigned *counter) {
    extern __shared__ double lds[];
    const int ntri = pp * (pp + 1) / 2;
    const int per = (ntri + gridDim.x - 1) / gridDim.x;
    const int e0 = blockIdx.x * per, e1 = (e0 + per < ntri) ? e0 + per : ntri;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nparts; ++w) s += partH[(int64_t)w * ntri + e];
        Hg[e] = s;
    }
    __threadfence();
    __syncthreads();
    __shared__ unsigned ticket;
    if (threadIdx.x == 0) ticket = atomicAdd(counter, 1u);
    __syncthreads();
    if (ticket != gridDim.x - 1) return;
    __threadfence();
    double *H = lds, *W = H + pp * pp;
    __shared__ double rot[EIG_MAXPP];
    __shared__ int pairs[EIG_MAXPP];
    __shared__ int perm[EIG_MAXPP];
    __shared__ double red4[4];
    for (int e = threadIdx.x; e < ntri; e += blockDim.x) {
        int a, b;
        tri_index(e, pp, a, b);
        // H_ab from X^T G X: symmetrise the two partial orders
        const double v = Hg[e];
        H[a * pp + b] = v;
        H[b * pp + a] = v;
    }
    __syncthreads();
    jacobi_eig_lds(H, W, pp, pp, rot, pairs, 40, red4);
    if (threadIdx.x == 0) sort_diag_desc(H, pp, pp, perm);
    __syncthreads();
    for (int e = threadIdx.x; e < pp * pp; e += blockDim.x) {
        const int i = e / pp, j = e % pp;
        Wout[e] = W[i * pp + perm[j]];
    }
    for (int j = threadIdx.x; j < pp; j += blockDim.x) theta[j] = H[perm[j] * pp + perm[j]];
    if (threadIdx.x == 0) *counter = 0u;
}

// U = X W (Ritz vectors), residual partials for the first k, and per-column
// max |U| with its row (ties: lowest row) for sign canonicalisation.
__global__ __launch_bounds__(256) void eig_res_kernel(const double *__restrict__ X, const double *__restrict__ GX,
                                                      const double *__restrict__ W, const double *__restrict__ theta,
                                                      int64_t m, int pp, int k, double *__restrict__ U,
                                                      double *__restrict__ part /* nblk x (3k) */) {
    __shared__ double Ws[EIG_MAXPP * EIG_MAXPP];
    __shared__ double res[EIG_RB * EIG_MAXPP];
    __shared__ double uu[EIG_RB * EIG_MAXPP];
    const int64_t r0 = (int64_t)blockIdx.x * EIG_RB;
    for (int e = threadIdx.x; e < pp * pp; e += blockDim.x) Ws[e] = W[e];
    __syncthreads();
    for (int e = threadIdx.x; e < EIG_RB * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        double u = 0.0, g = 0.0;
        if (r0 + i < m) {
            const double *xr = X + (r0 + i) * pp, *gr = GX + (r0 + i) * pp;
            for (int t = 0; t < pp; ++t) {
                u += xr[t] * Ws[t * pp + j];
                g += gr[t] * Ws[t * pp + j];
            }
            U[(r0 + i) * k + j] = u;
        }
        const double rr = g - theta[j] * u;
        res[i * k + j] = rr * rr;
        uu[i * k + j] = u;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0, best = -1.0;
        int64_t bi = 0;
        for (int i = 0; i < EIG_RB; ++i) {
            s += res[i * k + j];
            const double a = fabs(uu[i * k + j]);
            if (r0 + i < m && a > best) {
                best = a;
                bi = r0 + i;
            }
        }
        double *o = part + (int64_t)blockIdx.x * 3 * k;
        o[j] = s;
        o[k + j] = best;
        o[2 * k + j] = (double)bi;
    }
}

// Final reduction of the residual / sign partials (one workgroup).
// small: [0] = converged flag, [1] = max relative residual,
//        [2 .. 2+k) = sign of each Ritz vector.
__global__ __launch_bounds__(256) void eig_conv_kernel(const double *__restrict__ part, int nblk, int k,
                                                       const double *__restrict__ theta,
                                                       const double *__restrict__ U, double tol,
                                                       double *__restrict__ small) {
    __shared__ double red[256];
    double worst = 0.0;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0, best = -1.0, bi = 0.0;
        for (int b = 0; b < nblk; ++b) {
            const double *o = part + (int64_t)b * 3 * k;
            s += o[j];
            if (o[k + j] > best) {
                best = o[k + j];
                bi = o[2 * k + j];
            }
        }
        const double rel = sqrt(s) / fmax(fabs(theta[0]), 1e-300);
        worst = fmax(worst, rel);
        const double sv = U[(int64_t)bi * k + j];
        small[2 + j] = (sv < 0.0) ? -1.0 : 1.0;
    }
    red[threadIdx.x] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) w = fmax(w, red[i]);
        small[0] = (w <= tol) ? 1.0 : 0.0;
        small[1] = w;
    }
}

// S[i][j] = sign_i * U[j][i]  (FP32, k x m)
__global__ void eig_emit_kernel(const double *__restrict__ U, const double *__restrict__ small, int64_t m, int k,
                                float *__restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * k) return;
    const int i = (int)(e / m);
    const int64_t j = e % m;
    S[e] = (float)(small[2 + i] * U[j * k + i]);
}

}  // namespace

tsk_status tsk_eig_enqueue(tsk_ctx c, const double *G, int64_t m, int k, float *S, double *lambda,
                           int32_t *iters_out) {
    int p = c->eig_block > 0 ? c->eig_block : k + (k / 2 > 12 ? k / 2 : 12);
    if (p < k + 1) p = k + 1;
    if (p > m) p = (int)m;
    int pp = (p + 15) / 16 * 16;
    if (pp > EIG_MAXPP) {
        pp = EIG_MAXPP;
        if (p > pp) p = pp;
    }
    if (k >= p) return tsk_fail(c, TSK_E_ARG, "tsk_eig_topk: k too large for the search block");
    const int nblk = (int)((m + EIG_RB - 1) / EIG_RB);
    const int ntri = pp * (pp + 1) / 2;
    TSK_TRY(tsk_grow(c, c->eig_Y0, sizeof(double) * m * pp));
    TSK_TRY(tsk_grow(c, c->eig_Y1, sizeof(double) * m * pp));
    TSK_TRY(tsk_grow(c, c->eig_X, sizeof(double) * m * pp));
    TSK_TRY(tsk_grow(c, c->eig_GX, sizeof(double) * m * pp));
    TSK_TRY(tsk_grow(c, c->eig_U, sizeof(double) * m * k));
    TSK_TRY(tsk_grow(c, c->eig_Rinv, sizeof(double) * pp * pp * 2));
    TSK_TRY(tsk_grow(c, c->eig_part, sizeof(double) * (size_t)nblk * (ntri > 3 * k ? ntri : 3 * k)));
    TSK_TRY(tsk_grow(c, c->eig_C, sizeof(double) * ntri));
    TSK_TRY(tsk_grow(c, c->eig_small, sizeof(double) * (4 + 2 * pp + k) + 64));
    TSK_TRY(tsk_grow(c, c->counters, 256));
    double *Y[2] = {(double *)c->eig_Y0.p, (double *)c->eig_Y1.p};
    double *Rinv = (double *)c->eig_Rinv.p;
    double *W = Rinv + pp * pp;
    double *X = (double *)c->eig_X.p, *GX = (double *)c->eig_GX.p, *U = (double *)c->eig_U.p;
    double *part = (double *)c->eig_part.p, *Cg = (double *)c->eig_C.p;
    double *small = (double *)c->eig_small.p;  // [0..2+k) conv info, then theta (pp)
    double *theta = small + 2 + k + 8;
    unsigned *counter = (unsigned *)c->counters.p;
    int *ndead = (int *)((char *)c->counters.p + 64);
    hipError_t e = hipMemsetAsync(c->counters.p, 0, 256, c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "memset");

    const size_t lds_iter = sizeof(double) * (64 * pp + 16 * pp + pp * pp + 16 * pp);
    const size_t lds_chol = sizeof(double) * (3 * pp * pp);
    const size_t lds_gx = sizeof(double) * (64 * pp + 16 * pp + 16 * pp);
    const size_t lds_rr = sizeof(double) * (2 * pp * pp);
    const double tol_chol = 1e-26;
    {
        // kernels whose dynamic LDS may exceed the 64 KiB default
        hipError_t a1 = hipFuncSetAttribute((const void *)eig_iter_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_iter);
        hipError_t a2 = hipFuncSetAttribute((const void *)eig_chol_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_chol);
        hipError_t a3 = hipFuncSetAttribute((const void *)eig_gx_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_gx);
        hipError_t a4 = hipFuncSetAttribute((const void *)eig_rr_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_rr);
        if (a1 != hipSuccess || a2 != hipSuccess || a3 != hipSuccess || a4 != hipSuccess)
            return tsk_hip(c, a1 != hipSuccess ? a1 : a2 != hipSuccess ? a2 : a3 != hipSuccess ? a3 : a4,
                           "LDS attribute");
    }

    TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
               hipLaunchKernelGGL(eig_init_kernel,
                                  dim3((unsigned)(((m > pp ? m : pp) * pp + 255) / 256)), dim3(256), 0,
                                  c->stream, Y[0], m, pp, p, Rinv, (uint64_t)0x5eed5eedull));
    int cur = 0, it = 0;
    bool converged = false;
    std::vector<double> hsmall(2 + k);
    std::vector<double> htheta(pp);
    const int check = c->eig_check > 0 ? c->eig_check : 16;
    const int max_iter = c->eig_max_iter > 0 ? c->eig_max_iter : 600;
    const double tol = c->eig_tol > 0 ? c->eig_tol : 1e-10;
    while (it < max_iter) {
        const int steps = (max_iter - it < check) ? max_iter - it : check;
        for (int s = 0; s < steps; ++s) {
            TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
                       hipLaunchKernelGGL(eig_iter_kernel, dim3(nblk), dim3(256), lds_iter, c->stream, G, m, pp,
                                          (const double *)Y[cur], (const double *)Rinv, Y[cur ^ 1], part));
            TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
                       hipLaunchKernelGGL(eig_chol_kernel, dim3(EIG_NRED), dim3(256), lds_chol, c->stream,
                                          (const double *)part, nblk, pp, p, Cg, Rinv, counter, tol_chol, ndead));
            cur ^= 1;
        }
        it += steps;
        // Rayleigh-Ritz on X = Y Rinv
        TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                   hipLaunchKernelGGL(eig_x_kernel, dim3(nblk), dim3(256), 0, c->stream, (const double *)Y[cur],
                                      (const double *)Rinv, m, pp, X));
        TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                   hipLaunchKernelGGL(eig_gx_kernel, dim3(nblk), dim3(256), lds_gx, c->stream, G, m, pp,
                                      (const double *)X, GX, part));
        TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                   hipLaunchKernelGGL(eig_rr_kernel, dim3(EIG_NRED), dim3(256), lds_rr, c->stream,
                                      (const double *)part, nblk, pp, Cg, W, theta, counter));
        TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                   hipLaunchKernelGGL(eig_res_kernel, dim3(nblk), dim3(256), 0, c->stream, (const double *)X,
                                      (const double *)GX, (const double *)W, (const double *)theta, m, pp, k, U,
                                      part));
        TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                   hipLaunchKernelGGL(eig_conv_kernel, dim3(1), dim3(256), 0, c->stream, (const double *)part,
                                      nblk, k, (const double *)theta, (const double *)U, tol, small));
        e = hipMemcpyAsync(hsmall.data(), small, sizeof(double) * (2 + k), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return tsk_hip(c, e, "memcpy");
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return tsk_hip(c, e, "eigensolver");
        if (hsmall[0] != 0.0) {
            converged = true;
            break;
        }
    }
    TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
               hipLaunchKernelGGL(eig_emit_kernel, dim3((unsigned)((m * k + 255) / 256)), dim3(256), 0, c->stream,
                                  (const double *)U, (const double *)small, m, k, S));
    e = hipMemcpyAsync(htheta.data(), theta, sizeof(double) * pp, hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "memcpy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "eigensolver");
    if (lambda)
        for (int i = 0; i <= k; ++i) lambda[i] = (i < pp) ? htheta[i] : 0.0;
    if (iters_out) *iters_out = it;
    if (!converged) {
        char buf[160];
        snprintf(buf, sizeof buf, "eigensolver: residual %.3e above tol %.1e after %d iterations", hsmall[1], tol, it);
        return tsk_fail(c, TSK_E_NOCONV, buf);
    }
    return TSK_OK;
}
