// Leading-k eigenvectors of the symmetric mode-1 Gram: the Tucker1 factor
// S* = (U^(1))_k^T of Section 3.1 (the first k left singular vectors of
// A_(1) are the top-k eigenvectors of G = A_(1) A_(1)^T).
//
// Method: block subspace iteration in FP64 on a block of p >= k columns
// (padded to pp, a multiple of 16; padding columns stay zero), accelerated by
// a degree-2 Chebyshev filter (Zhou & Saad's filtered subspace iteration):
//     L = (G - c I) / e,   Y1 = L X,   Y2 = 2 L Y1 - X  (= T_2(L) X)
// with [0, b] the damped interval, c = e = b / 2 and b the smallest Ritz value
// of the block (every wanted eigenvalue lies above b and is amplified,
// everything in [0, b] is bounded by 1).  Y2 is orthonormalised by
// CholeskyQR2 in FP64.  Every few filter steps a Rayleigh-Ritz step
// diagonalises H = X^T G X (Jacobi), rotates the block to Ritz vectors, resets
// the filter interval and tests ||G u_i - theta_i u_i|| <= tol theta_1, i < k.
//
// Kernels (FP64 throughout)
//  eig_mv     : P = G In, FP64 MFMA 16x16x4, grid = 16-row blocks x K-splits,
//               operands prefetched one step ahead.
//  eig_filter : sums the K-split partials, Y2 = 2/e (G Y1 - c Y1) - X,
//               partial Gram of Y2.
//  eig_apply  : Out = In Rinv (+ partial Gram).
//  eig_chol   : one 1024-thread workgroup: sums the partial Grams in order,
//               Cholesky + triangular inverse -> Rinv.
//  eig_gx     : GX = G X, Y1 = (GX - c X)/e, or the Rayleigh-Ritz variant:
//               partial X^T G X.
//  eig_rr     : one 1024-thread workgroup: sums the partials of X^T G X and
//               runs the Jacobi eigensolver.
//  eig_rot    : X <- X W, GX <- GX W (Ritz vectors), Y1, residuals and the
//               sign convention; last workgroup sets the convergence flag.
//  eig_emit   : S (k x m, FP32) from the converged Ritz vectors.
// Reductions across workgroups go through per-workgroup partials summed in a
// fixed order, so results are bitwise reproducible.
#include <type_traits>

#include "tsk_common.hpp"

namespace {

constexpr int MV_RB = 16;      // rows per matvec workgroup (one MFMA tile)
// Rows per row-kernel workgroup: 60 workgroups at m = 1920.  64 rows (30
// workgroups) took 10.20 / 5.45 ms per 1920 x 1080 bf16 / 1024 x 768 FP32
// training, 32 rows 9.85 / 5.26, 16 rows 9.92 / 5.20.
constexpr int RW_RB = 32;
constexpr int RR_THREADS = 1024;  // threads of the one-workgroup small-matrix kernels
constexpr int EIG_MAXPP = 64;  // largest padded block
constexpr int NT_MAX = EIG_MAXPP / 16;

// device scalar block (doubles)
enum {
    SM_CONV = 0,   // 1.0 once converged
    SM_RES = 1,    // max relative residual of the last check
    SM_C = 2,      // filter centre
    SM_E = 3,      // filter half width
    SM_THETA = 8,  // Ritz values, descending (EIG_MAXPP)
    SM_SIGN = SM_THETA + EIG_MAXPP,
    SM_W = SM_SIGN + EIG_MAXPP,              // Ritz rotation (pp x pp)
    SM_RINV = SM_W + EIG_MAXPP * EIG_MAXPP,  // inverse Cholesky factor (pp x pp)
    SM_TOTAL = SM_RINV + EIG_MAXPP * EIG_MAXPP
};

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Last-workgroup election: every workgroup publishes its partials, fences and
// takes a ticket; the one that draws the last ticket sees all partials.
__device__ __forceinline__ bool last_block(unsigned *counter) {
    __shared__ unsigned s_ticket;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_ticket = atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned total = gridDim.x * gridDim.y * gridDim.z;
    if (s_ticket != total - 1) return false;
    __threadfence();
    if (threadIdx.x == 0) *counter = 0u;
    return true;
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

__global__ void eig_init_kernel(double *Y, int64_t m, int pp, int p, double *small, uint64_t seed) {
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
        small[SM_RINV + e] = (i == j && i < p) ? 1.0 : 0.0;
    }
    if (e < SM_THETA) small[e] = 0.0;
}

// P[ks][r0:r0+16][:] = G[r0:r0+16, K_ks] * In[K_ks, :]
// (G and In without __restrict__: with it the compiler treats their loads as
// invariant and sinks the next step's loads to their use, which leaves no
// load in flight during the MFMAs)
template <int NT>
__global__ __launch_bounds__(256) void eig_mv_kernel(const double *G, int64_t m, int pp, const double *In,
                                                     double *__restrict__ P, int64_t kchunk) {
    __shared__ double wpart[4 * MV_RB * EIG_MAXPP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, ii = lane & 15;
    const int nt = NT;
    const int64_t r0 = (int64_t)blockIdx.x * MV_RB;
    const int ks = blockIdx.y;
    const int64_t row = r0 + ii;
    const bool rv = row < m;
    const double *grow = G + (rv ? row : 0) * m;
    const int64_t kw = kchunk >> 2;
    const int64_t kb = (int64_t)ks * kchunk + wv * kw;
    int64_t ke = kb + kw;
    if (ke > m) ke = m;
    v4d acc[NT];
#pragma unroll
    for (int x = 0; x < NT; ++x) acc[x] = v4d{0.0, 0.0, 0.0, 0.0};
    // whole steps of 16 and a row block inside m (uniform per wave): a loop
    // whose loads carry no conditions, so the next step's stay in flight
    // during this step's MFMAs; otherwise every load is guarded
    const bool whole = r0 + MV_RB <= m && (ke - kb) % 16 == 0;
    auto run = [&](auto whole_tag) {
        constexpr bool WHOLE = decltype(whole_tag)::value;
        auto load = [&](int64_t k0, double (&aa)[4], double (&bb)[4][NT]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t kk = k0 + 4 * q + u;
                if constexpr (WHOLE) {
                    aa[u] = grow[kk];
                    const double *yr = In + kk * pp + ii;
#pragma unroll
                    for (int x = 0; x < NT; ++x) bb[u][x] = yr[x * 16];
                } else {
                    const bool kv = kk < ke;
                    aa[u] = (rv && kv) ? grow[kk] : 0.0;
                    const double *yr = In + (kv ? kk : 0) * pp + ii;
#pragma unroll
                    for (int x = 0; x < NT; ++x) bb[u][x] = kv ? yr[x * 16] : 0.0;
                }
            }
        };
        auto mma = [&](const double (&aa)[4], const double (&bb)[4][NT]) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int x = 0; x < NT; ++x) acc[x] = mfma16x16x4_f64(aa[u], bb[u][x], acc[x]);
        };
        // two register sets used in turn (copying the next step's values
        // into the current set would wait for its loads at once): steps in
        // pairs, a0 holding the first of a pair, a1 the second
        double a0[4], b0[4][NT], a1[4], b1[4][NT];
        int64_t k0 = kb;
        if (kb < ke) load(kb, a0, b0);
        for (; k0 + 16 < ke; k0 += 32) {
            load(k0 + 16, a1, b1);
            // the loads above are issued here, ahead of the MFMAs
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(a0, b0);
            // past the last step the loads repeat step k0 + 16 (in range, unused)
            load(k0 + 32 < ke ? k0 + 32 : k0 + 16, a0, b0);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(a1, b1);
        }
        if (k0 < ke) mma(a0, b0);
    };
    if (whole)
        run(std::true_type{});
    else
        run(std::false_type{});
    // f64 result layout: lane holds D[q + 4r][ii]
#pragma unroll
    for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) wpart[(wv * 16 + q + 4 * r) * pp + x * 16 + ii] = acc[x][r];
    __syncthreads();
    double *out = P + ((int64_t)ks * m + r0) * pp;
    for (int e = threadIdx.x; e < MV_RB * pp; e += blockDim.x) {
        if (r0 + e / pp >= m) continue;
        out[e] = wpart[e] + wpart[16 * pp + e] + wpart[32 * pp + e] + wpart[48 * pp + e];
    }
}

// ---------------------------------------------------------------------------
// Row-kernel helpers
// ---------------------------------------------------------------------------

// Sum of the KS partial matvec products for this workgroup's rows into Zs.
// Elements are processed four at a time per thread, with all of their loads
// (up to 4 x 8 splits) issued before the first add.
__device__ inline void load_mv_rows(const double *__restrict__ P, int KS, int64_t m, int pp, int64_t r0, double *Zs) {
    const int nel = RW_RB * pp;
    for (int base = 0; base < nel; base += 4 * 256) {
        double v[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = base + threadIdx.x + 256 * u;
            const bool ok = e < nel && r0 + e / pp < m;
            const double *p = P + r0 * pp + e;
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) v[u][ks] = (ok && ks < KS) ? p[(int64_t)ks * m * pp] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = base + threadIdx.x + 256 * u;
            double s = 0.0;
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) s += v[u][ks];
            if (e < nel) Zs[e] = s;
        }
    }
}

// Upper triangle of A^T B over the block's rows (A, B: RW_RB x pp in LDS)
// into part (ntri doubles, row-major upper triangle).  FP64 MFMA 16x16x4:
// the 16x16 tile pairs (ta <= tb) are dealt to the four waves, K runs over
// the rows in steps of 4 (lane (q, i) supplies A[k0 + q][16 ta + i] and
// B[k0 + q][16 tb + i]; the result lane holds D[q + 4r][i]).
__device__ inline void block_gram(const double *As, const double *Bs, int pp, double *part) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, ii = lane & 15;
    const int nt = pp >> 4, npair = nt * (nt + 1) / 2;
    for (int pr = wv; pr < npair; pr += (int)(blockDim.x >> 6)) {
        int ta = 0, rem = pr;
        while (rem >= nt - ta) {
            rem -= nt - ta;
            ++ta;
        }
        const int tb = ta + rem;
        v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k0 = 0; k0 < RW_RB; k0 += 4)
            acc = mfma16x16x4_f64(As[(k0 + q) * pp + 16 * ta + ii], Bs[(k0 + q) * pp + 16 * tb + ii], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ga = 16 * ta + q + 4 * r, gb = 16 * tb + ii;
            if (ga <= gb) part[ga * pp - ga * (ga - 1) / 2 + (gb - ga)] = acc[r];
        }
    }
}

// Sum nparts upper-triangle partials into the full symmetric C (LDS), in
// partial order; an entry's partials are loaded 32 at a time, each group
// before any of its adds.
__device__ inline void reduce_tri(const double *__restrict__ part, int nparts, int pp, double *C) {
    const int ntri = pp * (pp + 1) / 2;
    for (int e = threadIdx.x; e < ntri; e += blockDim.x) {
        double s = 0.0;
        for (int w0 = 0; w0 < nparts; w0 += 32) {
            double v[32];
#pragma unroll
            for (int w = 0; w < 32; ++w) v[w] = (w0 + w < nparts) ? part[(int64_t)(w0 + w) * ntri + e] : 0.0;
#pragma unroll
            for (int w = 0; w < 32; ++w) s += v[w];
        }
        int a, b;
        tri_index(e, pp, a, b);
        C[a * pp + b] = s;
        C[b * pp + a] = s;
    }
    __syncthreads();
}

// C (LDS, full symmetric, destroyed) -> Rinv (global, pp x pp), see
// chol_factor_inverse.  lds: 2*pp*pp doubles of scratch.
__device__ inline void chol_inverse(double *C, int pp, double tol_rel, double *lds, double *Rinv) {
    __shared__ int dead[EIG_MAXPP];
    double *R = lds, *X = lds + pp * pp;
    chol_factor_inverse<(EIG_MAXPP * EIG_MAXPP + RR_THREADS - 1) / RR_THREADS>(C, pp, pp, tol_rel, R, X, dead);
    for (int e = threadIdx.x; e < pp * pp; e += blockDim.x) Rinv[e] = X[e];
}

// ---------------------------------------------------------------------------
// Row kernels (RW_RB rows per workgroup, 256 threads)
// ---------------------------------------------------------------------------

// Y2 = 2/e (G Y1 - c Y1) - X; partial Gram(Y2) (the Cholesky follows in
// eig_chol_kernel)
__global__ __launch_bounds__(256) void eig_filter_kernel(const double *__restrict__ P, int KS, int64_t m, int pp,
                                                         const double *__restrict__ Y1, const double *__restrict__ X,
                                                         double *__restrict__ Y2, double *__restrict__ part,
                                                         const double *__restrict__ small) {
    extern __shared__ __align__(16) double lds[];
    double *Zs = lds;  // RW_RB x pp
    const int64_t r0 = (int64_t)blockIdx.x * RW_RB;
    load_mv_rows(P, KS, m, pp, r0, Zs);
    const double c = small[SM_C], e = small[SM_E];
    const double al = 2.0 / e;
    __syncthreads();
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int64_t row = r0 + t / pp;
        double v = 0.0;
        if (row < m) {
            const int64_t g = r0 * pp + t;
            v = al * (Zs[t] - c * Y1[g]) - X[g];
            Y2[g] = v;
        }
        Zs[t] = v;
    }
    __syncthreads();
    const int ntri = pp * (pp + 1) / 2;
    block_gram(Zs, Zs, pp, part + (int64_t)blockIdx.x * ntri);
}

// Out = In Rinv; optionally Gram(Out) (the Cholesky follows in eig_chol_kernel)
__global__ __launch_bounds__(256) void eig_apply_kernel(const double *__restrict__ In, int64_t m, int pp,
                                                        double *__restrict__ Out, int want_gram,
                                                        double *__restrict__ part, const double *__restrict__ small) {
    extern __shared__ __align__(16) double lds[];
    double *Rs = lds;              // pp x pp
    double *Is = Rs + pp * pp;     // RW_RB x pp
    double *Os = Is + RW_RB * pp;  // RW_RB x pp
    const int64_t r0 = (int64_t)blockIdx.x * RW_RB;
    for (int t = threadIdx.x; t < pp * pp; t += blockDim.x) Rs[t] = small[SM_RINV + t];
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int64_t row = r0 + t / pp;
        Is[t] = row < m ? In[r0 * pp + t] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int i = t / pp, j = t % pp;
        double s = 0.0;
        for (int u = 0; u <= j; ++u) s += Is[i * pp + u] * Rs[u * pp + j];
        Os[t] = s;
        if (r0 + i < m) Out[r0 * pp + t] = s;
    }
    if (!want_gram) return;
    __syncthreads();
    const int ntri = pp * (pp + 1) / 2;
    block_gram(Os, Os, pp, part + (int64_t)blockIdx.x * ntri);
}

// Sum of the nparts partial Grams (in order) -> Cholesky -> Rinv, by one
// workgroup of RR_THREADS threads in a kernel of its own (it ran as the last
// row workgroup, 256 threads, while the rest of the GPU waited).  lds: 3 pp^2
// doubles.
__global__ __launch_bounds__(RR_THREADS) void eig_chol_kernel(const double *__restrict__ part, int nparts, int pp,
                                                              double *__restrict__ small, double tol_chol) {
    extern __shared__ __align__(16) double lds[];
    double *C = lds;
    reduce_tri(part, nparts, pp, C);
    chol_inverse(C, pp, tol_chol, lds + pp * pp, small + SM_RINV);
}

// After a single-pass Cholesky QR of Y2 (Rinv from eig_filter) and P = G Y2:
// X = Y2 Rinv, GX = P Rinv = G X, Y1 = (GX - c X)/e.  X is only
// well-conditioned here (one Cholesky pass), which is all that the next
// filtered step needs; the spans are exact.
__global__ __launch_bounds__(256) void eig_gxr_kernel(const double *__restrict__ P, int KS, int64_t m, int pp,
                                                      const double *__restrict__ Y2, double *__restrict__ X,
                                                      double *__restrict__ GX, double *__restrict__ Y1,
                                                      const double *__restrict__ small) {
    extern __shared__ __align__(16) double lds[];
    double *Rs = lds, *Zs = Rs + pp * pp, *Ys = Zs + RW_RB * pp;
    const int64_t r0 = (int64_t)blockIdx.x * RW_RB;
    for (int t = threadIdx.x; t < pp * pp; t += blockDim.x) Rs[t] = small[SM_RINV + t];
    load_mv_rows(P, KS, m, pp, r0, Zs);
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int64_t row = r0 + t / pp;
        Ys[t] = row < m ? Y2[r0 * pp + t] : 0.0;
    }
    const double c = small[SM_C], e = small[SM_E];
    __syncthreads();
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int i = t / pp, j = t % pp;
        if (r0 + i >= m) continue;
        double x = 0.0, g = 0.0;
        for (int u = 0; u <= j; ++u) {
            const double rv = Rs[u * pp + j];
            x += Ys[i * pp + u] * rv;
            g += Zs[i * pp + u] * rv;
        }
        X[r0 * pp + t] = x;
        GX[r0 * pp + t] = g;
        Y1[r0 * pp + t] = (g - c * x) / e;
    }
}

// GX = G X.  rr = 0: Y1 = (GX - c X)/e.  rr = 1: partial X^T GX per
// workgroup (eig_rr_kernel sums them and diagonalises).
__global__ __launch_bounds__(256) void eig_gx_kernel(const double *__restrict__ P, int KS, int64_t m, int pp, int live,
                                                     const double *__restrict__ X, double *__restrict__ GX,
                                                     double *__restrict__ Y1, int rr, double *__restrict__ part,
                                                     const double *__restrict__ small) {
    extern __shared__ __align__(16) double lds[];
    double *Zs = lds, *Xs = lds + RW_RB * pp;
    const int64_t r0 = (int64_t)blockIdx.x * RW_RB;
    load_mv_rows(P, KS, m, pp, r0, Zs);
    const double c = small[SM_C], e = small[SM_E];
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int64_t row = r0 + t / pp;
        Xs[t] = row < m ? X[r0 * pp + t] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        if (r0 + t / pp >= m) continue;
        GX[r0 * pp + t] = Zs[t];
        if (!rr) Y1[r0 * pp + t] = (Zs[t] - c * Xs[t]) / e;
    }
    if (!rr) return;
    const int ntri = pp * (pp + 1) / 2;
    block_gram(Xs, Zs, pp, part + (int64_t)blockIdx.x * ntri);
}

// Rayleigh-Ritz on the block: one workgroup of RR_THREADS threads sums the
// nparts partial Grams (in order), diagonalizes the pp x pp projection by
// cyclic Jacobi, and writes the Ritz vectors (descending) and values and the
// damped interval of the next filter to small.  A kernel of its own, so the
// Jacobi, which one workgroup runs while the rest of the GPU waits, has four
// times the threads of a row workgroup.  lds: 2 pp^2 doubles.
__global__ __launch_bounds__(RR_THREADS) void eig_rr_kernel(const double *__restrict__ part, int nparts, int pp,
                                                            int live, double *__restrict__ small) {
    extern __shared__ __align__(16) double lds[];
    __shared__ __align__(16) double rot[EIG_MAXPP];
    __shared__ int perm[EIG_MAXPP];
    __shared__ double red[RR_THREADS / 64];
    double *H = lds, *W = lds + pp * pp;
    reduce_tri(part, nparts, pp, H);
    jacobi_eig_wg<(EIG_MAXPP * (EIG_MAXPP + 2) / 8 + RR_THREADS - 1) / RR_THREADS,
                  (EIG_MAXPP * EIG_MAXPP / 4 + RR_THREADS - 1) / RR_THREADS, RR_THREADS>(H, W, pp, pp, rot, 40,
                                                                                        red);
    // W holds the eigenvectors transposed
    if (threadIdx.x == 0) sort_diag_desc(H, pp, pp, perm);
    __syncthreads();
    for (int t = threadIdx.x; t < pp * pp; t += blockDim.x) {
        const int i = t / pp, j = t % pp;
        small[SM_W + t] = W[perm[j] * pp + i];
    }
    for (int j = threadIdx.x; j < pp; j += blockDim.x) small[SM_THETA + j] = H[perm[j] * pp + perm[j]];
    if (threadIdx.x == 0) {
        // damped interval [0, b], b = smallest live Ritz value (kept positive)
        const double th1 = H[perm[0] * pp + perm[0]];
        double b = H[perm[live - 1] * pp + perm[live - 1]];
        b = fmax(b, 1e-6 * fabs(th1));
        if (!(b > 0.0)) b = 1.0;
        small[SM_C] = 0.5 * b;
        small[SM_E] = 0.5 * b;
    }
}

// X <- X W, GX <- GX W (rows in place), Y1 = (GX - c X)/e; residuals of the
// first k Ritz pairs and the per-column sign convention; last workgroup sets
// the convergence flag.
__global__ __launch_bounds__(256) void eig_rot_kernel(int64_t m, int pp, int k, double *__restrict__ X,
                                                      double *__restrict__ GX, double *__restrict__ Y1,
                                                      double *__restrict__ part, unsigned *counter,
                                                      double *__restrict__ small, double tol) {
    extern __shared__ __align__(16) double lds[];
    double *Ws = lds, *Xs = Ws + pp * pp, *Gs = Xs + RW_RB * pp, *Rs = Gs + RW_RB * pp;
    const int64_t r0 = (int64_t)blockIdx.x * RW_RB;
    for (int t = threadIdx.x; t < pp * pp; t += blockDim.x) Ws[t] = small[SM_W + t];
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const bool v = r0 + t / pp < m;
        Xs[t] = v ? X[r0 * pp + t] : 0.0;
        Gs[t] = v ? GX[r0 * pp + t] : 0.0;
    }
    const double c = small[SM_C], e = small[SM_E];
    __syncthreads();
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const int i = t / pp, j = t % pp;
        double x = 0.0, g = 0.0;
        for (int u = 0; u < pp; ++u) {
            const double w = Ws[u * pp + j];
            x += Xs[i * pp + u] * w;
            g += Gs[i * pp + u] * w;
        }
        const double th = small[SM_THETA + j];
        Rs[t] = g - th * x;
        if (r0 + i < m) {
            X[r0 * pp + t] = x;
            GX[r0 * pp + t] = g;
            Y1[r0 * pp + t] = (g - c * x) / e;
        }
    }
    __syncthreads();
    // rotated rows, for the sign convention (Xs is free once all threads
    // have finished the rotation above)
    for (int t = threadIdx.x; t < RW_RB * pp; t += blockDim.x) {
        const bool v = r0 + t / pp < m;
        Xs[t] = v ? X[r0 * pp + t] : 0.0;
    }
    __syncthreads();
    double *o = part + (int64_t)blockIdx.x * 3 * k;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0, best = -1.0;
        int64_t bi = 0;
        for (int i = 0; i < RW_RB; ++i) {
            if (r0 + i >= m) break;
            s += Rs[i * pp + j] * Rs[i * pp + j];
            const double a = fabs(Xs[i * pp + j]);
            if (a > best) {
                best = a;
                bi = r0 + i;
            }
        }
        o[j] = s;
        o[k + j] = best;
        o[2 * k + j] = (double)bi;
    }
    if (!last_block(counter)) return;
    __shared__ double red[256];
    double worst = 0.0;
    const double th1 = fmax(fabs(small[SM_THETA]), 1e-300);
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0, best = -1.0, bi = 0.0;
        for (int b = 0; b < (int)gridDim.x; ++b) {
            const double *pb = part + (int64_t)b * 3 * k;
            s += pb[j];
            if (pb[k + j] > best) {
                best = pb[k + j];
                bi = pb[2 * k + j];
            }
        }
        worst = fmax(worst, sqrt(s) / th1);
        const double sv = X[(int64_t)bi * pp + j];
        small[SM_SIGN + j] = sv < 0.0 ? -1.0 : 1.0;
    }
    red[threadIdx.x] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) w = fmax(w, red[i]);
        small[SM_RES] = w;
        small[SM_CONV] = (w <= tol) ? 1.0 : 0.0;
    }
}

// S[i][j] = sign_i * X[j][i]  (FP32, k x m)
__global__ void eig_emit_kernel(const double *__restrict__ X, const double *__restrict__ small, int64_t m, int pp, int k,
                                float *__restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * k) return;
    const int i = (int)(e / m);
    const int64_t j = e % m;
    S[e] = (float)(small[SM_SIGN + i] * X[j * pp + i]);
}

}  // namespace

tsk_status tsk_eig_enqueue(tsk_ctx c, const double *G, int64_t m, int k, float *S, double *lambda,
                           int32_t *iters_out, double tol_default) {
    const int qx = k / 2 > 12 ? k / 2 : 12;  // guard columns beyond k
    int p = c->eig_block > 0 ? c->eig_block : k + qx;
    if (p > EIG_MAXPP) p = EIG_MAXPP;
    if (p > m) p = (int)m;
    if (p < k + 1) return tsk_fail(c, TSK_E_ARG, "tsk_eig_topk: search block too small for k");
    const int pp = (p + 15) / 16 * 16;
    const int ntri = pp * (pp + 1) / 2;
    const int nmv = (int)((m + MV_RB - 1) / MV_RB);
    const int nrw = (int)((m + RW_RB - 1) / RW_RB);
    // K-split of the matvec: aim for >= 256 workgroups, chunks multiples of 64
    int KS = (256 + nmv - 1) / nmv;
    if (KS > 8) KS = 8;
    int64_t kchunk = ((m + KS - 1) / KS + 63) / 64 * 64;
    KS = (int)((m + kchunk - 1) / kchunk);
    const size_t mp = (size_t)m * pp;
    TSK_TRY(tsk_grow(c, c->eig_Y0, sizeof(double) * mp * 3));  // X, GX, Y1
    TSK_TRY(tsk_grow(c, c->eig_Y1, sizeof(double) * mp * 2));  // Y2, X1
    TSK_TRY(tsk_grow(c, c->eig_X, sizeof(double) * mp * KS));  // matvec partials
    TSK_TRY(tsk_grow(c, c->eig_part, sizeof(double) * (size_t)nrw * (ntri > 3 * k ? ntri : 3 * k)));
    TSK_TRY(tsk_grow(c, c->eig_small, sizeof(double) * SM_TOTAL));
    TSK_TRY(tsk_grow(c, c->counters, 256));
    double *X = (double *)c->eig_Y0.p, *GX = X + mp, *Y1 = GX + mp;
    double *Y2 = (double *)c->eig_Y1.p, *X1 = Y2 + mp;
    double *P = (double *)c->eig_X.p, *part = (double *)c->eig_part.p, *small = (double *)c->eig_small.p;
    unsigned *counter = (unsigned *)c->counters.p;
    hipError_t e = hipMemsetAsync(c->counters.p, 0, 256, c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "memset");

    const size_t lds_filter = sizeof(double) * RW_RB * pp;
    const size_t lds_apply = sizeof(double) * (pp * pp + 2 * RW_RB * pp);
    const size_t lds_gx = sizeof(double) * 2 * RW_RB * pp;
    const size_t lds_rr = sizeof(double) * 2 * pp * pp;
    const size_t lds_chol = sizeof(double) * 3 * pp * pp;
    const size_t lds_rot = sizeof(double) * (pp * pp + 3 * RW_RB * pp);
    {
        hipError_t a1 = hipFuncSetAttribute((const void *)eig_filter_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_filter);
        hipError_t a2 = hipFuncSetAttribute((const void *)eig_apply_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_apply);
        hipError_t a3 = hipFuncSetAttribute((const void *)eig_gx_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_gx);
        hipError_t a4 = hipFuncSetAttribute((const void *)eig_rot_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_rot);
        if (a4 == hipSuccess)
            a4 = hipFuncSetAttribute((const void *)eig_rr_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_rr);
        if (a4 == hipSuccess)
            a4 = hipFuncSetAttribute((const void *)eig_chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_chol);
        if (a1 != hipSuccess || a2 != hipSuccess || a3 != hipSuccess || a4 != hipSuccess)
            return tsk_hip(c, a1 != hipSuccess ? a1 : a2 != hipSuccess ? a2 : a3 != hipSuccess ? a3 : a4,
                           "LDS attribute");
    }
    const double tol_chol = 1e-26;
    const double tol = c->eig_tol > 0 ? c->eig_tol : tol_default;
    const dim3 gmv((unsigned)nmv, (unsigned)KS);

    auto mv = [&](const double *in) -> tsk_status {
#define TSK_MV(NTV)                                                                                     \
    TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,                                                                  \
               hipLaunchKernelGGL(eig_mv_kernel<NTV>, gmv, dim3(256), 0, c->stream, G, m, pp, in, P, kchunk))
        switch (pp / 16) {  // pp is a multiple of 16, at most EIG_MAXPP
            case 1: TSK_MV(1); break;
            case 2: TSK_MV(2); break;
            case 3: TSK_MV(3); break;
            default: TSK_MV(4); break;
        }
#undef TSK_MV
        return TSK_OK;
    };
    auto chol = [&]() -> tsk_status {
        TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
                   hipLaunchKernelGGL(eig_chol_kernel, dim3(1), dim3(RR_THREADS), lds_chol, c->stream,
                                      (const double *)part, nrw, pp, small, tol_chol));
        return TSK_OK;
    };
    auto apply = [&](const double *in, double *out, int gram) -> tsk_status {
        TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
                   hipLaunchKernelGGL(eig_apply_kernel, dim3(nrw), dim3(256), lds_apply, c->stream, in, m, pp, out,
                                      gram, part, (const double *)small));
        return gram ? chol() : TSK_OK;
    };
    auto gx = [&](int rr) -> tsk_status {
        TSK_LAUNCH(c, rr ? TSK_KERNEL_EIG_RR : TSK_KERNEL_EIG_ITER,
                   hipLaunchKernelGGL(eig_gx_kernel, dim3(nrw), dim3(256), lds_gx, c->stream, (const double *)P, KS,
                                      m, pp, p, (const double *)X, GX, Y1, rr, part,
                                      (const double *)small));
        if (rr)
            TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                       hipLaunchKernelGGL(eig_rr_kernel, dim3(1), dim3(RR_THREADS), lds_rr, c->stream,
                                          (const double *)part, nrw, pp, p, small));
        return TSK_OK;
    };
    auto rot = [&]() -> tsk_status {
        TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
                   hipLaunchKernelGGL(eig_rot_kernel, dim3(nrw), dim3(256), lds_rot, c->stream, m, pp, k, X, GX, Y1,
                                      part, counter, small, tol));
        return TSK_OK;
    };
    const size_t lds_gxr = sizeof(double) * (pp * pp + 2 * RW_RB * pp);
    {
        hipError_t a5 = hipFuncSetAttribute((const void *)eig_gxr_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_gxr);
        if (a5 != hipSuccess) return tsk_hip(c, a5, "LDS attribute");
    }
    // one filtered step: Y2 = T_2(L) X; a single Cholesky QR pass keeps the
    // block well conditioned; before a Rayleigh-Ritz check (rr = 1) the block
    // is made orthonormal with CholeskyQR2.
    auto filter_step = [&](int rr) -> tsk_status {
        TSK_TRY(mv(Y1));
        TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
                   hipLaunchKernelGGL(eig_filter_kernel, dim3(nrw), dim3(256), lds_filter, c->stream,
                                      (const double *)P, KS, m, pp, (const double *)Y1, (const double *)X, Y2, part,
                                      (const double *)small));
        TSK_TRY(chol());
        if (!rr) {
            TSK_TRY(mv(Y2));
            TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
                       hipLaunchKernelGGL(eig_gxr_kernel, dim3(nrw), dim3(256), lds_gxr, c->stream,
                                          (const double *)P, KS, m, pp, (const double *)Y2, X, GX, Y1,
                                          (const double *)small));
            return TSK_OK;
        }
        TSK_TRY(apply(Y2, X1, 1));
        TSK_TRY(apply(X1, X, 0));
        TSK_TRY(mv(X));
        return gx(1);
    };

    // start: random block, CholeskyQR2, Rayleigh-Ritz
    const size_t ninit = (size_t)(m > pp ? m : pp) * pp;
    TSK_LAUNCH(c, TSK_KERNEL_EIG_ITER,
               hipLaunchKernelGGL(eig_init_kernel, dim3((unsigned)((ninit + 255) / 256)), dim3(256), 0, c->stream,
                                  Y2, m, pp, p, small, (uint64_t)0x5eed5eedull));
    TSK_TRY(apply(Y2, X1, 1));  // Rinv = I: copy + Gram
    TSK_TRY(apply(X1, Y2, 1));
    TSK_TRY(apply(Y2, X, 0));
    TSK_TRY(mv(X));
    TSK_TRY(gx(1));
    TSK_TRY(rot());

    // Convergence checks (Rayleigh-Ritz + residuals) are spaced adaptively:
    // after two checks the per-step decay of the largest residual predicts
    // how many filtered steps remain, and the next check is placed there
    // (at least 1, at most 4 x `check` steps away).
    const int check = c->eig_check > 0 ? c->eig_check : 6;
    const int max_steps = c->eig_max_iter > 0 ? c->eig_max_iter : 300;
    int steps = 0;
    double hs[2] = {0.0, 0.0};
    bool converged = false;
    int next = check;
    double prev_res = -1.0;
    while (steps < max_steps) {
        const int nb = (max_steps - steps < next) ? max_steps - steps : next;
        for (int s = 0; s < nb; ++s) TSK_TRY(filter_step(s == nb - 1));
        TSK_TRY(rot());
        steps += nb;
        e = hipMemcpyAsync(hs, small, sizeof(hs), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return tsk_hip(c, e, "memcpy");
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return tsk_hip(c, e, "eigensolver");
        if (hs[SM_CONV] != 0.0) {
            converged = true;
            break;
        }
        const double res = hs[SM_RES];
        next = check;
        if (prev_res > 0.0 && res > 0.0 && res < prev_res) {
            const double rate = pow(res / prev_res, 1.0 / nb);  // per filtered step
            const double need = log(tol / res) / log(rate);
            if (need > 0.0 && need < 1e6) next = (int)ceil(need);
            if (next < 1) next = 1;
            if (next > 4 * check) next = 4 * check;
        }
        prev_res = res;
    }
    TSK_LAUNCH(c, TSK_KERNEL_EIG_RR,
               hipLaunchKernelGGL(eig_emit_kernel, dim3((unsigned)((m * k + 255) / 256)), dim3(256), 0, c->stream,
                                  (const double *)X, (const double *)small, m, pp, k, S));
    std::vector<double> th(k + 1);
    e = hipMemcpyAsync(th.data(), small + SM_THETA, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "memcpy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return tsk_hip(c, e, "eigensolver");
    if (lambda)
        for (int i = 0; i <= k; ++i) lambda[i] = th[i];
    // block products with G: 1 to start + 2 per filtered step
    if (iters_out) *iters_out = 1 + 2 * steps;
    if (!converged) {
        char buf[160];
        snprintf(buf, sizeof buf, "eigensolver: residual %.3e above tol %.1e after %d filtered steps", hs[SM_RES], tol,
                 steps);
        return tsk_fail(c, TSK_E_NOCONV, buf);
    }
    return TSK_OK;
}
