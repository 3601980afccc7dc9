// Shared device helpers and the context structure of libtsk (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tsk.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

#define TSK_WAVE 64

// ---------------------------------------------------------------------------
// MFMA wrappers.  Operand layout of the 16x16x4 shapes (one wave of 64 lanes,
// lane = 16*q + i with q = lane/16, i = lane%16), measured on gfx950:
//   A operand: lane supplies A[i][q]      (16 x 4)
//   B operand: lane supplies B[q][i]      (4 x 16)
//   D result, f32: lane holds D[4q + r][i]  for r = 0..3
//   D result, f64: lane holds D[q + 4r][i]  for r = 0..3
// ---------------------------------------------------------------------------
__device__ __forceinline__ v4f mfma16x16x4_f32(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma16x16x4_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16x16x32 bf16 (FP32 accumulate), measured on gfx950: lane 16*q + i
// supplies A[i][8q .. 8q+7] and B[8q .. 8q+7][i] (8 consecutive bf16 in 4
// dwords, element 2t in the low half of dword t); D as for the f32 shape.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4f mfma16x16x32_bf16(v4u a, v4u b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

// 16x16x128 e4m3 x e4m3 with block scales (FP32 accumulate), measured on
// gfx950: lane 16*q + i supplies 32 bytes of row i of A and of column i of
// B; byte e of lane (q, i) of A pairs with byte e of lane (q, i') of B (the
// contraction order is the same on both operands); D as for the f32 shape.
// sa, sb: E8M0 exponents (127 = 1.0) multiplying the A and B operands.
typedef int v8i __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v4f mfma16x16x128_e4m3(v8i a, v8i b, v4f c, int sa, int sb) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
}
// The same with per-lane scales taken from byte OA of sa and byte OB of sb:
// lane (q, i) supplies the E8M0 scale of row i of A (column i of B) for the
// MFMA's K block q, and K block g is bytes 0..15 of lane groups 2(g & 1)
// and 2(g & 1) + 1 for g < 2, their bytes 16..31 for g >= 2 (measured).
template <int OA, int OB>
__device__ __forceinline__ v4f mfma16x16x128_e4m3_sel(v8i a, v8i b, v4f c, int sa, int sb) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, OA, sa, OB, sb);
}
// Two e4m3 bytes of w (bytes 0,1, or 2,3 when hi) to two bf16 packed in a
// dword, multiplied by the power of two sc (exact: e4m3 values are bf16
// values).
__device__ __forceinline__ unsigned e4m3x2_to_bf16(unsigned w, float sc, bool hi) {
    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
    const v2bf b = hi ? __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, sc, true)
                      : __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, sc, false);
    return __builtin_bit_cast(unsigned, b);
}
// 8 e4m3 bytes (two dwords) -> 8 bf16 (four dwords), times sc.
__device__ __forceinline__ v4u e4m3x8_to_bf16(uint2 w, float sc) {
    return v4u{e4m3x2_to_bf16(w.x, sc, false), e4m3x2_to_bf16(w.x, sc, true), e4m3x2_to_bf16(w.y, sc, false),
               e4m3x2_to_bf16(w.y, sc, true)};
}

// bf16 bits <-> float (bf16 is the upper half of a binary32).
__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
// Round-to-nearest-even float -> bf16 of two values packed into one dword
// (x in the low half), by the hardware conversion.
__device__ __forceinline__ unsigned pack_bf16(float x, float y) {
    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2bf h = __builtin_convertvector(v2f{x, y}, v2bf);
    return __builtin_bit_cast(unsigned, h);
}
// Sum of squares of the 8 bf16 values of a 16-byte vector, in FP32.
__device__ __forceinline__ float sumsq_bf16x8(v4u v) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float a = bf16_lo(v[t]), b = bf16_hi(v[t]);
        s = fmaf(a, a, s);
        s = fmaf(b, b, s);
    }
    return s;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide FP64 sum over NW waves (blockDim.x == 64 NW), the wave sums
// added in wave order; result valid in every thread.  scratch: NW doubles.
template <int NW>
__device__ __forceinline__ double block_sum_nw(double v, double *scratch) {
    v = wave_sum_f64(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double t = scratch[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) t += scratch[i];
    __syncthreads();
    return t;
}

// Block-wide FP64 sum for blockDim.x == 256; result valid in every thread.
__device__ __forceinline__ double block_sum_f64(double v, double *scratch4) {
    v = wave_sum_f64(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch4[w] = v;
    __syncthreads();
    double t = scratch4[0] + scratch4[1] + scratch4[2] + scratch4[3];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver pieces (Golub & Van Loan, Section 8.5): parallel
// round-robin ordering, each round rotates p/2 disjoint index pairs, p-1
// rounds per sweep.  Because the pairs are disjoint, H' = J^T H J splits
// into independent 2x2 blocks J_P^T H_PQ J_Q.  The Frobenius norm is
// invariant, so the stopping test needs only the off-diagonal mass.
// ---------------------------------------------------------------------------
// Reciprocal and reciprocal square root from the hardware FP64 estimates
// refined by Newton-Raphson steps (each step squares the relative error).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * fma(-x, r, 2.0);
    r = r * fma(-x, r, 2.0);
    return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

// Rotation (c, s) that zeroes H[a][b] in J^T H J.  t only has to be accurate
// enough for the sweep to converge; c = (1+t^2)^-1/2 and s = t c are what
// make the rotation orthogonal, so c is refined to full precision.
__device__ __forceinline__ void jacobi_rot(const double *H, int ld, int a, int b, double &c, double &s) {
    const double haa = H[a * ld + a], hbb = H[b * ld + b], hab = H[a * ld + b];
    c = 1.0;
    s = 0.0;
    // |hab| > 1e-18 sqrt(|haa hbb|), compared squared (no square root on the
    // round's critical path)
    if (hab != 0.0 && hab * hab > 1e-36 * fabs(haa * hbb)) {
        // t from the hardware estimates (an angle that is slightly off still
        // shrinks H[a][b] by the estimates' relative error, so the sweeps
        // converge); c refined so that c^2 + s^2 = 1 to rounding
        const double tau = (hbb - haa) * __builtin_amdgcn_rcp(2.0 * hab);
        const double q = 1.0 + tau * tau;
        const double root = q * __builtin_amdgcn_rsq(q);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) * __builtin_amdgcn_rcp(fabs(tau) + root);
        c = rsq_nr(1.0 + t * t);
        s = t * c;
    }
}

// Slot t of round rd of the round-robin pairing of p players (player 0
// fixed, the others rotated by rd): returns (a, b), a < b.  Pure arithmetic,
// so no pairing table has to be read in the inner loops.
__device__ __forceinline__ void rr_pair(int t, int rd, int p, int &a, int &b) {
    int ia = 0;
    if (t != 0) {
        ia = t - 1 + rd;
        if (ia >= p - 1) ia -= p - 1;
        ia += 1;
    }
    int ib = p - 2 - t + rd;
    if (ib >= p - 1) ib -= p - 1;
    ib += 1;
    a = ia < ib ? ia : ib;
    b = ia < ib ? ib : ia;
}

// Cyclic Jacobi for a symmetric p x p FP64 matrix in LDS, one workgroup of
// NTH threads (256 or 1024), in place.  Each round rotates the p/2 disjoint
// pairs of the round-robin ordering: the rotations are computed by p/2
// threads into rot,
// then every 2x2 block (P, Q), P <= Q, of J^T H J is rewritten by one thread
// together with its mirror image (the blocks are disjoint, so no second
// buffer is needed) and the eigenvector matrix is updated, W <- W J, stored
// TRANSPOSED (Wt[j][i] = W[i][j]).  A thread's blocks and items are fixed
// pair SLOTS; the indices occupying a slot advance by one (cyclically over
// 1..p-1, index 0 fixed) from round to round, so they are updated by an
// increment instead of being recomputed, and every load of a round is issued
// before its arithmetic.  Stops when the off-diagonal mass is below
// 1e-18 ||H||_F^2: eigenvalues are then exact to rounding (their error is
// second order in the off-diagonal part) and eigenvectors to 1e-9 of the
// relative gap.  A rotation is stored as one (c, s) pair and a W item
// covers two adjacent entries (16-byte accesses).  MAXB >= ceil(p(p+2)/8 /
// NTH), MAXW >= ceil(p^2/4 / NTH).  On exit H is diagonal to rounding and
// H_in = W diag W^T.  p even <= 64, ld even; rot: p doubles; Wt and rot
// 16-byte aligned; red: NTH/64 doubles.
template <int MAXB, int MAXW, int NTH = 256>
__device__ inline void jacobi_eig_wg(double *H, double *Wt, int p, int ld, double *rot, int max_sweeps,
                                     double *red4) {
    const int tid = threadIdx.x;
    const int half = p / 2;
    double tot = 0.0;
    for (int e = tid; e < p * p; e += NTH) {
        const int i = e / p, j = e % p;
        Wt[i * ld + j] = (i == j) ? 1.0 : 0.0;
        const double h = H[i * ld + j];
        tot += h * h;
    }
    tot = block_sum_nw<NTH / 64>(tot, red4);
    // slot -> indices at round 0 (rr_pair(t, 0)); ordered pairs (first,
    // second) are kept as produced, the rotation convention only needs the
    // same order in every use
    auto slot0 = [&](int t, int &a, int &b) {
        a = t == 0 ? 0 : t;
        b = p - 1 - t;
    };
    auto adv = [&](int x) { return x == 0 ? 0 : (x == p - 1 ? 1 : x + 1); };
    // fixed work items: blocks along the diagonals Q - P = 0, 1, ... and W
    // items row-fastest, so neighbouring threads touch different rows AND
    // columns (the row stride may be a multiple of the LDS bank count)
    const int nblk = half * (half + 1) / 2;
    // item slots that hold work for some thread (MAXB, MAXW cover the largest
    // p; the loops below skip the rest, a uniform test)
    const int nbu = (nblk + NTH - 1) / NTH, nwu = (half * half + NTH - 1) / NTH;
    bool bv[MAXB], wv_[MAXW];
    int bA[MAXB], bB[MAXB], bX[MAXB], bY[MAXB], bP[MAXB], bQ[MAXB];
    int wI[MAXW], wX[MAXW], wY[MAXW], wQ[MAXW];
    {
        int dg = 0, off = 0;
#pragma unroll
        for (int u = 0; u < MAXB; ++u) {
            const int e = tid + NTH * u;
            int P = 0, Q = 0;
            bv[u] = e < nblk;
            if (bv[u]) {
                while (e - off >= half - dg) {
                    off += half - dg;
                    ++dg;
                }
                P = e - off;
                Q = P + dg;
            }
            bP[u] = P;
            bQ[u] = Q;
        }
    }
    // W items: entry pairs (column 2c, 2c + 1) of the two rows of a slot
#pragma unroll
    for (int u = 0; u < MAXW; ++u) {
        const int e = tid + NTH * u;
        wv_[u] = e < half * half;
        wI[u] = wv_[u] ? 2 * (e % half) : 0;
        wQ[u] = wv_[u] ? e / half : 0;
    }
    int tA = 0, tB = 1;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0;
        for (int e = tid; e < p * p; e += NTH) {
            const int i = e / p, j = e % p;
            const double h = H[i * ld + j];
            if (i != j) off += h * h;
        }
        off = block_sum_nw<NTH / 64>(off, red4);
        if (off <= 1e-18 * tot || tot == 0.0) break;
        // indices of every slot at round 0 (the cycle returns there after
        // p - 1 rounds)
        if (tid < half) slot0(tid, tA, tB);
#pragma unroll
        for (int u = 0; u < MAXB; ++u) {
            slot0(bP[u], bA[u], bB[u]);
            slot0(bQ[u], bX[u], bY[u]);
        }
#pragma unroll
        for (int u = 0; u < MAXW; ++u) slot0(wQ[u], wX[u], wY[u]);
#pragma nounroll
        for (int rd = 0; rd < p - 1; ++rd) {
            if (tid < half) {
                double cc, ss;
                jacobi_rot(H, ld, tA, tB, cc, ss);
                *reinterpret_cast<double2 *>(rot + 2 * tid) = double2{cc, ss};
            }
            __syncthreads();
            // gather the blocks' entries (unused slots read block (0, 0): in
            // bounds, never stored) and the W items' rows together, so the
            // round waits for one set of LDS reads; then compute and write
            double hv[MAXB][4], rv[MAXB][4];
#pragma unroll
            for (int u = 0; u < MAXB; ++u) {
                if (u >= nbu) break;
                const int a = bA[u], b = bB[u], x = bX[u], y = bY[u];
                const double2 rp = *reinterpret_cast<const double2 *>(rot + 2 * bP[u]);
                const double2 rq = *reinterpret_cast<const double2 *>(rot + 2 * bQ[u]);
                rv[u][0] = rp.x; rv[u][1] = rp.y;
                rv[u][2] = rq.x; rv[u][3] = rq.y;
                hv[u][0] = H[a * ld + x]; hv[u][1] = H[a * ld + y];
                hv[u][2] = H[b * ld + x]; hv[u][3] = H[b * ld + y];
            }
            double2 w0v[MAXW], w1v[MAXW], wr[MAXW];
#pragma unroll
            for (int u = 0; u < MAXW; ++u) {
                if (u >= nwu) break;
                wr[u] = *reinterpret_cast<const double2 *>(rot + 2 * wQ[u]);
                w0v[u] = *reinterpret_cast<const double2 *>(Wt + wX[u] * ld + wI[u]);
                w1v[u] = *reinterpret_cast<const double2 *>(Wt + wY[u] * ld + wI[u]);
            }
#pragma unroll
            for (int u = 0; u < MAXB; ++u) {
                if (u >= nbu) break;
                const double cp = rv[u][0], sp = rv[u][1], cq = rv[u][2], sq = rv[u][3];
                const double hax = hv[u][0], hay = hv[u][1], hbx = hv[u][2], hby = hv[u][3];
                const double tax = cq * hax - sq * hay, tay = sq * hax + cq * hay;
                const double tbx = cq * hbx - sq * hby, tby = sq * hbx + cq * hby;
                const double nax = cp * tax - sp * tbx, nay = cp * tay - sp * tby;
                const double nbx = sp * tax + cp * tbx, nby = sp * tay + cp * tby;
                const int a = bA[u], b = bB[u], x = bX[u], y = bY[u];
                if (bv[u]) {
                    H[a * ld + x] = nax;
                    H[a * ld + y] = nay;
                    H[b * ld + x] = nbx;
                    H[b * ld + y] = nby;
                    if (bP[u] != bQ[u]) {  // off-diagonal block: its mirror image too
                        H[x * ld + a] = nax;
                        H[y * ld + a] = nay;
                        H[x * ld + b] = nbx;
                        H[y * ld + b] = nby;
                    }
                }
            }
            // W items: compute, write (two adjacent entries of each row)
#pragma unroll
            for (int u = 0; u < MAXW; ++u) {
                if (u >= nwu) break;
                const double cq = wr[u].x, sq = wr[u].y;
                if (wv_[u]) {
                    *reinterpret_cast<double2 *>(Wt + wX[u] * ld + wI[u]) =
                        double2{cq * w0v[u].x - sq * w1v[u].x, cq * w0v[u].y - sq * w1v[u].y};
                    *reinterpret_cast<double2 *>(Wt + wY[u] * ld + wI[u]) =
                        double2{sq * w0v[u].x + cq * w1v[u].x, sq * w0v[u].y + cq * w1v[u].y};
                }
            }
            // next round: every slot's indices advance
            tA = adv(tA);
            tB = adv(tB);
#pragma unroll
            for (int u = 0; u < MAXB; ++u) {
                bA[u] = adv(bA[u]); bB[u] = adv(bB[u]); bX[u] = adv(bX[u]); bY[u] = adv(bY[u]);
            }
#pragma unroll
            for (int u = 0; u < MAXW; ++u) {
                wX[u] = adv(wX[u]);
                wY[u] = adv(wY[u]);
            }
            __syncthreads();
        }
    }
}

// Stable descending order of the diagonal of H (p entries) into perm; run by
// thread 0 only, callers sync afterwards.
__device__ inline void sort_diag_desc(const double *H, int p, int ld, int *perm) {
    for (int i = 0; i < p; ++i) perm[i] = i;
    for (int i = 1; i < p; ++i) {
        int v = perm[i];
        double hv = H[v * ld + v];
        int j = i - 1;
        while (j >= 0 && H[perm[j] * ld + perm[j]] < hv) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

// ---------------------------------------------------------------------------
// Blocked inverse of an upper-triangular pp x pp matrix R (LDS) into X (LDS),
// pp a multiple of 8: 8x8 diagonal blocks inverted by one thread each, then
// neighbouring blocks merged level by level with X12 = -X11 R12 X22.  Zero
// diagonal entries (dead pivots) give zero rows/columns in X.  T: LDS scratch
// of pp*pp doubles.
// ---------------------------------------------------------------------------
__device__ inline void upper_tri_inverse(const double *R, double *X, int pp, double *T) {
    const int tid = threadIdx.x;
    for (int e = tid; e < pp * pp; e += blockDim.x) X[e] = 0.0;
    __syncthreads();
    // reciprocal diagonal, kept on the diagonal of X until the leaves use it
    for (int i = tid; i < pp; i += blockDim.x) {
        const double rii = R[i * pp + i];
        X[i * pp + i] = rii == 0.0 ? 0.0 : 1.0 / rii;
    }
    __syncthreads();
    // 8x8 diagonal blocks: one thread per (block, column); back substitution.
    // All reads of X's reciprocal diagonal happen before the barrier, all
    // writes after it; the barriers sit outside the branches.
    const int nblk = pp / 8;
    const bool act = tid < nblk * 8;
    const int o = (tid >> 3) * 8, j = tid & 7;
    double col[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) col[i] = 0.0;
    if (act) {
        const double dj = X[(o + j) * pp + (o + j)];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = (i == j) ? dj : 0.0;
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            if (i < j) {
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (t > i && t <= j) s += R[(o + i) * pp + (o + t)] * col[t];
                col[i] = -s * X[(o + i) * pp + (o + i)];
            }
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int i = 0; i < 8; ++i) X[(o + i) * pp + (o + j)] = (i <= j) ? col[i] : 0.0;
    }
    __syncthreads();
    for (int s = 8; s < pp; s *= 2) {
        const int ngroups = (pp + 2 * s - 1) / (2 * s);
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

// ---------------------------------------------------------------------------
// Cholesky C = R^T R of a symmetric positive semi-definite pp x pp matrix in
// LDS (row stride ld; only the upper triangle is read, C is destroyed), then
// X = R^-1 (LDS, stride pp).  A pivot <= tol_rel * max(diag) marks the index
// dead: its row of R and its row and column of X are zero.  R, X: LDS pp*pp
// each; dead: LDS pp ints.  Returns (in every thread) the number of dead
// indices below `live`.  MAXU: entries per thread, at least
// ceil(pp^2 / blockDim.x) (a compile-time bound keeps them in registers).
// Right-looking, one barrier per column: each thread keeps the upper-triangle
// entries it owns in registers for the whole factorisation; at step j the
// owners of row j (final by then) publish it into one of two LDS row buffers
// (the first 2 pp doubles of X), and every owner of an entry (a, b), a > j,
// subtracts C[j][a] C[j][b] / C[j][j] from it, all its reads of the row
// issued before the first use.  R = rows / sqrt(pivots) is formed after the
// loop (the pivots are kept in X), off the per-column path.  (Updating the
// entries in LDS made each thread's three accesses per entry wait on one
// another: 1.1 us per column at pp = 64.)
// ---------------------------------------------------------------------------
template <int MAXU>
__device__ inline int chol_factor_inverse(double *C, int ld, int pp, double tol_rel, double *R, double *X, int *dead,
                                          int live = 1 << 30) {
    __shared__ double s_maxd;
    __shared__ int s_nd;
    __shared__ double s_inv[2];
    const int tid = threadIdx.x;
    const int nth = (int)blockDim.x;
    if (tid < 64) {  // largest diagonal entry (wave 0)
        double v = tid < pp ? C[tid * ld + tid] : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if (tid == 0) {
            s_maxd = v;
            s_nd = 0;
        }
    }
    // each thread owns the upper-triangle entries e = tid + nth u, u < MAXU,
    // of the pp x pp matrix
    int ea[MAXU], eb[MAXU];
    double cv[MAXU];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
        const int e = tid + nth * u;
        const int a = e / pp, b = e % pp;
        const bool own = e < pp * pp && a <= b;
        ea[u] = own ? a : -1;
        eb[u] = own ? b : 0;
        cv[u] = own ? C[a * ld + b] : 0.0;
    }
    for (int e = tid; e < pp * pp; e += nth)
        if (e % pp < e / pp) R[e] = 0.0;
    __syncthreads();
    const double thr = tol_rel * s_maxd;
    double *pv = X + 2 * pp;  // the pivots, for R once the loop is done
    double ra[MAXU], rc[MAXU];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) ra[u] = rc[u] = 0.0;
    for (int j = 0; j < pp; ++j) {
        double *rb = X + (j & 1) * pp;
        // row j is published with the reciprocal of its pivot, formed once
        // by the pivot's owner instead of by every thread (5% of the
        // kernel at pp = 64 and 1024 threads)
#pragma unroll
        for (int u = 0; u < MAXU; ++u)
            if (ea[u] == j) {
                rb[eb[u]] = cv[u];
                if (eb[u] == j) s_inv[j & 1] = (cv[u] > thr && cv[u] > 0.0) ? rcp_nr(cv[u]) : 0.0;
            }
        __syncthreads();
        // the column's reads are all issued before any of them is used
        const double piv = rb[j], inv = s_inv[j & 1];
#pragma unroll
        for (int u = 0; u < MAXU; ++u)
            if (ea[u] > j) {
                ra[u] = rb[ea[u]];
                rc[u] = rb[eb[u]];
            }
        asm volatile("" ::: "memory");
        const bool dj = !(piv > thr) || !(piv > 0.0);
        if (tid == 0) {
            dead[j] = dj;
            pv[j] = piv;
            if (dj && j < live) ++s_nd;
        }
        if (!dj) {
#pragma unroll
            for (int u = 0; u < MAXU; ++u)
                if (ea[u] > j) cv[u] -= ra[u] * rc[u] * inv;
        }
    }
    __syncthreads();
    // row a of R: the final row a of the update divided by sqrt(pivot a)
#pragma unroll
    for (int u = 0; u < MAXU; ++u)
        if (ea[u] >= 0) {
            const int a = ea[u];
            R[a * pp + eb[u]] = dead[a] ? 0.0 : cv[u] / sqrt(pv[a]);
        }
    __syncthreads();
    // C is free now: scratch of the inverse (needs ld >= pp)
    upper_tri_inverse(R, X, pp, C);
    return s_nd;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct TskBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Per-shape-class tuning of the apply (tsk_set_tuning): 0 = default.
struct TskTune {
    int groups = 0;   // pipeline groups of tsk_apply
    int pj_cols = 0;  // bf16 projection: columns per step (64 or 128)
};

struct TskEvent {
    int cls;
    hipEvent_t a, b;
};

// Pipeline streams.  HIP maps streams onto a few hardware queues (four by
// default), and the caller's stream takes one: with three pipeline streams
// every stream has a queue of its own.  On the 8-stream batch (8 captured
// plans of 256 matrices) two streams gave 326k matrices/s, three 386k and
// four 324k (two of them then share a queue).
constexpr int TSK_MAX_PIPE = 4;      // pipeline streams at most
constexpr int TSK_DEFAULT_PIPE = 3;  // pipeline streams by default

struct tsk_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // workspaces
    TskBuf gram_part, gram_G;
    TskBuf eig_Y0, eig_Y1, eig_Rinv, eig_part, eig_C, eig_X, eig_GX, eig_small, eig_U;
    TskBuf counters;
    TskBuf ap_ws;         // workspace of tsk_apply (one buffer, carved per call)
    TskBuf mt_ws;         // tsk_opt_tail: eigenvector block and trace
    TskBuf ap2_ws;        // tsk_apply2: C1, W slots, Zl, Zr
    TskBuf t2_ws;         // tsk_train2: Grams, transposed slices, projections
    void *scratch = nullptr;  // device address of the no-allocation scratch on this device
    TskBuf er_part, st_part;
    TskBuf mp_ws, mp_tab;            // batched apply: workspace, descriptors + items
    void *mp_pin = nullptr;          // pinned host copy of the batch tables
    size_t mp_pin_bytes = 0;
    hipEvent_t mp_ev = nullptr;      // recorded after the last batch table copy
    hipEvent_t switch_ev = nullptr;  // orders the old stream before a new one (tsk_set_stream)
    // pipelined apply and plan launches: npl (2..TSK_MAX_PIPE) context-owned
    // streams (default priority), forked from and joined back into the
    // caller's stream
    hipStream_t pl[TSK_MAX_PIPE] = {};
    hipEvent_t pl_fork = nullptr, pl_join[TSK_MAX_PIPE] = {};
    int npl = 0;
    // tuning entries by shape class (m, n, kp, dtype)
    std::map<std::tuple<int64_t, int64_t, int, int>, TskTune> tune;
    // eigensolver controls
    int eig_block = 0, eig_max_iter = 300, eig_check = 6;
    double eig_tol = 0.0;  // 0: TSK_EIG_TOL_F32 / TSK_EIG_TOL_BF16 by the Gram's precision
    // timing
    uint32_t timing = 0;  // bit i: bracket launches of kernel class i with events
    std::vector<TskEvent> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches[TSK_KERNEL_COUNT] = {};
    double ms[TSK_KERNEL_COUNT] = {};
};

// Default residual tolerances of the eigensolver, relative to theta_1, by the
// precision of the Gram's products.  FP32: the rounding level of FP32
// accumulation.  bf16: rounding the data to bf16 perturbs G by about
// 1e-4 theta_1 (2 ||E|| ||A|| with ||E|| ~ 2^-9 / sqrt(3) rms(A)
// (sqrt(m) + sqrt(nN))), so iterating below 1e-5 theta_1 cannot bring the
// Ritz vectors closer to those of the exact Gram.
constexpr double TSK_EIG_TOL_F32 = 1e-7;
constexpr double TSK_EIG_TOL_BF16 = 1e-5;
// e4m3 keeps 4 significant bits (relative rounding 2^-4 against bf16's
// 2^-8): the Gram moves about 2^4 times further, so the tolerance is 2^4
// times looser (rounded).
constexpr double TSK_EIG_TOL_F8 = 1e-4;

// No-allocation scratch (tsk_apply_noalloc): bytes of the file-scope device
// array, and the number of devices whose addresses are kept.
constexpr size_t TSK_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int TSK_MAX_DEVICES = 64;

// host helpers (runtime.hip)
tsk_status tsk_fail(tsk_ctx c, tsk_status st, const std::string &msg);
tsk_status tsk_hip(tsk_ctx c, hipError_t e, const char *what);
tsk_status tsk_grow(tsk_ctx c, TskBuf &b, size_t bytes);
tsk_status tsk_check_dev(tsk_ctx c, const void *p, size_t bytes, const char *name);
tsk_status tsk_check_stack(tsk_ctx c, const tsk_stack *s, const char *name);
tsk_status tsk_pipeline_streams(tsk_ctx c);
TskTune tsk_tuning(tsk_ctx c, int64_t m, int64_t n, int kp, int dtype);
void tsk_ev_begin(tsk_ctx c, int cls, hipEvent_t *a);
void tsk_ev_end(tsk_ctx c, int cls, hipEvent_t a);

// Launch wrapper: optional event bracket + launch error check.
#define TSK_LAUNCH(ctx, cls, ...)                                           \
    do {                                                                    \
        hipEvent_t _ev_a = nullptr;                                         \
        tsk_ev_begin((ctx), (cls), &_ev_a);                                 \
        __VA_ARGS__;                                                        \
        hipError_t _e = hipGetLastError();                                  \
        tsk_ev_end((ctx), (cls), _ev_a);                                    \
        if (_e != hipSuccess) return tsk_hip((ctx), _e, #cls);              \
    } while (0)

#define TSK_TRY(x)                          \
    do {                                    \
        tsk_status _s = (x);                \
        if (_s != TSK_OK) return _s;        \
    } while (0)
