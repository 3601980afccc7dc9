// Shared device helpers and the context structure of libtsk (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
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

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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
// Cyclic Jacobi eigensolver for a symmetric p x p FP64 matrix held in LDS,
// run by one whole workgroup.  Parallel (round-robin) ordering: each round
// rotates p/2 disjoint index pairs, p-1 rounds per sweep, so the rotations of
// a round commute and are applied together.  On exit H is (numerically)
// diagonal and W holds the eigenvectors as columns (H_in = W diag W^T).
// p must be even (pad with a zero row/column); ld is the LDS row stride.
// rot: LDS scratch of 4*(p/2) entries.
// ---------------------------------------------------------------------------
__device__ inline void jacobi_eig_lds(double *H, double *W, int p, int ld, double *rot,
                                      int *pairs, int max_sweeps, double *red4) {
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int e = tid; e < p * p; e += nth) {
        int i = e / p, j = e % p;
        W[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int half = p / 2;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal mass vs total mass
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < p * p; e += nth) {
            int i = e / p, j = e % p;
            double h = H[i * ld + j];
            tot += h * h;
            if (i != j) off += h * h;
        }
        off = block_sum_f64(off, red4);
        tot = block_sum_f64(tot, red4);
        if (off <= 1e-30 * tot || tot == 0.0) break;
        for (int round = 0; round < p - 1; ++round) {
            if (tid < half) {
                // player list: 0 fixed, the rest rotated by `round`
                int ia = (tid == 0) ? 0 : 1 + ((tid - 1 + round) % (p - 1));
                int ib = 1 + ((p - 2 - tid + round) % (p - 1));
                int a = ia < ib ? ia : ib, b = ia < ib ? ib : ia;
                double haa = H[a * ld + a], hbb = H[b * ld + b], hab = H[a * ld + b];
                double c = 1.0, s = 0.0;
                if (hab != 0.0 && fabs(hab) > 1e-18 * sqrt(fabs(haa * hbb))) {
                    double tau = (hbb - haa) / (2.0 * hab);
                    double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                rot[2 * tid] = c;
                rot[2 * tid + 1] = s;
                pairs[2 * tid] = a;
                pairs[2 * tid + 1] = b;
            }
            __syncthreads();
            // H <- H J and W <- W J (columns a, b)
            for (int e = tid; e < p * half; e += nth) {
                int i = e / half, t = e % half;
                int a = pairs[2 * t], b = pairs[2 * t + 1];
                double c = rot[2 * t], s = rot[2 * t + 1];
                double ha = H[i * ld + a], hb = H[i * ld + b];
                H[i * ld + a] = c * ha - s * hb;
                H[i * ld + b] = s * ha + c * hb;
                double wa = W[i * ld + a], wb = W[i * ld + b];
                W[i * ld + a] = c * wa - s * wb;
                W[i * ld + b] = s * wa + c * wb;
            }
            __syncthreads();
            // H <- J^T H (rows a, b)
            for (int e = tid; e < p * half; e += nth) {
                int j = e / half, t = e % half;
                int a = pairs[2 * t], b = pairs[2 * t + 1];
                double c = rot[2 * t], s = rot[2 * t + 1];
                double ha = H[a * ld + j], hb = H[b * ld + j];
                H[a * ld + j] = c * ha - s * hb;
                H[b * ld + j] = s * ha + c * hb;
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
// Context
// ---------------------------------------------------------------------------
struct TskBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct TskEvent {
    int cls;
    hipEvent_t a, b;
};

struct tsk_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // workspaces
    TskBuf gram_part, gram_G;
    TskBuf eig_Y0, eig_Y1, eig_Rinv, eig_part, eig_C, eig_X, eig_GX, eig_small, eig_U;
    TskBuf counters;
    TskBuf ap_St, ap_B, ap_Vt, ap_C, ap_fro, ap_qflag;
    TskBuf er_part;
    // eigensolver controls
    int eig_block = 0, eig_max_iter = 300, eig_check = 4;
    double eig_tol = 1e-7;
    // timing
    bool timing = false;
    std::vector<TskEvent> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches[TSK_KERNEL_COUNT] = {};
    double ms[TSK_KERNEL_COUNT] = {};
};

// host helpers (runtime.hip)
tsk_status tsk_fail(tsk_ctx c, tsk_status st, const std::string &msg);
tsk_status tsk_hip(tsk_ctx c, hipError_t e, const char *what);
tsk_status tsk_grow(tsk_ctx c, TskBuf &b, size_t bytes);
tsk_status tsk_check_dev(tsk_ctx c, const void *p, size_t bytes, const char *name);
tsk_status tsk_check_stack(tsk_ctx c, const tsk_stack *s, const char *name);
void tsk_ev_begin(tsk_ctx c, hipEvent_t *a);
void tsk_ev_end(tsk_ctx c, int cls, hipEvent_t a);

// Launch wrapper: optional event bracket + launch error check.
#define TSK_LAUNCH(ctx, cls, ...)                                           \
    do {                                                                    \
        hipEvent_t _ev_a = nullptr;                                         \
        tsk_ev_begin((ctx), &_ev_a);                                        \
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
