// Data-free sketches for the SCW baseline: the randomly drawn sketching
// matrices the paper contrasts with its trained one (Section 1: Gaussian or
// Rademacher entries; Section 2: the sparse random sign matrix that
// initialises IVY's learned sketch).  Counter-based, so every entry is a pure
// function of (seed, position): the value of counter c is the c-th output
// (from 0) of SplitMix64 seeded with `seed` (Steele, Lea and Flood, OOPSLA
// 2014): state seed + (c + 1) * 0x9E3779B97F4A7C15, mixed by two
// xor-shift-multiply rounds and a final xor-shift.
#include <cmath>

#include "tsk_common.hpp"

namespace {

__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Dense kinds, one thread per entry (i, j), counter c = i m + j:
// kind 0 Gaussian N(0, 1/k) by Box-Muller on counters 2c and 2c + 1
// (u1 in (0, 1], u2 in [0, 1), 53 bits each, FP64, rounded once to FP32);
// kind 1 Rademacher +-1/sqrt(k) by the top bit of output c.
__global__ void dense_sketch_kernel(int kind, int64_t k, int64_t m, uint64_t seed, double scale,
                                    float *__restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * m) return;
    const uint64_t c = (uint64_t)e;
    double v;
    if (kind == 1) {
        v = (sm64(seed, c) >> 63) ? -1.0 : 1.0;
    } else {
        const double u1 = (double)((sm64(seed, 2 * c) >> 11) + 1) * 0x1p-53;
        const double u2 = (double)(sm64(seed, 2 * c + 1) >> 11) * 0x1p-53;
        v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
    }
    S[e] = (float)(v * scale);
}

// Sparse random sign (CountSketch): one thread per column j writes the whole
// column: +-1 (bit 0 of output j) in row (output j >> 32) mod k, zeros
// elsewhere.
__global__ void sparse_sketch_kernel(int64_t k, int64_t m, uint64_t seed, float *__restrict__ S) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint64_t h = sm64(seed, (uint64_t)j);
    const int64_t row = (int64_t)((h >> 32) % (uint64_t)k);
    const float v = (h & 1u) ? -1.f : 1.f;
    for (int64_t i = 0; i < k; ++i) S[i * m + j] = i == row ? v : 0.f;
}

}  // namespace

tsk_status tsk_random_sketch_enqueue(tsk_ctx c, int kind, int64_t k, int64_t m, uint64_t seed, float *S) {
    if (kind == TSK_SKETCH_SPARSE) {
        TSK_LAUNCH(c, TSK_KERNEL_SKETCH,
                   hipLaunchKernelGGL(sparse_sketch_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream,
                                      k, m, seed, S));
    } else {
        TSK_LAUNCH(c, TSK_KERNEL_SKETCH,
                   hipLaunchKernelGGL(dense_sketch_kernel, dim3((unsigned)((k * m + 255) / 256)), dim3(256), 0,
                                      c->stream, kind, k, m, seed, 1.0 / std::sqrt((double)k), S));
    }
    return TSK_OK;
}
