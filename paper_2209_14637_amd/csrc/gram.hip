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
//  * The workgroup stages 32 columns of its 256 operand rows in LDS per
//    step (coalesced 128-byte row reads), double buffered: the next step's
//    global loads are in flight while this step's MFMAs run.
//  * The contraction index (slice, column) can be visited in any order as
//    long as both operands use the same order, so each lane reads 2 float4
//    (columns 4q..+3 and 16+4q..+3 of one staged row) and feeds component u
//    of them to MFMA number u.
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

// Stage = 32 columns of one slice for the tile's 128 row-block rows (Ra) and
// 128 column-block rows (Rb), staged in LDS and double buffered.  LDS rows
// are padded to 36 floats so that the 16 rows read by one ds_read_b128
// quarter-wave start in distinct bank groups.
constexpr int GK = 32;           // columns per stage
constexpr int GLD = GK + 4;      // padded LDS row length
constexpr int GBUF = 2 * GT * GLD;  // floats per stage buffer (Ra and Rb)

__device__ __forceinline__ void gram_fetch(const float *__restrict__ Ad, int64_t m, int64_t n, int64_t ld,
                                           int64_t rb0, int64_t cb0, int64_t c0, float4 (&v)[8]) {
    // thread t: row (t >> 3) + 32 u of each block, columns c0 + 4 (t & 7) .. +3
    const int t = threadIdx.x;
    const int64_t cc = c0 + 4 * (t & 7);
    const bool fullc = cc + 3 < n;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t row = (u < 4 ? rb0 : cb0) + (t >> 3) + 32 * (u & 3);
        float4 x = float4{0.f, 0.f, 0.f, 0.f};
        if (row < m && cc < n) {
            const float *p = Ad + row * ld + cc;
            if (fullc) {
                x = *reinterpret_cast<const float4 *>(p);
            } else {
                x.x = p[0];
                if (cc + 1 < n) x.y = p[1];
                if (cc + 2 < n) x.z = p[2];
            }
        }
        v[u] = x;
    }
}

__device__ __forceinline__ void gram_stash(float *buf, const float4 (&v)[8]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = (u < 4 ? 0 : GT) + (t >> 3) + 32 * (u & 3);
        *reinterpret_cast<float4 *>(buf + r * GLD + 4 * (t & 7)) = v[u];
    }
}

__global__ __launch_bounds__(256) void gram_f32_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                       int64_t ld, int64_t stride, int64_t count, int T,
                                                       int nchunks, int per_xcd, float *__restrict__ part) {
    __shared__ float lds[2 * GBUF];
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
    const int64_t rb0 = (int64_t)bi * GT, cb0 = (int64_t)bj * GT;
    const int wr = (wv >> 1) * 64, wc = GT + (wv & 1) * 64;  // LDS row offsets of this wave's operands

    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    const int64_t spd = (n + GK - 1) / GK;  // stages per slice
    const int64_t nst = (d1 - d0) * spd;
    float4 pre[8];
    gram_fetch(A + d0 * stride, m, n, ld, rb0, cb0, 0, pre);
    gram_stash(lds, pre);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
        const float *cur = lds + (st & 1) * GBUF;
        const bool more = st + 1 < nst;
        if (more) {
            const int64_t s1 = st + 1;
            const int64_t d = d0 + s1 / spd;
            gram_fetch(A + d * stride, m, n, ld, rb0, cb0, (s1 % spd) * GK, pre);
        }
        float a[4][8], b[4][8];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const float *ra = cur + (wr + x * 16 + ii) * GLD + 4 * q;
            const float *rc = cur + (wc + x * 16 + ii) * GLD + 4 * q;
            const float4 a0 = *reinterpret_cast<const float4 *>(ra), a1 = *reinterpret_cast<const float4 *>(ra + 16);
            const float4 b0 = *reinterpret_cast<const float4 *>(rc), b1 = *reinterpret_cast<const float4 *>(rc + 16);
            a[x][0] = a0.x; a[x][1] = a0.y; a[x][2] = a0.z; a[x][3] = a0.w;
            a[x][4] = a1.x; a[x][5] = a1.y; a[x][6] = a1.z; a[x][7] = a1.w;
            b[x][0] = b0.x; b[x][1] = b0.y; b[x][2] = b0.z; b[x][3] = b0.w;
            b[x][4] = b1.x; b[x][5] = b1.y; b[x][6] = b1.z; b[x][7] = b1.w;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x4_f32(a[x][u], b[y][u], acc[x][y]);
        if (more) gram_stash(lds + ((st + 1) & 1) * GBUF, pre);
        __syncthreads();
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

// ---------------------------------------------------------------------------
// BF16 products (the precision form): same tiling, chunking and partial
// layout as the FP32 kernel; a stage is 64 bf16 columns (128 bytes of every
// staged row, the same LDS geometry), and each lane feeds the 16x16x32 bf16
// MFMA with two 16-byte reads per staged row.  The source is either bf16
// (read as stored) or FP32 rounded to bf16 (nearest-even) on the way into
// LDS, so training can consume an FP32 stack directly.
// ---------------------------------------------------------------------------
constexpr int HK = 64;            // bf16 columns per stage
constexpr int HLD = HK + 8;       // padded LDS row, bf16 elements (144 bytes)
constexpr int HBUF = 2 * GT * HLD;  // bf16 elements per stage buffer

// Per-thread staged data: 8 row chunks of 8 columns (thread t: chunk t & 7,
// rows (t >> 3) + 32 u of the row block (u < 4) or column block (u >= 4)).
template <typename SrcT> struct HRaw;
template <> struct HRaw<uint16_t> { v4u v[8]; };
template <> struct HRaw<float> { float4 v[16]; };

__device__ __forceinline__ void hfetch(const uint16_t *__restrict__ Ad, int64_t m, int64_t n, int64_t ld,
                                       int64_t rb0, int64_t cb0, int64_t c0, HRaw<uint16_t> &raw) {
    const int t = threadIdx.x;
    const int64_t cc = c0 + 8 * (t & 7);
    const bool fullc = cc + 7 < n;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t row = (u < 4 ? rb0 : cb0) + (t >> 3) + 32 * (u & 3);
        v4u x = v4u{0u, 0u, 0u, 0u};
        if (row < m && cc < n) {
            const uint16_t *p = Ad + row * ld + cc;
            if (fullc) {
                x = *reinterpret_cast<const v4u *>(p);
            } else {
                unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (cc + e < n) w[e >> 1] |= (unsigned)p[e] << (16 * (e & 1));
                x = v4u{w[0], w[1], w[2], w[3]};
            }
        }
        raw.v[u] = x;
    }
}

__device__ __forceinline__ void hfetch(const float *__restrict__ Ad, int64_t m, int64_t n, int64_t ld, int64_t rb0,
                                       int64_t cb0, int64_t c0, HRaw<float> &raw) {
    const int t = threadIdx.x;
    const int64_t cc = c0 + 8 * (t & 7);
    const bool fullc = cc + 7 < n;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t row = (u < 4 ? rb0 : cb0) + (t >> 3) + 32 * (u & 3);
        float4 x0 = float4{0.f, 0.f, 0.f, 0.f}, x1 = x0;
        if (row < m && cc < n) {
            const float *p = Ad + row * ld + cc;
            if (fullc) {
                x0 = *reinterpret_cast<const float4 *>(p);
                x1 = *reinterpret_cast<const float4 *>(p + 4);
            } else {
                float w[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (cc + e < n) w[e] = p[e];
                x0 = float4{w[0], w[1], w[2], w[3]};
                x1 = float4{w[4], w[5], w[6], w[7]};
            }
        }
        raw.v[2 * u] = x0;
        raw.v[2 * u + 1] = x1;
    }
}

__device__ __forceinline__ v4u hpack(const HRaw<uint16_t> &raw, int u) { return raw.v[u]; }
__device__ __forceinline__ v4u hpack(const HRaw<float> &raw, int u) {
    const float4 a = raw.v[2 * u], b = raw.v[2 * u + 1];
    return v4u{pack_bf16(a.x, a.y), pack_bf16(a.z, a.w), pack_bf16(b.x, b.y), pack_bf16(b.z, b.w)};
}

template <typename SrcT>
__device__ __forceinline__ void hstash(uint16_t *buf, const HRaw<SrcT> &raw) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = (u < 4 ? 0 : GT) + (t >> 3) + 32 * (u & 3);
        *reinterpret_cast<v4u *>(buf + r * HLD + 8 * (t & 7)) = hpack(raw, u);
    }
}

template <typename SrcT>
__global__ __launch_bounds__(256, 2 * (sizeof(SrcT) == 2) + (sizeof(SrcT) != 2)) void gram_bf16_kernel(const SrcT *__restrict__ A, int64_t m, int64_t n,
                                                        int64_t ld, int64_t stride, int64_t count, int T,
                                                        int nchunks, int per_xcd, float *__restrict__ part) {
    __shared__ uint16_t lds[2 * HBUF];
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
    const int64_t rb0 = (int64_t)bi * GT, cb0 = (int64_t)bj * GT;
    const int wr = (wv >> 1) * 64, wc = GT + (wv & 1) * 64;

    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    const int64_t spd = (n + HK - 1) / HK;
    const int64_t nst = (d1 - d0) * spd;
    // bf16 source: global loads run two stages ahead of the MFMAs (two
    // register sets, used alternately): a stage's MFMA time is far shorter
    // than the memory latency, so one stage of lookahead leaves every stage
    // waiting.
    auto fetch = [&](int64_t s1, HRaw<SrcT> &dst) {
        const int64_t d = d0 + s1 / spd;
        hfetch(A + d * stride, m, n, ld, rb0, cb0, (s1 % spd) * HK, dst);
    };
    auto mma_stage = [&](const uint16_t *cur) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            v4u a[4], b[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[x] = *reinterpret_cast<const v4u *>(cur + (wr + x * 16 + ii) * HLD + 8 * q + 32 * h);
                b[x] = *reinterpret_cast<const v4u *>(cur + (wc + x * 16 + ii) * HLD + 8 * q + 32 * h);
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x32_bf16(a[x], b[y], acc[x][y]);
        }
    };
    if constexpr (sizeof(SrcT) == 2) {
        HRaw<SrcT> p0, p1;
        fetch(0, p0);
        hstash(lds, p0);
        if (nst > 1) fetch(1, p1);
        __syncthreads();
        // pairs of stages: stage st lives in buffer 0, st + 1 in buffer 1; p1
        // carries stage st + 1 (issued a stage earlier), p0 receives st + 2
        int64_t st = 0;
        for (; st + 1 < nst; st += 2) {
            if (st + 2 < nst) fetch(st + 2, p0);
            mma_stage(lds);
            hstash(lds + HBUF, p1);
            __syncthreads();
            if (st + 3 < nst) fetch(st + 3, p1);
            mma_stage(lds + HBUF);
            if (st + 2 < nst) hstash(lds, p0);
            __syncthreads();
        }
        if (st < nst) mma_stage(lds);
    } else {
        // FP32 source: twice the registers per staged stage, so one stage of
        // lookahead (the conversion to bf16 happens on the way into LDS)
        HRaw<SrcT> pre;
        fetch(0, pre);
        hstash(lds, pre);
        __syncthreads();
        for (int64_t st = 0; st < nst; ++st) {
            const bool more = st + 1 < nst;
            if (more) fetch(st + 1, pre);
            mma_stage(lds + (st & 1) * HBUF);
            if (more) hstash(lds + ((st + 1) & 1) * HBUF, pre);
            __syncthreads();
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

// ---------------------------------------------------------------------------
// Wide-tile Gram for a bf16 stack (16x16x32 bf16 MFMA) or an e4m3 stack
// (16x16x128 e4m3 MFMA whose E8M0 operand scales fold the slice's scale in
// exactly): 256x256 tiles of G's lower triangle, 8 waves, each owning a
// 128x64 block (8x4 MFMA 16x16 tiles).  A tile reads half the operand bytes
// per flop of a 128x128 tile, which is what the per-CU path from L2 allows at
// full MFMA rate.  The tile's 128x128 quarters are written as the same
// per-chunk partials as the 128x128 kernels (quarter (2I+a, 2J+b) of tile
// (I, J)), so one reduction serves both.  Waves whose quarter lies above the
// diagonal or past the last row skip their MFMAs; a diagonal tile stages its
// 256 rows once and reads both operands from them.  A stage is 128 bytes of
// every operand row: 64 bf16 or 128 e4m3 columns (an e4m3 stage never
// straddles slices, so one scale serves it).
// ---------------------------------------------------------------------------
constexpr int WT = 256;                 // tile edge
constexpr int WROW = 128;               // LDS row: 128 bytes, unpadded
constexpr int WBUF = 2 * WT * WROW;     // bytes per stage buffer
constexpr int W_THREADS = 512;
constexpr size_t W_LDS = 2 * WBUF;

// LDS bank layout (measured on gfx950: 16-byte accesses are served 32 lanes
// at a time over 128 four-byte banks).  The 16-byte chunk c of LDS row r is
// stored at chunk c ^ wswz(r): the 32 lanes of an MFMA operand read (16
// rows of one 16-row block; chunks q and q + 4h of bf16 operands, chunks 2q
// or 2q + 1 of e4m3 operands, q < 2) then fall on 32 distinct 16-byte bank
// groups, and so do the 32 lanes of a store (4 whole rows).
template <typename ET>
__device__ __forceinline__ int wswz(int r) {
    const int a = (r >> 2) & 3;
    return sizeof(ET) == 2 ? 2 * a : (a & 1) + 4 * (a >> 1);
}

// Mask of the valid bytes of a 16-byte chunk whose first nb bytes are valid.
__device__ __forceinline__ v4u colmask(int nb) {
    v4u k;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = nb - 4 * j;
        k[j] = v >= 4 ? 0xffffffffu : (v <= 0 ? 0u : (1u << (8 * v)) - 1u);
    }
    return k;
}

// ---------------------------------------------------------------------------
// The kernel loads the operand rows straight into LDS (global_load_lds, 16
// bytes per lane): no register staging and no LDS store instructions (a
// register-staged version with loads two stages ahead was 5-10% slower).  The compiler waits for every such load in flight
// before any later LDS read, so a stage reads all its MFMA operands into
// registers first, then issues the next stage's loads into the other buffer,
// then runs its MFMAs; the loads are waited for at the end of the stage.
// Lane l of a load writes LDS row 8u + (l >> 3) of its wave's 64, physical
// chunk l & 7, so it loads the logical chunk (l & 7) ^ wswz(row).  Rows
// past m load row m - 1 (they only feed entries the reduction discards);
// chunks reaching past column n load in-bounds columns and are rewritten
// masked by the wave that loaded them once its loads have landed.
// ---------------------------------------------------------------------------
template <typename ET>
__global__ __launch_bounds__(W_THREADS) void gram_wide_kernel(const ET *__restrict__ A, const float *__restrict__ scale,
                                                             int64_t m, int64_t n, int64_t ld, int64_t stride,
                                                             int64_t count, int TW, int T, int nchunks, int per_xcd,
                                                             float *__restrict__ part) {
    constexpr int EB = (int)sizeof(ET);
    constexpr int SC = WROW / EB;  // columns per stage
    constexpr int CE = 16 / EB;    // columns per 16-byte chunk
    extern __shared__ __align__(16) uint8_t wlds[];
    const int w = blockIdx.x;
    const int xcd = w & 7, local = w >> 3;
    const int t = local % TW, sub = local / TW;
    const int chunk = xcd * per_xcd + sub;
    const int64_t d0 = (int64_t)chunk * count / nchunks;
    const int64_t d1 = (int64_t)(chunk + 1) * count / nchunks;
    if (d0 >= d1) return;
    int bi, bj;
    tile_coords(t, bi, bj);
    const bool diag = bi == bj;
    const int nb = (int)((m + GT - 1) / GT);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, ii = lane & 15;
    const int wr = wv >> 2, wc = wv & 3;
    const int qa = 2 * bi + wr, qb = 2 * bj + (wc >> 1);
    const bool active = qa < nb && qb <= qa;
    const int ra = wr * 128, rb = (diag ? 0 : WT) + wc * 64;
    const bool stager = !diag || wv < 4;
    const int64_t rbase = (wv < 4 ? (int64_t)bi * WT : (int64_t)bj * WT - WT) + 64 * wv;
    const int rl0 = 64 * wv;
    const uint32_t ldb = (uint32_t)(ld * EB);
    // load u of this thread: logical chunk lcu(u) of LDS row rl0 + 8u +
    // (lane >> 3), matrix row row0 + 8u, recomputed at every use from values
    // passed through an empty asm (hoisted out of the loop they hold 16
    // VGPRs and the kernel spills)
    const int row0 = (int)(rbase + (lane >> 3));
    auto lcu = [&](int u, int ln) { return (ln & 7) ^ wswz<ET>(rl0 + 8 * u + (ln >> 3)); };

    v4f acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    const int64_t spd = (n + SC - 1) / SC;
    const int64_t nst = (d1 - d0) * spd;
    const bool ragged = n % SC != 0;
    // the stage after the current one: slice nd, first column nc
    int64_t nd = d0, nc = 0;
    auto advance = [&]() {
        nc += SC;
        if (nc >= n) {
            nc = 0;
            ++nd;
        }
    };
    auto issue = [&](uint8_t *buf) {
        const char *base = reinterpret_cast<const char *>(A + nd * stride);
        int ln = lane, r0 = row0;
        asm volatile("" : "+v"(ln), "+v"(r0));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t col = nc + (int64_t)CE * lcu(u, ln);
            const uint32_t roff = (uint32_t)min(r0 + 8 * u, (int)(m - 1)) * ldb;
            const char *src = base + (roff + (uint32_t)(col < n ? col * EB : 0));
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src),
                                             (__attribute__((address_space(3))) void *)(buf + (rl0 + 8 * u) * WROW),
                                             16, 0, 0);
        }
    };
    // once this wave's loads of the stage at column c have landed: its chunks
    // reaching past n keep their valid bytes only
    auto fix = [&](uint8_t *buf, int64_t c) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t col = c + (int64_t)CE * lcu(u, lane);
            if (col + CE > n) {
                v4u *pch = reinterpret_cast<v4u *>(buf + (rl0 + 8 * u + (lane >> 3)) * WROW + 16 * (lane & 7));
                const int nvb = (int)min(max(n - col, (int64_t)0), (int64_t)CE) * EB;
                *pch = *pch & colmask(nvb);
            }
        }
    };
    auto escale = [&](int64_t d) {
        int es = 127;
        if constexpr (EB == 1) {
            int j;
            frexpf(scale[d], &j);
            es = 127 - (j - 1);
        }
        return es;
    };
    // stage 0
    if (stager) issue(wlds);
    int64_t cd = nd, cc = nc;  // the current stage
    advance();
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's loads have landed
    if (stager && ragged && cc + SC > n) fix(wlds, cc);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
        const uint8_t *cur = wlds + (st & 1) * WBUF;
        uint8_t *nxt = wlds + ((st + 1) & 1) * WBUF;
        const bool more = st + 1 < nst;
        const int es = escale(cd);
        if constexpr (EB == 2) {
            // every operand of the stage into registers, then the next
            // stage's loads, then the MFMAs
            v4u a[2][8], b[2][4];
            if (active) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int co = 16 * ((q + 4 * h) ^ wswz<ET>(ii));
#pragma unroll
                    for (int x = 0; x < 8; ++x)
                        a[h][x] = *reinterpret_cast<const v4u *>(cur + (ra + x * 16 + ii) * WROW + co);
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        b[h][y] = *reinterpret_cast<const v4u *>(cur + (rb + y * 16 + ii) * WROW + co);
                }
            }
            if (stager && more) issue(nxt);
            if (active) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int x = 0; x < 8; ++x)
#pragma unroll
                        for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x32_bf16(a[h][x], b[h][y], acc[x][y]);
            }
        } else {
            const int c0 = 16 * ((2 * q) ^ wswz<ET>(ii)), c1 = 16 * ((2 * q + 1) ^ wswz<ET>(ii));
            auto frag = [&](int row) {
                const v4u lo = *reinterpret_cast<const v4u *>(cur + row * WROW + c0);
                const v4u hi = *reinterpret_cast<const v4u *>(cur + row * WROW + c1);
                return v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            };
            v8i a[8], b[4];
            if (active) {
#pragma unroll
                for (int y = 0; y < 4; ++y) b[y] = frag(rb + y * 16 + ii);
#pragma unroll
                for (int x = 0; x < 8; ++x) a[x] = frag(ra + x * 16 + ii);
            }
            if (stager && more) issue(nxt);
            if (active) {
#pragma unroll
                for (int x = 0; x < 8; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x128_e4m3(a[x], b[y], acc[x][y], es, es);
            }
        }
        // the MFMAs stay ahead of the wait, which covers the loads' latency
        __builtin_amdgcn_sched_barrier(0);
        cd = nd;
        cc = nc;
        advance();
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
        if (stager && more && ragged && cc + SC > n) fix(nxt, cc);
        __syncthreads();
    }
    if (!active) return;
    const int tq = qa * (qa + 1) / 2 + qb;
    float *P = part + ((int64_t)chunk * T + tq) * (GT * GT);
    const int lc0 = (wc & 1) * 64;
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) P[(x * 16 + 4 * q + r) * GT + lc0 + y * 16 + ii] = acc[x][y][r];
}

// ---------------------------------------------------------------------------
// e4m3 products (the e4m3 form): same tiling; a stage is 128 e4m3 columns
// (again 128 bytes of every staged row), one 16x16x128 MFMA per tile per
// stage.  Slice d is stored as A_d s_d with s_d = 2^j_d, so each product is
// multiplied by 2^-2j_d through the MFMA's own operand scales (E8M0, exact);
// stages never straddle slices.
// ---------------------------------------------------------------------------
constexpr int QK = 128;  // e4m3 columns per stage

__device__ __forceinline__ void qfetch(const uint8_t *__restrict__ Ad, int64_t m, int64_t n, int64_t ld,
                                       int64_t rb0, int64_t cb0, int64_t c0, v4u (&v)[8]) {
    const int t = threadIdx.x;
    const int64_t cc = c0 + 16 * (t & 7);
    const bool fullc = cc + 15 < n;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t row = (u < 4 ? rb0 : cb0) + (t >> 3) + 32 * (u & 3);
        v4u x = v4u{0u, 0u, 0u, 0u};
        if (row < m && cc < n) {
            const uint8_t *p = Ad + row * ld + cc;
            if (fullc) {
                x = *reinterpret_cast<const v4u *>(p);
            } else {
                unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (cc + e < n) w[e >> 2] |= (unsigned)p[e] << (8 * (e & 3));
                x = v4u{w[0], w[1], w[2], w[3]};
            }
        }
        v[u] = x;
    }
}

__device__ __forceinline__ void qstash(uint8_t *buf, const v4u (&v)[8]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = (u < 4 ? 0 : GT) + (t >> 3) + 32 * (u & 3);
        *reinterpret_cast<v4u *>(buf + r * (2 * HLD) + 16 * (t & 7)) = v[u];
    }
}

// MX: a block-scaled stack (one E8M0 exponent per 32 consecutive elements of
// a row, bscale[(d m + i) nbk + b]); every lane loads the exponents of its
// four A rows and four B rows at its 32-column block of a stage together
// with the stage's data, packs them one byte per operand tile once they
// have landed, and hands them to the MFMA, which selects the byte.
template <bool MX>
__global__ __launch_bounds__(256, 2) void gram_e4m3_kernel(const uint8_t *__restrict__ A,
                                                           const float *__restrict__ scale,
                                                           const uint8_t *__restrict__ bscale, int nbk, int64_t m,
                                                           int64_t n, int64_t ld, int64_t stride, int64_t count,
                                                           int T, int nchunks, int per_xcd,
                                                           float *__restrict__ part) {
    constexpr int QLD = 2 * HLD;        // padded LDS row, bytes (144)
    constexpr int QBUF = 2 * GT * QLD;  // bytes per stage buffer
    __shared__ uint8_t lds[2 * QBUF];
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
    const int64_t rb0 = (int64_t)bi * GT, cb0 = (int64_t)bj * GT;
    const int wr = (wv >> 1) * 64, wc = GT + (wv & 1) * 64;
    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t spd = (n + QK - 1) / QK;
    const int64_t nst = (d1 - d0) * spd;
    auto fetch = [&](int64_t s1, v4u (&dst)[8]) {
        const int64_t d = d0 + s1 / spd;
        qfetch(A + d * stride, m, n, ld, rb0, cb0, (s1 % spd) * QK, dst);
    };
    // E8M0 operand scale 2^-j of the stage's slice (scale[d] = 2^j)
    auto escale = [&](int64_t s1) {
        if constexpr (MX) return 0;
        int j;
        frexpf(scale[d0 + s1 / spd], &j);
        return 127 - (j - 1);
    };
    // block-scaled form: this lane's exponents of stage s1 (rows past m read
    // row m - 1, blocks past n the last block: their data is zero)
    auto sfetch = [&](int64_t s1, unsigned (&sr)[8]) {
        const int64_t d = d0 + s1 / spd;
        const int64_t blk = min((s1 % spd) * (QK / 32) + q, (int64_t)nbk - 1);
        const uint8_t *base = bscale + d * m * nbk + blk;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t row = min((u < 4 ? rb0 + wr : cb0 + (wc - GT)) + 16 * (u & 3) + ii, m - 1);
            sr[u] = base[row * nbk];
        }
    };
    auto spack = [&](const unsigned (&sr)[8], unsigned &pa, unsigned &pb) {
        pa = sr[0] | (sr[1] << 8) | (sr[2] << 16) | (sr[3] << 24);
        pb = sr[4] | (sr[5] << 8) | (sr[6] << 16) | (sr[7] << 24);
    };
    // The MFMA's K blocks (measured): block g, whose scale lane group g
    // supplies, is bytes 0..15 of lane groups 2(g & 1) and 2(g & 1) + 1 for
    // g < 2 and their bytes 16..31 for g >= 2.  So lane group q takes the
    // stage's 16-byte chunks q (bytes 0..15) and q + 4 (bytes 16..31): block
    // g then holds columns 32g .. 32g + 31 of the stage, the MX block whose
    // exponent lane group g passes.
    auto mma_mx = [&](const uint8_t *cur, unsigned pa, unsigned pb) {
        v8i a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const uint8_t *ra = cur + (wr + x * 16 + ii) * QLD + 16 * q;
            const uint8_t *rc = cur + (wc + x * 16 + ii) * QLD + 16 * q;
            const v4u a0 = *reinterpret_cast<const v4u *>(ra), a1 = *reinterpret_cast<const v4u *>(ra + 64);
            const v4u b0 = *reinterpret_cast<const v4u *>(rc), b1 = *reinterpret_cast<const v4u *>(rc + 64);
            a[x] = v8i{(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
            b[x] = v8i{(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
        }
        const int sa = (int)pa, sb = (int)pb;
#define TSK_MXM(X, Y) acc[X][Y] = mfma16x16x128_e4m3_sel<X, Y>(a[X], b[Y], acc[X][Y], sa, sb);
        TSK_MXM(0, 0) TSK_MXM(0, 1) TSK_MXM(0, 2) TSK_MXM(0, 3)
        TSK_MXM(1, 0) TSK_MXM(1, 1) TSK_MXM(1, 2) TSK_MXM(1, 3)
        TSK_MXM(2, 0) TSK_MXM(2, 1) TSK_MXM(2, 2) TSK_MXM(2, 3)
        TSK_MXM(3, 0) TSK_MXM(3, 1) TSK_MXM(3, 2) TSK_MXM(3, 3)
#undef TSK_MXM
    };
    auto mma_stage = [&](const uint8_t *cur, int es) {
        v8i a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const uint8_t *ra = cur + (wr + x * 16 + ii) * QLD + 32 * q;
            const uint8_t *rc = cur + (wc + x * 16 + ii) * QLD + 32 * q;
            const v4u a0 = *reinterpret_cast<const v4u *>(ra), a1 = *reinterpret_cast<const v4u *>(ra + 16);
            const v4u b0 = *reinterpret_cast<const v4u *>(rc), b1 = *reinterpret_cast<const v4u *>(rc + 16);
            a[x] = v8i{(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
            b[x] = v8i{(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x128_e4m3(a[x], b[y], acc[x][y], es, es);
    };
    v4u p0[8], p1[8];
    if constexpr (MX) {
        // the pipeline below, with each stage's exponents beside its data
        unsigned s0[8], s1[8], pa0, pb0, pa1 = 0u, pb1 = 0u;
        fetch(0, p0);
        sfetch(0, s0);
        qstash(lds, p0);
        spack(s0, pa0, pb0);
        if (nst > 1) {
            fetch(1, p1);
            sfetch(1, s1);
        }
        __syncthreads();
        int64_t st = 0;
        for (; st + 1 < nst; st += 2) {
            if (st + 2 < nst) {
                fetch(st + 2, p0);
                sfetch(st + 2, s0);
            }
            mma_mx(lds, pa0, pb0);
            qstash(lds + QBUF, p1);
            spack(s1, pa1, pb1);
            __syncthreads();
            if (st + 3 < nst) {
                fetch(st + 3, p1);
                sfetch(st + 3, s1);
            }
            mma_mx(lds + QBUF, pa1, pb1);
            if (st + 2 < nst) {
                qstash(lds, p0);
                spack(s0, pa0, pb0);
            }
            __syncthreads();
        }
        if (st < nst) mma_mx(lds, pa0, pb0);
    } else {
        fetch(0, p0);
        qstash(lds, p0);
        if (nst > 1) fetch(1, p1);
        __syncthreads();
        int64_t st = 0;
        for (; st + 1 < nst; st += 2) {
            if (st + 2 < nst) fetch(st + 2, p0);
            mma_stage(lds, escale(st));
            qstash(lds + QBUF, p1);
            __syncthreads();
            if (st + 3 < nst) fetch(st + 3, p1);
            mma_stage(lds + QBUF, escale(st + 1));
            if (st + 2 < nst) qstash(lds, p0);
            __syncthreads();
        }
        if (st < nst) mma_stage(lds, escale(st));
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
// With at least as many slices as chunks every chunk holds one, so the
// per-chunk emptiness test (two 64-bit divisions) is skipped and the loads
// are issued eight chunks at a time; the sum keeps the chunk order.
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
    const float *p = part + (int64_t)t * (GT * GT) + e;
    const int64_t cs = (int64_t)T * (GT * GT);  // chunk stride
    double s = 0.0;
    if (count >= nchunks) {
        int c = 0;
        for (; c + 8 <= nchunks; c += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(c + u) * cs];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += (double)v[u];
        }
        for (; c < nchunks; ++c) s += (double)p[c * cs];
    } else {
        for (int c = 0; c < nchunks; ++c) {
            const int64_t d0 = (int64_t)c * count / nchunks, d1 = (int64_t)(c + 1) * count / nchunks;
            if (d0 >= d1) continue;
            s += (double)p[c * cs];
        }
    }
    G[i * m + j] = s;
    G[j * m + i] = s;
}

}  // namespace

// Chunks per XCD for tiles tiles, res workgroups resident per XCD: at least
// 2048 workgroups in all, and among up to four times that minimum the count
// whose workgroups fill whole rounds of the resident ones, so no round runs
// part-empty; at most count / 8 (every chunk holds a slice).
static int pick_per_xcd(int tiles, int res, int64_t count) {
    const int pmin = (2048 + 8 * tiles - 1) / (8 * tiles);
    int per_xcd = pmin;
    double best = 1.0;
    for (int pc = pmin; pc <= 4 * pmin; ++pc) {
        const int64_t wg = (int64_t)pc * tiles;
        const int64_t full = (wg + res - 1) / res * res;
        const double waste = (double)(full - wg) / (double)full;
        if (waste < best - 1e-12) {
            best = waste;
            per_xcd = pc;
        }
    }
    const int64_t cap = count / 8;
    if (per_xcd > cap) per_xcd = (int)(cap > 1 ? cap : 1);
    return per_xcd < 1 ? 1 : per_xcd;
}

// Chunks per XCD for the 256x256 tiles: chunks of about W_CHUNK_STAGES
// stages (128 bytes of every row each), between the 2048-workgroup minimum
// above and four times it (the bound the rule above keeps: a chunk writes
// about 2 m^2 bytes of partials, so large m keeps chunks long), and at most
// count / 8.  A workgroup's 256 rows drift away from those of
// the other tiles of its chunk as it runs, so a long chunk is fetched from
// beyond the XCD's L2 more often; short chunks add partial tiles to write and
// reduce.  On 1920 x 1080 bf16 slices (17 stages each) the Gram with its
// reduction took 5.42 / 5.20 / 5.18 / 5.30 ms at 8 / 10 / 12 / 16 chunks per
// XCD for 1000 slices (8 is what the rounds rule above picks), and 22.9 /
// 21.7 / 20.6 / 20.4 / 20.3 ms at 8 / 16 / 24 / 32 / 40 for 4000 slices.
constexpr int64_t W_CHUNK_STAGES = 200;
static int pick_per_xcd_wide(int tiles, int64_t count, int64_t stages_per_slice) {
    const int64_t pmin = (2048 + 8 * tiles - 1) / (8 * tiles);
    int64_t pc = (count * stages_per_slice + 4 * W_CHUNK_STAGES) / (8 * W_CHUNK_STAGES);
    if (pc < pmin) pc = pmin;
    if (pc > 4 * pmin) pc = 4 * pmin;
    const int64_t cap = count / 8;
    if (pc > cap) pc = cap;
    return pc < 1 ? 1 : (int)pc;
}

// Enqueue the Gram of a validated stack into device G (m x m FP64).
// compute TSK_F32: FP32 stack, FP32 products.  compute TSK_BF16: FP32 stack
// rounded to bf16 on load, or a bf16 stack as stored.  compute TSK_F8E4M3:
// an e4m3 stack with its per-slice scales.
tsk_status tsk_gram_enqueue(tsk_ctx c, const tsk_stack *s, int compute, double *G) {
    const int64_t m = s->m, count = s->count;
    const int nb = (int)((m + GT - 1) / GT);
    const int T = nb * (nb + 1) / 2;
    // bf16 and e4m3 stacks (slices under 4 GiB) take the 256x256 tiles
    const int eb = s->dtype == TSK_BF16 ? 2 : 1;
    // TSK_GRAM_TILE128 (diagnostic) forces the 128x128 kernels, which
    // otherwise serve only slices of 4 GiB and more, so tests can check them
    // on small stacks
    const bool force128 = getenv("TSK_GRAM_TILE128") != nullptr;
    const bool wide = ((compute == TSK_BF16 && s->dtype == TSK_BF16) || compute == TSK_F8E4M3) &&
                      m * s->ld * eb < ((int64_t)1 << 32) && !force128;
    const int nbw = (int)((m + WT - 1) / WT);
    const int TW = nbw * (nbw + 1) / 2;
    // 128x128 tiles: two per CU, 64 resident per XCD
    const int per_xcd = wide ? pick_per_xcd_wide(TW, count, (s->n * eb + WROW - 1) / WROW)
                             : pick_per_xcd(T, 64, count);
    const int nchunks = 8 * per_xcd;
    const size_t part_bytes = (size_t)nchunks * T * GT * GT * sizeof(float);
    TSK_TRY(tsk_grow(c, c->gram_part, part_bytes));
    float *part = (float *)c->gram_part.p;
    const unsigned grid = (unsigned)(8 * per_xcd * T);
    if (wide) {
        const void *fn = eb == 2 ? (const void *)gram_wide_kernel<uint16_t> : (const void *)gram_wide_kernel<uint8_t>;
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)W_LDS);
        if (e != hipSuccess) return tsk_hip(c, e, "Gram LDS attribute");
        const dim3 gw((unsigned)(8 * per_xcd * TW));
        if (eb == 2)
            TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                       hipLaunchKernelGGL(gram_wide_kernel<uint16_t>, gw, dim3(W_THREADS), W_LDS, c->stream,
                                          (const uint16_t *)s->A, nullptr, m, s->n, s->ld, s->stride, count, TW, T,
                                          nchunks, per_xcd, part));
        else
            TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                       hipLaunchKernelGGL(gram_wide_kernel<uint8_t>, gw, dim3(W_THREADS), W_LDS, c->stream,
                                          (const uint8_t *)s->A, s->scale, m, s->n, s->ld, s->stride, count, TW, T,
                                          nchunks, per_xcd, part));
    } else if (compute == TSK_F32) {
        TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                   hipLaunchKernelGGL(gram_f32_kernel, dim3(grid), dim3(256), 0, c->stream,
                                      (const float *)s->A, m, s->n, s->ld, s->stride, count, T, nchunks,
                                      per_xcd, part));
    } else if (compute == TSK_F8E4M3) {
        TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                   hipLaunchKernelGGL(gram_e4m3_kernel<false>, dim3(grid), dim3(256), 0, c->stream,
                                      (const uint8_t *)s->A, s->scale, (const uint8_t *)nullptr, 0, m, s->n, s->ld,
                                      s->stride, count, T, nchunks, per_xcd, part));
    } else if (compute == TSK_MXE4M3) {
        TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                   hipLaunchKernelGGL(gram_e4m3_kernel<true>, dim3(grid), dim3(256), 0, c->stream,
                                      (const uint8_t *)s->A, (const float *)nullptr,
                                      reinterpret_cast<const uint8_t *>(s->scale), (int)((s->n + 31) / 32), m,
                                      s->n, s->ld, s->stride, count, T, nchunks, per_xcd, part));
    } else if (s->dtype == TSK_F32) {
        TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                   hipLaunchKernelGGL(gram_bf16_kernel<float>, dim3(grid), dim3(256), 0, c->stream,
                                      (const float *)s->A, m, s->n, s->ld, s->stride, count, T, nchunks,
                                      per_xcd, part));
    } else {
        TSK_LAUNCH(c, TSK_KERNEL_GRAM,
                   hipLaunchKernelGGL(gram_bf16_kernel<uint16_t>, dim3(grid), dim3(256), 0, c->stream,
                                      (const uint16_t *)s->A, m, s->n, s->ld, s->stride, count, T, nchunks,
                                      per_xcd, part));
    }
    TSK_LAUNCH(c, TSK_KERNEL_GRAM_REDUCE,
               hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)(T * (GT * GT / 256))), dim3(256), 0,
                                  c->stream, (const float *)part, m, count, T, nchunks, G));
    return TSK_OK;
}
