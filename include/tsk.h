/*
 * tsk.h -- C ABI of the MI355X (gfx950) implementation of the tensor-based
 * sketching method for low-rank approximation of matrix data streams
 * (Liu, Xiao, Ding, Yang).
 *
 * Problem (Section 1, eq. 1.1): for every matrix A_d (m x n) of a stream,
 *     min_B ||A_d - B||_F   subject to   rank(B) <= r.
 * Method (Algorithm 2): stack the training matrices into an m x n x N tensor,
 * take its mode-1 Tucker1 factor as the sketch S (k x m, S S^T = I_k;
 * Section 3.1, eqs. 3.1-3.3 and the sentence after 3.3), then run SCW
 * (Algorithm 1) on every test matrix with that S.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every matrix is dense ROW-MAJOR.  Pointers documented "device" must be
 *   device memory of the context's GPU (for example torch.Tensor.data_ptr()
 *   of a CUDA tensor); pointers documented "host" are ordinary host memory.
 * - The caller allocates and owns every input and output.  The library owns
 *   only the context and its workspace (grown on demand, freed by
 *   tsk_destroy); it keeps no caller pointer after a call returns.
 * - All GPU work is enqueued on the context's stream; a call returns after
 *   enqueueing unless it documents a host output, in which case it
 *   synchronises that stream before returning.  Device outputs are valid
 *   once the stream has been synchronised.
 * - Arguments are validated before anything is launched; a violation returns
 *   TSK_E_ARG or TSK_E_SHAPE, launches nothing and sets tsk_last_error().
 * - One context per host thread; calls on one context must not overlap.
 */
/*
 * Diagnostics (environment; TSK_PIPELINE_STREAMS is described at
 * tsk_plan_launch, the others are read at each call): TSK_GRAM_TILE128 makes tsk_gram use
 * its 128 x 128-tile kernels for bf16 and e4m3 stacks (otherwise used only
 * for slices of 4 GiB and more); TSK_FAULT_NOMEM makes every workspace
 * allocation fail with TSK_E_NOMEM.  Both exist so tests can reach those
 * paths.
 */
#ifndef TSK_H
#define TSK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TSK_OK = 0,
    TSK_E_ARG = 1,     /* null pointer, bad enum, bad rank/sketch size      */
    TSK_E_SHAPE = 2,   /* inconsistent shapes, strides or alignment          */
    TSK_E_NOMEM = 3,   /* workspace allocation failed                         */
    TSK_E_DEVICE = 4,  /* HIP runtime error (message in tsk_last_error)       */
    TSK_E_NOCONV = 5   /* eigensolver hit its iteration cap; S still written  */
} tsk_status;

typedef enum {
    TSK_F64 = 0,
    TSK_F32 = 1,
    TSK_BF16 = 2,
    TSK_F8E4M3 = 3,
    TSK_MXE4M3 = 4
} tsk_dtype;

/* Per-matrix condition bits written to `flags` by tsk_apply. */
#define TSK_FLAG_RANKDEF 1 /* S A_d numerically rank deficient: V has fewer than k
                              directions (the missing ones are zero columns)   */
#define TSK_FLAG_TIE     2 /* sigma_r(A_d V) == sigma_{r+1}(A_d V) to rounding:
                              the rank-r factor is not unique (the error is)   */
#define TSK_FLAG_NONFIN  4 /* non-finite value in A_d; outputs are NaN          */

typedef struct tsk_ctx_s *tsk_ctx;

/* A stack of `count` row-major m x n slices (the training tensor of
 * Section 3.1, or a batch of test matrices).  Element (i, j) of slice d is at
 * A[d * stride + i * ld + j].  Requirements: m, n, count >= 1, ld >= n,
 * stride >= m * ld, A 16-byte aligned, ld and stride multiples of 16 bytes
 * (4 FP32, 8 bf16 or 16 e4m3 elements).  A row stride that is a multiple of
 * 128 bytes (a cache line) lets the streaming kernels read whole lines: at
 * 1920 x 1080 bf16 they run 5-8% faster than at a 2160-byte stride.
 * dtype: TSK_F32, TSK_BF16 (bfloat16 bits), TSK_F8E4M3 (OCP e4m3 bytes,
 * largest finite 448) or TSK_MXE4M3 (e4m3 bytes with one power-of-two scale
 * per block of 32 consecutive elements of a row, the MX layout; the last
 * block of a row is the ragged rest).  scale: NULL for TSK_F32 and TSK_BF16.
 * TSK_F8E4M3: a device array of `count` floats, slice d holds A_d * scale[d]
 * (tsk_stage writes such stacks).  TSK_MXE4M3: the pointer holds bytes, not
 * floats -- count * m * ceil(n / 32) E8M0 exponents, byte
 * (d * m + i) * ceil(n / 32) + b for block b of row i of slice d; element
 * (i, j) holds A_d(i, j) * 2^(127 - e) for its block's exponent e
 * (tsk_stage_mx writes such stacks).  Block-scaled stacks are accepted by
 * tsk_gram, tsk_train and tsk_opt_tail only. */
typedef struct {
    const void *A;     /* device */
    int32_t dtype;     /* tsk_dtype of the stored elements */
    const float *scale;/* device, count values, TSK_F8E4M3 only; else NULL */
    int64_t m, n, count;
    int64_t ld, stride;/* in elements */
} tsk_stack;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (NULL: the device's null stream).  The context does not own the
 * stream. */
tsk_status tsk_create(tsk_ctx *out, int device, void *hip_stream);
void tsk_destroy(tsk_ctx ctx);
/* Replace the stream used by later calls (same device).  The context's
 * workspace is shared by all its calls, so work enqueued after the switch
 * waits (hipStreamWaitEvent) for everything the context enqueued on the
 * previous stream. */
tsk_status tsk_set_stream(tsk_ctx ctx, void *hip_stream);
/* Message of the last failure on this context ("" when none). */
const char *tsk_last_error(tsk_ctx ctx);

/* Staging into a reduced-precision storage format (the precision forms; the
 * paper fixes no number format).  src: an FP32 stack.  dtype: TSK_BF16
 * (round to nearest even) or TSK_F8E4M3 (slice d is multiplied by the
 * power of two s_d = 2^floor(log2(448 / max|A_d|)), clamped to
 * [2^-126, 2^127], 1 for an all-zero slice, then rounded to nearest even;
 * no value saturates).  dst: device, element (i, j) of slice d at
 * dst[d * stride + i * ld + j] in the new format; ld >= n, stride >= m * ld,
 * both multiples of 16 bytes, dst 16-byte aligned; columns n..ld-1 are not
 * written.  scale: device, count floats (written: s_d), required for
 * TSK_F8E4M3, must be NULL for TSK_BF16.  norm2: device, count doubles,
 * nullable: ||A_d||_F^2 of the FP32 source in FP64.  Enqueue only. */
tsk_status tsk_stage(tsk_ctx ctx, const tsk_stack *src, int32_t dtype, void *dst, int64_t ld,
                     int64_t stride, float *scale, double *norm2);

/* Staging into block-scaled e4m3 (TSK_MXE4M3; the reading of the e4m3 form
 * with one scale per block of 32 consecutive elements of a row, the MX
 * layout).  Block b of row i of slice d is multiplied by its own power of
 * two 2^j, j = floor(log2(448 / max|block|)) clamped to [-126, 127] (0 for an
 * all-zero block), and rounded to nearest even e4m3; no value saturates.
 * src: an FP32 stack.  dst: device, codes at dst[d * stride + i * ld + c]
 * (ld >= n, stride >= m * ld, both multiples of 16, dst 16-byte aligned;
 * columns n..ld-1 not written).  bscale: device, count * m * ceil(n / 32)
 * bytes, written 127 - j per block in (slice, row, block) order.  Enqueue
 * only. */
tsk_status tsk_stage_mx(tsk_ctx ctx, const tsk_stack *src, void *dst, int64_t ld, int64_t stride,
                        uint8_t *bscale);

/* Mode-1 Gram (Section 3.1, eqs. 3.2-3.3; tensor basics in Section 2):
 *     G = A_(1) A_(1)^T = sum_{d<count} A_d A_d^T,   A_(1) = [A_1|...|A_N].
 * G: device, m x m FP64, full symmetric matrix.  Products accumulate in FP32
 * inside a chunk of slices and in FP64 across chunks.  compute:
 *   TSK_F32    : FP32 stack, FP32 products;
 *   TSK_BF16   : bf16 products, from a TSK_BF16 stack as stored or from an
 *                FP32 stack rounded to bf16 (nearest even) as it is loaded;
 *   TSK_F8E4M3 : e4m3 products of a TSK_F8E4M3 stack, each slice's products
 *                multiplied exactly by 1/scale[d]^2 (power of two);
 *   TSK_MXE4M3 : e4m3 products of a TSK_MXE4M3 stack, every 32-element
 *                block of each operand multiplied exactly by its own
 *                2^(e - 127) through the MFMA's per-lane operand scales
 *                (128 x 128 tiles).
 * Enqueue only. */
tsk_status tsk_gram(tsk_ctx ctx, const tsk_stack *train, int32_t compute, double *G);

/* Leading-k eigenvectors of a symmetric positive semi-definite m x m matrix
 * (the Tucker1 factor, S* = (U^(1))_k^T, Section 3.1).  G: device FP64 m x m
 * (full symmetric).  S: device FP32, k x m row-major, rows orthonormal, in
 * descending eigenvalue order, sign-canonical (largest-magnitude entry of
 * each row positive).  lambda: host, k+1 doubles: the Ritz values
 * theta_1..theta_{k+1} of the search block.  iters: host, nullable: number of
 * block products with G used.  Stops when every one of the first k Ritz pairs
 * has ||G u - theta u|| <= tol * theta_1 (tol of tsk_set_eig_params).
 * Requires 1 <= k < m, k <= 52.  Synchronises the stream.
 * Returns TSK_E_NOCONV when the residual test was not met within the cap
 * (S and lambda are still written from the last Rayleigh-Ritz step). */
tsk_status tsk_eig_topk(tsk_ctx ctx, const double *G, int64_t m, int32_t k,
                        float *S, double *lambda, int32_t *iters);

/* Training (the first half of Algorithm 2): tsk_gram (same stack/compute rules)
 * followed by tsk_eig_topk on the context's workspace.  S: device FP32
 * k x m.  lambda: host k+1.  iters: host, nullable.  Requires 1 <= k < m,
 * k <= 52.  Synchronises the stream. */
tsk_status tsk_train(tsk_ctx ctx, const tsk_stack *train, int32_t k, int32_t compute,
                     float *S, double *lambda, int32_t *iters);

/* Data-free sketches for the SCW baseline: the randomly drawn sketching
 * matrices the paper contrasts with its trained one (Section 1: entries
 * from a distribution such as the Gaussian or the Rademacher one; Section 2:
 * the sparse random sign matrix that initialises IVY's learned sketch).
 * S: device FP32, k x m row-major, written; usable as the sketch of
 * tsk_apply (whose basis step needs only that S A_d have full row rank).
 * Counter-based: entry values are a pure function of (seed, position); the
 * value of counter c is the c-th output (from 0) of SplitMix64 seeded with
 * `seed`.  kind:
 *   TSK_SKETCH_GAUSSIAN : N(0, 1/k) entries, Box-Muller on the outputs of
 *                         counters 2c and 2c + 1 (c = i m + j), FP64,
 *                         rounded to FP32;
 *   TSK_SKETCH_SIGN     : +-1/sqrt(k) by the top bit of output c;
 *   TSK_SKETCH_SPARSE   : one +-1 per column j (bit 0 of output j) in row
 *                         (output j >> 32) mod k, zeros elsewhere.
 * Requires 1 <= k <= m.  Enqueue only. */
typedef enum { TSK_SKETCH_GAUSSIAN = 0, TSK_SKETCH_SIGN = 1, TSK_SKETCH_SPARSE = 2 } tsk_sketch_kind;
tsk_status tsk_random_sketch(tsk_ctx ctx, int32_t kind, int32_t k, int64_t m, uint64_t seed, float *S);

/* SCW, Algorithm 1, on every slice of `test` with the sketch S (k x m,
 * device FP32; the trained sketch has orthonormal rows, but any S for which
 * S A_d has full row rank serves, e.g. those of tsk_random_sketch):
 *   1. B_d = S A_d (k x n);  V_d = orthonormal basis of the row space of B_d
 *      (n x k), by CholeskyQR2 -- the QR replacement for Algorithm 1's SVD
 *      that Section 3.2 allows;
 *   2. C_d = A_d V_d (m x k) and its rank-r truncation via the eigen-
 *      decomposition C_d^T C_d = Y diag(sigma^2) Y^T;
 *   3. A_hat_d = [A_d V_d]_r V_d^T = L_d R_d^T with
 *      L_d = C_d Y_r = U_r Sigma_r (m x r), R_d = V_d Y_r (n x r).
 * Outputs (device): L (count*m*r FP32), R (count*n*r FP32),
 * sigma (count*r FP32, descending), relerr (count FP64, nullable):
 *      relerr_d = ||A_d - L_d R_d^T||_F / ||A_d||_F,
 * first from the Pythagorean identity of the proof of Theorem 1,
 *      sqrt(max(0, ||A_d||^2 - sum_{i<=r} sigma_i^2)) / ||A_d||,
 * whose subtraction cancels as the error shrinks (its rounding is about
 * 2u / relerr^2 relative, u = 2^-24); where relerr^2 < 0.25 (FP32 form) or
 * < 1e-2 (bf16, e4m3 forms) it is recomputed from the explicit residual of
 * the stored values (FP32 products, FP64 sum), an extra pass over those
 * matrices only.  flags (count int32, nullable, TSK_FLAG_*).  Requires 1 <= r < k <= min(m, n), k <= 64.
 * compute must match the stack's dtype:
 *   TSK_F32    : FP32 products S A_d and A_d V_d;
 *   TSK_BF16   : bf16 stack; products with bf16 A_d and S, V_d each split
 *                into a bf16 pair (hi + lo), so the only rounding beyond
 *                FP32 is that of the stored A_d; ||A_d|| is that of the
 *                stored values;
 *   TSK_F8E4M3 : e4m3 stack; the stored values divided by scale[d] are
 *                widened exactly to bf16 and multiplied as in TSK_BF16 (the
 *                apply is bound by memory traffic, which the 1-byte storage
 *                halves; rounding S or V_d to e4m3 would add error and save
 *                nothing).
 * The small factorizations (CholeskyQR2, C^T C eigenproblem) are FP64 in
 * every form.  Enqueue only. */
tsk_status tsk_apply(tsk_ctx ctx, const float *S, int32_t k, const tsk_stack *test, int32_t r,
                     int32_t compute, float *L, float *R, float *sigma, double *relerr,
                     int32_t *flags);

/* tsk_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, validation and results (bit for bit) as tsk_apply, but the
 * workspace is a fixed 64 MiB device array inside the library (one per GPU,
 * held until the process ends) instead of the context's grown workspace;
 * nothing is allocated or freed.  The stack is processed in groups of as
 * many matrices as fit (about 60 of 1920 x 1080 at k = 40), one after
 * another on the context's stream.  A single matrix whose workspace exceeds
 * the array returns TSK_E_SHAPE (launches nothing).  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other contexts or threads) race and must be serialised by the caller.
 * Enqueue only. */
tsk_status tsk_apply_noalloc(tsk_ctx ctx, const float *S, int32_t k, const tsk_stack *test, int32_t r,
                             int32_t compute, float *L, float *R, float *sigma, double *relerr,
                             int32_t *flags);

/* One problem of a batch: the test matrices of one stream (any shape), its
 * sketch and outputs, exactly as the arguments of tsk_apply. */
typedef struct {
    tsk_stack A;          /* test matrices (device) */
    const float *S;       /* k x A.m sketch, device FP32, rows orthonormal */
    int32_t k, r;         /* 1 <= r < k <= min(A.m, A.n), k <= 64 */
    float *L, *R, *sigma; /* device outputs, layouts as tsk_apply */
    double *relerr;       /* device, nullable */
    int32_t *flags;       /* device, nullable */
} tsk_problem;

/* The batching form of SCW (Algorithm 1): tsk_apply on every problem of
 * `probs` -- matrices of different shapes and sketch sizes, e.g. from
 * several streams -- in a fixed number of launches for the whole batch
 * (one sketch-preparation launch, then one launch of each later phase --
 * sketch, basis, project, eig, outputs -- over all problems and sketch
 * sizes, and the error refinement per class ceil(r/16)), work items of all
 * problems sharing each launch.  Results are identical to tsk_apply on each
 * problem.  compute: as tsk_apply, and every stack's dtype must equal it.
 * nprobs >= 1.  The problems' outputs must not overlap.  Enqueue only (the
 * batch tables are copied from context-owned pinned memory; a later call
 * waits for that copy before reusing it). */
tsk_status tsk_apply_multi(tsk_ctx ctx, const tsk_problem *probs, int32_t nprobs, int32_t compute);

/* Captured batches of the batching form, for serving loops that apply the
 * same batch layout again and again.  tsk_apply_multi_plan builds the
 * batch's tables and workspace in plan-owned device memory once, runs the
 * batch once (the problems' outputs are written), and captures its launch
 * sequence into a HIP graph; the problems' pointers are fixed in the plan,
 * so later launches read the then-current contents of the same inputs and
 * overwrite the same outputs.  Arguments as tsk_apply_multi.  Synchronises
 * the context's stream.  The plan belongs to the context's device and must
 * be destroyed with tsk_plan_destroy.
 * tsk_plan_launch replays `nplans` plans (graph launches) after all work
 * enqueued on the context's stream; plans go in turn to three
 * context-owned streams (TSK_PIPELINE_STREAMS, 2..4, read when the context
 * first needs them, overrides the number) so consecutive batches overlap
 * (each plan has its
 * own workspace; plans whose outputs overlap must not be launched
 * together), and the context's stream waits for all of them.  Enqueue only. */
typedef struct tsk_plan_s *tsk_plan;
tsk_status tsk_apply_multi_plan(tsk_ctx ctx, const tsk_problem *probs, int32_t nprobs, int32_t compute,
                                tsk_plan *plan);
tsk_status tsk_plan_launch(tsk_ctx ctx, const tsk_plan *plans, int32_t nplans);
void tsk_plan_destroy(tsk_plan plan);

/* The two-sided method (Section 3.2, problem 3.6).
 *
 * tsk_train2 (Algorithm 3, line 2): the Tucker2 decomposition of the
 * training tensor along modes 1 and 2 by HOOI (Appendix, Algorithm 5) from
 * the HOSVD guess (S = top-k eigenvectors of sum_d A_d A_d^T, W = top-l of
 * sum_d A_d^T A_d); a sweep updates S to the top-k eigenvectors of
 * sum_d (A_d W^T)(A_d W^T)^T, then W to the top-l of sum_d (S A_d)^T (S A_d),
 * and stops when ||G||^2 = sum_d ||S A_d W^T||_F^2 (the top-l eigenvalue sum
 * of the second Gram) changes by at most max(tol, 1e-8) ||G||^2 (tol <= 0:
 * 1e-10; the FP32 Grams and the eigensolver's tolerance fix ||G||^2 to about
 * 1e-8) or after max_sweeps sweeps.  train: FP32 stack.  S: device FP32 k x m,
 * W: device FP32 l x n (rows orthonormal, descending, sign-canonical).
 * core2: host, nullable, max_sweeps doubles: ||G||^2 after each sweep.
 * sweeps: host, nullable.  Requires 1 <= k < m, 1 <= l < n, k, l <= 52.
 * Every Gram as tsk_gram (FP32), every eigensolve as tsk_eig_topk
 * (residual 1e-7 theta_1).  Synchronises the stream.
 *
 * tsk_apply2 (Algorithm 4, two-sided SCW) on every slice of `test` with S
 * (k x m) and W (l x n), device FP32:
 *   Q = orthonormal basis of the row space of S A_d (CholeskyQR2 of S A_d,
 *       as tsk_apply; Algorithm 4 takes a QR of A_d^T S^T, which spans the
 *       same space);
 *   P = orthonormal basis of the columns of A_d W^T (Cholesky QR, a second
 *       pass when ill-conditioned);
 *   M = P^T A_d Q (l x k), M^T M = Y diag(sigma^2) Y^T (FP64 Jacobi);
 *   A_hat_d = P [M]_r Q^T = L_d R_d^T, L_d = P M Y_r (m x r), R_d = Q Y_r.
 * Outputs, forms and relerr (with its exact recomputation where the
 * Pythagorean form cancels) as tsk_apply.  Requires 1 <= r < min(k, l),
 * k, l <= min(m, n), k, l <= 64.  Enqueue only. */
tsk_status tsk_train2(tsk_ctx ctx, const tsk_stack *train, int32_t k, int32_t l, int32_t max_sweeps, double tol,
                      float *S, float *W, double *core2, int32_t *sweeps);
tsk_status tsk_apply2(tsk_ctx ctx, const float *S, int32_t k, const float *W, int32_t l, const tsk_stack *test,
                      int32_t r, int32_t compute, float *L, float *R, float *sigma, double *relerr,
                      int32_t *flags);

/* Explicit relative error ||A_d - L_d R_d^T||_F / ||A_d||_F for every slice
 * (the quantity whose rank-r minimum is problem 1.1).  A: an FP32 stack.
 * L, R: device FP32 with the layout tsk_apply writes.  relerr: device FP64,
 * count values.  r >= 1.  Enqueue only. */
tsk_status tsk_error(tsk_ctx ctx, const tsk_stack *A, const float *L, const float *R,
                     int32_t r, double *relerr);

/* The optimum that metric (4.1) of Section 4 compares each SCW output with:
 * for every slice, tail_d = ||A_d - [A_d]_r||_F (the best rank-r error,
 * Eckart-Young, Section 1) and fro_d = ||A_d||_F, from the Gram
 * G_d = A_d A_d^T of the stored values (FP32 accumulation of exact products)
 * and its top-r eigenvalues (the filtered subspace iteration of
 * tsk_eig_topk, residual tolerance 1e-7 theta_1):
 *     tail_d^2 = trace(G_d) - sum_{i <= r} lambda_i(G_d).
 * Metric (4.1) of an output with relative error e_d is then
 * (e_d fro_d - tail_d) / tail_d.  A: any stack (FP32, bf16, e4m3 with its
 * scales: the stored values).  tail, fro: host, count doubles each.
 * Requires 1 <= r < m, r <= 52, m <= 65536.  Processes one slice after
 * another and synchronises the stream (an evaluation step, not the hot
 * path). */
tsk_status tsk_opt_tail(tsk_ctx ctx, const tsk_stack *A, int32_t r, double *tail, double *fro);

/* Eigensolver controls (defaults in brackets): block = search-block width p
 * [k + max(12, k/2), at most 64 and at most m]; max_iter = cap on filtered
 * subspace steps [300]; tol = residual tolerance relative to theta_1 [by
 * the precision of the Gram's products: 1e-7 for FP32 (the rounding level
 * of FP32 accumulation, so the Ritz vectors are exact eigenvectors of a
 * matrix within that distance of G), 1e-5 for bf16 (rounding the data to
 * bf16 already moves G by about 1e-4 theta_1), 1e-4 for e4m3 (16 times
 * coarser rounding than bf16); tsk_eig_topk uses 1e-7];
 * check = filtered steps to the first convergence test [6]; later tests are
 * placed where the observed residual decay predicts convergence (at most
 * 4 * check steps apart).  A value <= 0 restores the default. */
tsk_status tsk_set_eig_params(tsk_ctx ctx, int32_t block, int32_t max_iter, double tol,
                              int32_t check);

/* Tuning of the apply for one shape class (m, n, ceil(k / 16), dtype of the
 * test stack), as chosen by an autotuner (paper_2209_14637_amd/autotune.py
 * times the candidates and keeps a JSON cache): groups = the number of
 * pipeline groups of tsk_apply (1..64; the groups go in turn to the
 * context-owned streams of tsk_plan_launch), pj_cols = columns per projection step of the bf16 form
 * (64 or 128; also used by the batched forms).  0 restores the default
 * (groups: 1, the whole stack; pj_cols: 64).  Results do not
 * depend on either (bit for bit).  Host only. */
tsk_status tsk_set_tuning(tsk_ctx ctx, int64_t m, int64_t n, int32_t k, int32_t dtype, int32_t groups,
                          int32_t pj_cols);

/* Kernel timing.  mask bit i (i = TSK_KERNEL_*) brackets every launch of
 * kernel class i with HIP events on the context's stream (0: off, -1: all
 * classes).  tsk_timing_read synchronises and returns, for each kernel class,
 * the number of timed launches and their summed milliseconds since the last
 * reset. */
enum {
    TSK_KERNEL_GRAM = 0,     /* Gram product kernel          */
    TSK_KERNEL_GRAM_REDUCE,  /* FP64 reduction of partials    */
    TSK_KERNEL_EIG_ITER,     /* subspace iteration step       */
    TSK_KERNEL_EIG_RR,       /* Rayleigh-Ritz / residual      */
    TSK_KERNEL_SKETCH,       /* B_d = S A_d                   */
    TSK_KERNEL_QR,           /* CholeskyQR2 of B_d^T          */
    TSK_KERNEL_PROJECT,      /* C_d = A_d V_d                 */
    TSK_KERNEL_FINISH,       /* small eigenproblem + outputs  */
    TSK_KERNEL_ERROR,        /* explicit residual             */
    TSK_KERNEL_STAGE,        /* format conversion (tsk_stage) */
    TSK_KERNEL_COUNT
};
tsk_status tsk_timing_enable(tsk_ctx ctx, int32_t mask);
tsk_status tsk_timing_read(tsk_ctx ctx, int32_t reset, int64_t *launches /* TSK_KERNEL_COUNT */,
                           double *ms /* TSK_KERNEL_COUNT */);

#ifdef __cplusplus
}
#endif
#endif
