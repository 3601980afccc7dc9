/*
 * tsko -- FP64 CPU oracle for the tensor-based sketching method
 * (Liu, Xiao, Ding, Yang: "Tensor-Based Sketching Method for the Low-Rank
 * Approximation of Data Streams").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * calls it and shares no source with it.
 *
 * All arithmetic is IEEE double.  Matrices are dense row-major.  Every routine
 * returns 0 on success and a negative value on bad arguments; none allocates
 * memory that outlives the call.  OpenMP is used only across independent
 * outputs (rows of the Gram, test matrices), so results do not depend on the
 * thread count.
 *
 * Parity status of each routine is stated at its declaration.
 */
#ifndef TSKO_H
#define TSKO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* flag bits reported per test matrix */
#define TSKO_FLAG_RANKDEF 1  /* sigma_k(SA) <= 1e-13 sigma_1(SA): row space of SA has dim < k */
#define TSKO_FLAG_TIE     2  /* sigma_r(AV) - sigma_{r+1}(AV) <= 1e-12 sigma_1(AV)            */
#define TSKO_FLAG_NONFIN  4  /* non-finite input entry                                         */

/* Mode-1 Gram of the training tensor (Section 3.1, eqs. 3.2-3.3):
 *   G = A_(1) A_(1)^T = sum_d A_d A_d^T,   A_(1) = [A_1 | ... | A_D'].
 * A: count slices of m x n, slice d at A + d*m*n.  G: m x m, full symmetric.
 * Summation in natural order (slice, then column).  Pinned by exact integer
 * inputs and trace(G) = ||A||_F^2. */
int tsko_gram_f32(const float *A, int64_t count, int64_t m, int64_t n, double *G);
int tsko_gram_f64(const double *A, int64_t count, int64_t m, int64_t n, double *G);

/* Full symmetric eigendecomposition G = V diag(w) V^T by Householder
 * tridiagonalisation and the implicit-shift symmetric QR iteration
 * (Golub & Van Loan, Matrix Computations, Sections 8.3.1-8.3.3).
 * w: m eigenvalues in descending order (ties: lower original index first).
 * V: m x m row-major, COLUMN j is the eigenvector of w[j], sign-canonical
 *    (largest-magnitude entry positive, ties to the lowest index).
 * Returns 1 if the QR iteration failed to converge.
 * Pinned by planted spectra, residuals, 2x2 closed form, numpy (tests). */
int tsko_eigh(const double *G, int64_t m, double *w, double *V);

/* Cyclic Jacobi eigensolver (Golub & Van Loan, Section 8.5), same output
 * convention as tsko_eigh.  Independent cross-check for small m. */
int tsko_eigh_jacobi(const double *G, int64_t m, double *w, double *V);

/* Thin SVD A = U diag(s) Vt by one-sided (Hestenes) Jacobi on the columns of
 * A (or of A^T when m < n), Golub & Van Loan Section 8.6.  p = min(m,n).
 * U: m x p, s: p descending, Vt: p x n.  Any output pointer may be NULL.
 * Singular vectors of zero singular values are returned as zero vectors. */
int tsko_svd(const double *A, int64_t m, int64_t n, double *U, double *s, double *Vt);

/* Householder thin QR (Golub & Van Loan Alg. 5.2.1), m >= n.
 * Q: m x n with orthonormal columns, R: n x n upper triangular. */
int tsko_qr(const double *A, int64_t m, int64_t n, double *Q, double *R);

/* Training (first half of Algorithm 2; Section 3.1): S = top-k eigenvectors of
 * the mode-1 Gram as rows (S S^T = I_k), in descending eigenvalue order,
 * sign-canonical.  lambda: k+1 leading eigenvalues (lambda_{k+1} is 0 when
 * k == m).  Also returns ||A||_F^2 in *fro2 (nullable). */
int tsko_train_f32(const float *A, int64_t count, int64_t m, int64_t n, int64_t k,
                   double *S, double *lambda, double *fro2);
int tsko_train_from_gram(const double *G, int64_t m, int64_t k, double *S, double *lambda);

/* Step 1 of Algorithm 1 alone: V (n x k, column-orthonormal) spans the row
 * space of S A (thin SVD of S A; vmode = 1: Householder QR of (S A)^T).
 * Directions with sigma_i(S A) <= 1e-13 sigma_1 are zero columns and set
 * flag RANKDEF in *flags (nullable).  This is the V that tsko_scw uses. */
int tsko_scw_basis(const double *A, int64_t m, int64_t n, const double *S, int64_t k, int vmode,
                   double *V, int32_t *flags);

/* SCW (Algorithm 1) on one matrix A (m x n) with sketch S (k x m), r < k:
 *   1. B = S A;  V = right singular vectors of B (thin SVD, n x k) -- or, with
 *      vmode = 1, the Q factor of a Householder QR of B^T (the QR variant the
 *      paper allows in Section 3.2).  Directions with sigma_i(B) below
 *      1e-13 sigma_1(B) are left out (zero columns), flag RANKDEF.
 *   2. C = A V (m x k);  C = U Sig Y^T (thin SVD);  [AV]_r = U_r Sig_r Y_r^T.
 *   3. A_hat = [AV]_r V^T = L R^T with L = U_r Sig_r (m x r), R = V Y_r (n x r).
 * relerr = ||A - A_hat||_F / ||A||_F, computed from the dense residual.
 * Any of L, R, sigma (r values), Ahat (m x n) may be NULL. */
int tsko_scw(const double *A, int64_t m, int64_t n, const double *S, int64_t k, int64_t r,
             int vmode, double *L, double *R, double *sigma, double *Ahat,
             double *relerr, int32_t *flags);

/* SCW over a stack of float slices (OpenMP across slices).  Output strides:
 * L: m*r per slice, R: n*r, sigma: r.  Any output may be NULL. */
int tsko_apply_f32(const float *A, int64_t count, int64_t m, int64_t n, const double *S,
                   int64_t k, int64_t r, double *L, double *R, double *sigma,
                   double *relerr, int32_t *flags);

/* Explicit ||A - L R^T||_F / ||A||_F for a stack of float slices; L, R in
 * double with strides m*r and n*r. */
int tsko_error_f32(const float *A, int64_t count, int64_t m, int64_t n, const double *L,
                   const double *R, int64_t r, double *relerr);

/* Optimal rank-r error (Eckart-Young, Section 1): ||A - [A]_r||_F for each
 * slice, by the one-sided Jacobi SVD of the slice.  Also ||A||_F in fro
 * (nullable).  OpenMP across slices. */
int tsko_opt_f32(const float *A, int64_t count, int64_t m, int64_t n, int64_t r,
                 double *tail, double *fro);

/* Storage formats of the reduced-precision forms.  The paper fixes no number
 * format; the reading used is round to nearest with ties to the even
 * significand, into
 *   bf16 : 8 significant bits, binary32 exponent range (smallest normal
 *          2^-126, subnormals below it), overflow to +-infinity;
 *   e4m3 : 4 significant bits, smallest normal 2^-6 (subnormal quantum 2^-9),
 *          largest finite 448, saturating to +-448, no infinity.
 * y[i] is the rounded value of x[i] (for e4m3: of x[i] * scale) as a float.
 * NaN stays NaN.  Pinned by exhaustive nearest-value search over every code
 * of the format (tests). */
int tsko_round_bf16(const float *x, int64_t n, float *y);
int tsko_round_e4m3(const float *x, int64_t n, float scale, float *y);

/* Per-matrix power-of-two scale of the e4m3 form: s = 2^j with
 * j = floor(log2(448 / amax)), amax = max |x[i]| over the n values, clamped
 * to -126 <= j <= 127; amax == 0 gives s = 1.  So amax * s <= 448 and,
 * unless clamped, 2 * amax * s > 448. */
int tsko_e4m3_scale(const float *x, int64_t n, float *scale);

/* e4m3 with block scales (the MX layout: one power-of-two scale per block of
 * 32 consecutive elements of a row; the last block of a row may be
 * shorter).  x: rows x n.  Each block is scaled by its own tsko_e4m3_scale
 * and rounded by tsko_round_e4m3.  y (rows x n): the decoded values,
 * rounded value / scale.  e (rows x ceil(n / 32) bytes): the E8M0 exponent
 * of each block, 127 - log2(scale), so that a stored code times
 * 2^(e - 127) is the decoded value.  Pinned by exhaustive nearest-value
 * search per element, block independence and power-of-two equivariance,
 * the scale's defining inequality per block, and block boundaries (tests). */
int tsko_round_e4m3_mx(const float *x, int64_t rows, int64_t n, float *y, uint8_t *e);

/* Data-free sketches of the SCW baseline (Sections 1 and 2), k x m, from a
 * counter-based generator: tsko_splitmix64(seed, c) is the c-th output (from
 * 0) of SplitMix64 seeded with `seed`.  kind 0: Gaussian entries N(0, 1/k)
 * (Box-Muller on the outputs of counters 2c and 2c + 1, c = i m + j);
 * kind 1: Rademacher entries +-1/sqrt(k) (sign of the top bit of output c);
 * kind 2: sparse random sign (CountSketch) -- column j has its one nonzero,
 * +-1 (bit 0 of output j), in row (output j >> 32) mod k. */
uint64_t tsko_splitmix64(uint64_t seed, uint64_t c);
int tsko_random_sketch(int kind, int64_t k, int64_t m, uint64_t seed, double *S);

/* The two-sided method (Section 3.2, problem 3.6; Algorithms 3-5).
 * tsko_gram2_f32: mode-2 Gram sum_d A_d^T A_d (n x n).
 * tsko_train2_f32: Tucker2 by HOOI from the HOSVD guess (see tsko.c):
 *   S (k x m) and W (l x n) with orthonormal rows; core2 (nullable,
 *   max_sweeps + 1 values): ||G||^2 after each sweep (index 0: the guess);
 *   *sweeps (nullable): sweeps done (stop when ||G||^2 changes by <= tol).
 * tsko_scw2: two-sided SCW (Algorithm 4) on one matrix, factors as tsko_scw
 *   (L = P U_r Sig_r, R = Q Y_r), explicit relerr, flags.
 * tsko_apply2_f32: tsko_scw2 over a stack of float slices (OpenMP). */
int tsko_gram2_f32(const float *A, int64_t count, int64_t m, int64_t n, double *G);
int tsko_train2_f32(const float *A, int64_t count, int64_t m, int64_t n, int64_t k, int64_t l,
                    int64_t max_sweeps, double tol, double *S, double *W, double *core2, int64_t *sweeps);
int tsko_scw2(const double *A, int64_t m, int64_t n, const double *S, int64_t k, const double *W, int64_t l,
              int64_t r, double *L, double *R, double *sigma, double *relerr, int32_t *flags);
int tsko_apply2_f32(const float *A, int64_t count, int64_t m, int64_t n, const double *S, int64_t k,
                    const double *W, int64_t l, int64_t r, double *L, double *R, double *sigma, double *relerr,
                    int32_t *flags);

/* Number of OpenMP threads the library will use. */
int tsko_threads(void);

#ifdef __cplusplus
}
#endif
#endif
