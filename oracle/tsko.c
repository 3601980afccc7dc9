/*
 * tsko.c -- FP64 CPU oracle for the tensor-based sketching method.
 *
 * TEST INFRASTRUCTURE ONLY (see tsko.h).  Plain, slow, obviously correct:
 * every routine follows a textbook definition or the paper's algorithm in
 * its own order, in double precision, with natural summation order.
 * OpenMP only splits independent outputs across threads.
 */
#include "tsko.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EPS DBL_EPSILON

/* Planted-mistake hooks for the pin suite's mutation test: the default build
 * has TSKO_MUTANT == 0 and every MUT(n) is false. */
#ifndef TSKO_MUTANT
#define TSKO_MUTANT 0
#endif
#define MUT(n) (TSKO_MUTANT == (n))

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

int tsko_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Mode-1 Gram, Section 3.1: G = sum_d A_d A_d^T (block form of A_(1)).      */
/* Slice-outer so that one slice is shared in cache by all threads; each    */
/* G[i][j] (j <= i) is owned by one thread and summed in slice order.       */
/* ------------------------------------------------------------------------ */
#define GRAM_BODY(T)                                                           \
    if (!A || !G || count < 0 || m <= 0 || n <= 0) return -1;                  \
    for (int64_t i = 0; i < m * m; i++) G[i] = 0.0;                            \
    for (int64_t d = 0; d < count; d++) {                                      \
        const T *Ad = A + d * m * n;                                           \
        _Pragma("omp parallel for schedule(dynamic, 8)")                       \
        for (int64_t i = 0; i < m; i++) {                                      \
            const T *ai = Ad + i * n;                                          \
            for (int64_t j = 0; j <= i; j++) {                                 \
                const T *aj = Ad + j * n;                                      \
                double s = 0.0;                                                \
                for (int64_t c = 0; c < n - MUT(1); c++) s += (double)ai[c] * (double)aj[c]; \
                G[i * m + j] += s;                                             \
            }                                                                  \
        }                                                                      \
    }                                                                          \
    for (int64_t i = 0; i < m && !MUT(2); i++)                                 \
        for (int64_t j = 0; j < i; j++) G[j * m + i] = G[i * m + j];           \
    return 0;

int tsko_gram_f32(const float *A, int64_t count, int64_t m, int64_t n, double *G) { GRAM_BODY(float) }
int tsko_gram_f64(const double *A, int64_t count, int64_t m, int64_t n, double *G) { GRAM_BODY(double) }

/* ------------------------------------------------------------------------ */
/* Householder vector: P = I - beta v v^T with v[0] = 1 maps x to alpha e1,  */
/* alpha = -sign(x0) ||x|| (no cancellation in v0 = x0 - alpha).             */
/* x is overwritten by v.  Returns beta (0 when x[1:] is already zero).      */
/* ------------------------------------------------------------------------ */
static double house(double *x, int64_t len, double *alpha) {
    double tail = 0.0;
    for (int64_t i = 1; i < len; i++) tail += x[i] * x[i];
    if (tail == 0.0) {
        *alpha = x[0];
        x[0] = 1.0;
        return 0.0;
    }
    double nrm = sqrt(x[0] * x[0] + tail);
    double a = (x[0] >= 0.0) ? -nrm : nrm;
    double v0 = x[0] - a;
    for (int64_t i = 1; i < len; i++) x[i] /= v0;
    x[0] = 1.0;
    /* beta = 2 / (v^T v) with v scaled to v0 = 1 */
    double vtv = 1.0 + tail / (v0 * v0);
    *alpha = a;
    return (MUT(3) ? 1.0 : 2.0) / vtv;
}

static void sort_desc(double *w, int64_t m, int64_t *perm) {
    /* stable insertion sort of indices by descending w */
    for (int64_t i = 0; i < m; i++) perm[i] = i;
    for (int64_t i = 1; i < m; i++) {
        int64_t p = perm[i];
        int64_t j = i - 1;
        while (j >= 0 && (MUT(5) ? w[perm[j]] > w[p] : w[perm[j]] < w[p])) {
            perm[j + 1] = perm[j];
            j--;
        }
        perm[j + 1] = p;
    }
}

/* Columns of V (m x m row-major) = eigenvectors; make each column's
 * largest-magnitude entry positive (ties: lowest index). */
static void canon_columns(double *V, int64_t rows, int64_t cols) {
    for (int64_t j = 0; j < cols; j++) {
        int64_t best = 0;
        double bv = -1.0;
        for (int64_t i = 0; i < rows; i++) {
            double a = fabs(V[i * cols + j]);
            if (a > bv) { bv = a; best = i; }
        }
        if (V[best * cols + j] < 0.0)
            for (int64_t i = 0; i < rows; i++) V[i * cols + j] = -V[i * cols + j];
    }
}

/* ------------------------------------------------------------------------ */
/* Symmetric eigensolver: Householder tridiagonalisation, then implicit      */
/* symmetric QR steps with the Wilkinson shift (GVL 8.3).                    */
/* Zt holds the eigenvector basis TRANSPOSED (row j = current basis vector j)*/
/* so that a plane rotation updates two contiguous rows.                     */
/* ------------------------------------------------------------------------ */
int tsko_eigh(const double *G, int64_t m, double *w, double *V) {
    if (!G || !w || m <= 0) return -1;
    double *a = dalloc((size_t)(m * m));
    double *d = dalloc((size_t)m), *e = dalloc((size_t)m), *beta = dalloc((size_t)m);
    double *p = dalloc((size_t)m);
    double *Zt = V ? dalloc((size_t)(m * m)) : NULL;
    memcpy(a, G, sizeof(double) * (size_t)(m * m));
    /* symmetrise defensively from the lower triangle */
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < i; j++) a[j * m + i] = a[i * m + j];

    /* --- tridiagonalisation: T = Q^T G Q, Q = H_0 H_1 ... H_{m-3} --- */
    double *v = dalloc((size_t)m);
    for (int64_t k = 0; k + 2 < m; k++) {
        int64_t L = m - k - 1; /* length of column below the diagonal */
        for (int64_t i = 0; i < L; i++) v[i] = a[(k + 1 + i) * m + k];
        double alpha;
        double b = house(v, L, &alpha);
        beta[k] = b;
        /* keep v (v[0]=1 implicit) in column k below the subdiagonal */
        for (int64_t i = 1; i < L; i++) a[(k + 1 + i) * m + k] = v[i];
        e[k] = alpha;
        if (b == 0.0) continue;
        /* p = beta * A22 v */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < L; i++) {
            const double *row = a + (k + 1 + i) * m + (k + 1);
            double s = 0.0;
            for (int64_t j = 0; j < L; j++) s += row[j] * v[j];
            p[i] = b * s;
        }
        /* w = p - (beta p^T v / 2) v, stored in p */
        double pv = 0.0;
        for (int64_t i = 0; i < L; i++) pv += p[i] * v[i];
        double K = 0.5 * b * pv;
        for (int64_t i = 0; i < L; i++) p[i] -= K * v[i];
        /* A22 -= v w^T + w v^T */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < L; i++) {
            double *row = a + (k + 1 + i) * m + (k + 1);
            for (int64_t j = 0; j < L; j++) row[j] -= v[i] * p[j] + p[i] * v[j];
        }
    }
    for (int64_t i = 0; i < m; i++) d[i] = a[i * m + i];
    if (m >= 2) e[m - 2] = a[(m - 1) * m + (m - 2)];
    e[m - 1] = 0.0;

    /* --- accumulate Q (backward), stored transposed in Zt --- */
    if (Zt) {
        /* Q built row-major in tmp, then transposed into Zt */
        double *Q = dalloc((size_t)(m * m));
        for (int64_t i = 0; i < m; i++) Q[i * m + i] = 1.0;
        for (int64_t k = m - 3; k >= 0; k--) {
            double b = beta[k];
            if (b == 0.0) continue;
            int64_t L = m - k - 1;
            v[0] = 1.0;
            for (int64_t i = 1; i < L; i++) v[i] = a[(k + 1 + i) * m + k];
            /* Q[k+1:, k+1:] -= beta v (v^T Q[k+1:, k+1:]) */
#pragma omp parallel for schedule(static)
            for (int64_t c = k + 1; c < m; c++) {
                double s = 0.0;
                for (int64_t i = 0; i < L; i++) s += v[i] * Q[(k + 1 + i) * m + c];
                s *= b;
                for (int64_t i = 0; i < L; i++) Q[(k + 1 + i) * m + c] -= s * v[i];
            }
        }
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < m; j++) Zt[j * m + i] = Q[i * m + j];
        free(Q);
    }

    /* --- implicit symmetric QR with Wilkinson shift --- */
    int status = 0;
    double *cs = dalloc((size_t)(2 * m));
    int64_t iter = 0, maxiter = 60 * m + 100;
    int64_t hi = m - 1;
    while (hi > 0) {
        for (int64_t i = 0; i < hi; i++)
            if (fabs(e[i]) <= EPS * (fabs(d[i]) + fabs(d[i + 1])) || fabs(e[i]) <= DBL_MIN) e[i] = 0.0;
        if (e[hi - 1] == 0.0) { hi--; continue; }
        int64_t lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) lo--;
        if (++iter > maxiter) { status = 1; break; }
        /* Wilkinson shift: eigenvalue of trailing 2x2 closer to d[hi] */
        double dl = 0.5 * (d[hi - 1] - d[hi]);
        double eh = e[hi - 1];
        double sg = (dl >= 0.0) ? 1.0 : -1.0;
        double mu = d[hi] - eh * eh / (dl + sg * hypot(dl, eh));
        double x = d[lo] - mu, z = e[lo];
        for (int64_t k = lo; k < hi; k++) {
            double r = hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) { c = x / r; s = z / r; }
            if (k > lo) e[k - 1] = r;
            double ak = d[k], bk = e[k], ck = d[k + 1];
            d[k] = ak * c * c + 2.0 * bk * c * s + ck * s * s;
            d[k + 1] = ak * s * s - 2.0 * bk * c * s + ck * c * c;
            e[k] = c * s * (ck - ak) + bk * (c * c - s * s);
            if (k + 1 < hi) {
                z = e[k + 1] * s; /* bulge at T[k+2][k] */
                e[k + 1] *= c;
                x = e[k];
            }
            cs[2 * (k - lo)] = c;
            cs[2 * (k - lo) + 1] = s;
        }
        if (Zt) {
            /* apply the sweep's rotations to basis rows lo..hi; split the
             * element range across threads, each applies all rotations in order */
            int64_t nrot = hi - lo;
#pragma omp parallel for schedule(static)
            for (int64_t blk = 0; blk < (m + 63) / 64; blk++) {
                int64_t i0 = blk * 64, i1 = i0 + 64 < m ? i0 + 64 : m;
                for (int64_t t = 0; t < nrot; t++) {
                    double c = cs[2 * t], s = cs[2 * t + 1];
                    double *r0 = Zt + (lo + t) * m, *r1 = r0 + m;
                    for (int64_t i = i0; i < i1; i++) {
                        double z0 = r0[i], z1 = r1[i];
                        r0[i] = c * z0 + s * z1;
                        r1[i] = (MUT(4) ? s : -s) * z0 + c * z1;
                    }
                }
            }
        }
    }

    int64_t *perm = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    sort_desc(d, m, perm);
    for (int64_t j = 0; j < m; j++) w[j] = d[perm[j]];
    if (V) {
        for (int64_t j = 0; j < m; j++)
            for (int64_t i = 0; i < m; i++) V[i * m + j] = Zt[perm[j] * m + i];
        canon_columns(V, m, m);
    }
    free(perm); free(cs); free(v); free(a); free(d); free(e); free(beta); free(p);
    if (Zt) free(Zt);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Cyclic Jacobi eigensolver (GVL 8.5): rotate each off-diagonal pair to    */
/* zero until the off-diagonal mass is negligible.  O(m^3) per sweep.        */
/* ------------------------------------------------------------------------ */
int tsko_eigh_jacobi(const double *G, int64_t m, double *w, double *V) {
    if (!G || !w || m <= 0) return -1;
    double *a = dalloc((size_t)(m * m)), *Z = dalloc((size_t)(m * m));
    memcpy(a, G, sizeof(double) * (size_t)(m * m));
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < i; j++) a[j * m + i] = a[i * m + j];
    for (int64_t i = 0; i < m; i++) Z[i * m + i] = 1.0;
    double fro = 0.0;
    for (int64_t i = 0; i < m * m; i++) fro += a[i] * a[i];
    fro = sqrt(fro);
    int status = 1;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < m; j++)
                if (i != j) off += a[i * m + j] * a[i * m + j];
        if (sqrt(off) <= 1e-15 * fro || fro == 0.0) { status = 0; break; }
        for (int64_t p = 0; p < m - 1; p++)
            for (int64_t q = p + 1; q < m; q++) {
                double apq = a[p * m + q];
                if (apq == 0.0) continue;
                double tau = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
                double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                        : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* A <- J^T A J with J = I except J_pp=c, J_pq=s, J_qp=-s, J_qq=c */
                for (int64_t k = 0; k < m; k++) { /* columns p,q: A J */
                    double akp = a[k * m + p], akq = a[k * m + q];
                    a[k * m + p] = c * akp - s * akq;
                    a[k * m + q] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < m; k++) { /* rows p,q: J^T (A J) */
                    double apk = a[p * m + k], aqk = a[q * m + k];
                    a[p * m + k] = c * apk - s * aqk;
                    a[q * m + k] = s * apk + c * aqk;
                }
                a[p * m + q] = a[q * m + p] = 0.0;
                for (int64_t k = 0; k < m; k++) { /* Z <- Z J */
                    double zkp = Z[k * m + p], zkq = Z[k * m + q];
                    Z[k * m + p] = c * zkp - s * zkq;
                    Z[k * m + q] = s * zkp + c * zkq;
                }
            }
    }
    double *dg = dalloc((size_t)m);
    for (int64_t i = 0; i < m; i++) dg[i] = a[i * m + i];
    int64_t *perm = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    sort_desc(dg, m, perm);
    for (int64_t j = 0; j < m; j++) w[j] = dg[perm[j]];
    if (V) {
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < m; j++) V[i * m + j] = Z[i * m + perm[j]];
        canon_columns(V, m, m);
    }
    free(perm); free(dg); free(a); free(Z);
    return status;
}

/* ------------------------------------------------------------------------ */
/* One-sided Jacobi SVD (Hestenes; GVL 8.6).  Works on W = X^T stored so     */
/* that each column of X is a contiguous row of W (c rows of length len).    */
/* Rotates pairs of columns until all are mutually orthogonal; the same      */
/* rotations accumulated in Vr (rows = columns of the right factor).         */
/* ------------------------------------------------------------------------ */
static int jacobi_columns(double *W, int64_t c, int64_t len, double *Vr) {
    for (int sweep = 0; sweep < 100; sweep++) {
        int64_t rotated = 0;
        for (int64_t i = 0; i < c - 1; i++)
            for (int64_t j = i + 1; j < c; j++) {
                double *wi = W + i * len, *wj = W + j * len;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int64_t t = 0; t < len; t++) {
                    al += wi[t] * wi[t];
                    be += wj[t] * wj[t];
                    ga += wi[t] * wj[t];
                }
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                double zeta = (be - al) / (2.0 * ga);
                double t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int64_t q = 0; q < len; q++) {
                    double x = wi[q], y = wj[q];
                    wi[q] = cs * x - sn * y;
                    wj[q] = (MUT(6) ? -sn : sn) * x + cs * y;
                }
                if (Vr) {
                    double *vi = Vr + i * c, *vj = Vr + j * c;
                    for (int64_t q = 0; q < c; q++) {
                        double x = vi[q], y = vj[q];
                        vi[q] = cs * x - sn * y;
                        vj[q] = sn * x + cs * y;
                    }
                }
                rotated++;
            }
        if (!rotated) return 0;
    }
    return 1;
}

int tsko_svd(const double *A, int64_t m, int64_t n, double *U, double *s, double *Vt) {
    if (!A || m <= 0 || n <= 0) return -1;
    int tall = m >= n;
    int64_t c = tall ? n : m;   /* number of columns rotated */
    int64_t len = tall ? m : n; /* their length */
    double *W = dalloc((size_t)(c * len)), *Vr = dalloc((size_t)(c * c));
    /* W rows = columns of X, where X = A (tall) or A^T (wide) */
    if (tall) {
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < n; j++) W[j * m + i] = A[i * n + j];
    } else {
        memcpy(W, A, sizeof(double) * (size_t)(m * n));
    }
    for (int64_t i = 0; i < c; i++) Vr[i * c + i] = 1.0;
    int st = jacobi_columns(W, c, len, Vr);
    double *sv = dalloc((size_t)c);
    for (int64_t j = 0; j < c; j++) {
        double q = 0.0;
        for (int64_t t = 0; t < len; t++) q += W[j * len + t] * W[j * len + t];
        sv[j] = sqrt(q);
    }
    int64_t *perm = (int64_t *)calloc((size_t)c, sizeof(int64_t));
    sort_desc(sv, c, perm);
    /* X = Wcols * Vr^T-ish: X Vcols = W  =>  X = sum_j (W_j/s_j) s_j Vcol_j^T.
     * Left vectors of X: W_j / s_j (length len).  Right vectors of X: rows of Vr. */
    for (int64_t o = 0; o < c; o++) {
        int64_t j = perm[o];
        double sj = sv[j];
        if (s) s[o] = sj;
        for (int64_t t = 0; t < len; t++) {
            double lv = sj > 0.0 ? W[j * len + t] / sj : 0.0;
            if (tall) { if (U) U[t * c + o] = lv; }   /* U: m x p */
            else      { if (Vt) Vt[o * n + t] = lv; } /* A^T = L S R^T -> Vt rows = L cols */
        }
        for (int64_t q = 0; q < c; q++) {
            double rv = sj > 0.0 ? Vr[j * c + q] : 0.0;
            if (tall) { if (Vt) Vt[o * n + q] = rv; }  /* right vectors of A */
            else      { if (U) U[q * c + o] = rv; }    /* left vectors of A   */
        }
    }
    free(perm); free(sv); free(W); free(Vr);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Householder thin QR, GVL Alg. 5.2.1, with backward accumulation of Q.     */
/* ------------------------------------------------------------------------ */
int tsko_qr(const double *A, int64_t m, int64_t n, double *Q, double *R) {
    if (!A || m <= 0 || n <= 0 || m < n) return -1;
    double *W = dalloc((size_t)(m * n)), *betas = dalloc((size_t)n), *v = dalloc((size_t)m);
    memcpy(W, A, sizeof(double) * (size_t)(m * n));
    for (int64_t j = 0; j < n; j++) {
        int64_t L = m - j;
        for (int64_t i = 0; i < L; i++) v[i] = W[(j + i) * n + j];
        double alpha;
        double b = house(v, L, &alpha);
        betas[j] = b;
        for (int64_t c = j + 1; c < n; c++) {
            double s = 0.0;
            for (int64_t i = 0; i < L; i++) s += v[i] * W[(j + i) * n + c];
            s *= b;
            for (int64_t i = 0; i < L; i++) W[(j + i) * n + c] -= s * v[i];
        }
        W[j * n + j] = MUT(12) ? fabs(alpha) : alpha;
        for (int64_t i = 1; i < L; i++) W[(j + i) * n + j] = v[i];
    }
    if (R) {
        for (int64_t i = 0; i < n; i++)
            for (int64_t c = 0; c < n; c++) R[i * n + c] = (c >= i) ? W[i * n + c] : 0.0;
    }
    if (Q) {
        for (int64_t i = 0; i < m * n; i++) Q[i] = 0.0;
        for (int64_t i = 0; i < n; i++) Q[i * n + i] = 1.0;
        for (int64_t j = n - 1; j >= 0; j--) {
            double b = betas[j];
            if (b == 0.0) continue;
            int64_t L = m - j;
            v[0] = 1.0;
            for (int64_t i = 1; i < L; i++) v[i] = W[(j + i) * n + j];
            for (int64_t c = j; c < n; c++) {
                double s = 0.0;
                for (int64_t i = 0; i < L; i++) s += v[i] * Q[(j + i) * n + c];
                s *= b;
                for (int64_t i = 0; i < L; i++) Q[(j + i) * n + c] -= s * v[i];
            }
        }
    }
    free(W); free(betas); free(v);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Training: first half of Algorithm 2.  S* = first k columns of U^(1) (eq. */
/* 3.3 and the sentence after it), i.e. the top-k eigenvectors of the Gram. */
/* ------------------------------------------------------------------------ */
int tsko_train_from_gram(const double *G, int64_t m, int64_t k, double *S, double *lambda) {
    if (!G || !S || k < 1 || k > m) return -1;
    double *w = dalloc((size_t)m), *V = dalloc((size_t)(m * m));
    int st = tsko_eigh(G, m, w, V);
    for (int64_t i = 0; i < k; i++)
        for (int64_t j = 0; j < m; j++) S[i * m + j] = V[j * m + i + (MUT(7) && i + 1 < m)];
    if (lambda)
        for (int64_t i = 0; i <= k; i++) lambda[i] = (i < m) ? w[i] : 0.0;
    free(w); free(V);
    return st;
}

int tsko_train_f32(const float *A, int64_t count, int64_t m, int64_t n, int64_t k,
                   double *S, double *lambda, double *fro2) {
    if (!A || !S || count < 1 || m <= 0 || n <= 0 || k < 1 || k > m) return -1;
    double *G = dalloc((size_t)(m * m));
    tsko_gram_f32(A, count, m, n, G);
    if (fro2) {
        double t = 0.0;
        for (int64_t i = 0; i < m; i++) t += G[i * m + i];
        *fro2 = t;
    }
    int st = tsko_train_from_gram(G, m, k, S, lambda);
    free(G);
    return st;
}

/* ------------------------------------------------------------------------ */
/* SCW, Algorithm 1.                                                         */
/* ------------------------------------------------------------------------ */
/* Step 1 of Algorithm 1: B = S A and an orthonormal basis V (n x k) of its
 * row space (thin SVD of B, or Householder QR of B^T with vmode = 1). */
int tsko_scw_basis(const double *A, int64_t m, int64_t n, const double *S, int64_t k, int vmode,
                   double *V, int32_t *flags) {
    if (!A || !S || !V || m <= 0 || n <= 0 || k < 1 || k > m || k > n) return -1;
    int32_t fl = 0;
    double *B = dalloc((size_t)(k * n));
    for (int64_t s = 0; s < k; s++)
        for (int64_t i = 0; i < m; i++) {
            double sv = MUT(11) ? S[i * k + s] : S[s * m + i];
            for (int64_t j = 0; j < n; j++) B[s * n + j] += sv * A[i * n + j];
        }
    memset(V, 0, sizeof(double) * (size_t)(n * k));
    if (vmode == 1) {
        double *Bt = dalloc((size_t)(n * k));
        for (int64_t s = 0; s < k; s++)
            for (int64_t j = 0; j < n; j++) Bt[j * k + s] = B[s * n + j];
        tsko_qr(Bt, n, k, V, NULL);
        free(Bt);
    } else {
        double *sb = dalloc((size_t)k), *Vtb = dalloc((size_t)(k * n));
        tsko_svd(B, k, n, NULL, sb, Vtb);
        for (int64_t s = 0; s < k; s++) {
            int keep = sb[s] > 1e-13 * sb[0];
            if (!keep) fl |= TSKO_FLAG_RANKDEF;
            for (int64_t j = 0; j < n; j++) V[j * k + s] = keep ? Vtb[s * n + j] : 0.0;
            if (MUT(8)) {
                double nb = 0.0;
                for (int64_t j = 0; j < n; j++) nb += B[s * n + j] * B[s * n + j];
                for (int64_t j = 0; j < n; j++) V[j * k + s] = B[s * n + j] / sqrt(nb);
            }
        }
        free(sb); free(Vtb);
    }
    free(B);
    if (flags) *flags = fl;
    return 0;
}

int tsko_scw(const double *A, int64_t m, int64_t n, const double *S, int64_t k, int64_t r,
             int vmode, double *L, double *R, double *sigma, double *Ahat,
             double *relerr, int32_t *flags) {
    if (!A || !S || m <= 0 || n <= 0 || r < 1 || k <= r || k > m || k > n) return -1;
    int32_t fl = 0;
    double fro2 = 0.0;
    for (int64_t i = 0; i < m * n; i++) {
        if (!isfinite(A[i])) fl |= TSKO_FLAG_NONFIN;
        fro2 += A[i] * A[i];
    }
    if (fl & TSKO_FLAG_NONFIN) {
        if (relerr) *relerr = NAN;
        if (flags) *flags = fl;
        return 0;
    }
    /* step 1: B = S A (k x n) and V (n x k), an orthonormal basis of row(B) */
    double *V = dalloc((size_t)(n * k));
    int32_t fb = 0;
    tsko_scw_basis(A, m, n, S, k, vmode, V, &fb);
    fl |= fb;
    /* step 2: C = A V (m x k), thin SVD C = U Sig Y^T */
    double *C = dalloc((size_t)(m * k));
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) {
            double a = A[i * n + j];
            for (int64_t s = 0; s < k; s++) C[i * k + s] += a * V[j * k + s];
        }
    double *Uc = dalloc((size_t)(m * k)), *sc = dalloc((size_t)k), *Yt = dalloc((size_t)(k * k));
    tsko_svd(C, m, k, Uc, sc, Yt);
    if (r < k && sc[r - 1] - sc[r] <= 1e-12 * sc[0]) fl |= TSKO_FLAG_TIE;
    /* step 3: L = U_r Sig_r, R = V Y_r, A_hat = L R^T */
    double *Lm = dalloc((size_t)(m * r)), *Rm = dalloc((size_t)(n * r));
    for (int64_t i = 0; i < m; i++)
        for (int64_t t = 0; t < r; t++) Lm[i * r + t] = Uc[i * k + t] * sc[t];
    for (int64_t j = 0; j < n; j++)
        for (int64_t t = 0; t < r; t++) {
            double acc = 0.0;
            for (int64_t s = 0; s < k; s++) acc += V[j * k + s] * (MUT(9) ? Yt[s * k + t] : Yt[t * k + s]);
            Rm[j * r + t] = acc;
        }
    double res2 = 0.0;
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) {
            double ah = 0.0;
            for (int64_t t = 0; t < r; t++) ah += Lm[i * r + t] * Rm[j * r + t];
            if (MUT(10)) ah += Uc[i * k + r] * sc[r] * V[j * k + r];
            if (Ahat) Ahat[i * n + j] = ah;
            double dlt = A[i * n + j] - ah;
            res2 += dlt * dlt;
        }
    if (L) memcpy(L, Lm, sizeof(double) * (size_t)(m * r));
    if (R) memcpy(R, Rm, sizeof(double) * (size_t)(n * r));
    if (sigma) memcpy(sigma, sc, sizeof(double) * (size_t)r);
    if (relerr) *relerr = fro2 > 0.0 ? sqrt(res2 / fro2) : 0.0;
    if (flags) *flags = fl;
    free(V); free(C); free(Uc); free(sc); free(Yt); free(Lm); free(Rm);
    return 0;
}

int tsko_apply_f32(const float *A, int64_t count, int64_t m, int64_t n, const double *S,
                   int64_t k, int64_t r, double *L, double *R, double *sigma,
                   double *relerr, int32_t *flags) {
    if (!A || !S || count < 0 || m <= 0 || n <= 0 || r < 1 || k <= r || k > m || k > n) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t d = 0; d < count; d++) {
        double *Ad = dalloc((size_t)(m * n));
        for (int64_t i = 0; i < m * n; i++) Ad[i] = (double)A[d * m * n + i];
        int st = tsko_scw(Ad, m, n, S, k, r, 0, L ? L + d * m * r : NULL, R ? R + d * n * r : NULL,
                          sigma ? sigma + d * r : NULL, NULL, relerr ? relerr + d : NULL,
                          flags ? flags + d : NULL);
        bad |= (st != 0);
        free(Ad);
    }
    return bad ? -1 : 0;
}

int tsko_error_f32(const float *A, int64_t count, int64_t m, int64_t n, const double *L,
                   const double *R, int64_t r, double *relerr) {
    if (!A || !L || !R || !relerr || count < 0 || m <= 0 || n <= 0 || r < 1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t d = 0; d < count; d++) {
        const float *Ad = A + d * m * n;
        const double *Ld = L + d * m * r, *Rd = R + d * n * r;
        double res2 = 0.0, fro2 = 0.0;
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < n; j++) {
                double ah = 0.0;
                for (int64_t t = 0; t < r; t++) ah += Ld[i * r + t] * Rd[j * r + t];
                double a = (double)Ad[i * n + j];
                fro2 += a * a;
                res2 += (a - ah) * (a - ah);
            }
        relerr[d] = fro2 > 0.0 ? sqrt(res2 / fro2) : 0.0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Number formats of the reduced-precision forms (no precision is fixed by  */
/* the paper).  Written from the format definitions: the value is scaled    */
/* by its quantum (a power of two, so the division is exact), rounded to an */
/* integer with ties to even (rint in the default rounding mode) and scaled */
/* back.  No bit manipulation.                                               */
/* ------------------------------------------------------------------------ */
static double round_to_format(double x, int p, int emin, double maxfin, int saturate) {
    if (isnan(x) || x == 0.0) return x;
    if (isinf(x)) return saturate ? copysign(maxfin, x) : x;
    int e;
    frexp(x, &e);              /* |x| = f 2^e, 1/2 <= f < 1: leading bit weighs 2^(e-1) */
    int lead = e - 1;
    if (lead < emin) lead = emin;  /* subnormal range: fixed quantum */
    const double q = ldexp(1.0, lead - (p - 1 - MUT(14)));
    const double t = x / q;
    const double y = (MUT(13) ? round(t) : rint(t)) * q;
    if (fabs(y) > maxfin) return saturate ? copysign(maxfin, x) : copysign(INFINITY, x);
    return y;
}

int tsko_round_bf16(const float *x, int64_t n, float *y) {
    if ((!x || !y) && n > 0) return -1;
    const double maxfin = ldexp(2.0 - ldexp(1.0, -7), 127);
    for (int64_t i = 0; i < n; i++) y[i] = (float)round_to_format((double)x[i], 8, -126, maxfin, 0);
    return 0;
}

int tsko_round_e4m3(const float *x, int64_t n, float scale, float *y) {
    if ((!x || !y) && n > 0) return -1;
    for (int64_t i = 0; i < n; i++)
        y[i] = (float)round_to_format((double)x[i] * (double)scale, 4, -6, 448.0, 1);
    return 0;
}

int tsko_e4m3_scale(const float *x, int64_t n, float *scale) {
    if ((!x && n > 0) || !scale) return -1;
    double amax = 0.0;
    for (int64_t i = 0; i < n; i++)
        if (fabs((double)x[i]) > amax) amax = fabs((double)x[i]);
    if (amax == 0.0) {
        *scale = 1.0f;
        return 0;
    }
    int e;
    frexp(448.0 / amax, &e);   /* 448/amax = f 2^e, 1/2 <= f < 1: floor(log2) = e - 1 */
    int j = e - 1 + MUT(15);
    if (j > 127) j = 127;
    if (j < -126) j = -126;
    *scale = (float)ldexp(1.0, j);
    return 0;
}

int tsko_round_e4m3_mx(const float *x, int64_t rows, int64_t n, float *y, uint8_t *e) {
    if (rows < 0 || n < 0 || ((!x || !y || !e) && rows * n > 0)) return -1;
    const int64_t bw = 32 - 16 * MUT(20);           /* block width along a row */
    const int64_t nb = (n + bw - 1) / bw;
    for (int64_t i = 0; i < rows; i++)
        for (int64_t b = 0; b < nb; b++) {
            const int64_t c0 = b * bw, w = n - c0 < bw ? n - c0 : bw;
            const float *xb = x + i * n + c0;
            float *yb = y + i * n + c0, s;
            tsko_e4m3_scale(xb, w, &s);
            tsko_round_e4m3(xb, w, s, yb);
            for (int64_t j = 0; j < w; j++) yb[j] = (float)((double)yb[j] / (double)s);
            int ex;
            frexp((double)s, &ex);                  /* s = 2^(ex - 1) */
            e[i * nb + b] = (uint8_t)(127 - (ex - 1));
        }
    return 0;
}

int tsko_opt_f32(const float *A, int64_t count, int64_t m, int64_t n, int64_t r,
                 double *tail, double *fro) {
    if (!A || !tail || count < 0 || m <= 0 || n <= 0 || r < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t d = 0; d < count; d++) {
        int64_t p = m < n ? m : n;
        double *Ad = dalloc((size_t)(m * n)), *s = dalloc((size_t)p);
        double f2 = 0.0;
        for (int64_t i = 0; i < m * n; i++) {
            Ad[i] = (double)A[d * m * n + i];
            f2 += Ad[i] * Ad[i];
        }
        tsko_svd(Ad, m, n, NULL, s, NULL);
        double t2 = 0.0;
        for (int64_t i = p - 1; i >= r; i--) t2 += s[i] * s[i];
        tail[d] = sqrt(t2);
        if (fro) fro[d] = sqrt(f2);
        free(Ad); free(s);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Data-free sketches for the SCW baseline (Section 1: sketching matrices
 * drawn from a distribution such as the Gaussian or the Rademacher one;
 * Section 2: the sparse random sign matrix that initialises IVY's sketch).
 * Counter-based: the value of counter c is the c-th output (from 0) of the
 * SplitMix64 generator seeded with `seed` (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): the state
 * advances by the odd constant 0x9E3779B97F4A7C15 and each state is mixed by
 * two xor-shift-multiply rounds and a final xor-shift.
 * ------------------------------------------------------------------------ */
uint64_t tsko_splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int tsko_random_sketch(int kind, int64_t k, int64_t m, uint64_t seed, double *S) {
    if (!S || k < 1 || m < 1 || kind < 0 || kind > 2) return -1;
    const double scale = 1.0 / sqrt((double)k);
    if (kind == 2) {
        /* one nonzero +-1 per column: row (h >> 32) mod k, sign from bit 0 */
        memset(S, 0, sizeof(double) * (size_t)(k * m));
        for (int64_t j = 0; j < m; j++) {
            const uint64_t h = tsko_splitmix64(seed, (uint64_t)j);
            const int64_t row = (int64_t)((h >> 32) % (uint64_t)(k - MUT(17) * (k > 1)));
            S[row * m + j] = (h & 1u) ? -1.0 : 1.0;
        }
        return 0;
    }
    for (int64_t i = 0; i < k; i++)
        for (int64_t j = 0; j < m; j++) {
            const uint64_t c = (uint64_t)(i * m + j);
            double v;
            if (kind == 1) {
                /* Rademacher: the sign of the top bit */
                v = (tsko_splitmix64(seed, c) >> 63) ? -1.0 : 1.0;
            } else {
                /* Gaussian by the Box-Muller transform of two uniforms,
                 * u1 in (0, 1] and u2 in [0, 1), 53 bits each */
                const double u1 = (double)((tsko_splitmix64(seed, 2 * c) >> 11) + 1) * 0x1p-53;
                const double u2 = (double)(tsko_splitmix64(seed, 2 * c + 1) >> 11) * 0x1p-53;
                v = sqrt((MUT(16) ? -1.0 : -2.0) * log(u1)) * cos(6.283185307179586477 * u2);
            }
            S[i * m + j] = v * scale;
        }
    return 0;
}

/* ------------------------------------------------------------------------
 * The two-sided method (Section 3.2, problem 3.6; Algorithms 3 and 4;
 * Appendix, Algorithm 5).
 * ------------------------------------------------------------------------ */

/* Mode-2 Gram: sum_d A_d^T A_d (n x n), natural slice order, FP64. */
int tsko_gram2_f32(const float *A, int64_t count, int64_t m, int64_t n, double *G) {
    if (!A || !G || count < 0 || m <= 0 || n <= 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j1 = 0; j1 < n; j1++)
        for (int64_t j2 = 0; j2 <= j1; j2++) {
            double s = 0.0;
            for (int64_t d = 0; d < count; d++) {
                const float *a = A + d * m * n;
                for (int64_t i = 0; i < m; i++) s += (double)a[i * n + j1] * (double)a[i * n + j2];
            }
            G[j1 * n + j2] = s;
            G[j2 * n + j1] = s;
        }
    return 0;
}

/* Top-p eigenvectors of the symmetric p0 x p0 matrix G as the rows of U
 * (p x p0) and the sum of the top-p eigenvalues. */
static double top_rows(const double *G, int64_t p0, int64_t p, double *U) {
    double *lam = dalloc((size_t)(p + 1));
    tsko_train_from_gram(G, p0, p, U, lam);
    double s = 0.0;
    for (int64_t i = 0; i < p; i++) s += lam[i];
    free(lam);
    return s;
}

/* Tucker2 of the m x n x N tensor by HOOI (Algorithm 5 restricted to modes
 * 1 and 2, the third mode left whole), from the HOSVD initial guess:
 *   S_0 = top-k eigenvectors of sum_d A_d A_d^T,  W_0 = top-l of sum_d A_d^T A_d;
 * one sweep updates S (mode 1, with the current W), then W (mode 2, with the
 * new S):
 *   S <- top-k eigenvectors of sum_d (A_d W^T)(A_d W^T)^T,
 *   W <- top-l eigenvectors of sum_d (S A_d)^T (S A_d),
 * and ||G||^2 = sum_d ||S A_d W^T||_F^2 is the sum of the top-l eigenvalues
 * of the second Gram.  Stops when ||G||^2 changes by at most tol ||G||^2 or
 * after max_sweeps sweeps.  core2: nullable, max_sweeps + 1 values (index 0:
 * the HOSVD guess); *sweeps: the sweeps done. */
int tsko_train2_f32(const float *A, int64_t count, int64_t m, int64_t n, int64_t k, int64_t l,
                    int64_t max_sweeps, double tol, double *S, double *W, double *core2, int64_t *sweeps) {
    if (!A || !S || !W || count < 1 || k < 1 || k > m || l < 1 || l > n || max_sweeps < 0) return -1;
    double *G1 = dalloc((size_t)(m * m)), *G2 = dalloc((size_t)(n * n));
    tsko_gram_f32(A, count, m, n, G1);
    top_rows(G1, m, k, S);
    tsko_gram2_f32(A, count, m, n, G2);
    top_rows(G2, n, l, W);
    /* ||G||^2 of the guess */
    double c2 = 0.0;
    for (int64_t d = 0; d < count; d++) {
        const float *a = A + d * m * n;
        for (int64_t s = 0; s < k; s++)
            for (int64_t t = 0; t < l; t++) {
                double v = 0.0;
                for (int64_t i = 0; i < m; i++) {
                    double ai = 0.0;
                    for (int64_t j = 0; j < n; j++) ai += (double)a[i * n + j] * W[t * n + j];
                    v += S[s * m + i] * ai;
                }
                c2 += v * v;
            }
    }
    if (core2) core2[0] = c2;
    double *Y = dalloc((size_t)(m * l)), *Z = dalloc((size_t)(k * n));
    int64_t sw = 0;
    while (sw < max_sweeps) {
        /* mode 1: sum_d (A_d W^T)(A_d W^T)^T */
        memset(G1, 0, sizeof(double) * (size_t)(m * m));
        for (int64_t d = 0; d < count; d++) {
            const float *a = A + d * m * n;
            for (int64_t i = 0; i < m; i++)
                for (int64_t t = 0; t < l; t++) {
                    double v = 0.0;
                    for (int64_t j = 0; j < n; j++) v += (double)a[i * n + j] * W[t * n + j];
                    Y[i * l + t] = v;
                }
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t i1 = 0; i1 < m; i1++)
                for (int64_t i2 = 0; i2 <= i1; i2++) {
                    double v = 0.0;
                    for (int64_t t = 0; t < l; t++) v += Y[i1 * l + t] * Y[i2 * l + t];
                    G1[i1 * m + i2] += v;
                }
        }
        for (int64_t i1 = 0; i1 < m; i1++)
            for (int64_t i2 = 0; i2 < i1; i2++) G1[i2 * m + i1] = G1[i1 * m + i2];
        if (!MUT(19)) top_rows(G1, m, k, S);
        /* mode 2: sum_d (S A_d)^T (S A_d) */
        memset(G2, 0, sizeof(double) * (size_t)(n * n));
        for (int64_t d = 0; d < count; d++) {
            const float *a = A + d * m * n;
            for (int64_t s = 0; s < k; s++)
                for (int64_t j = 0; j < n; j++) {
                    double v = 0.0;
                    for (int64_t i = 0; i < m; i++) v += S[s * m + i] * (double)a[i * n + j];
                    Z[s * n + j] = v;
                }
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t j1 = 0; j1 < n; j1++)
                for (int64_t j2 = 0; j2 <= j1; j2++) {
                    double v = 0.0;
                    for (int64_t s = 0; s < k; s++) v += Z[s * n + j1] * Z[s * n + j2];
                    G2[j1 * n + j2] += v;
                }
        }
        for (int64_t j1 = 0; j1 < n; j1++)
            for (int64_t j2 = 0; j2 < j1; j2++) G2[j2 * n + j1] = G2[j1 * n + j2];
        const double c2n = top_rows(G2, n, l, W);
        sw++;
        if (core2) core2[sw] = c2n;
        const int done = fabs(c2n - c2) <= tol * c2n;
        c2 = c2n;
        if (done) break;
    }
    if (sweeps) *sweeps = sw;
    free(G1); free(G2); free(Y); free(Z);
    return 0;
}

/* Two-sided SCW (Algorithm 4) on one matrix A (m x n) with S (k x m) and
 * W (l x n), r < min(k, l):
 *   1. Q = Q factor of a Householder QR of A^T S^T (n x k);
 *   2. P = Q factor of a Householder QR of A W^T (m x l);
 *   3. M = P^T A Q (l x k), thin SVD M = U Sig Y^T, [M]_r = U_r Sig_r Y_r^T;
 *   4. A_hat = P [M]_r Q^T = L R^T with L = P U_r Sig_r (m x r),
 *      R = Q Y_r (n x r).
 * relerr = ||A - A_hat||_F / ||A||_F from the dense residual.  Flags: RANKDEF
 * when a diagonal entry of either R factor is at most 1e-13 of that
 * factor's largest; TIE when sigma_r - sigma_{r+1} <= 1e-12 sigma_1. */
int tsko_scw2(const double *A, int64_t m, int64_t n, const double *S, int64_t k, const double *W, int64_t l,
              int64_t r, double *L, double *R, double *sigma, double *relerr, int32_t *flags) {
    if (!A || !S || !W || m <= 0 || n <= 0 || r < 1 || r >= k || r >= l || k > n || l > m || k > m || l > n)
        return -1;
    int32_t fl = 0;
    double fro2 = 0.0;
    for (int64_t i = 0; i < m * n; i++) {
        if (!isfinite(A[i])) fl |= TSKO_FLAG_NONFIN;
        fro2 += A[i] * A[i];
    }
    if (fl & TSKO_FLAG_NONFIN) {
        if (relerr) *relerr = NAN;
        if (flags) *flags = fl;
        return 0;
    }
    double *At = dalloc((size_t)(n * k)), *Q = dalloc((size_t)(n * k)), *R1 = dalloc((size_t)(k * k));
    for (int64_t j = 0; j < n; j++)
        for (int64_t s = 0; s < k; s++) {
            double v = 0.0;
            for (int64_t i = 0; i < m; i++) v += A[i * n + j] * S[s * m + i];
            At[j * k + s] = v;
        }
    tsko_qr(At, n, k, Q, R1);
    double *Aw = dalloc((size_t)(m * l)), *P = dalloc((size_t)(m * l)), *R2 = dalloc((size_t)(l * l));
    for (int64_t i = 0; i < m; i++)
        for (int64_t t = 0; t < l; t++) {
            double v = 0.0;
            for (int64_t j = 0; j < n; j++) v += A[i * n + j] * W[t * n + j];
            Aw[i * l + t] = v;
        }
    tsko_qr(Aw, m, l, P, R2);
    double d1 = 0.0, d2 = 0.0;
    for (int64_t s = 0; s < k; s++) d1 = fmax(d1, fabs(R1[s * k + s]));
    for (int64_t t = 0; t < l; t++) d2 = fmax(d2, fabs(R2[t * l + t]));
    for (int64_t s = 0; s < k; s++)
        if (fabs(R1[s * k + s]) <= 1e-13 * d1) fl |= TSKO_FLAG_RANKDEF;
    for (int64_t t = 0; t < l; t++)
        if (fabs(R2[t * l + t]) <= 1e-13 * d2) fl |= TSKO_FLAG_RANKDEF;
    /* M = P^T A Q */
    double *AQ = dalloc((size_t)(m * k)), *M = dalloc((size_t)(l * k));
    for (int64_t i = 0; i < m; i++)
        for (int64_t s = 0; s < k; s++) {
            double v = 0.0;
            for (int64_t j = 0; j < n; j++) v += A[i * n + j] * Q[j * k + s];
            AQ[i * k + s] = v;
        }
    for (int64_t t = 0; t < l; t++)
        for (int64_t s = 0; s < k; s++) {
            double v = 0.0;
            for (int64_t i = 0; i < m; i++) v += P[i * l + t] * AQ[i * k + s];
            M[t * k + s] = v;
        }
    const int64_t p = l < k ? l : k;
    double *Um = dalloc((size_t)(l * p)), *sm = dalloc((size_t)p), *Yt = dalloc((size_t)(p * k));
    tsko_svd(M, l, k, Um, sm, Yt);
    if (r < p && sm[r - 1] - sm[r] <= 1e-12 * sm[0]) fl |= TSKO_FLAG_TIE;
    double *Lm = dalloc((size_t)(m * r)), *Rm = dalloc((size_t)(n * r));
    for (int64_t i = 0; i < m; i++)
        for (int64_t c = 0; c < r; c++) {
            double v = 0.0;
            for (int64_t t = 0; t < l; t++) v += P[i * l + t] * Um[t * p + c];
            Lm[i * r + c] = MUT(18) ? v : v * sm[c];
        }
    for (int64_t j = 0; j < n; j++)
        for (int64_t c = 0; c < r; c++) {
            double v = 0.0;
            for (int64_t s = 0; s < k; s++) v += Q[j * k + s] * Yt[c * k + s];
            Rm[j * r + c] = v;
        }
    double res2 = 0.0;
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) {
            double ah = 0.0;
            for (int64_t c = 0; c < r; c++) ah += Lm[i * r + c] * Rm[j * r + c];
            const double dl = A[i * n + j] - ah;
            res2 += dl * dl;
        }
    if (L) memcpy(L, Lm, sizeof(double) * (size_t)(m * r));
    if (R) memcpy(R, Rm, sizeof(double) * (size_t)(n * r));
    if (sigma) memcpy(sigma, sm, sizeof(double) * (size_t)r);
    if (relerr) *relerr = fro2 > 0.0 ? sqrt(res2 / fro2) : 0.0;
    if (flags) *flags = fl;
    free(At); free(Q); free(R1); free(Aw); free(P); free(R2); free(AQ); free(M);
    free(Um); free(sm); free(Yt); free(Lm); free(Rm);
    return 0;
}

int tsko_apply2_f32(const float *A, int64_t count, int64_t m, int64_t n, const double *S, int64_t k,
                    const double *W, int64_t l, int64_t r, double *L, double *R, double *sigma, double *relerr,
                    int32_t *flags) {
    if (!A || !S || !W || count < 0) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t d = 0; d < count; d++) {
        double *a = dalloc((size_t)(m * n));
        for (int64_t i = 0; i < m * n; i++) a[i] = (double)A[d * m * n + i];
        bad |= tsko_scw2(a, m, n, S, k, W, l, r, L ? L + d * m * r : NULL, R ? R + d * n * r : NULL,
                         sigma ? sigma + d * r : NULL, relerr ? relerr + d : NULL, flags ? flags + d : NULL) != 0;
        free(a);
    }
    return bad ? -1 : 0;
}
