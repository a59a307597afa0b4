/*
 * oracle_core.c -- plain FP64 (and one FP32) reference loops for the
 * orthogonalization-free Rayleigh-Ritz method of Xu, Zhang, Chen, Saad and
 * Xi, "Mixed Precision Orthogonalization-Free Projection Methods for
 * Eigenvalue and Singular Value Problems" (arXiv 2505.00281).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: it
 * is built into liborc_core.so and loaded by oracle/ofrr_oracle.py, which
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may import.  It shares no code, header or constant with the HIP
 * library and includes nothing from it.
 *
 * Everything is column-major with a leading dimension, 0-based indices.
 * Nothing is blocked, fused or reordered beyond what the cited passage
 * states; each routine is written to be checked against the paper by eye.
 *
 * Routines
 *   orc_jacobi_eig     cyclic two-sided Jacobi for a symmetric matrix
 *                      (textbook symmetric Schur rotations), used for the
 *                      small projected problems (Alg. "Rayleigh-Ritz with
 *                      orthogonal bases", Sec. 2) and for brute force.
 *   orc_cholesky       lower Cholesky factor, used to reduce the symmetric
 *                      definite pencil of eq. (geig) to standard form.
 *   orc_mgs2           modified Gram-Schmidt with one re-orthogonalisation
 *                      pass triggered by the sqrt(2)/2 norm-drop test
 *                      (Sec. 5.1, implementation details).
 *   orc_hessenberg_f64 the right-looking Hessenberg process for a block
 *   orc_hessenberg_f32 (Sec. 4.2, Algorithm "Computing non-orthogonal bases
 *                      from the Hessenberg Process"), in FP64 and in FP32;
 *   orc_hessenberg_f16s the same with binary16 storage and FP32 arithmetic
 *                      (orc_round_binary16: round to nearest binary16).
 *   orc_csr_mm         Y = A X for A in CSR (Sec. 5.1 uses CSR for sparse A).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------
 * Cyclic Jacobi eigenvalue algorithm for a symmetric n x n matrix S.
 *
 * One rotation J(p,q) (identity except J_pp = J_qq = c, J_pq = s,
 * J_qp = -s) is chosen so that the (p,q) entry of J^T S J vanishes:
 *   tau = (S_qq - S_pp) / (2 S_pq),
 *   t   = sign(tau) / (|tau| + sqrt(1 + tau^2))   (the smaller root),
 *   c   = 1 / sqrt(1 + t^2),   s = t c.
 * Columns p, q of S and Z are replaced by c*col_p - s*col_q and
 * s*col_p + c*col_q; rows p, q of S likewise.  Sweeps visit all pairs
 * p < q in row order until the off-diagonal Frobenius norm is at most
 * 1e-15 times the Frobenius norm of S.
 *
 * On return w[i] = S_ii (unsorted) and the columns of Z are the
 * eigenvectors.  S is overwritten.  Returns the number of sweeps used, or
 * -1 if max_sweeps was not enough.
 * ---------------------------------------------------------------------- */
int orc_jacobi_eig(int64_t n, double *S, int64_t lds, double *w, double *Z,
                   int64_t ldz, int max_sweeps)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            Z[IDX(i, j, ldz)] = (i == j) ? 1.0 : 0.0;

    double frob2 = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            frob2 += S[IDX(i, j, lds)] * S[IDX(i, j, lds)];
    const double tol2 = 1e-30 * frob2;

    int sweep = 0;
    for (;;) {
        double off2 = 0.0;
        for (int64_t q = 1; q < n; ++q)
            for (int64_t p = 0; p < q; ++p)
                off2 += 2.0 * S[IDX(p, q, lds)] * S[IDX(p, q, lds)];
        if (off2 <= tol2 || off2 == 0.0) break;
        if (sweep >= max_sweeps) {
            for (int64_t i = 0; i < n; ++i) w[i] = S[IDX(i, i, lds)];
            return -1;
        }
        ++sweep;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                const double apq = S[IDX(p, q, lds)];
                if (apq == 0.0) continue;
                const double app = S[IDX(p, p, lds)];
                const double aqq = S[IDX(q, q, lds)];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) /
                                 (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* S <- S J : columns p and q */
                for (int64_t k = 0; k < n; ++k) {
                    const double skp = S[IDX(k, p, lds)];
                    const double skq = S[IDX(k, q, lds)];
                    S[IDX(k, p, lds)] = c * skp - s * skq;
                    S[IDX(k, q, lds)] = s * skp + c * skq;
                }
                /* S <- J^T S : rows p and q */
                for (int64_t k = 0; k < n; ++k) {
                    const double spk = S[IDX(p, k, lds)];
                    const double sqk = S[IDX(q, k, lds)];
                    S[IDX(p, k, lds)] = c * spk - s * sqk;
                    S[IDX(q, k, lds)] = s * spk + c * sqk;
                }
                /* the rotation annihilates (p,q) exactly in exact
                 * arithmetic; store the exact zero */
                S[IDX(p, q, lds)] = 0.0;
                S[IDX(q, p, lds)] = 0.0;
                /* Z <- Z J */
                for (int64_t k = 0; k < n; ++k) {
                    const double zkp = Z[IDX(k, p, ldz)];
                    const double zkq = Z[IDX(k, q, ldz)];
                    Z[IDX(k, p, ldz)] = c * zkp - s * zkq;
                    Z[IDX(k, q, ldz)] = s * zkp + c * zkq;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) w[i] = S[IDX(i, i, lds)];
    return sweep;
}

/* ------------------------------------------------------------------------
 * Lower Cholesky factor G = L L^T, written over the lower triangle of G
 * (the strict upper triangle is set to zero).  Returns 0 on success, or
 * j+1 when the j-th pivot is not positive.
 * ---------------------------------------------------------------------- */
int orc_cholesky(int64_t n, double *G, int64_t ldg)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = G[IDX(j, j, ldg)];
        for (int64_t k = 0; k < j; ++k)
            d -= G[IDX(j, k, ldg)] * G[IDX(j, k, ldg)];
        if (!(d > 0.0)) return (int)(j + 1);
        const double ljj = sqrt(d);
        G[IDX(j, j, ldg)] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double v = G[IDX(i, j, ldg)];
            for (int64_t k = 0; k < j; ++k)
                v -= G[IDX(i, k, ldg)] * G[IDX(j, k, ldg)];
            G[IDX(i, j, ldg)] = v / ljj;
        }
        for (int64_t i = 0; i < j; ++i) G[IDX(i, j, ldg)] = 0.0;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Modified Gram-Schmidt QR, X = Q R, with re-orthogonalisation: when the
 * projection of column j against q_0..q_{j-1} reduces its 2-norm below
 * sqrt(2)/2 of what it was, the projection loop is run once more and its
 * coefficients are added to R (Sec. 5.1: the sqrt(2)/2 threshold).
 * X is overwritten by Q; R is b x b upper triangular.  Returns the number
 * of columns processed before a zero column was met (b on success).
 * ---------------------------------------------------------------------- */
static double col_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

int64_t orc_mgs2(int64_t n, int64_t b, double *X, int64_t ldx, double *R,
                 int64_t ldr)
{
    for (int64_t j = 0; j < b; ++j)
        for (int64_t i = 0; i < b; ++i) R[IDX(i, j, ldr)] = 0.0;

    for (int64_t j = 0; j < b; ++j) {
        double *v = X + IDX(0, j, ldx);
        double before = sqrt(col_dot(n, v, v));
        for (int pass = 0; pass < 2; ++pass) {
            for (int64_t i = 0; i < j; ++i) {
                const double *qi = X + IDX(0, i, ldx);
                const double r = col_dot(n, qi, v);
                R[IDX(i, j, ldr)] += r;
                for (int64_t t = 0; t < n; ++t) v[t] -= r * qi[t];
            }
            const double after = sqrt(col_dot(n, v, v));
            if (pass == 0 && after < (sqrt(2.0) / 2.0) * before) {
                before = after;
                continue; /* lost orthogonality: project once more */
            }
            break;
        }
        const double nrm = sqrt(col_dot(n, v, v));
        if (!(nrm > 0.0)) return j;
        R[IDX(j, j, ldr)] = nrm;
        for (int64_t t = 0; t < n; ++t) v[t] /= nrm;
    }
    return b;
}

/* ------------------------------------------------------------------------
 * Right-looking Hessenberg process on an n x k block Q (Sec. 4.2).
 *
 * For j = 0..k-1:
 *   r   = first index of the entry of largest magnitude in column j;
 *   if |Q_rj| >= tol:  column j := column j / Q_rj   (so Q_rj becomes 1),
 *                      piv[j] = r, keep[j] = 1, U_jj = old Q_rj, and every
 *                      trailing column i > j is updated as
 *                      Q_:i := Q_:i - Q_ri * Q_:j   with U_ji = Q_ri;
 *   else               keep[j] = 0, piv[j] = -1 and nothing else changes.
 * Each elementwise update is one fused multiply-add (one rounding), written
 * as fma(-Q_ri, Q_tj, Q_ti).
 *
 * The entries of rows already chosen as pivots become exact zeros in every
 * later column, so searching the whole column is the same as searching the
 * rows not yet used.  On return the kept columns of Q equal P^T L of the
 * row-pivoted LU factorisation of the input (Sec. 4.2, last paragraphs),
 * and input = Q(:,keep) * U(keep,:) up to rounding.
 * U (k x k, may be NULL) receives the multipliers; unset entries are 0.
 * Returns the number of kept columns.
 * ---------------------------------------------------------------------- */
int64_t orc_hessenberg_f64(int64_t n, int64_t k, double *Q, int64_t ldq,
                           double tol, int32_t *piv, int32_t *keep,
                           double *U, int64_t ldu)
{
    int64_t kept = 0;
    if (U)
        for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < k; ++i) U[IDX(i, j, ldu)] = 0.0;
    for (int64_t j = 0; j < k; ++j) {
        double *q = Q + IDX(0, j, ldq);
        int64_t r = 0;
        double best = fabs(q[0]);
        for (int64_t t = 1; t < n; ++t)
            if (fabs(q[t]) > best) { best = fabs(q[t]); r = t; }
        if (best >= tol && best > 0.0) {
            const double pivot = q[r];
            for (int64_t t = 0; t < n; ++t) q[t] = q[t] / pivot;
            piv[j] = (int32_t)r;
            keep[j] = 1;
            ++kept;
            if (U) U[IDX(j, j, ldu)] = pivot;
            for (int64_t i = j + 1; i < k; ++i) {
                double *qi = Q + IDX(0, i, ldq);
                const double wgt = qi[r];
                if (U) U[IDX(j, i, ldu)] = wgt;
                for (int64_t t = 0; t < n; ++t) qi[t] = fma(-wgt, q[t], qi[t]);
            }
        } else {
            keep[j] = 0;
            piv[j] = -1;
        }
    }
    return kept;
}

/* Same process, every quantity held and rounded in IEEE binary32 (FP32):
 * pivot search on FP32 magnitudes, correctly rounded FP32 division and
 * FP32 fused multiply-add.  U (may be NULL) is returned in FP32. */
int64_t orc_hessenberg_f32(int64_t n, int64_t k, float *Q, int64_t ldq,
                           float tol, int32_t *piv, int32_t *keep,
                           float *U, int64_t ldu)
{
    int64_t kept = 0;
    if (U)
        for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < k; ++i) U[IDX(i, j, ldu)] = 0.0f;
    for (int64_t j = 0; j < k; ++j) {
        float *q = Q + IDX(0, j, ldq);
        int64_t r = 0;
        float best = fabsf(q[0]);
        for (int64_t t = 1; t < n; ++t)
            if (fabsf(q[t]) > best) { best = fabsf(q[t]); r = t; }
        if (best >= tol && best > 0.0f) {
            const float pivot = q[r];
            for (int64_t t = 0; t < n; ++t) q[t] = q[t] / pivot;
            piv[j] = (int32_t)r;
            keep[j] = 1;
            ++kept;
            if (U) U[IDX(j, j, ldu)] = pivot;
            for (int64_t i = j + 1; i < k; ++i) {
                float *qi = Q + IDX(0, i, ldq);
                const float wgt = qi[r];
                if (U) U[IDX(j, i, ldu)] = wgt;
                for (int64_t t = 0; t < n; ++t) qi[t] = fmaf(-wgt, q[t], qi[t]);
            }
        } else {
            keep[j] = 0;
            piv[j] = -1;
        }
    }
    return kept;
}

/* ------------------------------------------------------------------------
 * x rounded to the nearest IEEE binary16 value, ties to even, returned as
 * FP32 (every binary16 value is an FP32 value).  binary16 has 11 significant
 * bits, normal numbers down to 2^-14 and subnormal multiples of 2^-24 below;
 * the largest finite value is 65504 = (2 - 2^-10) 2^15, and anything from
 * 65520 (the midpoint to 2^16, which ties to the even 2^16) up overflows to
 * infinity.  With |x| = f 2^e, f in [1/2, 1), a value in that binade is a
 * multiple of 2^(e-11) (of 2^-24 below the normal range); x / 2^q is exact
 * and is rounded to an integer by nearbyint in the default (nearest-even)
 * rounding mode.
 * ---------------------------------------------------------------------- */
float orc_round_binary16(float x)
{
    if (isnan(x) || isinf(x)) return x;
    const double a = fabs((double)x);
    if (a >= 65520.0) return copysignf(INFINITY, x);
    if (a == 0.0) return x;
    int e;
    (void)frexp(a, &e);
    int q = e - 11;
    if (q < -24) q = -24;
    const double r = nearbyint(ldexp(a, -q));
    return (float)copysign(ldexp(r, q), (double)x);
}

/* orc_round_binary16 applied to x[0..count-1] in place. */
void orc_round_binary16_array(int64_t count, float *x)
{
    for (int64_t i = 0; i < count; ++i) x[i] = orc_round_binary16(x[i]);
}

/* The Hessenberg process with binary16 storage and FP32 arithmetic (the
 * paper's FP16 runs compute in FP32 on FP16 data): as orc_hessenberg_f32,
 * but every value written back to Q (the divided column and each updated
 * entry) is rounded to binary16 first.  Q holds binary16 values on entry.
 * U (may be NULL) receives the multipliers as read from Q. */
int64_t orc_hessenberg_f16s(int64_t n, int64_t k, float *Q, int64_t ldq,
                            float tol, int32_t *piv, int32_t *keep,
                            float *U, int64_t ldu)
{
    int64_t kept = 0;
    if (U)
        for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < k; ++i) U[IDX(i, j, ldu)] = 0.0f;
    for (int64_t j = 0; j < k; ++j) {
        float *q = Q + IDX(0, j, ldq);
        int64_t r = 0;
        float best = fabsf(q[0]);
        for (int64_t t = 1; t < n; ++t)
            if (fabsf(q[t]) > best) { best = fabsf(q[t]); r = t; }
        if (best >= tol && best > 0.0f) {
            const float pivot = q[r];
            for (int64_t t = 0; t < n; ++t) q[t] = orc_round_binary16(q[t] / pivot);
            piv[j] = (int32_t)r;
            keep[j] = 1;
            ++kept;
            if (U) U[IDX(j, j, ldu)] = pivot;
            for (int64_t i = j + 1; i < k; ++i) {
                float *qi = Q + IDX(0, i, ldq);
                const float wgt = qi[r];
                if (U) U[IDX(j, i, ldu)] = wgt;
                for (int64_t t = 0; t < n; ++t) qi[t] = orc_round_binary16(fmaf(-wgt, q[t], qi[t]));
            }
        } else {
            keep[j] = 0;
            piv[j] = -1;
        }
    }
    return kept;
}

/* ------------------------------------------------------------------------
 * Y = A X for an n_rows x n_cols CSR matrix (0-based row_ptr/col_idx) and
 * an n_cols x b block X.  Each Y_ij is the sum over the stored entries of
 * row i in storage order.
 * ---------------------------------------------------------------------- */
void orc_csr_mm(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                const double *val, int64_t b, const double *X, int64_t ldx,
                double *Y, int64_t ldy)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        for (int64_t j = 0; j < b; ++j) {
            double s = 0.0;
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                s += val[e] * X[IDX(col_idx[e], j, ldx)];
            Y[IDX(i, j, ldy)] = s;
        }
    }
}
