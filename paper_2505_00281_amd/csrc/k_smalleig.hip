// k_smalleig.hip -- the small FP64 problems of the projection step, on the
// GPU in one workgroup (Sec. 4, mixed-precision plan: the projected pencil
// is promoted to and solved in FP64).
//
//   pencil_eig   H y = theta G y (eq. (geig)): Cholesky G = L L^T, symmetric
//                eigen-decomposition of C = L^{-1} H L^{-T}, Y = L^{-T} Z.
//                If G is not numerically positive definite, G itself is
//                diagonalised first and its negligible directions are
//                dropped (G-eigen truncation).
//   svd_pencil   the augmented pencil of Sec. 3.2 via block Cholesky:
//                C = L_U^{-1} B L_V^{-T}; the positive eigenvalues of
//                [0 C; C^T 0] are the singular values, with unit eigenvectors
//                [u; v] / sqrt(2); y = L_U^{-T} u / sqrt(2),
//                z = L_V^{-T} v / sqrt(2) meet [y; z]^T M [y; z] = 1.  The
//                SVD of C comes from one-sided Jacobi (relative accuracy of
//                the singular values; one or two sweeps once C is nearly
//                diagonal, as it is for a converging subspace).
//
// Symmetric eigen-decomposition, organised for one 1024-thread workgroup:
//   1. Householder reduction to tridiagonal form T = Q^T C Q (the matrix in
//      LDS when it fits): per column one reflector H = I - beta v v^T, the
//      symmetric rank-2 update C22 -= v w^T + w v^T with
//      w = p - (beta/2)(v^T p) v, p = beta C22 v.
//   2. Eigenvalues of T by Sturm-count multisection: 8 lanes per eigenvalue
//      probe 7 interior points of its bracket per step (3 bits per step,
//      19 steps: the bracket shrinks below 2^-55 of the Gershgorin width).
//   3. Eigenvectors of T by inverse iteration (row-pivoted tridiagonal LU,
//      three solves), with modified Gram-Schmidt inside clusters of nearly
//      equal eigenvalues so degenerate pairs stay independent.
//   4. Z = Q Z_T by applying the reflectors in reverse order.
#include <set>
#include <type_traits>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

constexpr int SE_THREADS = 1024;
constexpr int SE_LDS_MAX_N = 120;  // C (n x n FP64) kept in LDS up to this size

__device__ double block_sum(double v, double *red) {
    v = wave_sum_f64(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += red[i];
    __syncthreads();
    return r;
}

__device__ double block_maxabs(double v, double *red) {
    v = fabs(v);
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r = fmax(r, red[i]);
    __syncthreads();
    return r;
}

struct EigWork {
    double *Vh;    // n x n: reflector j in column j, rows j+1..n-1
    double *beta;  // n
    double *d;     // n   diagonal of T
    double *e;     // n   off-diagonal of T (e[k] couples k and k+1)
    double *e2;    // n   e^2
    double *p;     // n
    double *w;     // n
    double *lam;   // n   eigenvalues of T, ascending
    double *scr;   // 6 n per eigenvector (inverse iteration)
    int *cstart;   // n   cluster start flags
};

// ---------------------------------------------------------------- step 1
// C (n x n, column-major, full symmetric storage) is overwritten.
__device__ void tridiagonalize(double *C, int n, EigWork &wk, double *red) {
    const int t = threadIdx.x, T = blockDim.x;
    const int wave = t >> 6, lane = t & 63, nw = T >> 6;
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;
        double s = 0.0;
        for (int i = j + 1 + t; i < n; i += T) s += C[i + j * n] * C[i + j * n];
        s = block_sum(s, red);
        const double x0 = C[(j + 1) + j * n];
        const double alpha = (s > 0.0) ? -copysign(sqrt(s), x0) : 0.0;
        const double beta = (s > 0.0) ? 1.0 / (alpha * (alpha - x0)) : 0.0;
        double *v = wk.Vh + (int64_t)j * n;
        for (int i = j + 1 + t; i < n; i += T) v[i] = (i == j + 1) ? x0 - alpha : C[i + j * n];
        if (t == 0) {
            wk.beta[j] = beta;
            wk.d[j] = C[j + j * n];
            wk.e[j] = (s > 0.0) ? alpha : x0;
        }
        __syncthreads();
        if (beta == 0.0) continue;  // column already reduced
        // p = beta C22 v, one wavefront per row (rows of C22 read contiguously
        // as columns, C being symmetric)
        for (int r = j + 1 + wave; r < n; r += nw) {
            double acc = 0.0;
            for (int c = j + 1 + lane; c < n; c += 64) acc += C[c + r * n] * v[c];
            acc = wave_sum_f64(acc);
            if (lane == 0) wk.p[r] = beta * acc;
        }
        __syncthreads();
        double vp = 0.0;
        for (int i = j + 1 + t; i < n; i += T) vp += v[i] * wk.p[i];
        vp = block_sum(vp, red);
        const double K = 0.5 * beta * vp;
        for (int i = j + 1 + t; i < n; i += T) wk.w[i] = wk.p[i] - K * v[i];
        __syncthreads();
        // C22 -= v w^T + w v^T on the lower triangle, mirrored (exactly symmetric)
        for (int e = t; e < m * m; e += T) {
            const int r = j + 1 + e % m, c = j + 1 + e / m;
            if (r >= c) {
                const double upd = v[r] * wk.w[c] + wk.w[r] * v[c];
                const double val = C[r + c * n] - upd;
                C[r + c * n] = val;
                C[c + r * n] = val;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        if (n >= 2) {
            wk.d[n - 2] = C[(n - 2) + (n - 2) * n];
            wk.e[n - 2] = C[(n - 1) + (n - 2) * n];
            wk.beta[n - 2] = 0.0;
        }
        wk.d[n - 1] = C[(n - 1) + (n - 1) * n];
        wk.beta[n - 1] = 0.0;
        wk.e[n - 1] = 0.0;
    }
    __syncthreads();
    for (int i = t; i < n; i += T) wk.e2[i] = wk.e[i] * wk.e[i];
    __syncthreads();
}

// ---------------------------------------------------------------- step 2
// Number of eigenvalues of the tridiagonal (d, e) below x.  It equals the
// number of sign changes in the leading principal minors p_k of T - x I,
// p_k = (d_k - x) p_{k-1} - e_{k-1}^2 p_{k-2}, i.e. the number of negative
// pivots p_k / p_{k-1} of its LDL^T factorisation.  The minors are carried
// as (p_{k-1}, p_k) 2^-E, renormalised every step by the exponent of p_k
// (exact, signs kept), so each step costs one fused multiply-add on the
// dependency chain instead of a division.  A minor below 2^-901 of its
// predecessor is replaced by that size with the opposite sign (a tiny
// negative pivot, as the pivot floor of the ratio form).
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int n, double x,
                                           double pivmin) {
    (void)pivmin;
    double pm = 1.0;
    double p = d[0] - x;
    if (fabs(p) < 0x1p-901) p = -0x1p-901;
    int c = p < 0.0 ? 1 : 0;
    {
        const int ex = __builtin_amdgcn_frexp_exp(p);
        p = __builtin_amdgcn_frexp_mant(p);
        pm = __builtin_ldexp(pm, -ex);
    }
    // unrolled so that the loads of d and e2 run ahead of the dependency chain
#pragma unroll 8
    for (int k = 1; k < n; ++k) {
        double pn = fma(d[k] - x, p, -(e2[k - 1] * pm));
        if (fabs(pn) < 0x1p-901) pn = p < 0.0 ? 0x1p-901 : -0x1p-901;
        c += ((pn < 0.0) != (p < 0.0)) ? 1 : 0;
        const int ex = __builtin_amdgcn_frexp_exp(pn);
        pm = __builtin_ldexp(p, -ex);
        p = __builtin_amdgcn_frexp_mant(pn);
    }
    return c;
}

__device__ void bisect_ptr(int n, const double *dg, const double *eo, const double *eo2,
                           double *lamo) {
    const int t = threadIdx.x, T = blockDim.x;
    const int lane = t & 63, grp = lane >> 3, sub = lane & 7;
    // Gershgorin interval and the pivot floor
    double lo = INFINITY, hi = -INFINITY, emax = 0.0;
    for (int k = t; k < n; k += T) {
        const double off = (k > 0 ? fabs(eo[k - 1]) : 0.0) + (k + 1 < n ? fabs(eo[k]) : 0.0);
        lo = fmin(lo, dg[k] - off);
        hi = fmax(hi, dg[k] + off);
        if (k + 1 < n) emax = fmax(emax, eo2[k]);
    }
    __shared__ double s_lo[16], s_hi[16], s_em[16];
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
        emax = fmax(emax, __shfl_xor(emax, o, 64));
    }
    if (lane == 0) {
        s_lo[t >> 6] = lo;
        s_hi[t >> 6] = hi;
        s_em[t >> 6] = emax;
    }
    __syncthreads();
    lo = s_lo[0];
    hi = s_hi[0];
    emax = s_em[0];
    for (int i = 1; i < (T >> 6); ++i) {
        lo = fmin(lo, s_lo[i]);
        hi = fmax(hi, s_hi[i]);
        emax = fmax(emax, s_em[i]);
    }
    __syncthreads();
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = 0x1.0p-1000 * fmax(1.0, emax);
    lo -= 4.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin;
    hi += 4.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin;
    const int per_pass = (T >> 6) * 8;
    for (int base = 0; base < n; base += per_pass) {
        const int idx = base + (t >> 6) * 8 + grp;  // eigenvalue handled by this lane group
        const bool active = idx < n;
        double a = lo, b = hi;
        for (int it = 0; it < 19; ++it) {  // 3 bits each: 57 bits of the Gershgorin interval
            const double x = a + (b - a) * (double)(sub + 1) * 0.125;
            int c = 0;
            if (active && sub < 7) c = sturm_count(dg, eo2, n, x, pivmin);
            const bool flag = active && sub < 7 && c > idx;
            const unsigned long long bal = __ballot(flag);
            const unsigned bits = (unsigned)((bal >> (grp * 8)) & 0x7Full);
            // first probe with more than idx eigenvalues below it
            const int s = bits ? __builtin_ctz(bits) : 7;
            const double na = (s == 0) ? a : a + (b - a) * (double)s * 0.125;
            const double nb = (s == 7) ? b : a + (b - a) * (double)(s + 1) * 0.125;
            a = na;
            b = nb;
        }
        if (active && sub == 0) lamo[idx] = 0.5 * (a + b);
    }
    __syncthreads();
}

__device__ void bisect_all(int n, EigWork &wk, double *red) {
    (void)red;
    bisect_ptr(n, wk.d, wk.e, wk.e2, wk.lam);
}

// ---------------------------------------------------------------- step 3
// Solves (T - lam I) x = x in place using the factorisation in f (computed
// by tri_factor); f layout: dl[n], dd[n], du[n], du2[n], piv[n] (as double).
__device__ void tri_factor(const double *d, const double *e, int n, double lam, double tiny,
                           double *f) {
    double *dl = f, *dd = f + n, *du = f + 2 * n, *du2 = f + 3 * n, *pv = f + 4 * n;
    for (int k = 0; k < n; ++k) {
        dd[k] = d[k] - lam;
        du[k] = (k + 1 < n) ? e[k] : 0.0;
        dl[k] = (k + 1 < n) ? e[k] : 0.0;
        du2[k] = 0.0;
        pv[k] = 0.0;
    }
    for (int k = 0; k + 1 < n; ++k) {
        const double sub = dl[k];
        if (fabs(dd[k]) >= fabs(sub)) {
            const double piv = dd[k] != 0.0 ? dd[k] : tiny;
            dd[k] = piv;
            const double mlt = sub / piv;
            dl[k] = mlt;
            dd[k + 1] -= mlt * du[k];
        } else {
            // swap rows k and k+1
            const double mlt = dd[k] / sub;
            dl[k] = mlt;
            dd[k] = sub;
            const double t0 = du[k];
            du[k] = dd[k + 1];
            dd[k + 1] = t0 - mlt * dd[k + 1];
            if (k + 2 < n) {
                du2[k] = du[k + 1];
                du[k + 1] = -mlt * du2[k];
            }
            pv[k] = 1.0;
        }
    }
    if (dd[n - 1] == 0.0) dd[n - 1] = tiny;
}

__device__ void tri_solve(const double *f, int n, double *x) {
    const double *dl = f, *dd = f + n, *du = f + 2 * n, *du2 = f + 3 * n, *pv = f + 4 * n;
    for (int k = 0; k + 1 < n; ++k) {
        if (pv[k] != 0.0) {
            const double t0 = x[k];
            x[k] = x[k + 1];
            x[k + 1] = t0 - dl[k] * x[k + 1];
        } else {
            x[k + 1] -= dl[k] * x[k];
        }
    }
    x[n - 1] /= dd[n - 1];
    if (n >= 2) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / dd[n - 2];
    for (int k = n - 3; k >= 0; --k) x[k] = (x[k] - du[k] * x[k + 1] - du2[k] * x[k + 2]) / dd[k];
}

__device__ void inverse_iteration(int n, EigWork &wk, double *Zt, double *red) {
    const int t = threadIdx.x, T = blockDim.x;
    double tn = 0.0;
    for (int i = t; i < n; i += T) tn = fmax(tn, fabs(wk.lam[i]));
    for (int k = t; k < n; k += T) tn = fmax(tn, fabs(wk.d[k]) + fabs(wk.e[k]));
    tn = block_maxabs(tn, red);
    const double ortol = 1e-7 * tn;
    const double tiny = 2.220446049250313e-16 * fmax(tn, 1e-300);
    for (int i = t; i < n; i += T) wk.cstart[i] = (i == 0 || wk.lam[i] - wk.lam[i - 1] > ortol) ? 1 : 0;
    __syncthreads();
    for (int i0 = t; i0 < n; i0 += T) {
        if (!wk.cstart[i0]) continue;
        int i1 = i0 + 1;
        while (i1 < n && !wk.cstart[i1]) ++i1;
        double *f = wk.scr + (int64_t)i0 * 6 * n;
        for (int i = i0; i < i1; ++i) {
            double *x = Zt + (int64_t)i * n;
            // perturb a repeated eigenvalue slightly so the factorisation differs
            const double lam = wk.lam[i] + (double)(i - i0) * 4.0 * tiny;
            tri_factor(wk.d, wk.e, n, lam, tiny, f);
            for (int k = 0; k < n; ++k) {
                // deterministic start vector in [-1, 1]
                uint32_t h = (uint32_t)(k * 2654435761u) ^ (uint32_t)(i * 40503u + 0x9E37u);
                h ^= h >> 15;
                h *= 0x2C1B3C6Du;
                h ^= h >> 12;
                x[k] = 0.5 + (double)(h & 0xFFFF) * (1.0 / 65536.0);
            }
            for (int it = 0; it < 3; ++it) {
                tri_solve(f, n, x);
                // orthogonalise against the earlier vectors of the cluster
                for (int q = i0; q < i; ++q) {
                    const double *y = Zt + (int64_t)q * n;
                    double s = 0.0;
                    for (int k = 0; k < n; ++k) s += y[k] * x[k];
                    for (int k = 0; k < n; ++k) x[k] -= s * y[k];
                }
                double mx = 0.0;
                for (int k = 0; k < n; ++k) mx = fmax(mx, fabs(x[k]));
                const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
                double nn = 0.0;
                for (int k = 0; k < n; ++k) {
                    x[k] *= inv;
                    nn += x[k] * x[k];
                }
                const double r = 1.0 / sqrt(nn);
                for (int k = 0; k < n; ++k) x[k] *= r;
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- step 4
__device__ void back_transform(int n, EigWork &wk, double *Z) {
    const int t = threadIdx.x, T = blockDim.x;
    const int lane = t & 63;
    // 8 lanes per column
    const int grp = t >> 3, sub = t & 7, ngrp = T >> 3;
    for (int j = n - 3; j >= 0; --j) {
        const double beta = wk.beta[j];
        if (beta == 0.0) continue;
        const double *v = wk.Vh + (int64_t)j * n;
        for (int c0 = 0; c0 < n; c0 += ngrp) {
            const int c = c0 + grp;
            double s = 0.0;
            if (c < n)
                for (int i = j + 1 + sub; i < n; i += 8) s += v[i] * Z[i + (int64_t)c * n];
            s += __shfl_xor(s, 1, 64);
            s += __shfl_xor(s, 2, 64);
            s += __shfl_xor(s, 4, 64);
            s *= beta;
            if (c < n)
                for (int i = j + 1 + sub; i < n; i += 8) Z[i + (int64_t)c * n] -= s * v[i];
        }
        (void)lane;
        __syncthreads();
    }
}

// C (n x n symmetric, destroyed) -> ascending eigenvalues w, eigenvectors Z.
__device__ void sym_eig(double *C, int n, double *w, double *Z, EigWork &wk, double *red) {
    const int t = threadIdx.x, T = blockDim.x;
    if (n == 1) {
        if (t == 0) {
            w[0] = C[0];
            Z[0] = 1.0;
        }
        __syncthreads();
        return;
    }
    tridiagonalize(C, n, wk, red);
    bisect_all(n, wk, red);
    inverse_iteration(n, wk, Z, red);
    back_transform(n, wk, Z);
    for (int i = t; i < n; i += T) w[i] = wk.lam[i];
    __syncthreads();
}

// In-place lower Cholesky (right-looking) of the n x n matrix A (ld n);
// returns false if a pivot is not positive.
__device__ double chol_floor(const double *A, int ld, int n);

// rel_floor: 1 applies the 1e-12 pivot floor (pencil), 0 only requires
// positive pivots (the SVD pencil, whose caller reports failure instead of
// falling back).
__device__ bool cholesky(double *A, int n, int rel_floor) {
    const int t = threadIdx.x, T = blockDim.x;
    const double floor_ = rel_floor ? chol_floor(A, n, n) : 0.0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double d = A[j + j * n];
        if (!(d > floor_)) {
            __syncthreads();
            return false;
        }
        const double l = sqrt(d);
        __syncthreads();
        for (int i = j + t; i < n; i += T) A[i + j * n] = (i == j) ? l : A[i + j * n] / l;
        __syncthreads();
        const int rem = n - j - 1;
        if (rem <= 256 && T == 1024) {
            // thread (tr, tc): trailing rows tr + 32 p, columns tc + 32 q; the
            // thread's entries of column j in registers, and two columns'
            // loads issued before their stores (independent, in flight together)
            const int tr = t & 31, tc = t >> 5;
            double lj[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int i0 = tr + 32 * p;
                lj[p] = i0 < rem ? A[(j + 1 + i0) + (int64_t)j * n] : 0.0;
            }
            for (int k0 = tc; k0 < rem; k0 += 64) {
                const int k1 = k0 + 32;
                const double lk0 = A[(j + 1 + k0) + (int64_t)j * n];
                const double lk1 = k1 < rem ? A[(j + 1 + k1) + (int64_t)j * n] : 0.0;
                double x0[8], x1[8];
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int i0 = tr + 32 * p;
                    x0[p] = (i0 < rem && i0 >= k0) ? A[(j + 1 + i0) + (int64_t)(j + 1 + k0) * n] : 0.0;
                    x1[p] = (i0 < rem && i0 >= k1) ? A[(j + 1 + i0) + (int64_t)(j + 1 + k1) * n] : 0.0;
                }
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int i0 = tr + 32 * p;
                    if (i0 < rem && i0 >= k0) A[(j + 1 + i0) + (int64_t)(j + 1 + k0) * n] = x0[p] - lj[p] * lk0;
                    if (i0 < rem && i0 >= k1) A[(j + 1 + i0) + (int64_t)(j + 1 + k1) * n] = x1[p] - lj[p] * lk1;
                }
            }
        } else {
            for (int e = t; e < rem * rem; e += T) {
                const int ii = j + 1 + e % rem, kk = j + 1 + e / rem;
                if (kk <= ii) A[ii + kk * n] -= A[ii + j * n] * A[kk + j * n];
            }
        }
        __syncthreads();
    }
    for (int e = t; e < n * n; e += T) {
        const int i = e % n, j = e / n;
        if (i < j) A[e] = 0.0;
    }
    __syncthreads();
    return true;
}

// X <- L^{-1} X for lower-triangular L (n x n) and X (n x m, ld n).
// Row by row: the update of rows below uses all threads.
__device__ void trsm_lower(const double *L, int n, double *X, int m) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int i = 0; i < n; ++i) {
        const double lii = L[i + i * n];
        for (int c = t; c < m; c += T) X[i + (int64_t)c * n] /= lii;
        __syncthreads();
        const int rem = n - i - 1;
        for (int e = t; e < rem * m; e += T) {
            const int r = i + 1 + e % rem, c = e / rem;
            X[r + (int64_t)c * n] -= L[r + i * n] * X[i + (int64_t)c * n];
        }
        __syncthreads();
    }
}

// X <- L^{-T} X (back substitution with L^T upper triangular).
__device__ void trsm_lower_t(const double *L, int n, double *X, int m) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int i = n - 1; i >= 0; --i) {
        const double lii = L[i + i * n];
        for (int c = t; c < m; c += T) X[i + (int64_t)c * n] /= lii;
        __syncthreads();
        for (int e = t; e < i * m; e += T) {
            const int r = e % i, c = e / i;  // rows above i: x_r -= L[i, r] x_i
            X[r + (int64_t)c * n] -= L[i + r * n] * X[i + (int64_t)c * n];
        }
        __syncthreads();
    }
}

__device__ void transpose_sq(double *A, int n) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int e = t; e < n * n; e += T) {
        const int i = e % n, j = e / n;
        if (i < j) {
            const double x = A[i + j * n];
            A[i + j * n] = A[j + i * n];
            A[j + i * n] = x;
        }
    }
    __syncthreads();
}

// ord[rank] = i for values v (descending if desc), ties by index.
__device__ void sort_order(const double *v, int n, bool desc, int *ord) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int i = t; i < n; i += T) {
        int rank = 0;
        const double vi = v[i];
        for (int j = 0; j < n; ++j) {
            const double vj = v[j];
            const bool before = desc ? (vj > vi || (vj == vi && j < i)) : (vj < vi || (vj == vi && j < i));
            rank += before ? 1 : 0;
        }
        ord[rank] = i;
    }
    __syncthreads();
}

struct PencilWork {
    double *C, *Z, *L, *T;  // n x n each (C may be replaced by an LDS copy)
    double *w;              // n
    int *ord, *flag;
    EigWork ek;
};

__global__ __launch_bounds__(SE_THREADS) void k_pencil(const double *__restrict__ H,
                                                       const double *__restrict__ G, int n,
                                                       int which_smallest, double *__restrict__ theta,
                                                       double *__restrict__ Y, PencilWork w,
                                                       int *status, int use_lds, int skip_if_done) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    __shared__ double red[16];
    const int t = threadIdx.x, T = blockDim.x;
    // after the fast path: nothing to do when it factorised G
    if (skip_if_done && status[0] == 0) return;
    __syncthreads();
    double *C = use_lds ? smem : w.C;
    for (int e = t; e < n * n; e += T) {
        const int i = e % n, j = e / n;
        w.L[e] = 0.5 * (G[i + j * n] + G[j + i * n]);
        C[e] = 0.5 * (H[i + j * n] + H[j + i * n]);
    }
    __syncthreads();
    int rank = n;
    const bool pd = cholesky(w.L, n, 1);
    if (pd) {
        // C <- L^{-1} C L^{-T}
        trsm_lower(w.L, n, C, n);
        transpose_sq(C, n);
        trsm_lower(w.L, n, C, n);
        for (int e = t; e < n * n; e += T) {
            const int i = e % n, j = e / n;
            if (i < j) {
                const double s = 0.5 * (C[i + j * n] + C[j + i * n]);
                C[i + j * n] = s;
                C[j + i * n] = s;
            }
        }
        __syncthreads();
        sym_eig(C, n, w.w, w.Z, w.ek, red);
        trsm_lower_t(w.L, n, w.Z, n);  // Z <- L^{-T} Z
    } else {
        // G-eigen truncation: G = U D U^T, keep d_i > 1e-14 max d
        for (int e = t; e < n * n; e += T) {
            const int i = e % n, j = e / n;
            w.L[e] = 0.5 * (G[i + j * n] + G[j + i * n]);
        }
        __syncthreads();
        sym_eig(w.L, n, w.w, w.T, w.ek, red);  // ascending d_i in w.w, U in w.T
        __shared__ double dmax;
        if (t == 0) {
            double m = 0.0;
            for (int i = 0; i < n; ++i) m = fmax(m, w.w[i]);
            dmax = m;
            int c = 0;
            for (int i = 0; i < n; ++i)
                if (w.w[i] > 1e-14 * m) w.ord[c++] = i;
            w.flag[0] = c;
        }
        __syncthreads();
        rank = w.flag[0];
        // Tk (n x rank) = U_i / sqrt(d_i) for kept i, into Z
        for (int e = t; e < n * rank; e += T) {
            const int row = e % n, c = e / n;
            const int i = w.ord[c];
            w.Z[row + c * n] = w.T[row + i * n] / sqrt(w.w[i]);
        }
        __syncthreads();
        // HT = H_sym Tk into T (n x rank)
        for (int e = t; e < n * rank; e += T) {
            const int row = e % n, c = e / n;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += C[row + k * n] * w.Z[k + c * n];
            w.T[row + c * n] = s;
        }
        __syncthreads();
        // C_r = Tk^T HT (rank x rank, ld rank) into L
        for (int e = t; e < rank * rank; e += T) {
            const int i = e % rank, j = e / rank;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += w.Z[k + i * n] * w.T[k + j * n];
            w.L[i + j * rank] = s;
        }
        __syncthreads();
        for (int e = t; e < rank * rank; e += T) {
            const int i = e % rank, j = e / rank;
            if (i < j) {
                const double s = 0.5 * (w.L[i + j * rank] + w.L[j + i * rank]);
                w.L[i + j * rank] = s;
                w.L[j + i * rank] = s;
            }
        }
        __syncthreads();
        sym_eig(w.L, rank, w.w, w.T, w.ek, red);  // eigvecs in T (ld rank)
        // Y_r = Tk Zr (n x rank) -> C (ld n), then back to Z
        for (int e = t; e < n * rank; e += T) {
            const int row = e % n, c = e / n;
            double s = 0.0;
            for (int k = 0; k < rank; ++k) s += w.Z[row + k * n] * w.T[k + c * rank];
            C[row + c * n] = s;
        }
        __syncthreads();
        for (int e = t; e < n * rank; e += T) w.Z[e] = C[e];
        __syncthreads();
        if (t == 0) *status = 1;
        (void)dmax;
    }
    // order the `rank` values; columns beyond rank are zero
    sort_order(w.w, rank, !which_smallest, w.ord);
    for (int i = t; i < n; i += T) theta[i] = (i < rank) ? w.w[w.ord[i]] : 0.0;
    for (int e = t; e < n * n; e += T) {
        const int row = e % n, c = e / n;
        Y[e] = (c < rank) ? w.Z[row + w.ord[c] * n] : 0.0;
    }
    if (t == 0) {
        w.flag[1] = rank;
        status[1] = rank;
    }
}

// One-sided (Hestenes) Jacobi SVD of M (m x q, column-major, m >= q,
// m <= 1024): the columns are rotated in pairs until every pair is
// orthogonal to tol, so that M V = U Sigma with orthogonal V (q x q,
// accumulated here).  Pairs follow a round-robin tournament (every pair
// once per sweep, q/2 disjoint pairs per step, a half wavefront per pair
// with the lanes over rows); a sweep without a rotation ends the iteration.  The
// singular values come out with high relative accuracy, and a nearly
// diagonal start (the projected matrix of a converging subspace) needs one
// or two sweeps; a sweep whose rotations were all tiny is the last.
// Returns the number of sweeps.
// One step of the tournament: pair pr goes to the 32-lane group pr mod 32
// (a half wavefront; the lanes hold rows l + 32 u), so 32 pairs are in
// flight at once.

__device__ double half_wave_sum(double v);  // defined with the DPP helpers below

template <int MAXR>
__device__ void jacobi_rotate_pairs(double *M, int m, double *V, int q, int mm, int step, double tol, int *s_rot,
                                    unsigned *s_cmax) {
    const int t = threadIdx.x, T = blockDim.x, grp = t >> 5, gl = t & 31, ng = T >> 5;
    auto pos = [&](int k) { return k == 0 ? 0 : ((k - 1 + step) % (mm - 1)) + 1; };
    for (int pr = grp; pr < mm / 2; pr += ng) {
        int i = pos(pr), j = pos(mm - 1 - pr);
        if (i > j) {
            const int x = i;
            i = j;
            j = x;
        }
        if (j >= q) continue;  // the dummy slot of an odd q
        double *gi = M + (int64_t)i * m, *gj = M + (int64_t)j * m;
        double *vi = V + (int64_t)i * q, *vj = V + (int64_t)j * q;
        double a[MAXR], b[MAXR], c[MAXR], d[MAXR];
#pragma unroll
        for (int u = 0; u < MAXR; ++u) {
            const int r = gl + 32 * u;
            a[u] = r < m ? gi[r] : 0.0;
            b[u] = r < m ? gj[r] : 0.0;
            c[u] = r < q ? vi[r] : 0.0;
            d[u] = r < q ? vj[r] : 0.0;
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < MAXR; ++u) {
            al += a[u] * a[u];
            be += b[u] * b[u];
            ga += a[u] * b[u];
        }
        al = half_wave_sum(al);
        be = half_wave_sum(be);
        ga = half_wave_sum(ga);
        // the largest cosine of the sweep (as FP32 bits: positive values
        // order as unsigned integers)
        const double nab = sqrt(al * be);
        if (gl == 0 && nab > 0.0) atomicMax(s_cmax, __float_as_uint((float)(fabs(ga) / nab)));
        if (!(fabs(ga) > tol * nab)) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
        for (int u = 0; u < MAXR; ++u) {
            const int r = gl + 32 * u;
            if (r < m) {
                gi[r] = cs * a[u] - sn * b[u];
                gj[r] = sn * a[u] + cs * b[u];
            }
            if (r < q) {
                vi[r] = cs * c[u] - sn * d[u];
                vj[r] = sn * c[u] + cs * d[u];
            }
        }
        if (gl == 0) atomicAdd(s_rot, 1);
    }
}

// MAXR = 0 picks the register depth at run time (8 for m <= 256, else 32)
template <int MAXR = 0>
__device__ int jacobi_svd(double *M, int m, int q, double *V, int *s_rot) {
    __shared__ unsigned s_cmax;
    const int t = threadIdx.x, T = blockDim.x;
    for (int e = t; e < q * q; e += T) V[e] = (e % q == e / q) ? 1.0 : 0.0;
    const int mm = q + (q & 1);
    const double tol = 0x1p-52 * sqrt((double)m);
    // a sweep whose largest cosine was below a tenth of sqrt(tol) leaves
    // cosines of order its square (quadratic convergence): no further sweep
    const float cfin = (float)(0.1 * sqrt(tol));
    int sweep = 0;
    __syncthreads();
    for (; sweep < 40; ++sweep) {
        if (t == 0) {
            *s_rot = 0;
            s_cmax = 0u;
        }
        __syncthreads();
        for (int step = 0; step < mm - 1; ++step) {
            if (MAXR == 8 || (MAXR == 0 && m <= 256))
                jacobi_rotate_pairs<8>(M, m, V, q, mm, step, tol, s_rot, &s_cmax);
            else
                jacobi_rotate_pairs<32>(M, m, V, q, mm, step, tol, s_rot, &s_cmax);
            __syncthreads();
        }
        const int nrot = *s_rot;
        const float cmax = __uint_as_float(s_cmax);
        __syncthreads();
        if (nrot == 0 || cmax <= cfin) break;
    }
    return sweep + 1;
}

__global__ __launch_bounds__(SE_THREADS) void k_svd_pencil(const double *__restrict__ B, int k1,
                                                           int k2, const double *__restrict__ MU,
                                                           const double *__restrict__ MV,
                                                           double *__restrict__ sigma,
                                                           double *__restrict__ Yo,
                                                           double *__restrict__ Zo, PencilWork w,
                                                           double *LU, double *LV, int *status) {
    __shared__ double red[16];
    const int t = threadIdx.x, T = blockDim.x;
    const int N = k1 + k2;
    for (int e = t; e < k1 * k1; e += T) {
        const int i = e % k1, j = e / k1;
        LU[e] = 0.5 * (MU[i + j * k1] + MU[j + i * k1]);
    }
    for (int e = t; e < k2 * k2; e += T) {
        const int i = e % k2, j = e / k2;
        LV[e] = 0.5 * (MV[i + j * k2] + MV[j + i * k2]);
    }
    __syncthreads();
    if (!cholesky(LU, k1, 0)) {
        if (t == 0) *status = 3;
        return;
    }
    if (!cholesky(LV, k2, 0)) {
        if (t == 0) *status = 4;
        return;
    }
    // Cm = LU^{-1} B LV^{-T}  (k1 x k2): T = B^T (k2 x k1), T <- LV^{-1} T,
    // transpose -> k1 x k2, <- LU^{-1}
    for (int e = t; e < k1 * k2; e += T) {
        const int i = e % k2, j = e / k2;  // T[i + j*k2] = B[j + i*k1]
        w.T[i + j * k2] = B[j + i * k1];
    }
    __syncthreads();
    trsm_lower(LV, k2, w.T, k1);
    for (int e = t; e < k1 * k2; e += T) {
        const int i = e % k1, j = e / k1;  // Cm[i + j*k1] = T[j + i*k2]
        w.L[i + j * k1] = w.T[j + i * k2];
    }
    __syncthreads();
    trsm_lower(LU, k1, w.L, k2);
    // SVD of Cm = U Sigma V^T (the positive eigenpairs of [0 Cm; Cm^T 0] are
    // (sigma, [u; v] / sqrt 2)) by one-sided Jacobi on the taller of Cm and
    // Cm^T
    const bool swap = k1 < k2;
    const int m = swap ? k2 : k1, q = swap ? k1 : k2;
    double *M = w.L;
    if (swap) {
        for (int e = t; e < k1 * k2; e += T) {
            const int i = e % k2, j = e / k2;  // M[i + j*k2] = Cm[j + i*k1]
            w.T[i + j * k2] = w.L[j + i * k1];
        }
        M = w.T;
    }
    __shared__ int s_rot;
    (void)jacobi_svd(M, m, q, w.Z, &s_rot);
    // column norms = singular values, descending
    for (int j = t; j < q; j += T) {
        double s2 = 0.0;
        for (int r = 0; r < m; ++r) s2 += M[r + (int64_t)j * m] * M[r + (int64_t)j * m];
        w.w[j] = sqrt(s2);
    }
    __syncthreads();
    sort_order(w.w, q, true, w.ord);
    const int r = q;
    for (int c = t; c < r; c += T) sigma[c] = w.w[w.ord[c]];
    // left singular vectors u = M_j / sigma_j (length m), right v = V_j
    // (length q); [y; z] = [u; v] / sqrt 2 before the L^{-T} transforms
    const double h = 0.70710678118654752440;
    for (int e = t; e < m * r; e += T) {
        const int row = e % m, c = e / m;
        const int j = w.ord[c];
        const double sj = w.w[j];
        const double uv = sj > 0.0 ? M[row + (int64_t)j * m] / sj * h : 0.0;
        if (swap)
            Zo[row + c * k2] = uv;
        else
            Yo[row + c * k1] = uv;
    }
    for (int e = t; e < q * r; e += T) {
        const int row = e % q, c = e / q;
        const double vv = w.Z[row + (int64_t)w.ord[c] * q] * h;
        if (swap)
            Yo[row + c * k1] = vv;
        else
            Zo[row + c * k2] = vv;
    }
    __syncthreads();
    trsm_lower_t(LU, k1, Yo, r);
    trsm_lower_t(LV, k2, Zo, r);
}

// ------------------------------------------------------------ fast path --
// n <= 128, as a pipeline of seven launches on the stream, each shaped for
// the parallelism its step has:
//
//   k_fp_chol     one 1024-thread workgroup.  G = L L^T, right-looking, with
//                 the n x n matrix in registers: thread t = 32 a + b holds
//                 rows a + 32 u and columns b + 32 v (u, v < 4), so column j
//                 reaches LDS from 32 threads and every rank-1 update is
//                 register-local; one barrier per column.
//   k_fp_solve    ceil(n / 16) workgroups of two waves: X = L^{-1} sym(H)
//                 (stored transposed), then C = L^{-1} X^T = L^{-1} H L^{-T}.
//                 A wave holds eight columns (lane l: column l % 8, rows
//                 l / 8 + 8 q), so a row's value reaches its column's other
//                 seven lanes by a shuffle and no barrier is needed.
//   k_fp_tridiag  one 1024-thread workgroup, the same register layout as the
//                 Cholesky: per column the reflector from a wave-redundant
//                 norm, p = beta C v by 16 register products and a butterfly
//                 sum over the 32 lanes sharing a row group, the rank-2
//                 update in registers; two barriers per column.
//   k_fp_bisect   one wave per eigenvalue: 63 Sturm counts per step split
//                 the bracket into 64 (6 bits per step, 10 steps).
//   k_fp_vectors  one wave per eigenvalue: an eigenvalue separated from its
//                 neighbours by more than 1e-7 |T| gets its vector from the
//                 twisted factorisation (forward pivots D+ of
//                 T - lam I = L+ D+ L+^T and backward pivots D- of U D- U^T
//                 on two lanes at once, gamma_k = D+_k + D-_k - (a_k - lam),
//                 twist r = argmin |gamma_k|, then z_r = 1 and the two one-term
//                 recurrences away from r); a cluster of closer eigenvalues
//                 goes through inverse iteration with Gram-Schmidt inside the
//                 cluster, on one lane of the cluster's first wave.
//   k_fp_back     ceil(n / 16) workgroups: Z = Q Z_T (reflectors in LDS,
//                 applied in reverse), Y = L^{-T} Z, output order.
//
// Every later launch reads the status word first and returns at once when
// the Cholesky factorisation gave up, so the host decides about the general
// kernel after one synchronisation.
constexpr int FP_NMAX = 128;
constexpr int FP_LD = 130;    // LDS leading dimension of the zero-padded 128 x 128 matrices
constexpr int FP_COLS = 32;   // columns per solve / back-transform workgroup (two waves)
constexpr int FP_WAVES = 4;   // waves (eigenvalues) per bisection / vector workgroup

struct FPWork {
    double *Lg;   // n x n  Cholesky factor, column-major, zero above the diagonal
    double *Xg;   // n x n  (L^{-1} sym(H))^T
    double *Cg;   // n x n  C = L^{-1} H L^{-T}
    double *Vg;   // n x n  reflector j in column j, zero in rows <= j
    double *Zt;   // n x n  eigenvectors of T
    double *tri;  // 4 n    d, e, beta, lam
    double *scr;  // 6 n per eigenvalue (inverse iteration inside clusters)
};

// r[i] for a register array, from the values through a tree of selects
// on the bits of i, so the array never needs an addressable (scratch) copy
__device__ __forceinline__ double pick8v(double r0, double r1, double r2, double r3, double r4, double r5,
                                         double r6, double r7, int i) {
    const bool b0 = (i & 1) != 0, b1 = (i & 2) != 0, b2 = (i & 4) != 0;
    const double a0 = b0 ? r1 : r0, a1 = b0 ? r3 : r2;
    const double a2 = b0 ? r5 : r4, a3 = b0 ? r7 : r6;
    const double c0 = b1 ? a1 : a0, c1 = b1 ? a3 : a2;
    return b2 ? c1 : c0;
}
#define pick8(r, i) pick8v((r)[0], (r)[1], (r)[2], (r)[3], (r)[4], (r)[5], (r)[6], (r)[7], (i))

// Cross-lane moves of an FP64 value through the DPP lane patterns (both
// 32-bit halves), and a uniform read of one lane.  Callers keep every lane
// of the wave active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <- 7 - i within each 8
constexpr int DPP_MIRROR = 0x140;      // lane i <- 15 - i within each 16

// value of lane 4 (l / 4) + s of each quad, s a compile-time constant after unrolling
__device__ __forceinline__ double quad_bcast(double v, int s) {
    switch (s) {
        case 0: return dpp_f64<0x00>(v);
        case 1: return dpp_f64<0x55>(v);
        case 2: return dpp_f64<0xAA>(v);
        default: return dpp_f64<0xFF>(v);
    }
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}

// Sum over each 32-lane half of the wave, in every lane of that half: DPP
// sums inside rows of 16 lanes, then the other row's sum by a swizzle (lane
// xor 16).  Only lanes of the same half are read, so the other half may be
// inactive.
__device__ double half_wave_sum(double v) {
    v += dpp_f64<DPP_XOR1>(v);
    v += dpp_f64<DPP_XOR2>(v);
    v += dpp_f64<DPP_HALF_MIRROR>(v);
    v += dpp_f64<DPP_MIRROR>(v);
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    constexpr int XOR16 = 0x1F | (0x10 << 10);  // bit mode: and 31, or 0, xor 16
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)u, XOR16);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(u >> 32), XOR16);
    return v + __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}

// Sum over the 64 lanes with a fixed pattern (rows of 16 lanes, then the
// four row sums in a fixed order): every lane, and every wave summing the
// same data, gets the same bits.
__device__ __forceinline__ double wave_sum_fixed(double v) {
    v += dpp_f64<DPP_XOR1>(v);
    v += dpp_f64<DPP_XOR2>(v);
    v += dpp_f64<DPP_HALF_MIRROR>(v);
    v += dpp_f64<DPP_MIRROR>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Orders this wave's LDS accesses before and after the call (lanes of one
// wave exchanging values through LDS).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_max_f64(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// 1 / sqrt(a) and 1 / a for positive normal a: the hardware estimates
// refined by two Newton steps each (a few ulps; the IEEE-exact sequences
// cost several times the latency on these serial chains)
__device__ __forceinline__ double rsqrt_nr(double a) {
    double r = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    r = fma(r, fma(-h * r, r, 0.5), r);
    r = fma(r, fma(-h * r, r, 0.5), r);
    return r;
}
__device__ __forceinline__ double rcp_nr(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = fma(r, fma(-a, r, 1.0), r);
    r = fma(r, fma(-a, r, 1.0), r);
    return r;
}

// Both Cholesky factorisations give up (and the caller falls back to the
// G-eigen truncation) when a pivot is not above 1e-12 of the largest
// diagonal entry: such a pivot bounds 1/kappa(G) from above, so G has a
// condition number beyond 1e12 and its factor would not be trustworthy.
__device__ double chol_floor(const double *A, int ld, int n) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, A[i + i * ld]);
    return 1e-12 * m;
}

constexpr size_t fp_lds_bytes() { return ((size_t)FP_NMAX * FP_LD + 2 * FP_NMAX) * sizeof(double); }

// M (n x n, column-major in global memory) into LDS as a 128 x 128 matrix,
// zero outside n x n, leading dimension FP_LD; 16 pairs of loads in flight
// per thread (blockDim.x must divide 512).
__device__ void fp_load_padded(const double *M, int n, double *S) {
    const int per = 64 * FP_NMAX / blockDim.x;
    for (int k0 = 0; k0 < per; k0 += 16) {
        double va[16], vb[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int el = threadIdx.x + (k0 + k) * blockDim.x;
            const int r = 2 * (el & 63), c = min(el >> 6, n - 1);
            va[k] = M[min(r, n - 1) + (size_t)c * n];
            vb[k] = M[min(r + 1, n - 1) + (size_t)c * n];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int el = threadIdx.x + (k0 + k) * blockDim.x;
            const int r = 2 * (el & 63), c = el >> 6;
            double2 v;
            v.x = (r < n && c < n) ? va[k] : 0.0;
            v.y = (r + 1 < n && c < n) ? vb[k] : 0.0;
            *reinterpret_cast<double2 *>(S + r + c * FP_LD) = v;
        }
    }
}

// X <- L^{-1} X and X <- L^{-T} X for the sixteen columns of a wave, L in
// LDS (zero-padded, FP_LD), invd[i] = 1 / L_ii.  Lane l holds rows
// (l & 3) + 4 q, q < 32, of column l / 4, so row i's value reaches the other
// three lanes of its column by one DPP move.  The updates run over whole
// register blocks: entries of L outside its triangle are zero, and the
// owner's own row is overwritten with the solved value afterwards.
__device__ __forceinline__ void fwd_solve_q4(const double *S, int n, double (&x)[32], const double *invd) {
    const int sl = threadIdx.x & 3;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        if (4 * q >= n) break;  // one uniform test per block of four rows
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = 4 * q + s;
            // rows past n in the last block: invd and the padded L are zero,
            // so xi = 0 and every update adds a zero (values unchanged up to
            // the sign of a zero); no branch inside the block
            const double xi = quad_bcast(x[q] * invd[i], s);
#pragma unroll
            for (int q2 = q; q2 < 32; ++q2) x[q2] = fma(-S[sl + 4 * q2 + i * FP_LD], xi, x[q2]);
            if (sl == s) x[q] = xi;
        }
    }
}

__device__ __forceinline__ void bwd_solve_q4(const double *S, int n, double (&x)[32], const double *invd) {
    const int sl = threadIdx.x & 3;
#pragma unroll
    for (int q = 31; q >= 0; --q) {
#pragma unroll
        for (int s = 3; s >= 0; --s) {
            const int i = 4 * q + s;
            // rows past n: as in the forward solve, no change and no branch
            const double xi = quad_bcast(x[q] * invd[i], s);
#pragma unroll
            for (int q2 = 0; q2 <= q; ++q2) x[q2] = fma(-S[i + (sl + 4 * q2) * FP_LD], xi, x[q2]);
            if (sl == s) x[q] = xi;
        }
    }
}

// second = 0: X = L^{-1} sym(H), written as X^T; second = 1: C = L^{-1} X^T.
__global__ __launch_bounds__(4 * FP_COLS) void k_fp_solve(const double *__restrict__ H, int n, int second,
                                                          FPWork w, const int *status) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    if (status[0] != 0) return;
    double *S = smem, *invd = S + FP_NMAX * FP_LD;
    fp_load_padded(w.Lg, n, S);
    __syncthreads();
    for (int i = threadIdx.x; i < FP_NMAX; i += blockDim.x) invd[i] = (i < n) ? 1.0 / S[i + i * FP_LD] : 0.0;
    __syncthreads();
    const int l = threadIdx.x & 63, sl = l & 3;
    const int c = blockIdx.x * FP_COLS + 16 * (threadIdx.x >> 6) + (l >> 2);
    const bool cin = c < n;
    double x[32];
    {
        const int cc = min(c, n - 1);
        double a[32], b[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int r = min(sl + 4 * q, n - 1);
            a[q] = second ? w.Xg[r + cc * n] : H[r + cc * n];
            b[q] = second ? 0.0 : H[cc + r * n];
        }
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const bool in = (sl + 4 * q < n) && cin;
            x[q] = in ? (second ? a[q] : 0.5 * (a[q] + b[q])) : 0.0;
        }
    }
    fwd_solve_q4(S, n, x, invd);
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int r = sl + 4 * q;
        if (r < n && cin) {
            if (second)
                w.Cg[r + c * n] = x[q];
            else
                w.Xg[c + r * n] = x[q];
        }
    }
}

// The 128 x 128 register layout of the one-workgroup factorisations: 256
// threads (one wave per SIMD), thread t = 16 A + B holds rows A + 16 u and
// columns B + 16 v, u, v < 8 (block (u, v) of 16 x 16, element (A, B)).
// Column loops run as eight unrolled sweeps of sixteen columns, so the
// blocks left of the current sweep are pruned at compile time and the
// block of column j + 1 is a static register index.
constexpr int RL_THREADS = 256;

__device__ __forceinline__ void rl_load_sym(const double *M, int n, int A, int B, double (&m)[8][8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        double a[8], b[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int r = min(A + 16 * u, n - 1), c = min(B + 16 * v, n - 1);
            a[v] = M[r + (size_t)c * n];
            b[v] = M[c + (size_t)r * n];
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const bool in = (A + 16 * u < n) && (B + 16 * v < n);
            m[u][v] = in ? 0.5 * (a[v] + b[v]) : 0.0;
        }
    }
}

// status[0]: 0 factorised, 1 G not positive definite (nothing else runs);
// status[1]: rank (= n when factorised).
__global__ __launch_bounds__(RL_THREADS) void k_fp_chol(const double *__restrict__ G, int n, FPWork w,
                                                        int *status) {
    __shared__ double col[2][FP_NMAX];
    const int t = threadIdx.x, A = t >> 4, B = t & 15, lane = t & 63;
    double m[8][8];
    rl_load_sym(G, n, A, B, m);
    const double dg0 = G[(size_t)min(lane, n - 1) * (n + 1)], dg1 = G[(size_t)min(lane + 64, n - 1) * (n + 1)];
    const double floor_ = 1e-12 * wave_max_f64(fmax(lane < n ? dg0 : 0.0, lane + 64 < n ? dg1 : 0.0));
    if (B == 0) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (A + 16 * u < n) col[0][A + 16 * u] = m[u][0];
    }
    __syncthreads();
#pragma unroll
    for (int jv = 0; jv < 8; ++jv) {
        for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * jv + jj;
            if (j >= n) break;
            const double *cj = col[j & 1];
            const double piv = cj[j];
            double cr[8], cc[8];
#pragma unroll
            for (int u = jv; u < 8; ++u) cr[u] = cj[A + 16 * u];
#pragma unroll
            for (int v = jv; v < 8; ++v) cc[v] = cj[B + 16 * v];
            if (!(piv > floor_)) {  // the same value in every thread
                if (t == 0) {
                    status[0] = 1;
                    status[1] = 0;
                }
                return;
            }
            const double il = rsqrt_nr(piv), lj = piv * il;
            double lr[8], lc[8];
#pragma unroll
            for (int u = jv; u < 8; ++u) {
                const int r = A + 16 * u;
                lr[u] = (r > j && r < n) ? cr[u] * il : 0.0;
            }
#pragma unroll
            for (int v = jv; v < 8; ++v) {
                const int c = B + 16 * v;
                lc[v] = (c > j && c < n) ? cc[v] * il : 0.0;
            }
#pragma unroll
            for (int u = jv; u < 8; ++u)
#pragma unroll
                for (int v = jv; v < 8; ++v) m[u][v] = fma(-lr[u], lc[v], m[u][v]);
            if (t < FP_NMAX && t < n) {
                const double lv = cj[t];
                w.Lg[t + j * n] = (t == j) ? lj : (t > j ? lv * il : 0.0);
            }
            if (j + 1 < n && B == ((j + 1) & 15)) {
                // column j + 1 lies in block jv, or jv + 1 after the sweep's last column
                const int vn = (jv < 7) ? jv + 1 : 7;
#pragma unroll
                for (int u = jv; u < 8; ++u)
                    if (A + 16 * u < n) col[(j + 1) & 1][A + 16 * u] = (jj == 15) ? m[u][vn] : m[u][jv];
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        status[0] = 0;
        status[1] = n;
    }
}

// Householder reduction of sym(C) to tridiagonal form with C in registers.
// Reflector j, H = I - beta v v^T with v = x - alpha e_{j+1} (x: column j
// below the diagonal, alpha = -sign(x_{j+1}) |x|), goes to column j of Vg;
// the trailing block takes C22 -= v w^T + w v^T with p = beta C22 v and
// w = p - (beta/2)(v^T p) v.  Since C22 v = C22 x - alpha C22 e_{j+1}, the
// product y = C22 x starts right after the previous column's barrier,
// before |x| is known, and v^T C22 v = x^T y - 2 alpha y_{j+1}
// + alpha^2 C_{j+1,j+1}.  Per column: 64 register products and a 16-lane
// DPP sum for y, one barrier to publish it, two wave-redundant sums
// (|x|^2, x^T y), v and w for all rows by the first 128 threads, one
// barrier to publish them, the register update, one barrier to publish the
// next two columns.  Each update entry is v_r w_c + w_r v_c with both
// products and the sum rounded separately, so entries (r, c) and (c, r)
// stay bit-identical and C stays exactly symmetric.
// One sweep of sixteen columns j = 16 JV .. 16 JV + 15 of the reduction
// below (JV a template parameter, so the register blocks left of the sweep
// are pruned and every register index is static).
template <int JV>
__device__ __forceinline__ void tri_sweep(double (&m)[8][8], int n, int &cur, double (*col)[FP_NMAX],
                                          double (*col1)[FP_NMAX], double *yb, double2 *vw, double *dg,
                                          double *eo, double *bo, double *Vg) {
    const int t = threadIdx.x, A = t >> 4, B = t & 15, lane = t & 63;
    for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * JV + jj;
        if (j + 2 >= n) return;
        const double *cj = col[cur], *c1 = col1[cur];
        // y = C22 x over the active blocks (x zero at rows <= j, >= n)
        {
            double xc[8];
#pragma unroll
            for (int v = JV; v < 8; ++v) {
                const int c = B + 16 * v;
                const double cv = cj[c];
                xc[v] = (c > j && c < n) ? cv : 0.0;
            }
            double y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) y[u] = 0.0;
#pragma unroll
            for (int u = JV; u < 8; ++u) {
                double ya = m[u][JV] * xc[JV], yc = 0.0;
#pragma unroll
                for (int v = JV + 1; v < 8; ++v) {
                    if ((v - JV) & 1)
                        yc = fma(m[u][v], xc[v], yc);
                    else
                        ya = fma(m[u][v], xc[v], ya);
                }
                y[u] = ya + yc;
            }
            // sum over the 16 lanes B of row group A: each stage pairs
            // lanes holding the same rows and halves what a lane carries
            const bool h8 = (B & 8) != 0, h4 = (B & 4) != 0, h2 = (B & 2) != 0;
            double k4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) k4[i] = (h8 ? y[4 + i] : y[i]) + dpp_f64<DPP_MIRROR>(h8 ? y[i] : y[4 + i]);
            double k2[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                k2[i] = (h4 ? k4[2 + i] : k4[i]) + dpp_f64<DPP_HALF_MIRROR>(h4 ? k4[i] : k4[2 + i]);
            double k1 = (h2 ? k2[1] : k2[0]) + dpp_f64<DPP_XOR2>(h2 ? k2[0] : k2[1]);
            k1 += dpp_f64<DPP_XOR1>(k1);
            const int prow = A + 16 * (B >> 1);  // lanes 2u, 2u + 1 hold row A + 16 u
            if ((B & 1) == 0 && prow < n) yb[prow] = k1;
        }
        __syncthreads();
        // |x|^2 and x^T y, the same bits in every wave
        const double xw0 = cj[lane], xw1 = cj[lane + 64], yw0 = yb[lane], yw1 = yb[lane + 64];
        const bool in0 = lane > j && lane < n, in1 = lane + 64 > j && lane + 64 < n;
        const double x0 = cj[j + 1], djj = cj[j], y1v = yb[j + 1], c11 = c1[j + 1];
        double s = (in0 ? xw0 * xw0 : 0.0) + (in1 ? xw1 * xw1 : 0.0);
        double q1 = (in0 ? xw0 * yw0 : 0.0) + (in1 ? xw1 * yw1 : 0.0);
        s = wave_sum_fixed(s);
        q1 = wave_sum_fixed(q1);
        const bool refl = s > 0.0;
        const double alpha = refl ? -copysign(s * rsqrt_nr(s), x0) : 0.0;
        const double bt = refl ? rcp_nr(alpha * (alpha - x0)) : 0.0;
        const double vj1 = x0 - alpha;
        if (t == 0) {
            dg[j] = djj;
            eo[j] = refl ? alpha : x0;
            bo[j] = bt;
        }
        // v_r (vj1 at row j+1, x_r below, zero elsewhere) to Vg; and
        // p_r = beta (y_r - alpha C_{r, j+1}), w_r = p_r - K v_r to LDS
        if (t < FP_NMAX) {
            const double xv = cj[t], yv = yb[t], cv = c1[t];
            const bool in = t > j && t < n;
            const double vr = in ? ((t == j + 1) ? vj1 : xv) : 0.0;
            if (t < n) Vg[t + j * n] = vr;
            const double vcv = (q1 - 2.0 * alpha * y1v) + alpha * alpha * c11;
            const double K = 0.5 * bt * (bt * vcv);
            const double pv = in ? bt * (yv - alpha * cv) : 0.0;
            vw[t] = make_double2(vr, pv - K * vr);
        }
        __syncthreads();
        if (refl) {  // the same value in every thread
            double vr[8], wr[8], vc[8], wc[8];
#pragma unroll
            for (int u = JV; u < 8; ++u) {
                const double2 q = vw[A + 16 * u];
                vr[u] = q.x;
                wr[u] = q.y;
            }
#pragma unroll
            for (int v = JV; v < 8; ++v) {
                const double2 q = vw[B + 16 * v];
                vc[v] = q.x;
                wc[v] = q.y;
            }
#pragma unroll
            for (int u = JV; u < 8; ++u)
#pragma unroll
                for (int v = JV; v < 8; ++v)
                    m[u][v] = __dsub_rn(m[u][v], __dadd_rn(__dmul_rn(vr[u], wc[v]), __dmul_rn(wr[u], vc[v])));
        }
        // the next two columns: j + 1 in block JV (JV + 1 after the
        // sweep's last column), j + 2 in block JV (JV + 1 from jj = 14)
        const int nx = cur ^ 1;
        const int vn = (JV < 7) ? JV + 1 : 7;
        if (B == ((j + 1) & 15)) {
#pragma unroll
            for (int u = JV; u < 8; ++u)
                if (A + 16 * u < n) col[nx][A + 16 * u] = (jj == 15) ? m[u][vn] : m[u][JV];
        }
        if (B == ((j + 2) & 15)) {
#pragma unroll
            for (int u = JV; u < 8; ++u)
                if (A + 16 * u < n) col1[nx][A + 16 * u] = (jj >= 14) ? m[u][vn] : m[u][JV];
        }
        __syncthreads();
        cur = nx;
    }
}

__global__ __launch_bounds__(RL_THREADS) void k_fp_tridiag(int n, FPWork w, const int *status) {
    __shared__ double col[2][FP_NMAX], col1[2][FP_NMAX], yb[FP_NMAX];
    __shared__ double2 vw[FP_NMAX];
    if (status[0] != 0) return;
    const int t = threadIdx.x, A = t >> 4, B = t & 15, lane = t & 63;
    double *dg = w.tri, *eo = w.tri + n, *bo = w.tri + 2 * n;
    double m[8][8];
    rl_load_sym(w.Cg, n, A, B, m);
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (A + 16 * u < n) {
            if (B == 0) col[0][A + 16 * u] = m[u][0];
            if (B == 1) col1[0][A + 16 * u] = m[u][0];
        }
    if (t < FP_NMAX) {
        yb[t] = 0.0;  // rows >= n stay zero
        vw[t] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    int cur = 0;
    tri_sweep<0>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<1>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<2>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<3>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<4>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<5>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<6>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    tri_sweep<7>(m, n, cur, col, col1, yb, vw, dg, eo, bo, w.Vg);
    // the trailing 2 x 2 (or 1 x 1) block: col[cur] holds column
    // max(n - 2, 0), col1[cur] the column after it
    if (t == 0) {
        if (n >= 2) {
            dg[n - 2] = col[cur][n - 2];
            eo[n - 2] = col[cur][n - 1];
            bo[n - 2] = 0.0;
            dg[n - 1] = col1[cur][n - 1];
        } else {
            dg[0] = col[cur][0];
        }
        eo[n - 1] = 0.0;
        bo[n - 1] = 0.0;
    }
}

// Inverse iteration for the eigenvalues lam[i0..i1) of one cluster, with
// Gram-Schmidt against the earlier members; vectors to Zt columns.
__device__ void cluster_vectors(const double *d, const double *e, int n, const double *lam, int i0,
                                int i1, double tiny, double *f, double *Zt) {
    for (int i = i0; i < i1; ++i) {
        double *x = Zt + (int64_t)i * n;
        const double lm = lam[i] + (double)(i - i0) * 4.0 * tiny;
        tri_factor(d, e, n, lm, tiny, f);
        for (int k = 0; k < n; ++k) {
            uint32_t h = (uint32_t)(k * 2654435761u) ^ (uint32_t)(i * 40503u + 0x9E37u);
            h ^= h >> 15;
            h *= 0x2C1B3C6Du;
            h ^= h >> 12;
            x[k] = 0.5 + (double)(h & 0xFFFF) * (1.0 / 65536.0);
        }
        for (int it = 0; it < 3; ++it) {
            tri_solve(f, n, x);
            for (int qv = i0; qv < i; ++qv) {
                const double *y = Zt + (int64_t)qv * n;
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += y[k] * x[k];
                for (int k = 0; k < n; ++k) x[k] -= s * y[k];
            }
            double mx = 0.0;
            for (int k = 0; k < n; ++k) mx = fmax(mx, fabs(x[k]));
            const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
            double nn = 0.0;
            for (int k = 0; k < n; ++k) {
                x[k] *= inv;
                nn += x[k] * x[k];
            }
            const double rr = 1.0 / sqrt(nn);
            for (int k = 0; k < n; ++k) x[k] *= rr;
        }
    }
}

// The same inverse iteration for one wavefront with the factorisation and
// the iterate in LDS (f: 5 n, x: n): the recurrences run on lane 0, the
// Gram-Schmidt steps against the cluster's earlier vectors and the
// normalisation on all lanes.
__device__ void cluster_vectors_wave(const double *d, const double *e, int n, const double *lam, int i0, int i1,
                                     double tiny, double *f, double *x, double *Zt) {
    const int lane = threadIdx.x & 63;
    for (int i = i0; i < i1; ++i) {
        const double lm = lam[i] + (double)(i - i0) * 4.0 * tiny;
        if (lane == 0) tri_factor(d, e, n, lm, tiny, f);
        for (int k = lane; k < n; k += 64) {
            uint32_t h = (uint32_t)(k * 2654435761u) ^ (uint32_t)(i * 40503u + 0x9E37u);
            h ^= h >> 15;
            h *= 0x2C1B3C6Du;
            h ^= h >> 12;
            x[k] = 0.5 + (double)(h & 0xFFFF) * (1.0 / 65536.0);
        }
        wave_lds_sync();
        for (int it = 0; it < 3; ++it) {
            if (lane == 0) tri_solve(f, n, x);
            wave_lds_sync();
            for (int qv = i0; qv < i; ++qv) {
                const double *y = Zt + (int64_t)qv * n;
                double sdot = 0.0;
                for (int k = lane; k < n; k += 64) sdot += y[k] * x[k];
                sdot = wave_sum_f64(sdot);
                for (int k = lane; k < n; k += 64) x[k] -= sdot * y[k];
                wave_lds_sync();
            }
            double mx = 0.0;
            for (int k = lane; k < n; k += 64) mx = fmax(mx, fabs(x[k]));
            mx = wave_max_f64(mx);
            const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
            double nn = 0.0;
            for (int k = lane; k < n; k += 64) {
                const double v = x[k] * inv;
                nn += v * v;
            }
            nn = wave_sum_f64(nn);
            const double rr = inv / sqrt(nn);
            for (int k = lane; k < n; k += 64) x[k] *= rr;
            wave_lds_sync();
        }
        double *zo = Zt + (int64_t)i * n;
        for (int k = lane; k < n; k += 64) zo[k] = x[k];
        // the next member's Gram-Schmidt reads this vector from global memory
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// Gershgorin interval of T widened by a few ulps, and the pivot floor;
// the same values in every lane of every wave.
__device__ void fp_gershgorin(const double *sd, const double *se, int n, double &lo, double &hi,
                              double &pivmin) {
    const int lane = threadIdx.x & 63;
    double l = INFINITY, h = -INFINITY, emax = 0.0;
    for (int k = lane; k < n; k += 64) {
        const double off = (k > 0 ? fabs(se[k - 1]) : 0.0) + (k + 1 < n ? fabs(se[k]) : 0.0);
        l = fmin(l, sd[k] - off);
        h = fmax(h, sd[k] + off);
        if (k + 1 < n) emax = fmax(emax, se[k] * se[k]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        l = fmin(l, __shfl_xor(l, o, 64));
        h = fmax(h, __shfl_xor(h, o, 64));
        emax = fmax(emax, __shfl_xor(emax, o, 64));
    }
    const double tnorm = fmax(fabs(l), fabs(h));
    pivmin = 0x1.0p-1000 * fmax(1.0, emax);
    lo = l - (4.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin);
    hi = h + (4.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin);
}

__global__ __launch_bounds__(64 * FP_WAVES) void k_fp_bisect(int n, FPWork w, const int *status) {
    __shared__ double sd[FP_NMAX], se[FP_NMAX], se2[FP_NMAX];
    if (status[0] != 0) return;
    const int t = threadIdx.x, lane = t & 63;
    for (int k = t; k < n; k += blockDim.x) {
        sd[k] = w.tri[k];
        se[k] = w.tri[n + k];
        se2[k] = w.tri[n + k] * w.tri[n + k];
    }
    __syncthreads();
    double lo, hi, pivmin;
    fp_gershgorin(sd, se, n, lo, hi, pivmin);
    const int idx = blockIdx.x * FP_WAVES + (t >> 6);  // eigenvalue of this wave (ascending)
    if (idx >= n) return;
    double lo_ = lo, hi_ = hi;
    for (int it = 0; it < 10; ++it) {  // 6 bits each: 60 bits of the Gershgorin interval
        const double x = lo_ + (hi_ - lo_) * (double)(lane + 1) * 0.015625;
        const int c = (lane < 63) ? sturm_count(sd, se2, n, x, pivmin) : 0;
        const unsigned long long bal = __ballot(lane < 63 && c > idx);
        // first probe with more than idx eigenvalues below it
        const int s = bal ? __builtin_ctzll(bal) : 63;
        const double na = (s == 0) ? lo_ : lo_ + (hi_ - lo_) * (double)s * 0.015625;
        const double nb = (s == 63) ? hi_ : lo_ + (hi_ - lo_) * (double)(s + 1) * 0.015625;
        lo_ = na;
        hi_ = nb;
    }
    if (lane == 0) w.tri[3 * n + idx] = 0.5 * (lo_ + hi_);
}

__global__ __launch_bounds__(64 * FP_WAVES) void k_fp_vectors(int n, FPWork w, const int *status) {
    __shared__ double sd[FP_NMAX], se[FP_NMAX], sl[FP_NMAX];
    __shared__ double dpm[FP_WAVES][2][FP_NMAX], zz[FP_WAVES][FP_NMAX];
    // factorisation of T - lam I for a cluster's inverse iteration, per wave
    __shared__ double fsc[FP_WAVES][5 * FP_NMAX];
    if (status[0] != 0) return;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int k = t; k < n; k += blockDim.x) {
        sd[k] = w.tri[k];
        se[k] = w.tri[n + k];
        sl[k] = w.tri[3 * n + k];
    }
    __syncthreads();
    double tn = 0.0;
    for (int k = lane; k < n; k += 64) tn = fmax(tn, fmax(fabs(sl[k]), fabs(sd[k]) + fabs(se[k])));
    tn = wave_max_f64(tn);
    const double ortol = 1e-7 * tn;
    const double tiny = 2.220446049250313e-16 * fmax(tn, 1e-300);
    const int i = blockIdx.x * FP_WAVES + wv;
    if (i >= n) return;
    if (i > 0 && !(sl[i] - sl[i - 1] > ortol)) return;  // inside a cluster: its first wave
    int i1 = i + 1;
    while (i1 < n && !(sl[i1] - sl[i1 - 1] > ortol)) ++i1;
    if (i1 > i + 1) {
        cluster_vectors_wave(sd, se, n, sl, i, i1, tiny, fsc[wv], zz[wv], w.Zt);
        return;
    }
    const double lm = sl[i];
    double *Dp = dpm[wv][0], *Dm = dpm[wv][1], *z = zz[wv];
    // lane 0: forward pivots D+, lane 1: backward pivots D-, the same
    // instruction stream with mirrored indices
    if (lane < 2) {
        const bool fw = lane == 0;
        double *dst = fw ? Dp : Dm;
        int k = fw ? 0 : n - 1;
        double q = sd[k] - lm;
        if (q == 0.0) q = tiny;
        dst[k] = q;
        for (int s = 1; s < n; ++s) {
            k = fw ? s : n - 1 - s;
            const double ec = fw ? se[k - 1] : se[k];
            q = (sd[k] - lm) - ec * ec / q;
            if (q == 0.0) q = tiny;
            dst[k] = q;
        }
    }
    wave_lds_sync();
    // twist r = argmin gamma_k (ties: the larger k), gamma_{n-1} = D+_{n-1}
    double gb = INFINITY;
    int rb = -1;
    for (int k = lane; k < n; k += 64) {
        double gk = (k == n - 1) ? fabs(Dp[k]) : fabs(Dp[k] + Dm[k] - (sd[k] - lm));
        if (!(gk == gk)) gk = INFINITY;
        if (gk < gb || (gk == gb && k > rb)) {
            gb = gk;
            rb = k;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double og = __shfl_xor(gb, o, 64);
        const int orr = __shfl_xor(rb, o, 64);
        if (og < gb || (og == gb && orr > rb)) {
            gb = og;
            rb = orr;
        }
    }
    const int r = rb < 0 ? n - 1 : rb;
    // one-term recurrences away from r: factors first (independent), then
    // the two products on lanes 0 (downwards) and 1 (upwards)
    for (int k = lane; k < n; k += 64) z[k] = (k < r) ? -(se[k] / Dp[k]) : ((k > r) ? -(se[k - 1] / Dm[k]) : 1.0);
    wave_lds_sync();
    if (lane < 2) {
        const bool dn = lane == 0;
        const int cnt = dn ? r : n - 1 - r;
        int k = dn ? r - 1 : r + 1;
        double zk = 1.0;
        for (int s = 0; s < cnt; ++s) {
            zk = z[k] * zk;
            z[k] = zk;
            k += dn ? -1 : 1;
        }
    }
    wave_lds_sync();
    double nn = 0.0;
    for (int k = lane; k < n; k += 64) nn += z[k] * z[k];
    nn = wave_sum_f64(nn);
    const double inv = 1.0 / sqrt(nn);
    for (int k = lane; k < n; k += 64) w.Zt[k + (size_t)i * n] = z[k] * inv;
}

__global__ __launch_bounds__(4 * FP_COLS) void k_fp_back(int n, int which_smallest, FPWork w,
                                                         double *__restrict__ theta, double *__restrict__ Y,
                                                         const int *status) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    if (status[0] != 0) return;
    double *S = smem, *aux = S + FP_NMAX * FP_LD;
    fp_load_padded(w.Vg, n, S);
    for (int k = threadIdx.x; k < FP_NMAX; k += blockDim.x) aux[k] = (k < n) ? w.tri[2 * n + k] : 0.0;
    __syncthreads();
    const int l = threadIdx.x & 63, sl = l & 3;
    const int c = blockIdx.x * FP_COLS + 16 * (threadIdx.x >> 6) + (l >> 2);
    const bool cin = c < n;
    double x[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) x[q] = w.Zt[min(sl + 4 * q, n - 1) + (size_t)min(c, n - 1) * n];
#pragma unroll
    for (int q = 0; q < 32; ++q) x[q] = (sl + 4 * q < n && cin) ? x[q] : 0.0;
    // Z = H_0 H_1 ... H_{n-3} Z_T, the last reflector first; reflector
    // entries above row j + 1 and beyond n are stored zeros
    for (int j = n - 3; j >= 0; --j) {
        const double bt = aux[j];
        if (bt == 0.0) continue;
        double vq[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) vq[q] = S[sl + 4 * q + j * FP_LD];
        double sa[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sa[k] = vq[k] * x[k];
#pragma unroll
        for (int q = 8; q < 32; ++q) sa[q & 7] = fma(vq[q], x[q], sa[q & 7]);
        // over the four lanes of the column, the same bits in all four
        double tot = ((sa[0] + sa[1]) + (sa[2] + sa[3])) + ((sa[4] + sa[5]) + (sa[6] + sa[7]));
        tot += dpp_f64<DPP_XOR1>(tot);
        tot += dpp_f64<DPP_XOR2>(tot);
        tot *= bt;
#pragma unroll
        for (int q = 0; q < 32; ++q) x[q] = fma(-tot, vq[q], x[q]);
    }
    __syncthreads();
    fp_load_padded(w.Lg, n, S);
    __syncthreads();
    for (int i = threadIdx.x; i < FP_NMAX; i += blockDim.x) aux[i] = (i < n) ? 1.0 / S[i + i * FP_LD] : 0.0;
    __syncthreads();
    bwd_solve_q4(S, n, x, aux);
    // eigenvalues ascending: column c of the result goes to position c
    // (smallest first) or n - 1 - c (largest first)
    const int pos = which_smallest ? c : n - 1 - c;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int r = sl + 4 * q;
        if (r < n && cin) Y[r + (size_t)pos * n] = x[q];
    }
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < n; k += blockDim.x) theta[which_smallest ? k : n - 1 - k] = w.tri[3 * n + k];
}

PencilWork make_work(Context *ctx, int n) {
    PencilWork w;
    const size_t nn = (size_t)n * n;
    double *base = ctx->buf<double>("pencil_work", 5 * nn + 12 * (size_t)n + 6 * nn + 64);
    w.C = base;
    w.Z = base + nn;
    w.L = base + 2 * nn;
    w.T = base + 3 * nn;
    w.ek.Vh = base + 4 * nn;
    double *v = base + 5 * nn;
    w.w = v;
    w.ek.beta = v + n;
    w.ek.d = v + 2 * n;
    w.ek.e = v + 3 * n;
    w.ek.e2 = v + 4 * n;
    w.ek.p = v + 5 * n;
    w.ek.w = v + 6 * n;
    w.ek.lam = v + 7 * n;
    w.ek.scr = v + 12 * n;  // 6 n per eigenvector
    int *ib = ctx->buf<int>("pencil_iwork", 3 * (size_t)n + 8);
    w.ord = ib;
    w.ek.cstart = ib + n;
    w.flag = ib + 2 * n;
    return w;
}

// ---------------------------------------------------------------------------
// Non-symmetric pencil H y = theta G y with H = V^T A V real non-symmetric
// and G = V^T V symmetric positive definite (Sec. 3.1: a real A has complex
// Ritz values; eq. (geig) on a non-orthogonal basis).  One workgroup:
//   1. G = L L^T; C = L^{-1} H L^{-T}, the standard problem with the same
//      eigenvalues (y = L^{-T} z for C z = theta z).
//   2. Householder reduction C = Q Hs Q^T to upper Hessenberg form, Q
//      accumulated (all threads; per column one reflector applied from the
//      left to the trailing columns and from the right to every row).
//   3. Francis double-shift QR iteration on Hs to the real Schur form
//      T = Z^T Hs Z (implicit double shift from the trailing 2 x 2 block,
//      an exceptional shift after every ten iterations without a
//      deflation, a 2 x 2 block with real eigenvalues rotated to triangular
//      form).  One wavefront chases the bulge; the reflectors and rotations
//      are logged and applied to Q afterwards by every thread, each taking
//      rows of Q (the transforms act on the rows independently).
//   4. Eigenvectors of the quasi-triangular T by back substitution, one
//      thread per real eigenvalue or conjugate pair (complex arithmetic,
//      2 x 2 diagonal blocks solved as 2 x 2 systems), then V = Q X_T, each
//      complex vector scaled to unit 2-norm, Y = L^{-T} V (so y^H G y = 1).
//   5. Output order: modulus descending, then real part, then imaginary
//      part descending; a conjugate pair is placed as one unit, + member
//      first.  Y is packed real: a real value's column is its vector; a
//      pair occupies two columns, Re y and Im y of the + member.
// status[0]: 0 ok, 1 G not positive definite, 2 the QR iteration did not
// converge; status[1]: QR iterations.
// ---------------------------------------------------------------------------

constexpr int GN_LOGW = 4;  // doubles per logged transform
// C kept in LDS up to this size (137 x 136 FP64 = 146 KiB with the odd
// leading dimension; with the static arrays below the 160 KiB of a CU)
constexpr int GN_LDS_MAX_N = 136;

struct GenWork {
    double *L, *C, *Q, *X;  // n x n each (C may be replaced by an LDS copy)
    double *wr, *wi;        // n
    double *lg;             // GN_LOGW * cap: v0, v1, v2, beta (rotation: c, s)
    int *lcode;             // cap: k | m << 16 (m = 2, 3: reflector; 0: rotation)
    int cap;
};

// orders the wavefront's memory accesses (LDS or global) before and after
__device__ __forceinline__ void gn_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// rows r = r0 + i * stride of Q (col-major, n) times the logged transforms
// [0, count), in order.  A transform at column k acts on columns k..k+2
// (k, k+1 for a rotation); a bulge chase logs k, k+1, k+2, ..., so each
// row keeps its three current columns in registers and slides them: one
// load and one store per transform, the load of the column after the
// window issued one transform ahead, the next entry read one ahead.
__device__ void gn_apply_log(double *Q, int n, const double *lg, const int *lcode, int count, int r0,
                             int stride) {
    for (int r = r0; r < n; r += stride) {
        double *q = Q + r;
        int base = -1;
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, pre = 0.0;
        int code = count > 0 ? lcode[0] : 0;
        double v0 = count > 0 ? lg[0] : 0.0, v1 = count > 0 ? lg[1] : 0.0;
        double v2 = count > 0 ? lg[2] : 0.0, beta = count > 0 ? lg[3] : 0.0;
        for (int e = 0; e < count; ++e) {
            // the next entry
            const int en = e + 1 < count ? e + 1 : e;
            const int code_n = lcode[en];
            const double n0 = lg[GN_LOGW * en], n1 = lg[GN_LOGW * en + 1];
            const double n2 = lg[GN_LOGW * en + 2], nb = lg[GN_LOGW * en + 3];
            const int k = code & 0xffff, m = code >> 16;
            if (base >= 0 && k == base + 1) {
                q[(int64_t)base * n] = w0;
                w0 = w1;
                w1 = w2;
                w2 = pre;
                base = k;
            } else if (k != base) {
                if (base >= 0) {
                    q[(int64_t)base * n] = w0;
                    q[(int64_t)(base + 1) * n] = w1;
                    if (base + 2 < n) q[(int64_t)(base + 2) * n] = w2;
                }
                base = k;
                w0 = q[(int64_t)k * n];
                w1 = q[(int64_t)(k + 1) * n];
                w2 = k + 2 < n ? q[(int64_t)(k + 2) * n] : 0.0;
            }
            // the column after the window, for a slide at the next entry
            // (columns beyond the window are not touched before then)
            pre = base + 3 < n ? q[(int64_t)(base + 3) * n] : 0.0;
            if (m == 0) {
                const double u = w0, w = w1;
                w0 = v0 * u + v1 * w;
                w1 = v0 * w - v1 * u;
            } else {
                const double t = beta * (v0 * w0 + v1 * w1 + (m == 3 ? v2 * w2 : 0.0));
                w0 -= t * v0;
                w1 -= t * v1;
                if (m == 3) w2 -= t * v2;
            }
            code = code_n;
            v0 = n0;
            v1 = n1;
            v2 = n2;
            beta = nb;
        }
        if (base >= 0) {
            q[(int64_t)base * n] = w0;
            q[(int64_t)(base + 1) * n] = w1;
            if (base + 2 < n) q[(int64_t)(base + 2) * n] = w2;
        }
    }
}

// The same product by the whole workgroup, row t of Q per thread (n <= the
// workgroup size): the log passes through LDS in chunks of GN_CHUNK entries
// (each chunk one batch of loads by all threads, read back as broadcasts),
// and a row holds the GN_PF columns after its window in registers, loaded
// GN_PF slides before they enter it.  Columns beyond the window are written
// only after they have entered it, and a jump reloads window and prefetch.
constexpr int GN_CHUNK = 64, GN_PF = 8;
__device__ void gn_apply_log_wg(double *Q, int n, const double *lg, const int *lcode, int count) {
    __shared__ double s_lg[GN_CHUNK * GN_LOGW];
    __shared__ int s_code[GN_CHUNK];
    const int t = threadIdx.x, T = blockDim.x;
    double *q = Q + t;
    const bool row = t < n;
    int base = -1;
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    double pf[GN_PF];
#pragma unroll
    for (int i = 0; i < GN_PF; ++i) pf[i] = 0.0;
    for (int c0 = 0; c0 < count; c0 += GN_CHUNK) {
        const int nc = min(GN_CHUNK, count - c0);
        __syncthreads();  // the previous chunk has been read by every row
        for (int e = t; e < nc * GN_LOGW; e += T) s_lg[e] = lg[(int64_t)c0 * GN_LOGW + e];
        for (int e = t; e < nc; e += T) s_code[e] = lcode[c0 + e];
        __syncthreads();
        if (!row) continue;
        for (int e = 0; e < nc; ++e) {
            const int code = s_code[e];
            const int k = code & 0xffff, m = code >> 16;
            const double v0 = s_lg[GN_LOGW * e], v1 = s_lg[GN_LOGW * e + 1];
            const double v2 = s_lg[GN_LOGW * e + 2], beta = s_lg[GN_LOGW * e + 3];
            if (base >= 0 && k == base + 1) {
                q[(int64_t)base * n] = w0;
                w0 = w1;
                w1 = w2;
                w2 = pf[0];
#pragma unroll
                for (int i = 0; i + 1 < GN_PF; ++i) pf[i] = pf[i + 1];
                const int cn = k + 2 + GN_PF;
                pf[GN_PF - 1] = cn < n ? q[(int64_t)cn * n] : 0.0;
                base = k;
            } else if (k != base) {
                if (base >= 0) {
                    q[(int64_t)base * n] = w0;
                    q[(int64_t)(base + 1) * n] = w1;
                    if (base + 2 < n) q[(int64_t)(base + 2) * n] = w2;
                }
                base = k;
                w0 = q[(int64_t)k * n];
                w1 = q[(int64_t)(k + 1) * n];
                w2 = k + 2 < n ? q[(int64_t)(k + 2) * n] : 0.0;
#pragma unroll
                for (int i = 0; i < GN_PF; ++i) pf[i] = k + 3 + i < n ? q[(int64_t)(k + 3 + i) * n] : 0.0;
            }
            if (m == 0) {
                const double u = w0, w = w1;
                w0 = v0 * u + v1 * w;
                w1 = v0 * w - v1 * u;
            } else {
                const double tt = beta * (v0 * w0 + v1 * w1 + (m == 3 ? v2 * w2 : 0.0));
                w0 -= tt * v0;
                w1 -= tt * v1;
                if (m == 3) w2 -= tt * v2;
            }
        }
    }
    if (row && base >= 0) {
        q[(int64_t)base * n] = w0;
        q[(int64_t)(base + 1) * n] = w1;
        if (base + 2 < n) q[(int64_t)(base + 2) * n] = w2;
    }
    __syncthreads();
}

template <bool LDS>
__device__ __forceinline__ void gn_sync() {
    if (LDS)
        wave_lds_sync();  // C in LDS: the wavefront's DS operations in order
    else
        gn_wave_sync();
}

// step 3 for wavefront 0: C (n x n, upper Hessenberg) -> T in place;
// eigenvalues in diagonal order to w.wr, w.wi
template <bool LDS>
__device__ void gn_francis(double *C, int n, int ldc, GenWork &w, int *status) {
    const int lane = threadIdx.x & 63;
    const double eps = 0x1p-52;
    double hn = 0.0;
    for (int e = lane; e < n * n; e += 64) {
        const int i = e % n, j = e / n;
        if (i <= j + 1) hn = fmax(hn, fabs(C[i + (int64_t)j * ldc]));
    }
    for (int o = 32; o > 0; o >>= 1) hn = fmax(hn, __shfl_xor(hn, o, 64));
    int nn = n - 1, it = 0, total = 0, nlog = 0, nbat = 0, fail = 0;
    const int itmax = 30 * (n > 10 ? n : 10);
    // transforms are logged 64 at a time: lane j holds entry j of the batch
    // in registers until the batch is written out with one store per lane
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    int pc = 0;
    auto write_batch = [&]() {
        if (lane < nbat) {
            const int64_t idx = nlog - nbat + lane;
            double *p = w.lg + (int64_t)GN_LOGW * idx;
            p[0] = p0;
            p[1] = p1;
            p[2] = p2;
            p[3] = p3;
            w.lcode[idx] = pc;
        }
        nbat = 0;
    };
    auto logt = [&](int k, int m, double a0, double a1, double a2, double a3) {
        if (lane == nbat) {
            p0 = a0;
            p1 = a1;
            p2 = a2;
            p3 = a3;
            pc = k | (m << 16);
        }
        ++nbat;
        ++nlog;
        if (nbat == 64) write_batch();
        if (nlog == w.cap) {
            // log full: this wavefront applies it to Q now
            write_batch();
            gn_wave_sync();
            gn_apply_log(w.Q, n, w.lg, w.lcode, nlog, lane, 64);
            gn_wave_sync();
            nlog = 0;
        }
    };
    while (nn >= 0) {
        // the largest l <= nn whose subdiagonal entry is negligible against
        // its two diagonal neighbours (l = 0: none)
        int l = 0;
        for (int base = nn; base >= 1; base -= 64) {
            const int c = base - lane;
            bool ok = false;
            if (c >= 1) {
                double s = fabs(C[(c - 1) + (int64_t)(c - 1) * ldc]) + fabs(C[c + (int64_t)c * ldc]);
                if (s == 0.0) s = hn;
                ok = fabs(C[c + (int64_t)(c - 1) * ldc]) <= eps * s;
            }
            const unsigned long long m = __ballot(ok);
            if (m) {
                l = base - (int)__builtin_ctzll(m);
                break;
            }
        }
        if (l > 0 && lane == 0) C[l + (int64_t)(l - 1) * ldc] = 0.0;
        gn_sync<LDS>();
        if (l == nn) {
            if (lane == 0) {
                w.wr[nn] = C[nn + (int64_t)nn * ldc];
                w.wi[nn] = 0.0;
            }
            --nn;
            it = 0;
            continue;
        }
        if (l == nn - 1) {
            const int a = nn - 1, b = nn;
            const double t11 = C[a + (int64_t)a * ldc], t12 = C[a + (int64_t)b * ldc];
            const double t21 = C[b + (int64_t)a * ldc], t22 = C[b + (int64_t)b * ldc];
            const double p = 0.5 * (t11 - t22);
            const double q = p * p + t12 * t21;
            if (q >= 0.0) {
                // real pair: rotate with the eigenvector (z, t21) of
                // t22 + z so the block becomes upper triangular
                const double z = p + copysign(sqrt(q), p);
                const double r = hypot(z, t21);
                const double cs = r > 0.0 ? z / r : 1.0, sn = r > 0.0 ? t21 / r : 0.0;
                for (int c = a + lane; c < n; c += 64) {
                    const double u = C[a + (int64_t)c * ldc], v = C[b + (int64_t)c * ldc];
                    C[a + (int64_t)c * ldc] = cs * u + sn * v;
                    C[b + (int64_t)c * ldc] = cs * v - sn * u;
                }
                gn_sync<LDS>();
                for (int rr = lane; rr <= b; rr += 64) {
                    const double u = C[rr + (int64_t)a * ldc], v = C[rr + (int64_t)b * ldc];
                    C[rr + (int64_t)a * ldc] = cs * u + sn * v;
                    C[rr + (int64_t)b * ldc] = cs * v - sn * u;
                }
                gn_sync<LDS>();
                if (lane == 0) {
                    C[b + (int64_t)a * ldc] = 0.0;
                    w.wr[a] = C[a + (int64_t)a * ldc];
                    w.wi[a] = 0.0;
                    w.wr[b] = C[b + (int64_t)b * ldc];
                    w.wi[b] = 0.0;
                }
                gn_sync<LDS>();
                logt(a, 0, cs, sn, 0.0, 0.0);
            } else if (lane == 0) {
                w.wr[a] = w.wr[b] = t22 + p;
                w.wi[a] = sqrt(-q);
                w.wi[b] = -w.wi[a];
            }
            nn -= 2;
            it = 0;
            continue;
        }
        if (total >= itmax) {
            fail = 1;
            break;
        }
        ++it;
        ++total;
        // shifts: the eigenvalues of the trailing 2 x 2 block (sum s,
        // product t), or an exceptional pair every tenth iteration
        double s, t;
        if (it % 10 == 0) {
            const double e = fabs(C[nn + (int64_t)(nn - 1) * ldc]) + fabs(C[(nn - 1) + (int64_t)(nn - 2) * ldc]);
            const double h = 0.75 * e + C[nn + (int64_t)nn * ldc];
            s = 2.0 * h;
            t = h * h + 0.4375 * e * e;
        } else {
            const double x = C[nn + (int64_t)nn * ldc], y = C[(nn - 1) + (int64_t)(nn - 1) * ldc];
            s = x + y;
            t = x * y - C[nn + (int64_t)(nn - 1) * ldc] * C[(nn - 1) + (int64_t)nn * ldc];
        }
        // first column of Hs^2 - s Hs + t I at row l
        const double h00 = C[l + (int64_t)l * ldc], h10 = C[(l + 1) + (int64_t)l * ldc];
        const double h01 = C[l + (int64_t)(l + 1) * ldc], h11 = C[(l + 1) + (int64_t)(l + 1) * ldc];
        const double h21 = C[(l + 2) + (int64_t)(l + 1) * ldc];
        double x = h00 * h00 + h01 * h10 - s * h00 + t;
        double y = h10 * (h00 + h11 - s);
        double z = h10 * h21;
        // with C in LDS (n <= 136: at most three rows per lane) the next
        // step's x, y, z (column k, rows k+1..k+3 after the right update)
        // come from the lanes that computed them
        bool have_next = false;
        // (named registers, not an array: an array the selects index would
        // be placed in scratch memory)
        double c0a = 0.0, c0b = 0.0, c0c = 0.0;
        for (int k = l; k <= nn - 1; ++k) {
            const int m = (k == nn - 1) ? 2 : 3;
            if (k > l) {
                if (LDS && have_next) {
                    const int ix = k >> 6, iy = (k + 1) >> 6, iz = (k + 2) >> 6;
                    const double vx = ix == 0 ? c0a : (ix == 1 ? c0b : c0c);
                    const double vy = iy == 0 ? c0a : (iy == 1 ? c0b : c0c);
                    const double vz = iz == 0 ? c0a : (iz == 1 ? c0b : c0c);
                    x = readlane_f64(vx, k & 63);
                    y = readlane_f64(vy, (k + 1) & 63);
                    z = (m == 3) ? readlane_f64(vz, (k + 2) & 63) : 0.0;
                } else {
                    x = C[k + (int64_t)(k - 1) * ldc];
                    y = C[(k + 1) + (int64_t)(k - 1) * ldc];
                    z = (m == 3) ? C[(k + 2) + (int64_t)(k - 1) * ldc] : 0.0;
                }
            }
            have_next = false;
            const double sc = fabs(x) + fabs(y) + fabs(z);
            if (sc == 0.0) continue;
            // scaled by the power of two that brings sc to [1/2, 1) (exact;
            // the exponent clamped so that both factors stay finite): the
            // sum of squares then lies in [1/12, 1) and alpha (alpha - xs)
            // in [1/12, 2), where the refined hardware estimates apply (a
            // few ulps: the reflector stays orthogonal to working accuracy)
            int se;
            (void)frexp(sc, &se);
            se = se < -1020 ? -1020 : (se > 1020 ? 1020 : se);
            const double rs = ldexp(1.0, -se), sb = ldexp(1.0, se);
            const double xs = x * rs, ys = y * rs, zs = z * rs;
            const double s2 = xs * xs + ys * ys + zs * zs;
            const double nr = s2 * rsqrt_nr(s2);
            const double alpha = -copysign(nr, xs);
            const double v0 = xs - alpha, v1 = ys, v2 = zs;
            const double beta = rcp_nr(alpha * (alpha - xs));
            const int c0 = (k > l) ? k - 1 : k;
            const int r1 = (k + 3 < nn) ? k + 3 : nn;
            // left: rows k..k+2 from column c0 on (column k-1 of a chase step
            // gets its exact result alpha sc, 0, 0)
            if (LDS) {
                // at most three columns per lane (n <= 136): every load first
                double ra[3], rb[3], rc[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int c = c0 + lane + 64 * q;
                    const double *p = C + k + (int64_t)(c < n ? c : n - 1) * ldc;
                    ra[q] = p[0];
                    rb[q] = p[1];
                    rc[q] = m == 3 ? p[2] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int c = c0 + lane + 64 * q;
                    if (c >= n) continue;
                    double *p = C + k + (int64_t)c * ldc;
                    double n0, n1, n2;
                    if (k > l && c == k - 1) {
                        n0 = alpha * sb;
                        n1 = 0.0;
                        n2 = 0.0;
                    } else {
                        const double tt = beta * (v0 * ra[q] + v1 * rb[q] + v2 * rc[q]);
                        n0 = ra[q] - tt * v0;
                        n1 = rb[q] - tt * v1;
                        n2 = rc[q] - tt * v2;
                    }
                    p[0] = n0;
                    p[1] = n1;
                    if (m == 3) p[2] = n2;
                }
            } else {
                for (int c = c0 + lane; c < n; c += 64) {
                    double *p = C + k + (int64_t)c * ldc;
                    if (k > l && c == k - 1) {
                        p[0] = alpha * sb;
                        p[1] = 0.0;
                        if (m == 3) p[2] = 0.0;
                        continue;
                    }
                    const double a = p[0], b = p[1], cc = m == 3 ? p[2] : 0.0;
                    const double tt = beta * (v0 * a + v1 * b + v2 * cc);
                    p[0] = a - tt * v0;
                    p[1] = b - tt * v1;
                    if (m == 3) p[2] = cc - tt * v2;
                }
            }
            gn_sync<LDS>();
            // right: columns k..k+2 of rows 0..r1
            if (LDS) {
                // rows lane, lane + 64, lane + 128: every load first
                double ra[3], rb[3], rc[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int r = lane + 64 * q;
                    const double *p = C + (r <= r1 ? r : r1) + (int64_t)k * ldc;
                    ra[q] = p[0];
                    rb[q] = p[ldc];
                    rc[q] = m == 3 ? p[2 * ldc] : 0.0;
                }
                double nk[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int r = lane + 64 * q;
                    const double tt = beta * (ra[q] * v0 + rb[q] * v1 + rc[q] * v2);
                    nk[q] = ra[q] - tt * v0;
                    if (r <= r1) {
                        double *p = C + r + (int64_t)k * ldc;
                        p[0] = nk[q];
                        p[ldc] = rb[q] - tt * v1;
                        if (m == 3) p[2 * ldc] = rc[q] - tt * v2;
                    }
                }
                c0a = nk[0];
                c0b = nk[1];
                c0c = nk[2];
                have_next = true;
            } else {
                for (int r = lane; r <= r1; r += 64) {
                    double *p = C + r + (int64_t)k * ldc;
                    const double a = p[0], b = p[ldc], cc = m == 3 ? p[2 * ldc] : 0.0;
                    const double tt = beta * (a * v0 + b * v1 + cc * v2);
                    p[0] = a - tt * v0;
                    p[ldc] = b - tt * v1;
                    if (m == 3) p[2 * ldc] = cc - tt * v2;
                }
            }
            gn_sync<LDS>();
            logt(k, m, v0, v1, v2, beta);
        }
    }
    write_batch();
    // the rest of the log: every thread applies it after the block barrier
    if (lane == 0) {
        status[0] = fail ? 2 : 0;
        status[1] = total;
        status[2] = nlog;
    }
}

// one thread per real eigenvalue or conjugate pair: the eigenvector of the
// quasi-triangular T (n x n) into X (packed real, col-major n)
__device__ void gn_tri_vector(const double *T, int n, int ldt, const double *wr, const double *wi, int k,
                              double tiny, double *X) {
    const bool pair = wi[k] > 0.0;
    const double lr = wr[k], li = wi[k];
    double *xr = X + (int64_t)k * n;
    double *xi = pair ? X + (int64_t)(k + 1) * n : nullptr;
    int top = k;
    if (!pair) {
        xr[k] = 1.0;
    } else {
        const int a = k, b = k + 1;
        const double t11 = T[a + (int64_t)a * ldt], t12 = T[a + (int64_t)b * ldt];
        const double t21 = T[b + (int64_t)a * ldt], t22 = T[b + (int64_t)b * ldt];
        if (fabs(t21) >= fabs(t12)) {
            // x_b = 1, x_a = (lambda - t22) / t21
            xr[b] = 1.0;
            xi[b] = 0.0;
            xr[a] = (lr - t22) / t21;
            xi[a] = li / t21;
        } else {
            // x_a = 1, x_b = (lambda - t11) / t12
            xr[a] = 1.0;
            xi[a] = 0.0;
            xr[b] = (lr - t11) / t12;
            xi[b] = li / t12;
        }
        top = b;
    }
    for (int i = k - 1; i >= 0; --i) {
        const bool blk2 = i >= 1 && wi[i] < 0.0;
        if (blk2) {
            const int a = i - 1, b = i;
            double rar = 0.0, rai = 0.0, rbr = 0.0, rbi = 0.0;
            for (int j = i + 1; j <= top; ++j) {
                const double ta = T[a + (int64_t)j * ldt], tb = T[b + (int64_t)j * ldt];
                const double vr = xr[j], vi = pair ? xi[j] : 0.0;
                rar += ta * vr;
                rai += ta * vi;
                rbr += tb * vr;
                rbi += tb * vi;
            }
            // [[m11, m12], [m21, m22]] [xa; xb] = -[ra; rb], m11 = t11 - lambda,
            // m22 = t22 - lambda (complex), m12, m21 real
            const double m11r = T[a + (int64_t)a * ldt] - lr, m11i = -li;
            const double m22r = T[b + (int64_t)b * ldt] - lr, m22i = -li;
            const double m12 = T[a + (int64_t)b * ldt], m21 = T[b + (int64_t)a * ldt];
            double detr = m11r * m22r - m11i * m22i - m12 * m21;
            double deti = m11r * m22i + m11i * m22r;
            if (detr == 0.0 && deti == 0.0) detr = tiny;
            // xa = (-ra m22 + rb m12) / det, xb = (-rb m11 + ra m21) / det
            const double nar = -(rar * m22r - rai * m22i) + rbr * m12;
            const double nai = -(rar * m22i + rai * m22r) + rbi * m12;
            const double nbr = -(rbr * m11r - rbi * m11i) + rar * m21;
            const double nbi = -(rbr * m11i + rbi * m11r) + rai * m21;
            const double dd = detr * detr + deti * deti;
            xr[a] = (nar * detr + nai * deti) / dd;
            xr[b] = (nbr * detr + nbi * deti) / dd;
            if (pair) {
                xi[a] = (nai * detr - nar * deti) / dd;
                xi[b] = (nbi * detr - nbr * deti) / dd;
            }
            --i;
        } else {
            double rr = 0.0, ri = 0.0;
            for (int j = i + 1; j <= top; ++j) {
                const double ti = T[i + (int64_t)j * ldt];
                rr += ti * xr[j];
                if (pair) ri += ti * xi[j];
            }
            double dr = T[i + (int64_t)i * ldt] - lr, di = -li;
            if (dr == 0.0 && di == 0.0) dr = tiny;
            const double dd = dr * dr + di * di;
            // x_i = -r / d
            xr[i] = -(rr * dr + ri * di) / dd;
            if (pair) xi[i] = -(ri * dr - rr * di) / dd;
        }
        // growth guard: the new entries (rows lo..i0) above 2^330 scale the
        // whole partial vector down
        const int lo = i, i0 = blk2 ? i + 1 : i;
        double mx = 0.0;
        for (int j = lo; j <= i0; ++j) mx = fmax(mx, fabs(xr[j]) + (pair ? fabs(xi[j]) : 0.0));
        if (mx > 0x1p330) {
            const double f = 1.0 / mx;
            for (int j = lo; j <= top; ++j) {
                xr[j] *= f;
                if (pair) xi[j] *= f;
            }
        }
    }
}

template <bool LDS>
__global__ __launch_bounds__(SE_THREADS) void k_pencil_general(const double *__restrict__ H,
                                                               const double *__restrict__ G, int n,
                                                               double *__restrict__ theta_re,
                                                               double *__restrict__ theta_im,
                                                               double *__restrict__ Y, GenWork w, int *status) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    __shared__ double red[16];
    __shared__ int s_slot[SE_THREADS];
    const int t = threadIdx.x, T = blockDim.x, wave = t >> 6;
    // the reduction C = L^{-1} H L^{-T} in the workspace (leading dimension
    // n), then C in LDS (n <= GN_LDS_MAX_N) with an odd leading dimension,
    // so that a wavefront reading a row (lanes over columns) spreads over the
    // banks, or left in the workspace
    double *Cg = w.C;
    for (int e = t; e < n * n; e += T) {
        const int i = e % n, j = e / n;
        w.L[e] = 0.5 * (G[i + j * n] + G[j + i * n]);
        Cg[e] = H[e];
    }
    if (t < 4) status[t] = 0;
    __syncthreads();
    if (!cholesky(w.L, n, 1)) {
        if (t == 0) status[0] = 1;
        for (int i = t; i < n; i += T) {
            theta_re[i] = 0.0;
            theta_im[i] = 0.0;
        }
        return;
    }
    // C <- L^{-1} H L^{-T}: L^{-1} H, transpose, L^{-1} (.), transpose
    trsm_lower(w.L, n, Cg, n);
    transpose_sq(Cg, n);
    trsm_lower(w.L, n, Cg, n);
    transpose_sq(Cg, n);
    const int ldc = LDS ? (n | 1) : n;
    double *C = LDS ? smem : Cg;
    if (LDS) {
        for (int e = t; e < n * n; e += T) {
            const int i = e % n, j = e / n;
            C[i + j * ldc] = Cg[e];
        }
        __syncthreads();
    }
    // ---- 2. Householder reduction to Hessenberg form, Q accumulated
    for (int e = t; e < n * n; e += T) w.Q[e] = (e % n == e / n) ? 1.0 : 0.0;
    double *v = w.wr;  // scratch vector (rows j+1..n-1) until step 3
    double *tv = w.wi;
    __syncthreads();
    for (int j = 0; j + 2 < n; ++j) {
        double sg = 0.0;
        for (int i = j + 2 + t; i < n; i += T) sg += C[i + (int64_t)j * ldc] * C[i + (int64_t)j * ldc];
        sg = block_sum(sg, red);
        if (sg == 0.0) continue;  // uniform: column already reduced
        const double x0 = C[(j + 1) + (int64_t)j * ldc];
        const double alpha = -copysign(sqrt(x0 * x0 + sg), x0);
        const double beta = 1.0 / (alpha * (alpha - x0));
        for (int i = j + 1 + t; i < n; i += T) v[i] = (i == j + 1) ? x0 - alpha : C[i + (int64_t)j * ldc];
        __syncthreads();
        // left: columns j+1..n-1, tv[c] = beta v^T C[:, c] (a wavefront per column)
        const int nw = T >> 6, lane = t & 63;
        for (int c = j + 1 + wave; c < n; c += nw) {
            double acc = 0.0;
            for (int i = j + 1 + lane; i < n; i += 64) acc += v[i] * C[i + (int64_t)c * ldc];
            acc = wave_sum_f64(acc);
            if (lane == 0) tv[c] = beta * acc;
        }
        __syncthreads();
        const int m = n - j - 1;
        for (int e = t; e < m * m; e += T) {
            const int i = j + 1 + e % m, c = j + 1 + e / m;
            C[i + (int64_t)c * ldc] -= tv[c] * v[i];
        }
        __syncthreads();
        for (int i = j + 1 + t; i < n; i += T) C[i + (int64_t)j * ldc] = (i == j + 1) ? alpha : 0.0;
        // right: every row r of C and of Q, tv[r] = beta C[r, :] v
        for (int r = t; r < 2 * n; r += T) {
            const double *M = r < n ? C : w.Q;
            const int rr = r < n ? r : r - n;
            const int ldm = r < n ? ldc : n;
            double acc = 0.0;
            for (int i = j + 1; i < n; ++i) acc += M[rr + (int64_t)i * ldm] * v[i];
            w.X[r] = beta * acc;
        }
        __syncthreads();
        for (int e = t; e < 2 * n * m; e += T) {
            const int r = e % (2 * n), i = j + 1 + e / (2 * n);
            double *M = r < n ? C : w.Q;
            const int rr = r < n ? r : r - n;
            const int ldm = r < n ? ldc : n;
            M[rr + (int64_t)i * ldm] -= w.X[r] * v[i];
        }
        __syncthreads();
    }
    // ---- 3. QR iteration (wavefront 0), then Q <- Q Z from the log
    if (wave == 0) gn_francis<LDS>(C, n, ldc, w, status);
    __syncthreads();
    if (status[0] != 0) {
        for (int i = t; i < n; i += T) {
            theta_re[i] = 0.0;
            theta_im[i] = 0.0;
        }
        return;
    }
    if (n <= T)
        gn_apply_log_wg(w.Q, n, w.lg, w.lcode, status[2]);
    else
        gn_apply_log(w.Q, n, w.lg, w.lcode, status[2], t, T);
    // ---- 4. eigenvectors of T, V = Q X_T
    double tn = 0.0;
    for (int e = t; e < n * n; e += T) tn = fmax(tn, fabs(C[e % n + (int64_t)(e / n) * ldc]));
    tn = block_maxabs(tn, red);
    const double tiny = 0x1p-52 * (tn > 0.0 ? tn : 1.0);
    for (int e = t; e < n * n; e += T) w.X[e] = 0.0;
    __syncthreads();
    for (int k = t; k < n; k += T)
        if (w.wi[k] >= 0.0) gn_tri_vector(C, n, ldc, w.wr, w.wi, k, tiny, w.X);
    __syncthreads();
    // V = Q X into C's storage... C (T) is no longer needed
    double *V = w.C;  // global n x n
    for (int e = t; e < n * n; e += T) {
        const int r = e % n, c = e / n;
        const int jmax = (c + 1 < n) ? c + 1 : n - 1;
        double s = 0.0;
        for (int j = 0; j <= jmax; ++j) s += w.Q[r + (int64_t)j * n] * w.X[j + (int64_t)c * n];
        V[e] = s;
    }
    __syncthreads();
    // unit 2-norm per real vector / complex pair
    for (int k = t; k < n; k += T) {
        if (w.wi[k] < 0.0) continue;
        const bool pair = w.wi[k] > 0.0;
        double s = 0.0;
        for (int r = 0; r < n; ++r) {
            const double a = V[r + (int64_t)k * n];
            s += a * a;
            if (pair) {
                const double b = V[r + (int64_t)(k + 1) * n];
                s += b * b;
            }
        }
        const double f = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        for (int r = 0; r < n; ++r) {
            V[r + (int64_t)k * n] *= f;
            if (pair) V[r + (int64_t)(k + 1) * n] *= f;
        }
    }
    __syncthreads();
    trsm_lower_t(w.L, n, V, n);  // Y = L^{-T} V
    // ---- 5. order the units (real values and + members of pairs)
    for (int g = t; g < n; g += T) {
        int slot = -1;
        if (w.wi[g] >= 0.0) {
            const double mg = hypot(w.wr[g], w.wi[g]), rg = w.wr[g], ig = w.wi[g];
            slot = 0;
            for (int h = 0; h < n; ++h) {
                if (w.wi[h] < 0.0 || h == g) continue;
                const double mh = hypot(w.wr[h], w.wi[h]), rh = w.wr[h], ih = w.wi[h];
                const bool before = mh > mg || (mh == mg && (rh > rg || (rh == rg && (ih > ig || (ih == ig && h < g)))));
                if (before) slot += ih > 0.0 ? 2 : 1;
            }
        }
        s_slot[g] = slot;
    }
    __syncthreads();
    for (int g = t; g < n; g += T) {
        const int s = s_slot[g];
        if (s < 0) continue;
        theta_re[s] = w.wr[g];
        theta_im[s] = w.wi[g];
        if (w.wi[g] > 0.0) {
            theta_re[s + 1] = w.wr[g];
            theta_im[s + 1] = -w.wi[g];
        }
    }
    for (int e = t; e < n * n; e += T) {
        const int r = e % n, c = e / n;
        // column c of V goes to slot s_slot[c] (a real value or Re of a pair)
        // or s_slot[c - 1] + 1 (Im of the pair starting at c - 1)
        int s;
        if (w.wi[c] >= 0.0)
            s = s_slot[c];
        else
            s = s_slot[c - 1] + 1;
        Y[r + (int64_t)s * n] = V[e];
    }
}

// ---------------------------------------------------------------------------
// SVD pencil as a pipeline of launches (k1, k2 <= 256):
//   k_svdp_chol    two workgroups: MU = L_U L_U^T and MV = L_V L_V^T at once,
//                  with the reciprocal diagonals and the transposed factors
//                  (the rows of L as columns, for the backward solves);
//   k_tri_cols     the triangular solves, one wavefront per right-hand
//                  column (lanes over rows, the column in registers, the
//                  factor's next column loaded one step ahead): no barrier;
//   k_svdp_jacobi  one workgroup: one-sided Jacobi SVD of the reduced matrix,
//                  singular values in descending order, the unit vectors
//                  divided by sqrt(2) before the last solves.
// status[0]: 3 / 4 when MU / MV is not positive definite (later launches
// return at once).
// ---------------------------------------------------------------------------
struct SvdpWork {
    double *LU, *LV, *LUt, *LVt;  // factors and their transposes
    double *iu, *iv;              // reciprocal diagonals
    double *T, *M, *V;            // k1 x k2 / k2 x k1 / q x q scratch
    double *w;                    // q singular values (unsorted)
    int *ord;
};

// Blocked right-looking Cholesky for n <= 256 with 1024 threads (positive
// pivots required): per panel of CP columns, the panel (rows j0..n-1) is
// factorised in LDS, written back, and the trailing lower triangle takes the
// panel's rank-CP update in one pass (thread (tr, tc): rows tr + 32 p,
// columns tc + 32 q of the trailing block), so global memory is visited once
// per panel instead of once per column.
constexpr int CP = 8;
__device__ bool cholesky_panel256(double *A, int n) {
    __shared__ double P[256 * CP];
    __shared__ int s_bad;
    const int t = threadIdx.x, T = blockDim.x;
    if (t == 0) s_bad = 0;
    for (int j0 = 0; j0 < n; j0 += CP) {
        const int nb = min(CP, n - j0), rows = n - j0;
        for (int e = t; e < rows * nb; e += T) {
            const int r = e % rows, c = e / rows;
            P[r + c * 256] = A[(j0 + r) + (int64_t)(j0 + c) * n];
        }
        __syncthreads();
        for (int jj = 0; jj < nb; ++jj) {
            const double d = P[jj + jj * 256];
            if (!(d > 0.0)) {
                if (t == 0) s_bad = 1;
                break;
            }
            const double l = sqrt(d);
            __syncthreads();
            for (int r = jj + t; r < rows; r += T) P[r + jj * 256] = (r == jj) ? l : P[r + jj * 256] / l;
            __syncthreads();
            // rank-1 update of the panel's later columns (rows >= their index)
            for (int e = t; e < rows * (nb - jj - 1); e += T) {
                const int r = e % rows, c = jj + 1 + e / rows;
                if (r >= c) P[r + c * 256] -= P[r + jj * 256] * P[c + jj * 256];
            }
            __syncthreads();
        }
        __syncthreads();
        if (s_bad) return false;
        for (int e = t; e < rows * nb; e += T) {
            const int r = e % rows, c = e / rows;
            A[(j0 + r) + (int64_t)(j0 + c) * n] = r >= c ? P[r + c * 256] : 0.0;
        }
        // trailing update: rows and columns j0 + nb .. n-1
        const int k0 = j0 + nb, rem = n - k0;
        if (rem > 0) {
            const int tr = t & 31, tc = t >> 5;
            for (int cq = tc; cq < rem; cq += 32) {
                double lc[CP];
#pragma unroll
                for (int jj = 0; jj < CP; ++jj) lc[jj] = jj < nb ? P[(nb + cq) + jj * 256] : 0.0;
                double x[8];
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int rp = tr + 32 * p;
                    x[p] = (rp < rem && rp >= cq) ? A[(k0 + rp) + (int64_t)(k0 + cq) * n] : 0.0;
                }
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int rp = tr + 32 * p;
                    if (rp < rem && rp >= cq) {
                        double s = x[p];
#pragma unroll
                        for (int jj = 0; jj < CP; ++jj) s -= P[(nb + rp) + jj * 256] * lc[jj];
                        A[(k0 + rp) + (int64_t)(k0 + cq) * n] = s;
                    }
                }
            }
        }
        __syncthreads();
    }
    // the strict upper triangle above the panels' diagonal blocks
    for (int e = t; e < n * n; e += T) {
        const int i = e % n, j = e / n;
        if (i < j) A[e] = 0.0;
    }
    __syncthreads();
    return true;
}

__global__ __launch_bounds__(SE_THREADS) void k_svdp_chol(const double *__restrict__ MU, int k1,
                                                          const double *__restrict__ MV, int k2, SvdpWork w,
                                                          int *status) {
    const bool u = blockIdx.x == 0;
    const int k = u ? k1 : k2;
    const double *Msrc = u ? MU : MV;
    double *L = u ? w.LU : w.LV, *Lt = u ? w.LUt : w.LVt, *inv = u ? w.iu : w.iv;
    const int t = threadIdx.x, T = blockDim.x;
    for (int e = t; e < k * k; e += T) {
        const int i = e % k, j = e / k;
        L[e] = 0.5 * (Msrc[i + j * k] + Msrc[j + i * k]);
    }
    __syncthreads();
    if (!cholesky_panel256(L, k)) {
        if (t == 0) atomicMax(status, u ? 3 : 4);
        return;
    }
    for (int e = t; e < k * k; e += T) {
        const int i = e % k, j = e / k;
        Lt[e] = L[j + i * k];
    }
    for (int i = t; i < k; i += T) inv[i] = 1.0 / L[i + i * k];
}

// column c of X (n x m, ld n) <- L^{-1} X_c (FWD, L lower, its columns) or
// L^{-T} X_c (backward, with Lt = L^T: column j of Lt is row j of L); one
// wavefront per column, n <= 256
template <bool FWD>
__global__ __launch_bounds__(256) void k_tri_cols(const double *__restrict__ Lc, const double *__restrict__ inv, int n,
                                                  double *__restrict__ X, int m, const int *status) {
    if (status[0] != 0) return;
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= m) return;
    double *x = X + (int64_t)c * n;
    double xr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = lane + 64 * u;
        xr[u] = r < n ? x[r] : 0.0;
    }
    // the factor's columns (and reciprocal diagonals) two steps ahead, loaded
    // unconditionally from clamped rows (a per-lane guard would wait for
    // every load); rows past n are never used
    auto col = [&](int j, double (&d)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = lane + 64 * u;
            d[u] = Lc[(r < n ? r : n - 1) + (int64_t)j * n];
        }
    };
    auto ahead = [&](int j, int d) { return FWD ? (j + d < n ? j + d : n - 1) : (j - d > 0 ? j - d : 0); };
    const int j0 = FWD ? 0 : n - 1;
    double lc[4], l1[4], l2[4];
    col(j0, lc);
    col(ahead(j0, 1), l1);
    double ic = inv[j0], i1 = inv[ahead(j0, 1)];
    for (int s = 0; s < n; ++s) {
        const int j = FWD ? s : n - 1 - s;
        const int j2 = ahead(j, 2);
        col(j2, l2);
        const double i2 = inv[j2];
        const int ju = j >> 6;
        const double own = ju == 0 ? xr[0] : (ju == 1 ? xr[1] : (ju == 2 ? xr[2] : xr[3]));
        const double xj = readlane_f64(own, j & 63) * ic;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = lane + 64 * u;
            if (r == j) xr[u] = xj;
            else if (FWD ? (r > j && r < n) : (r < j)) xr[u] = fma(-lc[u], xj, xr[u]);
            lc[u] = l1[u];
            l1[u] = l2[u];
        }
        ic = i1;
        i1 = i2;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = lane + 64 * u;
        if (r < n) x[r] = xr[u];
    }
}

// dst (cols x rows) = src^T (src rows x cols, both column-major)
__global__ void k_transpose_f64(const double *__restrict__ src, int rows, int cols, double *__restrict__ dst,
                                const int *status) {
    if (status[0] != 0) return;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % cols), j = (int)(e / cols);  // dst[i + j cols] = src[j + i rows]
        dst[e] = src[j + (int64_t)i * rows];
    }
}

// One-sided Jacobi SVD of M (m x q, m >= q) -> sigma (descending), the
// left vectors (length m) and right vectors (length q) divided by sqrt 2
// into Lo (ld lo_ld) and Ro (ld ro_ld).
__global__ __launch_bounds__(SE_THREADS) void k_svdp_jacobi(double *__restrict__ M, int m, int q, SvdpWork w,
                                                            double *__restrict__ sigma, double *__restrict__ Lo,
                                                            int lo_ld, double *__restrict__ Ro, int ro_ld,
                                                            int run_jacobi, const int *status) {
    if (status[0] != 0) return;
    __shared__ int s_rot;
    const int t = threadIdx.x, T = blockDim.x, wave = t >> 6, lane = t & 63, nw = T >> 6;
    // (run_jacobi = 0: the block Jacobi launch before this one left the
    // rotated M and its V)
    if (run_jacobi) (void)jacobi_svd<8>(M, m, q, w.V, &s_rot);  // launched for m <= 256 only
    // column norms: a wavefront per column
    for (int j = wave; j < q; j += nw) {
        double s2 = 0.0;
        for (int r = lane; r < m; r += 64) s2 += M[r + (int64_t)j * m] * M[r + (int64_t)j * m];
        s2 = wave_sum_f64(s2);
        if (lane == 0) w.w[j] = sqrt(s2);
    }
    __syncthreads();
    sort_order(w.w, q, true, w.ord);
    for (int c = t; c < q; c += T) sigma[c] = w.w[w.ord[c]];
    const double h = 0.70710678118654752440;
    for (int e = t; e < m * q; e += T) {
        const int row = e % m, c = e / m;
        const int j = w.ord[c];
        const double sj = w.w[j];
        Lo[row + (int64_t)c * lo_ld] = sj > 0.0 ? M[row + (int64_t)j * m] / sj * h : 0.0;
    }
    for (int e = t; e < q * q; e += T) {
        const int row = e % q, c = e / q;
        Ro[row + (int64_t)c * ro_ld] = w.V[row + (int64_t)w.ord[c] * q] * h;
    }
}

// The same one-sided Jacobi spread over workgroups (q >= BJ_MIN_Q, m <= 256,
// cooperative launch of nblk / 2 workgroups).  The q columns form nblk
// blocks of at most BJ_NB (nblk even; a block past q is empty).  A sweep is
// one inner round and nblk - 1 cross rounds, each ended by a grid barrier:
//   inner: workgroup g copies blocks 2g and 2g + 1 (their columns of M and
//          of V) into LDS and rotates every pair among them once (a local
//          round-robin tournament, a half wavefront per pair);
//   cross: a round-robin tournament pairs the blocks; of its pair (I, J)
//          a workgroup keeps one column of I in each half wavefront's
//          registers and J in LDS, and in BJ_NB steps every half wavefront
//          meets every column of J (step s: column (p + s) mod BJ_NB).
// So every pair of columns is rotated in each sweep.  The stopping rule is
// the single-workgroup one, on the sweep's largest cosine and rotation
// count, gathered by global atomics into slot `sweep` of cmax / nrot (zeroed
// by the host with the barrier words) and read by every workgroup after the
// sweep's last barrier, so all leave together.  status[0] = 5 when a
// barrier wait timed out.
constexpr int BJ_NB = 7, BJ_THREADS = 256, BJ_MIN_Q = 24, BJ_MAX_SWEEPS = 40;

struct BjSync {
    unsigned *bar;   // barrier counter
    int *err;        // barrier time-out flag
    unsigned *cmax;  // BJ_MAX_SWEEPS slots: largest cosine (FP32 bits)
    int *nrot;       // BJ_MAX_SWEEPS slots: rotations
};

// One Jacobi rotation of a column pair held by a half wavefront (a, c: the
// lower-numbered column of M and of V; b, d: the other; row gl + 32 u in
// slot u).  The cosine of the pair goes to s_cmax, a rotation to s_rot.
// Reciprocals and square roots are hardware estimates refined by Newton
// steps (a few ulps: the rotation stays orthogonal to working accuracy).
__device__ __forceinline__ void bj_rotate(double (&a)[8], double (&b)[8], double (&c)[8], double (&d)[8], double tol,
                                          int gl, unsigned *s_cmax, int *s_rot) {
    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        al = fma(a[u], a[u], al);
        be = fma(b[u], b[u], be);
        ga = fma(a[u], b[u], ga);
    }
    al = half_wave_sum(al);
    be = half_wave_sum(be);
    ga = half_wave_sum(ga);
    const double pab = al * be;
    // (columns of norm below 2^-500 are left alone)
    if (!(pab > 0x1p-1000)) return;
    const double cosv = fabs(ga) * rsqrt_nr(pab);
    if (gl == 0) atomicMax(s_cmax, __float_as_uint((float)cosv));
    if (!(cosv > tol)) return;
    const double zeta = (be - al) * 0.5 * rcp_nr(ga);
    double tt;
    if (fabs(zeta) > 0x1p500) {
        tt = 0.5 * rcp_nr(zeta);
    } else {
        const double z2 = fma(zeta, zeta, 1.0);
        tt = copysign(rcp_nr(fabs(zeta) + z2 * rsqrt_nr(z2)), zeta);
    }
    const double cs = rsqrt_nr(fma(tt, tt, 1.0)), sn = cs * tt;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double x = a[u], y = b[u], z = c[u], w = d[u];
        a[u] = cs * x - sn * y;
        b[u] = sn * x + cs * y;
        c[u] = cs * z - sn * w;
        d[u] = sn * z + cs * w;
    }
    if (gl == 0) atomicAdd(s_rot, 1);
}

__global__ __launch_bounds__(BJ_THREADS) void k_svdp_bjacobi(double *__restrict__ M, int m, int q,
                                                             double *__restrict__ V, int nblk, BjSync sy,
                                                             int *status) {
    if (status[0] != 0) return;
    __shared__ double s_m[2 * BJ_NB * 256], s_v[2 * BJ_NB * 256];
    __shared__ unsigned s_cmax;
    __shared__ int s_rot;
    const int t = threadIdx.x, g = blockIdx.x, G = gridDim.x;
    const int grp = t >> 5, gl = t & 31;
    constexpr int LS = 2 * BJ_NB;  // slots of the inner round: BJ_NB of each block
    unsigned epoch = 0;
    for (int e = g * BJ_THREADS + t; e < q * q; e += G * BJ_THREADS) V[e] = (e % q == e / q) ? 1.0 : 0.0;
    if (!grid_barrier(sy.bar, (unsigned)G, epoch, sy.err)) {
        if (g == 0 && t == 0) status[0] = 5;
        return;
    }
    const double tol = 0x1p-52 * sqrt((double)m);
    const float cfin = (float)(0.1 * sqrt(tol));
    // thread t moves row t of slots [0, ns) between the columns col(slot)
    // and LDS (m, q <= BJ_THREADS); every global load before the first store
    auto to_lds = [&](auto col, auto ns_tag) {
        constexpr int NS = decltype(ns_tag)::value;
        double xm[NS], xv[NS];
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int c = col(sl);
            xm[sl] = (c >= 0 && t < m) ? M[(int64_t)c * m + t] : 0.0;
            xv[sl] = (c >= 0 && t < q) ? V[(int64_t)c * q + t] : 0.0;
        }
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            if (t < m) s_m[sl * m + t] = xm[sl];
            if (t < q) s_v[sl * q + t] = xv[sl];
        }
    };
    auto from_lds = [&](auto col, auto ns_tag) {
        constexpr int NS = decltype(ns_tag)::value;
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int c = col(sl);
            if (c >= 0 && t < m) M[(int64_t)c * m + t] = s_m[sl * m + t];
            if (c >= 0 && t < q) V[(int64_t)c * q + t] = s_v[sl * q + t];
        }
    };
    using NSInner = std::integral_constant<int, LS>;
    using NSBlock = std::integral_constant<int, BJ_NB>;
    for (int sweep = 0; sweep < BJ_MAX_SWEEPS; ++sweep) {
        for (int round = -1; round < nblk - 1; ++round) {
            int bi, bj;
            if (round < 0) {
                bi = 2 * g;
                bj = 2 * g + 1;
            } else {
                auto bpos = [&](int k) { return k == 0 ? 0 : ((k - 1 + round) % (nblk - 1)) + 1; };
                bi = bpos(g);
                bj = bpos(nblk - 1 - g);
                if (bi > bj) {
                    const int x = bi;
                    bi = bj;
                    bj = x;
                }
            }
            const int i0 = bi * BJ_NB, j0 = bj * BJ_NB;
            const int ci = min(max(q - i0, 0), BJ_NB), cj = min(max(q - j0, 0), BJ_NB);
            if (t == 0) {
                s_cmax = 0u;
                s_rot = 0;
            }
            if (round < 0) {
                // inner round: slots of block bi first, so slot order is column order
                auto gcol = [&](int sl) {
                    return sl < BJ_NB ? (sl < ci ? i0 + sl : -1) : (sl - BJ_NB < cj ? j0 + sl - BJ_NB : -1);
                };
                to_lds(gcol, NSInner{});
                __syncthreads();
                for (int step = 0; step < LS - 1; ++step) {
                    auto lpos = [&](int k) { return k == 0 ? 0 : ((k - 1 + step) % (LS - 1)) + 1; };
                    if (grp < LS / 2) {
                        int a0 = lpos(grp), b0 = lpos(LS - 1 - grp);
                        if (a0 > b0) {
                            const int x = a0;
                            a0 = b0;
                            b0 = x;
                        }
                        if (gcol(a0) >= 0 && gcol(b0) >= 0) {
                            double *gi = s_m + a0 * m, *gj = s_m + b0 * m;
                            double *vi = s_v + a0 * q, *vj = s_v + b0 * q;
                            double a[8], b[8], c[8], d[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int r = gl + 32 * u;
                                a[u] = r < m ? gi[r] : 0.0;
                                b[u] = r < m ? gj[r] : 0.0;
                                c[u] = r < q ? vi[r] : 0.0;
                                d[u] = r < q ? vj[r] : 0.0;
                            }
                            bj_rotate(a, b, c, d, tol, gl, &s_cmax, &s_rot);
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int r = gl + 32 * u;
                                if (r < m) {
                                    gi[r] = a[u];
                                    gj[r] = b[u];
                                }
                                if (r < q) {
                                    vi[r] = c[u];
                                    vj[r] = d[u];
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
                from_lds(gcol, NSInner{});
            } else {
                // cross round: J in LDS, column i0 + grp of I in registers
                auto jcol = [&](int sl) { return sl < cj ? j0 + sl : -1; };
                to_lds(jcol, NSBlock{});
                const int ic = (grp < BJ_NB && grp < ci) ? i0 + grp : -1;
                double a[8], c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int r = gl + 32 * u;
                    a[u] = (ic >= 0 && r < m) ? M[(int64_t)ic * m + r] : 0.0;
                    c[u] = (ic >= 0 && r < q) ? V[(int64_t)ic * q + r] : 0.0;
                }
                __syncthreads();
                for (int step = 0; step < BJ_NB; ++step) {
                    const int s = (grp + step) % BJ_NB;
                    if (ic >= 0 && s < cj) {
                        double *gj = s_m + s * m, *vj = s_v + s * q;
                        double b[8], d[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int r = gl + 32 * u;
                            b[u] = r < m ? gj[r] : 0.0;
                            d[u] = r < q ? vj[r] : 0.0;
                        }
                        bj_rotate(a, b, c, d, tol, gl, &s_cmax, &s_rot);
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int r = gl + 32 * u;
                            if (r < m) gj[r] = b[u];
                            if (r < q) vj[r] = d[u];
                        }
                    }
                    __syncthreads();
                }
                if (ic >= 0) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int r = gl + 32 * u;
                        if (r < m) M[(int64_t)ic * m + r] = a[u];
                        if (r < q) V[(int64_t)ic * q + r] = c[u];
                    }
                }
                from_lds(jcol, NSBlock{});
            }
            if (t == 0) {
                atomicMax(sy.cmax + sweep, s_cmax);
                atomicAdd(sy.nrot + sweep, s_rot);
            }
            if (!grid_barrier(sy.bar, (unsigned)G, epoch, sy.err)) {
                if (g == 0 && t == 0) status[0] = 5;
                return;
            }
        }
        const int nrot = __hip_atomic_load(sy.nrot + sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const float cm = __uint_as_float(__hip_atomic_load(sy.cmax + sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (nrot == 0 || cm <= cfin) break;
    }
}

// Dynamic-LDS limits are per kernel and device; raising them once per
// device to the largest size the launches below ask for keeps the attribute
// calls off the per-iteration path.
void pencil_attributes(Context *ctx) {
    static std::set<int> done;
    if (done.count(ctx->device)) return;
    OFRR_HIP(hipFuncSetAttribute((const void *)k_fp_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)fp_lds_bytes()));
    OFRR_HIP(hipFuncSetAttribute((const void *)k_fp_back, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)fp_lds_bytes()));
    OFRR_HIP(hipFuncSetAttribute((const void *)k_pencil, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)((size_t)SE_LDS_MAX_N * SE_LDS_MAX_N * sizeof(double))));
    OFRR_HIP(hipFuncSetAttribute((const void *)k_pencil_general<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)((size_t)(GN_LDS_MAX_N | 1) * GN_LDS_MAX_N * sizeof(double))));
    done.insert(ctx->device);
}

}  // namespace

const int32_t *pencil_eig_async(Context *ctx, int32_t b, const double *H, const double *G, ofrr_which which,
                                double *theta, double *Y) {
    OFRR_CHECK_ARG(b >= 1 && b <= 1024, "pencil: 1 <= b <= 1024");
    pencil_attributes(ctx);
    int *status = ctx->buf<int>("pencil_status", 4);
    const int ws = which == OFRR_SMALLEST ? 1 : 0;
    PencilWork w = make_work(ctx, b + 1);
    const int use_lds = b <= SE_LDS_MAX_N ? 1 : 0;
    const size_t gshmem = use_lds ? (size_t)b * b * sizeof(double) : 0;
    KTimer tm(ctx, "small_eig");
    if (b <= FP_NMAX) {
        // fast path; the general kernel behind it returns at once unless G
        // was not positive definite
        const size_t nn = (size_t)b * b;
        double *base = ctx->buf<double>("pencil_fast", 5 * nn + 4 * (size_t)b + 6 * nn + 8);
        FPWork fw;
        fw.Lg = base;
        fw.Xg = base + nn;
        fw.Cg = base + 2 * nn;
        fw.Vg = base + 3 * nn;
        fw.Zt = base + 4 * nn;
        fw.tri = base + 5 * nn;
        fw.scr = fw.tri + 4 * b;
        const size_t shmem = fp_lds_bytes();
        const int ncb = (b + FP_COLS - 1) / FP_COLS, nwb = (b + FP_WAVES - 1) / FP_WAVES;
        hipLaunchKernelGGL(k_fp_chol, dim3(1), dim3(RL_THREADS), 0, ctx->stream, G, b, fw, status);
        hipLaunchKernelGGL(k_fp_solve, dim3(ncb), dim3(4 * FP_COLS), shmem, ctx->stream, H, b, 0, fw, status);
        hipLaunchKernelGGL(k_fp_solve, dim3(ncb), dim3(4 * FP_COLS), shmem, ctx->stream, H, b, 1, fw, status);
        hipLaunchKernelGGL(k_fp_tridiag, dim3(1), dim3(RL_THREADS), 0, ctx->stream, b, fw, status);
        hipLaunchKernelGGL(k_fp_bisect, dim3(nwb), dim3(64 * FP_WAVES), 0, ctx->stream, b, fw, status);
        hipLaunchKernelGGL(k_fp_vectors, dim3(nwb), dim3(64 * FP_WAVES), 0, ctx->stream, b, fw, status);
        hipLaunchKernelGGL(k_fp_back, dim3(ncb), dim3(4 * FP_COLS), shmem, ctx->stream, b, ws, fw, theta, Y,
                           status);
        hipLaunchKernelGGL(k_pencil, dim3(1), dim3(SE_THREADS), gshmem, ctx->stream, H, G, b, ws, theta, Y, w,
                           status, use_lds, 1);
    } else {
        zero_bytes(ctx, status, 16);
        hipLaunchKernelGGL(k_pencil, dim3(1), dim3(SE_THREADS), gshmem, ctx->stream, H, G, b, ws, theta, Y, w,
                           status, use_lds, 0);
    }
    OFRR_HIP(hipGetLastError());
    return status + 1;
}

int32_t pencil_eig(Context *ctx, int32_t b, const double *H, const double *G, ofrr_which which,
                   double *theta, double *Y, bool want_rank) {
    (void)want_rank;
    const int32_t *rank = pencil_eig_async(ctx, b, H, G, which, theta, Y);
    int32_t *host = ctx->host_stage<int32_t>(1);
    OFRR_HIP(hipMemcpyAsync(host, rank, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    return host[0];
}

const int32_t *pencil_general_async(Context *ctx, int32_t b, const double *H, const double *G, double *theta_re,
                                    double *theta_im, double *Y) {
    OFRR_CHECK_ARG(b >= 1 && b <= SE_THREADS, "general pencil: 1 <= b <= 1024");
    pencil_attributes(ctx);
    const size_t nn = (size_t)b * b;
    GenWork w;
    double *base = ctx->buf<double>("gpencil_work", 4 * nn + 2 * (size_t)b + 8);
    w.L = base;
    w.C = base + nn;
    w.Q = base + 2 * nn;
    w.X = base + 3 * nn;
    w.wr = base + 4 * nn;
    w.wi = w.wr + b;
    // transforms logged before Q is updated: about two sweeps of b steps per
    // eigenvalue are usual; a full log is applied by the chasing wavefront
    w.cap = (int)std::min<size_t>(4 * nn + 64, (size_t)1 << 22);
    w.lg = ctx->buf<double>("gpencil_log", (size_t)GN_LOGW * w.cap);
    w.lcode = ctx->buf<int>("gpencil_lcode", (size_t)w.cap);
    int *status = ctx->buf<int>("gpencil_status", 4);
    const int use_lds = b <= GN_LDS_MAX_N ? 1 : 0;
    const size_t shmem = use_lds ? (size_t)(b | 1) * b * sizeof(double) : 0;
    KTimer tm(ctx, "small_eig");
    if (use_lds)
        hipLaunchKernelGGL(k_pencil_general<true>, dim3(1), dim3(SE_THREADS), shmem, ctx->stream, H, G, b, theta_re,
                           theta_im, Y, w, status);
    else
        hipLaunchKernelGGL(k_pencil_general<false>, dim3(1), dim3(SE_THREADS), 0, ctx->stream, H, G, b, theta_re,
                           theta_im, Y, w, status);
    OFRR_HIP(hipGetLastError());
    return status;
}

void pencil_general(Context *ctx, int32_t b, const double *H, const double *G, double *theta_re, double *theta_im,
                    double *Y) {
    const int32_t *st = pencil_general_async(ctx, b, H, G, theta_re, theta_im, Y);
    int32_t *host = ctx->host_stage<int32_t>(2);
    OFRR_HIP(hipMemcpyAsync(host, st, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    if (host[0] == 1) fail(OFRR_ERR_NUMERIC, "general pencil: G is not positive definite");
    if (host[0] == 2) fail(OFRR_ERR_NUMERIC, "general pencil: the QR iteration did not converge");
}

void svd_pencil(Context *ctx, int32_t k1, int32_t k2, const double *B, const double *MU,
                const double *MV, double *sigma, double *Y, double *Z) {
    OFRR_CHECK_ARG(k1 >= 1 && k2 >= 1 && k1 + k2 <= 1024, "svd pencil sizes");
    if (k1 <= 256 && k2 <= 256) {
        // the pipeline of launches: block Cholesky, C^T = L_V^{-1} (L_U^{-1} B)^T
        // by column solves, one-sided Jacobi on the taller of C and C^T, the
        // L^{-T} transforms by column solves
        const size_t kk = (size_t)256 * 256;
        double *base = ctx->buf<double>("svdp2_work", 9 * kk + 2 * 256 + 256);
        SvdpWork w;
        w.LU = base;
        w.LV = base + kk;
        w.LUt = base + 2 * kk;
        w.LVt = base + 3 * kk;
        w.T = base + 4 * kk;
        w.M = base + 5 * kk;
        w.V = base + 6 * kk;
        w.iu = base + 9 * kk;
        w.iv = w.iu + 256;
        w.w = w.iv + 256;
        w.ord = ctx->buf<int>("svdp2_ord", 256);
        int *status = ctx->buf<int>("pencil_status", 4);
        zero_bytes(ctx, status, 16);
        KTimer tm(ctx, "small_eig");
        hipLaunchKernelGGL(k_svdp_chol, dim3(2), dim3(SE_THREADS), 0, ctx->stream, MU, k1, MV, k2, w, status);
        // T = L_U^{-1} B (k1 x k2: k2 columns)
        OFRR_HIP(hipMemcpyAsync(w.T, B, sizeof(double) * k1 * k2, hipMemcpyDeviceToDevice, ctx->stream));
        hipLaunchKernelGGL(k_tri_cols<true>, dim3((k2 + 3) / 4), dim3(256), 0, ctx->stream, w.LU, w.iu, k1, w.T,
                           k2, status);
        // C^T = L_V^{-1} T^T (k2 x k1: k1 columns)
        double *Ct = w.M;
        hipLaunchKernelGGL(k_transpose_f64, dim3(64), dim3(256), 0, ctx->stream, w.T, k1, k2, Ct, status);
        hipLaunchKernelGGL(k_tri_cols<true>, dim3((k1 + 3) / 4), dim3(256), 0, ctx->stream, w.LV, w.iv, k2, Ct,
                           k1, status);
        const int r = k1 < k2 ? k1 : k2;
        unsigned *bj = ctx->buf<unsigned>("svdp_bj_sync", 2 + 2 * BJ_MAX_SWEEPS);
        // Jacobi on Mx (mr x qc, mr >= qc): across workgroups when qc is
        // large enough to pay for the grid barriers, then norms, order and
        // the scaled vectors in one workgroup
        auto jacobi = [&](double *Mx, int mr, int qc, double *Lo, int lo_ld, double *Ro, int ro_ld) {
            int run = 1;
            if (qc >= BJ_MIN_Q) {
                int nblk = (qc + BJ_NB - 1) / BJ_NB;
                nblk += nblk & 1;
                BjSync sy;
                sy.bar = bj;
                sy.err = reinterpret_cast<int *>(bj + 1);
                sy.cmax = bj + 2;
                sy.nrot = reinterpret_cast<int *>(bj + 2 + BJ_MAX_SWEEPS);
                zero_bytes(ctx, bj, sizeof(unsigned) * (2 + 2 * BJ_MAX_SWEEPS));
                double *Vp = w.V;
                int *stp = status;
                void *args[] = {&Mx, &mr, &qc, &Vp, &nblk, &sy, &stp};
                OFRR_HIP(hipLaunchCooperativeKernel((const void *)k_svdp_bjacobi, dim3(nblk / 2), dim3(BJ_THREADS),
                                                    args, 0, ctx->stream));
                run = 0;
            }
            hipLaunchKernelGGL(k_svdp_jacobi, dim3(1), dim3(SE_THREADS), 0, ctx->stream, Mx, mr, qc, w, sigma, Lo,
                               lo_ld, Ro, ro_ld, run, status);
        };
        if (k2 >= k1) {
            // Jacobi on C^T (k2 x k1): C^T V' = U' S, so C = V' S U'^T: the left
            // vectors of C are V' (length k1), the right ones U' (length k2)
            jacobi(Ct, k2, k1, Z, k2, Y, k1);
        } else {
            double *C = w.T;
            hipLaunchKernelGGL(k_transpose_f64, dim3(64), dim3(256), 0, ctx->stream, Ct, k2, k1, C, status);
            jacobi(C, k1, k2, Y, k1, Z, k2);
        }
        // y = L_U^{-T} (u / sqrt 2), z = L_V^{-T} (v / sqrt 2)
        hipLaunchKernelGGL(k_tri_cols<false>, dim3((r + 3) / 4), dim3(256), 0, ctx->stream, w.LUt, w.iu, k1, Y, r,
                           status);
        hipLaunchKernelGGL(k_tri_cols<false>, dim3((r + 3) / 4), dim3(256), 0, ctx->stream, w.LVt, w.iv, k2, Z, r,
                           status);
        OFRR_HIP(hipGetLastError());
        int host = 0;
        OFRR_HIP(hipMemcpyAsync(&host, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        if (host == 3) fail(OFRR_ERR_NUMERIC, "svd pencil: U^T U not positive definite");
        if (host == 4) fail(OFRR_ERR_NUMERIC, "svd pencil: V^T V not positive definite");
        if (host == 5) fail(OFRR_ERR_HIP, "svd pencil: a grid barrier of the Jacobi sweeps timed out");
        return;
    }
    const int N = k1 + k2;
    PencilWork w = make_work(ctx, N + 1);
    double *LU = ctx->buf<double>("svdp_LU", (size_t)k1 * k1);
    double *LV = ctx->buf<double>("svdp_LV", (size_t)k2 * k2);
    int *status = ctx->buf<int>("pencil_status", 4);
    zero_bytes(ctx, status, 16);
    {
        KTimer tm(ctx, "small_eig");
        hipLaunchKernelGGL(k_svd_pencil, dim3(1), dim3(SE_THREADS), 0, ctx->stream, B, k1, k2, MU,
                           MV, sigma, Y, Z, w, LU, LV, status);
        OFRR_HIP(hipGetLastError());
    }
    int host = 0;
    OFRR_HIP(hipMemcpyAsync(&host, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    if (host == 3) fail(OFRR_ERR_NUMERIC, "svd pencil: U^T U not positive definite");
    if (host == 4) fail(OFRR_ERR_NUMERIC, "svd pencil: V^T V not positive definite");
}

}  // namespace ofrr
