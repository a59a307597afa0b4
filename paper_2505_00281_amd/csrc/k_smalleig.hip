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
//                z = L_V^{-T} v / sqrt(2) meet [y; z]^T M [y; z] = 1.
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
        for (int e = t; e < rem * rem; e += T) {
            const int ii = j + 1 + e % rem, kk = j + 1 + e / rem;
            if (kk <= ii) A[ii + kk * n] -= A[ii + j * n] * A[kk + j * n];
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
                                                       int *status, int use_lds) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    __shared__ double red[16];
    const int t = threadIdx.x, T = blockDim.x;
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
    if (t == 0) w.flag[1] = rank;
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
    // augmented symmetric [0 Cm; Cm^T 0] (N x N)
    for (int e = t; e < N * N; e += T) {
        const int i = e % N, j = e / N;
        double v = 0.0;
        if (i < k1 && j >= k1) v = w.L[i + (j - k1) * k1];
        if (i >= k1 && j < k1) v = w.L[j + (i - k1) * k1];
        w.C[e] = v;
    }
    __syncthreads();
    sym_eig(w.C, N, w.w, w.Z, w.ek, red);
    sort_order(w.w, N, true, w.ord);
    const int r = k1 < k2 ? k1 : k2;
    // top r (positive) eigenpairs: u part (k1), v part (k2) of unit eigvecs
    for (int c = t; c < r; c += T) sigma[c] = w.w[w.ord[c]];
    for (int e = t; e < k1 * r; e += T) {
        const int row = e % k1, c = e / k1;
        Yo[row + c * k1] = w.Z[row + w.ord[c] * N];
    }
    for (int e = t; e < k2 * r; e += T) {
        const int row = e % k2, c = e / k2;
        Zo[row + c * k2] = w.Z[k1 + row + w.ord[c] * N];
    }
    __syncthreads();
    trsm_lower_t(LU, k1, Yo, r);
    trsm_lower_t(LV, k2, Zo, r);
}

// ------------------------------------------------------------ fast path --
// n <= 128.  One 1024-thread workgroup keeps the active n x n matrix in LDS
// (leading dimension n + 1, so row and column walks are both free of bank
// conflicts) and a second n x n matrix in registers: lane l of wave w holds
// column c = 8 w + l % 8, rows r = l / 8 + 8 q, q = 0..15.  The eight lanes
// of one column sit in one wavefront, so the triangular solves and the
// back-transform exchange values with cross-lane shuffles and need no
// workgroup barrier at all.  Every phase then works
// out of LDS and registers; global memory only carries the Cholesky factor
// while LDS holds the tridiagonal reduction, one transpose, and the
// eigenvectors of T between their computation and the back-transform.
//
// Eigenvectors of T: for an eigenvalue separated from its neighbours by
// more than 1e-7 |T| the twisted factorisation gives the vector in one pass
// (forward pivots D+ of T - lam I = L+ D+ L+^T, backward pivots D- of the
// U D- U^T factorisation, gamma_k = D+_k + D-_k - (a_k - lam), twist
// r = argmin |gamma_k|, then z_r = 1 and the two one-term recurrences away
// from r); clusters of closer eigenvalues go through inverse iteration with
// Gram-Schmidt inside the cluster.
constexpr int FP_NMAX = 128;

struct FastWork {
    double *Lg;   // n x n, the Cholesky factor (column-major)
    double *Tg;   // n x n, transpose scratch
    double *Zt;   // n x n, eigenvectors of T (column-major)
    double *dpm;  // 2 n x n, twisted-factorisation pivots, [k][i]
    double *scr;  // 6 n per eigenvector (inverse iteration inside clusters)
    int *cstart;  // n
};

// one-sync block sum over 1024 threads (red: 16 doubles, alternate buffers
// between consecutive calls)
__device__ __forceinline__ double bsum1(double v, double *red) {
    v = wave_sum_f64(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    // pairwise tree (fixed order, 4 dependent adds instead of 16)
    double r[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = red[2 * i] + red[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = r[2 * i] + r[2 * i + 1];
    return (r[0] + r[1]) + (r[2] + r[3]);
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

__device__ bool chol_lds(double *S, int ld, int n) {
    const int t = threadIdx.x, tx = t & 31, ty = t >> 5;
    const double floor_ = chol_floor(S, ld, n);
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double dj = S[j + j * ld];
        if (!(dj > floor_)) return false;  // every thread read the same value
        const double l = sqrt(dj), il = 1.0 / l;
        __syncthreads();
        for (int i = j + t; i < n; i += SE_THREADS) S[i + j * ld] = (i == j) ? l : S[i + j * ld] * il;
        __syncthreads();
        // lower triangle of the trailing block: column kk (per ty), rows
        // ii >= kk (per tx)
        for (int kk = j + 1 + ty; kk < n; kk += 32) {
            const double lk = S[kk + j * ld];
            // rows ii = kk + tx + 32 u (u < 4 covers n <= 128 in one pass):
            // loads first, then the stores
            for (int i0 = kk + tx; i0 < n; i0 += 128) {
                double a[4], l[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ii = min(i0 + 32 * u, n - 1);
                    a[u] = S[ii + kk * ld];
                    l[u] = S[ii + j * ld];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + 32 * u < n) S[i0 + 32 * u + kk * ld] = a[u] - l[u] * lk;
            }
        }
        __syncthreads();
    }
    return true;
}

// X <- L^{-1} X, L lower triangular in LDS (S, ld), X in registers (wave-
// local column layout), invd[i] = 1 / L_ii.  Fully unrolled so every
// register index is static; row i's owner scales it and a shuffle hands
// it to the other seven lanes of its column.
__device__ __forceinline__ void fwd_solve_reg(const double *S, int ld, int n, double (&x)[16], const double *invd) {
    const int l = threadIdx.x & 63, g = l >> 3, cl = l & 7;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
#pragma unroll 1
        for (int sidx = 0; sidx < 8; ++sidx) {
            const int i = 8 * q + sidx;
            if (i < n) {
                const double own = x[q] * invd[i];
                if (g == sidx) x[q] = own;
                const double xi = __shfl(own, cl + 8 * sidx, 64);
#pragma unroll
                for (int q2 = q; q2 < 16; ++q2) {
                    const int r = g + 8 * q2;
                    const double lv = S[min(r, n - 1) + i * ld];
                    x[q2] = (r > i && r < n) ? fma(-lv, xi, x[q2]) : x[q2];
                }
            }
        }
    }
}

// X <- L^{-T} X, same layout.
__device__ __forceinline__ void bwd_solve_reg(const double *S, int ld, int n, double (&x)[16], const double *invd) {
    const int l = threadIdx.x & 63, g = l >> 3, cl = l & 7;
#pragma unroll
    for (int q = 15; q >= 0; --q) {
#pragma unroll 1
        for (int sidx = 7; sidx >= 0; --sidx) {
            const int i = 8 * q + sidx;
            if (i < n) {
                const double own = x[q] * invd[i];
                if (g == sidx) x[q] = own;
                const double xi = __shfl(own, cl + 8 * sidx, 64);
#pragma unroll
                for (int q2 = 0; q2 <= q; ++q2) {
                    const int r = g + 8 * q2;
                    const double lv = S[i + min(r, n - 1) * ld];
                    x[q2] = (r < i) ? fma(-lv, xi, x[q2]) : x[q2];
                }
            }
        }
    }
}

// Householder reduction of the symmetric matrix in S (LDS, ld) to
// tridiagonal form; reflector j is left in S rows j+1..n-1 of column j.
__device__ void tridiag_lds(double *S, int ld, int n, double *d, double *e, double *beta,
                            double *pv, double *red2) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int rb = 0;
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;
        double s = 0.0;
        for (int i = j + 1 + t; i < n; i += SE_THREADS) s += S[i + j * ld] * S[i + j * ld];
        s = bsum1(s, red2 + 16 * rb);
        rb ^= 1;
        const double x0 = S[(j + 1) + j * ld];
        const double alpha = (s > 0.0) ? -copysign(sqrt(s), x0) : 0.0;
        const double bt = (s > 0.0) ? 1.0 / (alpha * (alpha - x0)) : 0.0;
        const double vj1 = x0 - alpha;
        if (t == 0) {
            d[j] = S[j + j * ld];
            e[j] = (s > 0.0) ? alpha : x0;
            beta[j] = bt;
        }
        if (bt == 0.0) continue;  // column already reduced; S untouched
        // p = beta C22 v: eight lanes per row (column r of the symmetric C22),
        // each over every eighth entry, then a 3-step shuffle sum; a wave
        // covers 8 rows at once
        double vp = 0.0;
        {
            const int rl = lane & 7, sub = lane >> 3;
            for (int r = j + 1 + 8 * wave + rl; r - rl < n; r += 128) {
                double a0 = 0.0, a1 = 0.0;
                if (r < n) {
                    int cc = j + 1 + sub;
                    for (; cc + 8 < n; cc += 16) {
                        const double v0 = (cc == j + 1) ? vj1 : S[cc + j * ld];
                        const double v1 = S[cc + 8 + j * ld];
                        a0 = fma(S[cc + r * ld], v0, a0);
                        a1 = fma(S[cc + 8 + r * ld], v1, a1);
                    }
                    if (cc < n) a0 = fma(S[cc + r * ld], (cc == j + 1) ? vj1 : S[cc + j * ld], a0);
                }
                double acc = a0 + a1;
                acc += __shfl_xor(acc, 8, 64);
                acc += __shfl_xor(acc, 16, 64);
                acc += __shfl_xor(acc, 32, 64);
                acc *= bt;
                if (sub == 0 && r < n) {
                    pv[r] = acc;
                    vp += ((r == j + 1) ? vj1 : S[r + j * ld]) * acc;
                }
            }
        }
        vp = bsum1(vp, red2 + 16 * rb);  // also publishes pv
        rb ^= 1;
        const double K = 0.5 * bt * vp;
        // C22 -= v w^T + w v^T, w = p - K v, over the whole trailing block on
        // a 32 x 32 thread grid; each entry's update is v_r w_c + w_r v_c
        // with both products rounded separately, so entries (r, c) and (c, r)
        // receive bit-identical updates and C22 stays exactly symmetric
        {
            const int tx = t & 31, ty = t >> 5;
            for (int cc = j + 1 + ty; cc < n; cc += 32) {
                const double vc = (cc == j + 1) ? vj1 : S[cc + j * ld];
                // w_x = p_x - K v_x with explicit roundings, so a value is the
                // same whether x indexes a row or a column
                const double wc = __dsub_rn(pv[cc], __dmul_rn(K, vc));
                // rows r = j + 1 + tx + 32 u, u < 4 (n <= 128: one pass):
                // every load before any store
                for (int r0 = j + 1 + tx; r0 < n; r0 += 128) {
                    double vr[4], pr[4], a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int r = min(r0 + 32 * u, n - 1);
                        vr[u] = (r == j + 1) ? vj1 : S[r + j * ld];
                        pr[u] = pv[r];
                        a[u] = S[r + cc * ld];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double wr = __dsub_rn(pr[u], __dmul_rn(K, vr[u]));
                        const double upd = __dadd_rn(__dmul_rn(vr[u], wc), __dmul_rn(wr, vc));
                        if (r0 + 32 * u < n) S[r0 + 32 * u + cc * ld] = a[u] - upd;
                    }
                }
            }
        }
        if (t == 0) S[(j + 1) + j * ld] = vj1;
        __syncthreads();
    }
    if (t == 0) {
        if (n >= 2) {
            d[n - 2] = S[(n - 2) + (n - 2) * ld];
            e[n - 2] = S[(n - 1) + (n - 2) * ld];
            beta[n - 2] = 0.0;
        }
        d[n - 1] = S[(n - 1) + (n - 1) * ld];
        beta[n - 1] = 0.0;
        e[n - 1] = 0.0;
    }
    __syncthreads();
}

// Eigenvector of the symmetric tridiagonal (d, e) for the isolated
// eigenvalue lam by the twisted factorisation; pivots go to dp/dm (stride
// `st` between consecutive k).  Writes the unit vector to z (stride 1).
__device__ void twisted_vector(const double *d, const double *e, int n, double lam, double tiny,
                               double *dp, double *dm, int64_t st, double *z) {
    double q = d[0] - lam;
    if (q == 0.0) q = tiny;
    dp[0] = q;
    for (int k = 1; k < n; ++k) {
        q = (d[k] - lam) - e[k - 1] * e[k - 1] / q;
        if (q == 0.0) q = tiny;
        dp[(int64_t)k * st] = q;
    }
    q = d[n - 1] - lam;
    if (q == 0.0) q = tiny;
    dm[(int64_t)(n - 1) * st] = q;
    double gbest = fabs(dp[(int64_t)(n - 1) * st]);  // gamma_{n-1} = D+_{n-1}
    int r = n - 1;
    for (int k = n - 2; k >= 0; --k) {
        q = (d[k] - lam) - e[k] * e[k] / q;
        if (q == 0.0) q = tiny;
        dm[(int64_t)k * st] = q;
        const double gk = fabs(dp[(int64_t)k * st] + q - (d[k] - lam));
        if (gk < gbest) {  // first minimum from the top; ties keep the larger k
            gbest = gk;
            r = k;
        }
    }
    z[r] = 1.0;
    double nn = 1.0;
    double zk = 1.0;
    for (int k = r - 1; k >= 0; --k) {
        zk = -(e[k] / dp[(int64_t)k * st]) * zk;
        z[k] = zk;
        nn += zk * zk;
    }
    zk = 1.0;
    for (int k = r + 1; k < n; ++k) {
        zk = -(e[k - 1] / dm[(int64_t)k * st]) * zk;
        z[k] = zk;
        nn += zk * zk;
    }
    const double inv = 1.0 / sqrt(nn);
    for (int k = 0; k < n; ++k) z[k] *= inv;
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

// status[0]: 0 solved, 1 G not positive definite (nothing written);
// status[1]: rank (= n when solved).
__global__ __launch_bounds__(SE_THREADS) void k_pencil_fast(const double *__restrict__ H,
                                                            const double *__restrict__ G, int n,
                                                            int which_smallest,
                                                            double *__restrict__ theta,
                                                            double *__restrict__ Y, FastWork fw,
                                                            int *status) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    __shared__ double red2[32];
    const int ld = n + 1;
    double *S = smem;
    double *invd = S + (size_t)n * ld;    // 1 / L_ii (128)
    double *part = invd + 256;            // spare (2 x 8 x 128)
    double *dd = part + 2048;             // d, e, e2, lam, beta, p: 128 each
    double *ee = dd + 128, *e2 = ee + 128, *lam = e2 + 128, *beta = lam + 128, *pv = beta + 128;
    const int t = threadIdx.x;
    const int c = 8 * (t >> 6) + (t & 7), g = (t & 63) >> 3;  // wave-local column layout
    const bool cin = c < n;

    // A. Cholesky of sym(G) in LDS
    for (int el = t; el < n * n; el += SE_THREADS) {
        const int i = el % n, j = el / n;
        S[i + j * ld] = 0.5 * (G[i + j * n] + G[j + i * n]);
    }
    __syncthreads();
    if (!chol_lds(S, ld, n)) {
        if (t == 0) {
            status[0] = 1;
            status[1] = 0;
        }
        return;
    }
    // B. keep L in global memory; reciprocal pivots for the solves
    for (int el = t; el < n * n; el += SE_THREADS) {
        const int i = el % n, j = el / n;
        fw.Lg[el] = (i >= j) ? S[i + j * ld] : 0.0;
    }
    for (int i = t; i < n; i += SE_THREADS) invd[i] = 1.0 / S[i + i * ld];
    __syncthreads();
    // C. X = sym(H) in registers; X <- L^{-1} X
    double x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = g + 8 * q;
        x[q] = (r < n && cin) ? 0.5 * (H[r + c * n] + H[c + r * n]) : 0.0;
    }
    fwd_solve_reg(S, ld, n, x, invd);
    // D. transpose through global memory, X <- L^{-1} X^T = L^{-1} H L^{-T}
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = g + 8 * q;
        if (r < n && cin) fw.Tg[c + r * n] = x[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = g + 8 * q;
        x[q] = (r < n && cin) ? fw.Tg[r + c * n] : 0.0;
    }
    fwd_solve_reg(S, ld, n, x, invd);
    __syncthreads();
    // E. C (symmetrised) into LDS over L
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = g + 8 * q;
        if (r < n && cin) S[r + c * ld] = x[q];
    }
    __syncthreads();
    for (int el = t; el < n * n; el += SE_THREADS) {
        const int i = el % n, j = el / n;
        if (i > j) {
            const double v = 0.5 * (S[i + j * ld] + S[j + i * ld]);
            S[i + j * ld] = v;
            S[j + i * ld] = v;
        }
    }
    __syncthreads();
    // F. tridiagonal T = Q^T C Q, eigenvalues by multisection
    tridiag_lds(S, ld, n, dd, ee, beta, pv, red2);
    for (int i = t; i < n; i += SE_THREADS) e2[i] = ee[i] * ee[i];
    __syncthreads();
    bisect_ptr(n, dd, ee, e2, lam);
    // G. eigenvectors of T
    double tn = 0.0;
    for (int i = t; i < n; i += SE_THREADS) tn = fmax(tn, fmax(fabs(lam[i]), fabs(dd[i]) + fabs(ee[i])));
    for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, 64));
    if ((t & 63) == 0) red2[t >> 6] = tn;
    __syncthreads();
    tn = 0.0;
    for (int i = 0; i < 16; ++i) tn = fmax(tn, red2[i]);
    const double ortol = 1e-7 * tn;
    const double tiny = 2.220446049250313e-16 * fmax(tn, 1e-300);
    for (int i = t; i < n; i += SE_THREADS)
        fw.cstart[i] = (i == 0 || lam[i] - lam[i - 1] > ortol) ? 1 : 0;
    __syncthreads();
    if (t < n) {
        const int i = t;
        if (fw.cstart[i]) {
            int i1 = i + 1;
            while (i1 < n && !fw.cstart[i1]) ++i1;
            if (i1 == i + 1)
                twisted_vector(dd, ee, n, lam[i], tiny, fw.dpm + i, fw.dpm + (int64_t)n * n + i, n,
                               fw.Zt + (int64_t)i * n);
            else
                cluster_vectors(dd, ee, n, lam, i, i1, tiny, fw.scr + (int64_t)i * 6 * n, fw.Zt);
        }
    }
    __syncthreads();
    // H. back-transform Z = Q Z_T with Z in registers
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = g + 8 * q;
        x[q] = (r < n && cin) ? fw.Zt[r + c * n] : 0.0;
    }
    for (int j = n - 3; j >= 0; --j) {
        const double bt = beta[j];
        if (bt == 0.0) continue;
        double vq[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = g + 8 * q;
            vq[q] = (r > j && r < n) ? S[min(r, n - 1) + j * ld] : 0.0;
        }
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < 16; q += 2) {
            s0 = fma(vq[q], x[q], s0);
            s1 = fma(vq[q + 1], x[q + 1], s1);
        }
        // sum over the eight lanes of the column (lane bits 3..5), fixed order
        double tot = s0 + s1;
        tot += __shfl_xor(tot, 8, 64);
        tot += __shfl_xor(tot, 16, 64);
        tot += __shfl_xor(tot, 32, 64);
        tot *= bt;
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = fma(-tot, vq[q], x[q]);
    }
    __syncthreads();
    // I. Y = L^{-T} Z with L back in LDS
    for (int el = t; el < n * n; el += SE_THREADS) {
        const int i = el % n, j = el / n;
        S[i + j * ld] = fw.Lg[el];
    }
    __syncthreads();
    bwd_solve_reg(S, ld, n, x, invd);
    // J. order: lam is ascending
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = g + 8 * q;
        if (r < n && cin) {
            const int pos = which_smallest ? c : n - 1 - c;
            Y[r + (int64_t)pos * n] = x[q];
        }
    }
    for (int i = t; i < n; i += SE_THREADS) theta[which_smallest ? i : n - 1 - i] = lam[i];
    if (t == 0) {
        status[0] = 0;
        status[1] = n;
    }
}

constexpr size_t fast_lds_bytes(int n) {
    return ((size_t)n * (n + 1) + 256 + 2048 + 6 * 128) * sizeof(double);
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

}  // namespace

int32_t pencil_eig(Context *ctx, int32_t b, const double *H, const double *G, ofrr_which which,
                   double *theta, double *Y, bool want_rank) {
    OFRR_CHECK_ARG(b >= 1 && b <= 1024, "pencil: 1 <= b <= 1024");
    int *status = ctx->buf<int>("pencil_status", 4);
    if (b <= FP_NMAX) {
        // fast path; falls through to the general kernel when G is not
        // positive definite
        const size_t nn = (size_t)b * b;
        double *base = ctx->buf<double>("pencil_fast", 11 * nn + 8);
        FastWork fw;
        fw.Lg = base;
        fw.Tg = base + nn;
        fw.Zt = base + 2 * nn;
        fw.dpm = base + 3 * nn;
        fw.scr = base + 5 * nn;
        fw.cstart = ctx->buf<int>("pencil_fast_i", (size_t)b + 8);
        const size_t shmem = fast_lds_bytes(b);
        OFRR_HIP(hipFuncSetAttribute((const void *)k_pencil_fast,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
        {
            KTimer tm(ctx, "small_eig");
            hipLaunchKernelGGL(k_pencil_fast, dim3(1), dim3(SE_THREADS), shmem, ctx->stream, H, G, b,
                               which == OFRR_SMALLEST ? 1 : 0, theta, Y, fw, status);
            OFRR_HIP(hipGetLastError());
        }
        int host[2] = {1, 0};
        OFRR_HIP(hipMemcpyAsync(host, status, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        if (host[0] == 0) return host[1];
    }
    PencilWork w = make_work(ctx, b + 1);
    zero_bytes(ctx, status, 16);
    const int use_lds = b <= SE_LDS_MAX_N ? 1 : 0;
    const size_t shmem = use_lds ? (size_t)b * b * sizeof(double) : 0;
    if (shmem > 0)
        OFRR_HIP(hipFuncSetAttribute((const void *)k_pencil, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shmem));
    {
        KTimer tm(ctx, "small_eig");
        hipLaunchKernelGGL(k_pencil, dim3(1), dim3(SE_THREADS), shmem, ctx->stream, H, G, b,
                           which == OFRR_SMALLEST ? 1 : 0, theta, Y, w, status, use_lds);
        OFRR_HIP(hipGetLastError());
    }
    int host[2] = {0, 0};
    OFRR_HIP(hipMemcpyAsync(&host[0], status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    OFRR_HIP(hipMemcpyAsync(&host[1], w.flag + 1, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    (void)want_rank;
    return host[1];
}

void svd_pencil(Context *ctx, int32_t k1, int32_t k2, const double *B, const double *MU,
                const double *MV, double *sigma, double *Y, double *Z) {
    OFRR_CHECK_ARG(k1 >= 1 && k2 >= 1 && k1 + k2 <= 1024, "svd pencil sizes");
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
