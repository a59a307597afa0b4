// k_smalleig.hip -- the small FP64 problems of the projection step, on the
// GPU in one workgroup (Sec. 4, mixed-precision plan: the projected pencil
// is promoted to and solved in FP64).
//
//   pencil_eig   H y = theta G y (eq. (geig)): Cholesky G = L L^T, cyclic
//                Jacobi on C = L^{-1} H L^{-T}, Y = L^{-T} Z.  If G is not
//                numerically positive definite, G is diagonalised first and
//                its negligible directions are dropped (G-eigen truncation).
//   svd_pencil   the augmented pencil of Sec. 3.2 via block Cholesky:
//                C = L_U^{-1} B L_V^{-T}; the positive eigenvalues of
//                [0 C; C^T 0] are the singular values, with unit eigenvectors
//                [u; v] / sqrt(2); y = L_U^{-T} u / sqrt(2),
//                z = L_V^{-T} v / sqrt(2) meet [y; z]^T M [y; z] = 1.
//
// The Jacobi sweeps use the parallel round-robin ordering: each round
// rotates n/2 disjoint (p, q) pairs at once, with the rotation chosen to
// annihilate C_pq (tau = (C_qq - C_pp) / (2 C_pq), t the smaller root of
// t^2 + 2 tau t - 1 = 0, c = 1/sqrt(1+t^2), s = t c).  Sweeps stop when the
// off-diagonal Frobenius norm is below 1e-15 times the Frobenius norm.
#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

constexpr int SE_THREADS = 1024;

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

// Round-robin pairing for m players (m even), round r in [0, m-1):
// pair 0 is (m-1, r), pair k>0 is ((r+k) mod (m-1), (r-k) mod (m-1)).
__device__ __forceinline__ void rr_pair(int m, int r, int k, int &p, int &q) {
    if (k == 0) {
        p = r;
        q = m - 1;
    } else {
        p = (r + k) % (m - 1);
        q = (r - k + (m - 1)) % (m - 1);
    }
    if (p > q) {
        int x = p;
        p = q;
        q = x;
    }
}

// Jacobi eigen-decomposition of the symmetric n x n matrix C (column-major,
// ld n) accumulating Z (initialised to I here).  Player m-1 is a dummy when
// n is odd.  Returns the number of sweeps (-1: not converged).
__device__ int jacobi(double *C, double *Z, int n, double *cs, double *sn, int *pp, int *qq,
                      double *red) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int e = t; e < n * n; e += T) Z[e] = ((e % n) == (e / n)) ? 1.0 : 0.0;
    double f2 = 0.0;
    for (int e = t; e < n * n; e += T) f2 += C[e] * C[e];
    f2 = block_sum(f2, red);
    const double tol2 = 1e-30 * f2;
    const int m = (n & 1) ? n + 1 : n;
    const int npair = m / 2;
    for (int sweep = 0; sweep <= 60; ++sweep) {
        double off = 0.0;
        for (int e = t; e < n * n; e += T) {
            const int i = e % n, j = e / n;
            if (i != j) off += C[e] * C[e];
        }
        off = block_sum(off, red);
        if (off <= tol2 || off == 0.0) return sweep;
        if (sweep == 60) return -1;
        for (int r = 0; r < m - 1; ++r) {
            // rotation parameters
            for (int k = t; k < npair; k += T) {
                int p, q;
                rr_pair(m, r, k, p, q);
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = C[p + q * n];
                    if (apq != 0.0) {
                        const double app = C[p + p * n], aqq = C[q + q * n];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                cs[k] = c;
                sn[k] = s;
                pp[k] = p;
                qq[k] = (q < n) ? q : -1;
            }
            __syncthreads();
            // columns: C <- C J
            for (int e = t; e < npair * n; e += T) {
                const int k = e / n, row = e - k * n;
                const int q = qq[k];
                if (q < 0 || sn[k] == 0.0) continue;
                const int p = pp[k];
                const double c = cs[k], s = sn[k];
                const double x = C[row + p * n], y = C[row + q * n];
                C[row + p * n] = c * x - s * y;
                C[row + q * n] = s * x + c * y;
            }
            __syncthreads();
            // rows: C <- J^T C ; and Z <- Z J
            for (int e = t; e < npair * n; e += T) {
                const int k = e / n, col = e - k * n;
                const int q = qq[k];
                if (q < 0 || sn[k] == 0.0) continue;
                const int p = pp[k];
                const double c = cs[k], s = sn[k];
                const double x = C[p + col * n], y = C[q + col * n];
                C[p + col * n] = c * x - s * y;
                C[q + col * n] = s * x + c * y;
                const double zx = Z[col + p * n], zy = Z[col + q * n];
                Z[col + p * n] = c * zx - s * zy;
                Z[col + q * n] = s * zx + c * zy;
            }
            __syncthreads();
            for (int k = t; k < npair; k += T) {
                const int q = qq[k];
                if (q < 0 || sn[k] == 0.0) continue;
                const int p = pp[k];
                C[p + q * n] = 0.0;
                C[q + p * n] = 0.0;
            }
            __syncthreads();
        }
    }
    return -1;
}

// In-place lower Cholesky (right-looking) of the n x n matrix A (ld n);
// returns false if a pivot is not positive.
__device__ bool cholesky(double *A, int n, int *flag) {
    const int t = threadIdx.x, T = blockDim.x;
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double d = A[j + j * n];
        if (!(d > 0.0)) {
            if (t == 0) *flag = 1;
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

// X <- L^{-1} X for lower-triangular L (n x n) and X (n x m), one column
// per thread group.
__device__ void trsm_lower(const double *L, int n, double *X, int m) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int c = t; c < m; c += T) {
        double *x = X + (int64_t)c * n;
        for (int i = 0; i < n; ++i) {
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= L[i + k * n] * x[k];
            x[i] = s / L[i + i * n];
        }
    }
    __syncthreads();
}

// X <- L^{-T} X (back substitution with L^T upper triangular).
__device__ void trsm_lower_t(const double *L, int n, double *X, int m) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int c = t; c < m; c += T) {
        double *x = X + (int64_t)c * n;
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int k = i + 1; k < n; ++k) s -= L[k + i * n] * x[k];
            x[i] = s / L[i + i * n];
        }
    }
    __syncthreads();
}

// in-place transpose of a square matrix
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

// Order of n values: rank[i] = position of value i (descending if desc),
// ties by index.  Written to ord[rank] = i.
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
    double *C, *Z, *L, *T;  // n x n each
    double *cs, *sn, *w;    // n
    int *pp, *qq, *ord, *flag;
};

__global__ __launch_bounds__(SE_THREADS) void k_pencil(const double *__restrict__ H,
                                                       const double *__restrict__ G, int n,
                                                       int which_smallest, double *__restrict__ theta,
                                                       double *__restrict__ Y, PencilWork w,
                                                       int *status) {
    __shared__ double red[16];
    const int t = threadIdx.x, T = blockDim.x;
    // symmetrised copies
    for (int e = t; e < n * n; e += T) {
        const int i = e % n, j = e / n;
        w.L[e] = 0.5 * (G[i + j * n] + G[j + i * n]);
        w.C[e] = 0.5 * (H[i + j * n] + H[j + i * n]);
    }
    __syncthreads();
    int rank = n;
    const bool pd = cholesky(w.L, n, w.flag);
    if (pd) {
        // C <- L^{-1} C L^{-T}
        trsm_lower(w.L, n, w.C, n);
        transpose_sq(w.C, n);
        trsm_lower(w.L, n, w.C, n);
        for (int e = t; e < n * n; e += T) {
            const int i = e % n, j = e / n;
            if (i < j) {
                const double s = 0.5 * (w.C[i + j * n] + w.C[j + i * n]);
                w.C[i + j * n] = s;
                w.C[j + i * n] = s;
            }
        }
        __syncthreads();
        const int sw = jacobi(w.C, w.Z, n, w.cs, w.sn, w.pp, w.qq, red);
        if (t == 0 && sw < 0) *status = 2;
        for (int i = t; i < n; i += T) w.w[i] = w.C[i + i * n];
        __syncthreads();
        trsm_lower_t(w.L, n, w.Z, n);  // Z <- L^{-T} Z
    } else {
        // G-eigen truncation: G = U D U^T, keep d_i > 1e-14 max d
        for (int e = t; e < n * n; e += T) {
            const int i = e % n, j = e / n;
            w.L[e] = 0.5 * (G[i + j * n] + G[j + i * n]);
        }
        __syncthreads();
        int sw = jacobi(w.L, w.T, n, w.cs, w.sn, w.pp, w.qq, red);
        if (t == 0 && sw < 0) *status = 2;
        // d_i = L_ii; scaled kept directions: T[:, i] *= 1/sqrt(d_i) or 0
        __shared__ double dmax;
        if (t == 0) {
            double m = 0.0;
            for (int i = 0; i < n; ++i) m = fmax(m, w.L[i + i * n]);
            dmax = m;
        }
        __syncthreads();
        // order kept directions first (by index among kept)
        if (t == 0) {
            int c = 0;
            for (int i = 0; i < n; ++i)
                if (w.L[i + i * n] > 1e-14 * dmax) w.ord[c++] = i;
            w.flag[0] = c;
        }
        __syncthreads();
        rank = w.flag[0];
        // Tk (n x rank) = U_i / sqrt(d_i) for kept i, into Z
        for (int e = t; e < n * rank; e += T) {
            const int row = e % n, c = e / n;
            const int i = w.ord[c];
            w.Z[row + c * n] = w.T[row + i * n] / sqrt(w.L[i + i * n]);
        }
        __syncthreads();
        // C_r = Tk^T H_sym Tk  (rank x rank, ld n): first HT = H Tk into T
        for (int e = t; e < n * rank; e += T) {
            const int row = e % n, c = e / n;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += w.C[row + k * n] * w.Z[k + c * n];
            w.T[row + c * n] = s;
        }
        __syncthreads();
        for (int e = t; e < rank * rank; e += T) {
            const int i = e % rank, j = e / rank;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += w.Z[k + i * n] * w.T[k + j * n];
            w.L[i + j * rank] = s;  // compact rank x rank, ld rank
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
        sw = jacobi(w.L, w.T, rank, w.cs, w.sn, w.pp, w.qq, red);  // eigvecs in T (ld rank)
        if (t == 0 && sw < 0) *status = 2;
        for (int i = t; i < rank; i += T) w.w[i] = w.L[i + i * rank];
        __syncthreads();
        // Y_r = Tk Zr  (n x rank) -> stash in C (ld n)
        for (int e = t; e < n * rank; e += T) {
            const int row = e % n, c = e / n;
            double s = 0.0;
            for (int k = 0; k < rank; ++k) s += w.Z[row + k * n] * w.T[k + c * rank];
            w.C[row + c * n] = s;
        }
        __syncthreads();
        for (int e = t; e < n * rank; e += T) w.Z[e] = w.C[e];
        __syncthreads();
        if (t == 0) *status = (*status == 2) ? 2 : 1;
    }
    // sort the `rank` values and write outputs; columns beyond rank are zero
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
    if (!cholesky(LU, k1, w.flag)) {
        if (t == 0) *status = 3;
        return;
    }
    if (!cholesky(LV, k2, w.flag)) {
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
    const int sw = jacobi(w.C, w.Z, N, w.cs, w.sn, w.pp, w.qq, red);
    if (t == 0 && sw < 0) *status = 2;
    for (int i = t; i < N; i += T) w.w[i] = w.C[i + i * N];
    __syncthreads();
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

PencilWork make_work(Context *ctx, int n) {
    PencilWork w;
    const size_t nn = (size_t)n * n;
    double *base = ctx->buf<double>("pencil_work", 4 * nn + 3 * n + 64);
    w.C = base;
    w.Z = base + nn;
    w.L = base + 2 * nn;
    w.T = base + 3 * nn;
    w.cs = base + 4 * nn;
    w.sn = w.cs + n;
    w.w = w.sn + n;
    int *ib = ctx->buf<int>("pencil_iwork", 3 * (size_t)n + 8);
    w.pp = ib;
    w.qq = ib + n;
    w.ord = ib + 2 * n;
    w.flag = ib + 3 * n;
    return w;
}

}  // namespace

int32_t pencil_eig(Context *ctx, int32_t b, const double *H, const double *G, ofrr_which which,
                   double *theta, double *Y, bool want_rank) {
    OFRR_CHECK_ARG(b >= 1 && b <= 1024, "pencil: 1 <= b <= 1024");
    PencilWork w = make_work(ctx, b + 1);
    int *status = ctx->buf<int>("pencil_status", 4);
    zero_bytes(ctx, status, 16);
    {
        KTimer tm(ctx, "small_eig");
        hipLaunchKernelGGL(k_pencil, dim3(1), dim3(SE_THREADS), 0, ctx->stream, H, G, b,
                           which == OFRR_SMALLEST ? 1 : 0, theta, Y, w, status);
        OFRR_HIP(hipGetLastError());
    }
    int host[2] = {0, 0};
    OFRR_HIP(hipMemcpyAsync(&host[0], status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    OFRR_HIP(hipMemcpyAsync(&host[1], w.flag + 1, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    if (host[0] == 2) fail(OFRR_ERR_NUMERIC, "pencil: Jacobi did not converge");
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
    if (host == 2) fail(OFRR_ERR_NUMERIC, "svd pencil: Jacobi did not converge");
}

}  // namespace ofrr
