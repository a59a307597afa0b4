// k_general.hip -- residuals and returned vectors of complex Ritz pairs for
// a real non-symmetric A (Sec. 3.1: the Galerkin condition admits complex
// Ritz values).
//
// The Ritz block is held real and packed: a real Ritz value's column is its
// vector; a conjugate pair lambda = a +- i b (b > 0, + member first) takes
// two adjacent columns, xr = Re x and xi = Im x of the + member's vector
// (the - member's vector is the conjugate).  With AX the same columns of
// A X, both members have the residual
//   ||A x - lambda x||^2 = ||AXr - a xr + b xi||^2 + ||AXi - b xr - a xi||^2
// and ||x||^2 = ||xr||^2 + ||xi||^2.
#include <algorithm>
#include <cstdint>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

// packed-column role of slot c: first column of its unit (p) and whether it
// is a pair; the - member of a pair reads the unit that starts one before it
__device__ __forceinline__ void gen_unit(const double *__restrict__ th_im, int c, int &p, bool &pair) {
    const double im = th_im[c];
    pair = im != 0.0;
    p = im < 0.0 ? c - 1 : c;
}

// Per 64-row block partial sums for every slot c < nc: res2[blk][c] the
// squared residual, xn2[blk][c] the squared norm (row-major X, AX, ld).
template <class T>
__global__ __launch_bounds__(256) void k_res_general(const T *__restrict__ X, const T *__restrict__ AX, int64_t ld,
                                                     int64_t n, int nc, const double *__restrict__ th_re,
                                                     const double *__restrict__ th_im, double *__restrict__ res2,
                                                     double *__restrict__ xn2) {
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int64_t r1 = r0 + 64 < n ? r0 + 64 : n;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        int p;
        bool pair;
        gen_unit(th_im, c, p, pair);
        const double a = th_re[p], b = pair ? th_im[p] : 0.0;
        double sr = 0.0, sx = 0.0;
        for (int64_t i = r0; i < r1; ++i) {
            const double xr = load_as_f64(X + i * ld + p), ar = load_as_f64(AX + i * ld + p);
            if (pair) {
                const double xi = load_as_f64(X + i * ld + p + 1), ai = load_as_f64(AX + i * ld + p + 1);
                const double u = ar - a * xr + b * xi, w = ai - b * xr - a * xi;
                sr += u * u + w * w;
                sx += xr * xr + xi * xi;
            } else {
                const double u = ar - a * xr;
                sr += u * u;
                sx += xr * xr;
            }
        }
        res2[(int64_t)blockIdx.x * nc + c] = sr;
        xn2[(int64_t)blockIdx.x * nc + c] = sx;
    }
}

// Final pass over the k wanted slots (one workgroup per slot; X, AX FP64
// row-major, ld): norm, residual, and the entry of largest modulus (first
// on ties) with its value.
__global__ __launch_bounds__(256) void k_final_general_cols(const double *__restrict__ X, const double *__restrict__ AX,
                                                            int64_t ld, int64_t n, const double *__restrict__ th_re,
                                                            const double *__restrict__ th_im,
                                                            double *__restrict__ tmp) {
    const int c = blockIdx.x, t = threadIdx.x;
    int p;
    bool pair;
    gen_unit(th_im, c, p, pair);
    const double a = th_re[p], b = pair ? th_im[p] : 0.0;
    double sx = 0.0, sr = 0.0, best = -1.0, bvr = 0.0, bvi = 0.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = t; i < n; i += 256) {
        const double xr = X[i * ld + p], ar = AX[i * ld + p];
        const double xi = pair ? X[i * ld + p + 1] : 0.0, ai = pair ? AX[i * ld + p + 1] : 0.0;
        const double u = ar - a * xr + b * xi, w = ai - b * xr - a * xi;
        const double m2 = xr * xr + xi * xi;
        sx += m2;
        sr += u * u + w * w;
        if (m2 > best) {
            best = m2;
            bi = i;
            bvr = xr;
            bvi = xi;
        }
    }
    __shared__ double s_best[256], s_vr[256], s_vi[256];
    __shared__ int64_t s_bi[256];
    s_best[t] = best;
    s_bi[t] = bi;
    s_vr[t] = bvr;
    s_vi[t] = bvi;
    const double tx = block_sum_f64(sx);
    const double tr = block_sum_f64(sr);
    __syncthreads();
    if (t == 0) {
        double bb = s_best[0], vr = s_vr[0], vi = s_vi[0];
        int64_t ii = s_bi[0];
        for (int q = 1; q < 256; ++q)
            if (s_best[q] > bb || (s_best[q] == bb && s_bi[q] < ii)) {
                bb = s_best[q];
                ii = s_bi[q];
                vr = s_vr[q];
                vi = s_vi[q];
            }
        // the - member's vector is the conjugate
        if (th_im[c] < 0.0) vi = -vi;
        double *o = tmp + 6 * (int64_t)c;
        o[0] = sqrt(tx);
        o[1] = sqrt(tr);
        o[2] = vr;
        o[3] = vi;
        o[4] = (double)ii;
    }
}

// evecs = x * conj(x_m) / (|x_m| ||x||) (x_m the largest entry), the x_m
// entry written as the exact real |x_m| / ||x||; evals, resid per slot
__global__ void k_final_general_write(const double *__restrict__ X, int64_t ld, int64_t n, int k,
                                      const double *__restrict__ th_re, const double *__restrict__ th_im,
                                      const double *__restrict__ tmp, double anorm, double *__restrict__ evals_re,
                                      double *__restrict__ evals_im, double *__restrict__ evecs_re,
                                      double *__restrict__ evecs_im, double *__restrict__ resid) {
    const int64_t total = n * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n);
        const int64_t i = e - (int64_t)c * n;
        int p;
        bool pair;
        gen_unit(th_im, c, p, pair);
        const double *o = tmp + 6 * (int64_t)c;
        const double nx = o[0] > 0.0 ? o[0] : 1.0;
        const double mr = o[2], mi = o[3];
        const double mm = sqrt(mr * mr + mi * mi);
        // phase factor conj(x_m) / |x_m| / ||x||
        const double fr = mm > 0.0 ? mr / mm / nx : 1.0 / nx, fi = mm > 0.0 ? -mi / mm / nx : 0.0;
        const double xr = X[i * ld + p];
        double xi = pair ? X[i * ld + p + 1] : 0.0;
        if (th_im[c] < 0.0) xi = -xi;
        double yr = xr * fr - xi * fi, yi = xr * fi + xi * fr;
        if (i == (int64_t)o[4]) {
            yr = mm / nx;
            yi = 0.0;
        }
        evecs_re[i + (int64_t)c * n] = yr;
        evecs_im[i + (int64_t)c * n] = yi;
        if (i == 0) {
            evals_re[c] = th_re[c];
            evals_im[c] = th_im[c];
            resid[c] = o[1] / nx / anorm;
        }
    }
}

inline int grid1(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

}  // namespace

void residual_partials_general(Context *ctx, ofrr_dtype t, int64_t n, int32_t nc, const void *X, const void *AX,
                               int64_t ld, const double *th_re, const double *th_im, double *res2, double *xn2) {
    KTimer tm(ctx, "residual");
    const unsigned nblk = (unsigned)((n + 63) / 64);
    switch (t) {
        case OFRR_F64:
            hipLaunchKernelGGL(k_res_general<double>, dim3(nblk), dim3(256), 0, ctx->stream, (const double *)X,
                               (const double *)AX, ld, n, nc, th_re, th_im, res2, xn2);
            break;
        case OFRR_F32:
            hipLaunchKernelGGL(k_res_general<float>, dim3(nblk), dim3(256), 0, ctx->stream, (const float *)X,
                               (const float *)AX, ld, n, nc, th_re, th_im, res2, xn2);
            break;
        default: fail(OFRR_ERR_UNSUPPORTED, "general residuals: FP32 or FP64 blocks");
    }
    OFRR_HIP(hipGetLastError());
}

void finalize_general(Context *ctx, int64_t n, int32_t k, const double *X, const double *AX, int64_t ld,
                      const double *th_re, const double *th_im, double anorm, double *evals_re,
                      double *evals_im, double *evecs_re, double *evecs_im, double *resid) {
    KTimer tm(ctx, "residual");
    double *tmp = ctx->buf<double>("general_final_tmp", 6 * (size_t)k + 8);
    hipLaunchKernelGGL(k_final_general_cols, dim3(k), dim3(256), 0, ctx->stream, X, AX, ld, n, th_re, th_im, tmp);
    OFRR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_final_general_write, dim3(grid1(n * k)), dim3(256), 0, ctx->stream, X, ld, n, k, th_re,
                       th_im, tmp, anorm, evals_re, evals_im, evecs_re, evecs_im, resid);
    OFRR_HIP(hipGetLastError());
}

}  // namespace ofrr
