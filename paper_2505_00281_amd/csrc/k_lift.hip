// k_lift.hip -- the Ritz lift X = V Y and A X = W Y (Alg. "Orthogonalization-
// Free Rayleigh-Ritz Projection", last line; Sec. 2: restart from all Ritz
// vectors), residual estimates R = A X - X Theta, the filter recurrences and
// the final normalisation of the returned eigenvectors.
//
// A X = W Y needs no product with A because W = A V is already formed; the
// same identity makes the first filter step of the next outer iteration
// free.  Blocks are row-major (i*ld + j); the small coefficient matrix Y is
// column-major FP64.
#include <set>
#include <type_traits>
#include <utility>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

// OUT1 = IN1 * S[:, :nc], OUT2 = IN2 * S[:, :nc] (IN2 optional), 64 x 64
// output tiles, 16-deep K slices; optional residual partial sums per tile
// row block: res2[blk][c] = sum_i (OUT2 - theta_c OUT1)^2, xn2[blk][c] =
// sum_i OUT1^2.
template <class TI1, class TI2, class TO>
__global__ __launch_bounds__(256) void k_tall_small(const TI1 *__restrict__ In1, int64_t ld1,
                                                    const TI2 *__restrict__ In2, int64_t ld2,
                                                    int64_t n, int b, int nc,
                                                    const double *__restrict__ S, int lds,
                                                    const double *__restrict__ theta,
                                                    TO *__restrict__ Out1, TO *__restrict__ Out2,
                                                    int64_t ldo, double *__restrict__ res2,
                                                    double *__restrict__ xn2) {
    __shared__ double A1[64][17];
    __shared__ double A2[64][17];
    __shared__ double Ss[16][65];
    __shared__ double red[2][16][64];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    const bool two = In2 != nullptr;
    double acc1[4][4] = {}, acc2[4][4] = {};
    for (int k0 = 0; k0 < b; k0 += 16) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = t + 256 * s;
            const int rr = e >> 4, kk = e & 15;
            const int64_t gi = i0 + rr;
            const int gk = k0 + kk;
            const bool ok = gi < n && gk < b;
            A1[rr][kk] = ok ? load_as_f64(In1 + gi * ld1 + gk) : 0.0;
            if (two) A2[rr][kk] = ok ? load_as_f64(In2 + gi * ld2 + gk) : 0.0;
            const int sk = e >> 6, sc = e & 63;
            Ss[sk][sc] = (k0 + sk < b && c0 + sc < nc) ? S[(k0 + sk) + (int64_t)(c0 + sc) * lds] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double s[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = Ss[kk][tx + 16 * q];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const double a1 = A1[ty + 16 * p][kk];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc1[p][q] = fma(a1, s[q], acc1[p][q]);
                if (two) {
                    const double a2 = A2[ty + 16 * p][kk];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc2[p][q] = fma(a2, s[q], acc2[p][q]);
                }
            }
        }
        __syncthreads();
    }
    double r2[4] = {0, 0, 0, 0}, x2[4] = {0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int64_t gi = i0 + ty + 16 * p;
        if (gi >= n) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gc = c0 + tx + 16 * q;
            if (gc >= nc) continue;
            store_as<TO>(Out1 + gi * ldo + gc, acc1[p][q]);
            if (two) store_as<TO>(Out2 + gi * ldo + gc, acc2[p][q]);
            if (res2) {
                const double x = acc1[p][q];
                const double r = acc2[p][q] - theta[gc] * x;
                r2[q] += r * r;
                x2[q] += x * x;
            }
        }
    }
    if (res2) {
        // column sums over the 16 ty-groups, fixed order
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            red[0][ty][tx + 16 * q] = r2[q];
            red[1][ty][tx + 16 * q] = x2[q];
        }
        __syncthreads();
        if (t < 64) {
            double a = 0.0, c = 0.0;
            for (int y = 0; y < 16; ++y) {
                a += red[0][y][t];
                c += red[1][y][t];
            }
            const int gc = c0 + t;
            if (gc < nc) {
                res2[(int64_t)blockIdx.x * nc + gc] = a;
                xn2[(int64_t)blockIdx.x * nc + gc] = c;
            }
        }
    }
}

// out[c] = sqrt(sum_blk res2[blk][c]) / sqrt(sum_blk xn2[blk][c]) / anorm
__global__ __launch_bounds__(256) void k_res_reduce(const double *__restrict__ res2,
                                                    const double *__restrict__ xn2, int nblk, int nc,
                                                    int count, double anorm, double *__restrict__ out,
                                                    const int32_t *__restrict__ extra,
                                                    const int32_t *__restrict__ extra2) {
    // one wavefront per column: lanes take every 64th partial, then a fixed
    // butterfly sum (deterministic)
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (extra && blockIdx.x == 0 && threadIdx.x == 0) out[count] = (double)extra[0];
    if (extra2 && blockIdx.x == 0 && threadIdx.x < 2) out[count + 1 + threadIdx.x] = (double)extra2[threadIdx.x];
    if (c >= count) return;
    double a = 0.0, x = 0.0;
    for (int i = lane; i < nblk; i += 64) {
        a += res2[(int64_t)i * nc + c];
        x += xn2[(int64_t)i * nc + c];
    }
    a = wave_sum_f64(a);
    x = wave_sum_f64(x);
    if (lane == 0) out[c] = (x > 0.0) ? sqrt(a) / sqrt(x) / anorm : 0.0;
}

// The same lift on FP64 MFMA (v_mfma_f64_16x16x4) for b, nc <= 128 and one
// input type: a workgroup takes 64 rows (16 per wave) and every column; Y is
// staged in LDS once (b x nc FP64).  Within each 16-deep K block, lane l
// holds row l % 16 of its wave's rows and the four consecutive K entries
// 4 (l / 16) .. +3 (one vector load), and MFMA step s uses K = 4 (l / 16) + s
// on both operands (any consistent K order gives the same sum up to
// rounding).  Accumulator register r of lane l is D[4 r + l / 16][l % 16].
typedef double lf_f64x4_t __attribute__((ext_vector_type(4)));
template <class TI>
struct LiftVec;
template <>
struct LiftVec<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
};
template <>
struct LiftVec<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
};

constexpr int LF_LDK = 129;  // LDS row stride of the coefficients (128 columns + 1)

template <class TI, class TO, bool TWO, int NQ>
__global__ __launch_bounds__(256) void k_lift_mfma(const TI *__restrict__ In1, int64_t ld1,
                                                   const TI *__restrict__ In2, int64_t ld2, int64_t n, int b,
                                                   int nc, const double *__restrict__ S, int lds,
                                                   const double *__restrict__ theta, TO *__restrict__ Out1,
                                                   TO *__restrict__ Out2, int64_t ldo, double *__restrict__ res2,
                                                   double *__restrict__ xn2) {
    extern __shared__ __attribute__((aligned(16))) double Ys[];  // [k][c], kpad x 128, row stride LF_LDK
    __shared__ double red[2][4][128];
    typedef typename LiftVec<TI>::v4 v4;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, cl = lane & 15;
    constexpr bool two = TWO;
    // NQ 16-column tiles (8 for nc <= 128, 4 for nc <= 64)
    // Y (column-major, leading dimension lds) into LDS as [k][c], zero-padded
    // to kpad = 16 ceil(b / 16) rows and 16 NQ columns, so every operand read
    // below is unconditional: consecutive threads read consecutive k of a
    // column (coalesced), eight loads in flight per thread; the odd row
    // stride spreads both the stores and the MFMA operand reads over the banks
    const int kpad = (b + 15) / 16 * 16;
    {
        const int tot = kpad * 16 * NQ;
        for (int e0 = 0; e0 < tot; e0 += 256 * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + 256 * u + t;
                const int c = e / kpad, k = e - c * kpad;
                v[u] = S[(k < b ? k : b - 1) + (int64_t)(c < nc ? c : nc - 1) * lds];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + 256 * u + t;
                const int c = e / kpad, k = e - c * kpad;
                if (e < tot) Ys[k * LF_LDK + c] = (k < b && c < nc) ? v[u] : 0.0;
            }
        }
    }
    __syncthreads();
    // the workgroup lifts 64-row blocks blockIdx.x, + gridDim.x, ... with the
    // coefficients staged once (a grid of at most a few workgroups per CU)
    const int64_t nblk = (n + 63) / 64;
    // residual partials of this workgroup's blocks (thread t < nc: column t),
    // summed over its blocks in order and written once
    double racc = 0.0, xacc = 0.0;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t rowA = blk * 64 + 16 * wave + cl;  // this lane's operand row
    const bool rok = rowA < n;
    const int ntile = (nc + 15) / 16;
    lf_f64x4_t acc1[NQ], acc2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc1[q] = acc2[q] = lf_f64x4_t{0.0, 0.0, 0.0, 0.0};
    // K blocks of 16; lane group g takes the block's entries 4g .. 4g + 3
    auto mfma_block = [&](int k0, const double (&a1)[4], const double (&a2)[4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * g + s;
            // all NQ column tiles (the padding is zero): the operand reads
            // are static and unconditional, so they are issued together
            double yq[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) yq[q] = Ys[k * LF_LDK + 16 * q + cl];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                acc1[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], yq[q], acc1[q], 0, 0, 0);
                if constexpr (TWO) acc2[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[s], yq[q], acc2[q], 0, 0, 0);
            }
        }
    };
    const auto vec_aligned = [](const TI *p, int64_t ld) {
        return ((uintptr_t)p & (sizeof(v4) - 1)) == 0 && (ld & 3) == 0;
    };
    const bool fast = (b & 15) == 0 && vec_aligned(In1, ld1) && (!two || vec_aligned(In2, ld2));
    if (fast) {
        // every load of the lane's row (clamped to the block, unconditional)
        // is issued D blocks ahead of its use; rows past n are zeroed where
        // the values are used
        constexpr int NKB = 8;  // b <= 128
        constexpr int D = sizeof(TI) == 4 ? 8 : 4;
        const int64_t rc = rok ? rowA : n - 1;
        const TI *p1 = In1 + rc * ld1;
        const TI *p2 = two ? In2 + rc * ld2 : p1;
        v4 xr[D], yr[D];
        auto fetch = [&](int kb8, v4 &x, v4 &y) {
            const int col = (16 * kb8 + 4 * g < b) ? 16 * kb8 + 4 * g : b - 4;
            x = *reinterpret_cast<const v4 *>(p1 + col);
            y = *reinterpret_cast<const v4 *>(p2 + col);
        };
#pragma unroll
        for (int q = 0; q < D; ++q) fetch(q, xr[q], yr[q]);
#pragma unroll
        for (int kb8 = 0; kb8 < NKB; ++kb8) {
            if (16 * kb8 >= b) break;
            const v4 x = xr[kb8 % D], y = yr[kb8 % D];
            if (kb8 + D < NKB) fetch(kb8 + D, xr[kb8 % D], yr[kb8 % D]);
            double a1[4], a2[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                a1[s] = rok ? (double)x[s] : 0.0;
                a2[s] = rok ? (double)y[s] : 0.0;
            }
            mfma_block(16 * kb8, a1, a2);
        }
    } else {
        for (int k0 = 0; k0 < b; k0 += 16) {
            const int kb = k0 + 4 * g;  // this lane's four K entries
            double a1[4], a2[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool ok = rok && kb + s < b;
                a1[s] = ok ? load_as_f64(In1 + rowA * ld1 + kb + s) : 0.0;
                a2[s] = (ok && two) ? load_as_f64(In2 + rowA * ld2 + kb + s) : 0.0;
            }
            mfma_block(k0, a1, a2);
        }
    }
    // outputs, and the residual partials of this 64-row block
    const int64_t rbase = blk * 64 + 16 * wave + g;  // + 4 r
    double r2[NQ], x2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) r2[q] = x2[q] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int c = 16 * q + cl;
        if (q >= ntile || c >= nc) continue;
        const double th = res2 ? theta[c] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gi = rbase + 4 * r;
            if (gi >= n) continue;
            const double x = acc1[q][r];
            store_as<TO>(Out1 + gi * ldo + c, x);
            if (two) store_as<TO>(Out2 + gi * ldo + c, acc2[q][r]);
            const double rr = acc2[q][r] - th * x;
            r2[q] += rr * rr;
            x2[q] += x * x;
        }
    }
    if (res2) {
        // over the four lane groups (fixed butterfly), then the four waves
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            r2[q] += __shfl_xor(r2[q], 16, 64);
            r2[q] += __shfl_xor(r2[q], 32, 64);
            x2[q] += __shfl_xor(x2[q], 16, 64);
            x2[q] += __shfl_xor(x2[q], 32, 64);
        }
        if (g == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                red[0][wave][16 * q + cl] = r2[q];
                red[1][wave][16 * q + cl] = x2[q];
            }
        }
        __syncthreads();
        if (t < nc) {
            racc += (red[0][0][t] + red[0][1][t]) + (red[0][2][t] + red[0][3][t]);
            xacc += (red[1][0][t] + red[1][1][t]) + (red[1][2][t] + red[1][3][t]);
        }
        __syncthreads();  // red is rewritten by the next block
    }
    }
    if (res2 && t < nc) {
        res2[(int64_t)blockIdx.x * nc + t] = racc;
        xn2[(int64_t)blockIdx.x * nc + t] = xacc;
    }
}

// Elementwise kernels over row-major n x b blocks: 256 / min(b, 256) rows per
// workgroup pass, threads over columns (no per-element integer division).
#define OFRR_ROWS_COLS_LOOP(BODY)                                                        \
    const int cols_ = b < 256 ? b : 256;                                                 \
    const int groups_ = 256 / cols_;                                                     \
    const int j0_ = threadIdx.x % cols_, g_ = threadIdx.x / cols_;                       \
    if (g_ < groups_)                                                                    \
        for (int64_t i = (int64_t)blockIdx.x * groups_ + g_; i < n; i += (int64_t)gridDim.x * groups_) \
            for (int j = j0_; j < b; j += cols_) { BODY }

template <class TI, class TO>
__global__ void k_axpby(const TI *__restrict__ AX, const TI *__restrict__ X, int64_t ld, int64_t n,
                        int b, double alpha, double beta, TO *__restrict__ Y, int64_t ldy) {
    OFRR_ROWS_COLS_LOOP(
        const double v = alpha * load_as_f64(AX + i * ld + j) + (beta != 0.0 ? beta * load_as_f64(X + i * ld + j) : 0.0);
        store_as<TO>(Y + i * ldy + j, v);)
}

template <class TP, class TS, class TN>
__global__ void k_cheb(const TP *__restrict__ P, const TS *__restrict__ Yc, const TS *__restrict__ Yp,
                       int64_t ld, int64_t n, int b, double alpha, double c, double beta,
                       TN *__restrict__ Yn) {
    OFRR_ROWS_COLS_LOOP(
        const int64_t o = i * ld + j;
        double v = alpha * fma(-c, load_as_f64(Yc + o), load_as_f64(P + o));
        if (beta != 0.0) v = fma(-beta, load_as_f64(Yp + o), v);
        store_as<TN>(Yn + o, v);)
}

// The recurrence with P = sum of nsplit split-K slabs, summed in slab order in
// the slab type (the reduction kernel's arithmetic, so the same P).
template <class TSL, class TS, class TN>
__global__ void k_cheb_slabs(const TSL *__restrict__ P, int nsplit, int64_t sstride, const TS *__restrict__ Yc,
                             const TS *__restrict__ Yp, int64_t ld, int64_t n, int b, double alpha, double c,
                             double beta, TN *__restrict__ Yn) {
    OFRR_ROWS_COLS_LOOP(
        const int64_t o = i * ld + j;
        TSL s = (TSL)0;
        for (int z = 0; z < nsplit; ++z) s += P[(int64_t)z * sstride + o];
        double v = alpha * fma(-c, load_as_f64(Yc + o), (double)s);
        if (beta != 0.0) v = fma(-beta, load_as_f64(Yp + o), v);
        store_as<TN>(Yn + o, v);)
}

// Final step: per column norms of X and of R = AX - theta X, sign of the
// entry of largest magnitude (first on ties).  One workgroup per column.
__global__ __launch_bounds__(256) void k_final_cols(const double *__restrict__ X, int64_t ldx,
                                                    const double *__restrict__ AX, int64_t ldax,
                                                    int64_t n, const double *__restrict__ theta,
                                                    double *__restrict__ xnorm,
                                                    double *__restrict__ rnorm,
                                                    double *__restrict__ sgn) {
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    double sx = 0.0, sr = 0.0, best = -1.0;
    int64_t bi = INT64_MAX;
    double bv = 0.0;
    for (int64_t i = t; i < n; i += 256) {
        const double x = X[i * ldx + c];
        const double r = AX[i * ldax + c] - theta[c] * x;
        sx += x * x;
        sr += r * r;
        if (fabs(x) > best) {
            best = fabs(x);
            bi = i;
            bv = x;
        }
    }
    __shared__ double s_best[256];
    __shared__ int64_t s_bi[256];
    __shared__ double s_bv[256];
    s_best[t] = best;
    s_bi[t] = bi;
    s_bv[t] = bv;
    const double tx = block_sum_f64(sx);
    const double tr = block_sum_f64(sr);
    __syncthreads();
    if (t == 0) {
        double bb = s_best[0];
        int64_t ii = s_bi[0];
        double vv = s_bv[0];
        for (int k = 1; k < 256; ++k)
            if (s_best[k] > bb || (s_best[k] == bb && s_bi[k] < ii)) {
                bb = s_best[k];
                ii = s_bi[k];
                vv = s_bv[k];
            }
        xnorm[c] = sqrt(tx);
        rnorm[c] = sqrt(tr);
        sgn[c] = vv < 0.0 ? -1.0 : 1.0;
    }
}

__global__ void k_final_write(const double *__restrict__ X, int64_t ldx, int64_t n, int k,
                              const double *__restrict__ theta, const double *__restrict__ xnorm,
                              const double *__restrict__ rnorm, const double *__restrict__ sgn,
                              double anorm, double *__restrict__ evals, double *__restrict__ evecs,
                              double *__restrict__ resid) {
    const int64_t total = n * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n);
        const int64_t i = e - (int64_t)c * n;
        const double nx = xnorm[c] > 0.0 ? xnorm[c] : 1.0;
        evecs[i + (int64_t)c * n] = X[i * ldx + c] * (sgn[c] / nx);
        if (i == 0) {
            evals[c] = theta[c];
            resid[c] = rnorm[c] / nx / anorm;
        }
    }
}

__global__ void k_scale_array(double *x, int64_t n, double f) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        x[e] *= f;
}

// out[c] = ||X1_c - s_c X2_c|| / ||X2_c|| / anorm, one workgroup per column
template <class T>
__global__ __launch_bounds__(256) void k_col_resid(const T *__restrict__ X1, const T *__restrict__ X2,
                                                   int64_t ld, int64_t n,
                                                   const double *__restrict__ s, double anorm,
                                                   double *__restrict__ out) {
    const int c = blockIdx.x;
    double a = 0.0, x = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v2 = load_as_f64(X2 + i * ld + c);
        const double r = load_as_f64(X1 + i * ld + c) - s[c] * v2;
        a += r * r;
        x += v2 * v2;
    }
    a = block_sum_f64(a);
    x = block_sum_f64(x);
    if (threadIdx.x == 0) out[c] = x > 0.0 ? sqrt(a) / sqrt(x) / anorm : 0.0;
}

// SVD final: norms of u, v (first pass), sign from v's largest entry
__global__ __launch_bounds__(256) void k_svd_norms(const double *__restrict__ Uv, int64_t m,
                                                   const double *__restrict__ Vv, int64_t n,
                                                   int64_t ld, double *__restrict__ un,
                                                   double *__restrict__ vn, double *__restrict__ sg) {
    const int c = blockIdx.x, t = threadIdx.x;
    double su = 0.0, sv = 0.0, best = -1.0, bv = 0.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = t; i < m; i += 256) su += Uv[i * ld + c] * Uv[i * ld + c];
    for (int64_t i = t; i < n; i += 256) {
        const double v = Vv[i * ld + c];
        sv += v * v;
        if (fabs(v) > best) {
            best = fabs(v);
            bi = i;
            bv = v;
        }
    }
    __shared__ double s_best[256], s_bv[256];
    __shared__ int64_t s_bi[256];
    s_best[t] = best;
    s_bi[t] = bi;
    s_bv[t] = bv;
    su = block_sum_f64(su);
    sv = block_sum_f64(sv);
    __syncthreads();
    if (t == 0) {
        double bb = s_best[0], vv = s_bv[0];
        int64_t ii = s_bi[0];
        for (int q = 1; q < 256; ++q)
            if (s_best[q] > bb || (s_best[q] == bb && s_bi[q] < ii)) {
                bb = s_best[q];
                ii = s_bi[q];
                vv = s_bv[q];
            }
        un[c] = sqrt(su);
        vn[c] = sqrt(sv);
        sg[c] = vv < 0.0 ? -1.0 : 1.0;
    }
}

// residual of the normalised pair and the column-major outputs
__global__ __launch_bounds__(256) void k_svd_final(const double *__restrict__ Uv,
                                                   const double *__restrict__ AV, int64_t m,
                                                   const double *__restrict__ Vv,
                                                   const double *__restrict__ ATU, int64_t n,
                                                   int64_t ld, const double *__restrict__ sig,
                                                   const double *__restrict__ un,
                                                   const double *__restrict__ vn,
                                                   const double *__restrict__ sg, double anorm,
                                                   double *__restrict__ sig_out,
                                                   double *__restrict__ Uo, double *__restrict__ Vo,
                                                   double *__restrict__ resid) {
    const int c = blockIdx.x, t = threadIdx.x;
    const double iu = un[c] > 0 ? 1.0 / un[c] : 1.0, iv = vn[c] > 0 ? 1.0 / vn[c] : 1.0;
    const double s = sig[c];
    double r1 = 0.0, r2 = 0.0;
    for (int64_t i = t; i < m; i += 256) {
        const double u = Uv[i * ld + c] * iu;
        const double r = AV[i * ld + c] * iv - s * u;
        r1 += r * r;
        Uo[i + (int64_t)c * m] = u * sg[c];
    }
    for (int64_t i = t; i < n; i += 256) {
        const double v = Vv[i * ld + c] * iv;
        const double r = ATU[i * ld + c] * iu - s * v;
        r2 += r * r;
        Vo[i + (int64_t)c * n] = v * sg[c];
    }
    r1 = block_sum_f64(r1);
    r2 = block_sum_f64(r2);
    if (t == 0) {
        resid[c] = sqrt(r1 + r2) / anorm;
        sig_out[c] = s;
    }
}

template <class F>
void dispatch_t(ofrr_dtype t, F &&f) {
    switch (t) {
        case OFRR_F64: f((double *)nullptr); break;
        case OFRR_F32: f((float *)nullptr); break;
        case OFRR_BF16: f((bf16_t *)nullptr); break;
        case OFRR_F16: f((f16_t *)nullptr); break;
        default: fail(OFRR_ERR_UNSUPPORTED, "lift: element type");
    }
}

inline int grid1(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

}  // namespace

int64_t lift(Context *ctx, int64_t n, int32_t b, int32_t nc, ofrr_dtype vt, const void *V,
             int64_t ldv, ofrr_dtype wt, const void *W, int64_t ldw, const double *Y, int32_t ldy,
             const double *theta, ofrr_dtype xt, void *X, void *AX, int64_t ldx, double *res2,
             double *xn2) {
    KTimer tm(ctx, "lift");
    int64_t prow = (n + 63) / 64;  // rows of residual partials written
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((nc + 63) / 64));
    if (vt != wt && W != nullptr) {
        // mixed input types: lift the two products separately
        lift(ctx, n, b, nc, vt, V, ldv, vt, nullptr, 0, Y, ldy, nullptr, xt, X, nullptr, ldx,
             nullptr, nullptr);
        lift(ctx, n, b, nc, wt, W, ldw, wt, nullptr, 0, Y, ldy, nullptr, xt, AX, nullptr, ldx,
             nullptr, nullptr);
        OFRR_CHECK_ARG(res2 == nullptr, "lift: residual partials need one input type");
        return 0;
    }
    // FP64 MFMA path when the coefficients fit one LDS stage and the input is
    // FP32 or FP64 (whose residual partials use the same 64-row blocks)
    const bool mfma = b <= 128 && nc <= 128 && (vt == OFRR_F32 || vt == OFRR_F64);
    if (mfma) {
        static std::set<std::pair<int, const void *>> lds_set;
        dispatch_t(vt, [&](auto *ip) {
            using TI = std::remove_pointer_t<decltype(ip)>;
            if constexpr (std::is_same<TI, float>::value || std::is_same<TI, double>::value) {
                dispatch_t(xt, [&](auto *op) {
                    using TO = std::remove_pointer_t<decltype(op)>;
                    auto launch = [&](auto kernel) {
                        const void *kern = (const void *)kernel;
                        if (!lds_set.count({ctx->device, kern})) {
                            OFRR_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                         128 * LF_LDK * (int)sizeof(double)));
                            lds_set.insert({ctx->device, kern});
                        }
                        const size_t shmem = (size_t)((b + 15) / 16 * 16) * LF_LDK * sizeof(double);
                        // at most two workgroups per CU (what its registers and
                        // LDS hold at once), each over several 64-row blocks
                        const int64_t nblk = (n + 63) / 64;
                        const int64_t cap = 2LL * (ctx->cu_count > 0 ? ctx->cu_count : 256);
                        const unsigned gl = (unsigned)(nblk < cap ? nblk : cap);
                        prow = gl;
                        hipLaunchKernelGGL(kernel, dim3(gl), dim3(256), shmem, ctx->stream,
                                           (const TI *)V, ldv, (const TI *)W, ldw, n, b, nc, Y, ldy, theta,
                                           (TO *)X, (TO *)AX, ldx, res2, xn2);
                    };
                    if (nc <= 64) {
                        if (W)
                            launch(k_lift_mfma<TI, TO, true, 4>);
                        else
                            launch(k_lift_mfma<TI, TO, false, 4>);
                    } else {
                        if (W)
                            launch(k_lift_mfma<TI, TO, true, 8>);
                        else
                            launch(k_lift_mfma<TI, TO, false, 8>);
                    }
                });
            }
        });
    } else {
        dispatch_t(vt, [&](auto *ip) {
            using TI = std::remove_pointer_t<decltype(ip)>;
            dispatch_t(xt, [&](auto *op) {
                using TO = std::remove_pointer_t<decltype(op)>;
                hipLaunchKernelGGL((k_tall_small<TI, TI, TO>), grid, dim3(256), 0, ctx->stream,
                                   (const TI *)V, ldv, (const TI *)W, ldw, n, b, nc, Y, ldy, theta,
                                   (TO *)X, (TO *)AX, ldx, res2, xn2);
            });
        });
    }
    OFRR_HIP(hipGetLastError());
    return prow;
}

void residual_reduce(Context *ctx, const double *res2, const double *xn2, int nblk, int stride,
                     int count, double anorm, double *out, const int32_t *extra, const int32_t *extra2) {
    hipLaunchKernelGGL(k_res_reduce, dim3((count + 3) / 4), dim3(256), 0, ctx->stream, res2, xn2,
                       nblk, stride, count, anorm, out, extra, extra2);
    OFRR_HIP(hipGetLastError());
}

void axpby_block(Context *ctx, int64_t n, int32_t b, ofrr_dtype it, const void *AX, const void *X,
                 int64_t ld, double alpha, double beta, ofrr_dtype yt, void *Y, int64_t ldy) {
    dispatch_t(it, [&](auto *ip) {
        using TI = std::remove_pointer_t<decltype(ip)>;
        dispatch_t(yt, [&](auto *op) {
            using TO = std::remove_pointer_t<decltype(op)>;
            hipLaunchKernelGGL((k_axpby<TI, TO>), dim3(grid1(n * b)), dim3(256), 0, ctx->stream,
                               (const TI *)AX, (const TI *)X, ld, n, b, alpha, beta, (TO *)Y, ldy);
        });
    });
    OFRR_HIP(hipGetLastError());
}

void cheb_combine(Context *ctx, int64_t n, int32_t b, ofrr_dtype pt, const void *P, ofrr_dtype st,
                  const void *Ycur, const void *Yprev, int64_t ld, double alpha, double c,
                  double beta, ofrr_dtype nt, void *Ynext) {
    dispatch_t(pt, [&](auto *pp) {
        using TP = std::remove_pointer_t<decltype(pp)>;
        dispatch_t(st, [&](auto *sp) {
            using TS = std::remove_pointer_t<decltype(sp)>;
            dispatch_t(nt, [&](auto *np) {
                using TN = std::remove_pointer_t<decltype(np)>;
                hipLaunchKernelGGL((k_cheb<TP, TS, TN>), dim3(grid1(n * b)), dim3(256), 0,
                                   ctx->stream, (const TP *)P, (const TS *)Ycur, (const TS *)Yprev,
                                   ld, n, b, alpha, c, beta, (TN *)Ynext);
            });
        });
    });
    OFRR_HIP(hipGetLastError());
}

void cheb_combine_slabs(Context *ctx, int64_t n, int32_t b, const SlabOut &P, ofrr_dtype st, const void *Ycur,
                        const void *Yprev, int64_t ld, double alpha, double c, double beta, ofrr_dtype nt,
                        void *Ynext) {
    OFRR_CHECK_ARG(P.t == OFRR_F32 || P.t == OFRR_F64, "slab type");
    auto go = [&](auto *slp) {
        using TSL = std::remove_pointer_t<decltype(slp)>;
        dispatch_t(st, [&](auto *sp) {
            using TS = std::remove_pointer_t<decltype(sp)>;
            dispatch_t(nt, [&](auto *np) {
                using TN = std::remove_pointer_t<decltype(np)>;
                hipLaunchKernelGGL((k_cheb_slabs<TSL, TS, TN>), dim3(grid1(n * b)), dim3(256), 0, ctx->stream,
                                   (const TSL *)P.p, P.nsplit, P.stride, (const TS *)Ycur, (const TS *)Yprev, ld, n,
                                   b, alpha, c, beta, (TN *)Ynext);
            });
        });
    };
    if (P.t == OFRR_F32)
        go((float *)nullptr);
    else
        go((double *)nullptr);
    OFRR_HIP(hipGetLastError());
}

void finalize_eig(Context *ctx, int64_t n, int32_t k, const double *X, int64_t ldx,
                  const double *AX, int64_t ldax, const double *theta, double anorm,
                  double *evals, double *evecs, double *resid) {
    KTimer tm(ctx, "residual");
    double *tmp = ctx->buf<double>("final_tmp", 3 * (size_t)k + 8);
    hipLaunchKernelGGL(k_final_cols, dim3(k), dim3(256), 0, ctx->stream, X, ldx, AX, ldax, n, theta,
                       tmp, tmp + k, tmp + 2 * k);
    OFRR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_final_write, dim3(grid1(n * k)), dim3(256), 0, ctx->stream, X, ldx, n, k,
                       theta, tmp, tmp + k, tmp + 2 * k, anorm, evals, evecs, resid);
    OFRR_HIP(hipGetLastError());
}

}  // namespace ofrr

namespace ofrr {

void scale_array(Context *ctx, int64_t count, double *x, double f) {
    hipLaunchKernelGGL(k_scale_array, dim3(grid1(count)), dim3(256), 0, ctx->stream, x, count, f);
    OFRR_HIP(hipGetLastError());
}

void col_resid(Context *ctx, ofrr_dtype t, int64_t n, int32_t count, const void *X1, const void *X2,
               int64_t ld, const double *s, double anorm, double *out) {
    dispatch_t(t, [&](auto *p) {
        using T = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_col_resid<T>), dim3(count), dim3(256), 0, ctx->stream, (const T *)X1,
                           (const T *)X2, ld, n, s, anorm, out);
    });
    OFRR_HIP(hipGetLastError());
}

void finalize_svd(Context *ctx, int64_t m, int64_t n, int32_t k, const double *Uv, const double *AV,
                  const double *Vv, const double *ATU, int64_t ld, const double *sigma,
                  double anorm, double *sig_out, double *Uo, double *Vo, double *resid) {
    KTimer tm(ctx, "residual");
    double *tmp = ctx->buf<double>("svd_final_tmp", 3 * (size_t)k + 8);
    hipLaunchKernelGGL(k_svd_norms, dim3(k), dim3(256), 0, ctx->stream, Uv, m, Vv, n, ld, tmp,
                       tmp + k, tmp + 2 * k);
    OFRR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_svd_final, dim3(k), dim3(256), 0, ctx->stream, Uv, AV, m, Vv, ATU, n, ld,
                       sigma, tmp, tmp + k, tmp + 2 * k, anorm, sig_out, Uo, Vo, resid);
    OFRR_HIP(hipGetLastError());
}

}  // namespace ofrr
