// k_gemm_i8.hip -- FP64-class block product W = op(A) V for the final,
// full-accuracy phase, on INT8 MFMA with exact integer accumulation.
//
// The final phase needs products accurate to far below the 1e-8 residual
// target, which FP32 accumulation cannot give (its rounding is about
// 2^-24 |A||V|).  MI355X runs FP64 at 78.6 TFLOP/s but INT8 MFMA at
// 5 POP/s, so the product is rebuilt from exact integer pieces:
//   op(A)[i][k] = 2^{e_i} sum_{s=1..6} a_s[i][k] 2^{-7s}   (+ |rest| < 2^{e_i-42})
//   V[k][j]     = 2^{f_j} sum_{t=1..6} v_t[k][j] 2^{-7t}   (+ |rest| < 2^{f_j-42})
// with signed 7-bit digits |a_s|, |v_t| <= 127 (truncation of the scaled
// value, exact in floating point), e_i the exponent bound of row i of
// op(A) and f_j that of column j of V.  Then
//   W[i][j] = 2^{e_i + f_j} sum_{p=2..7} 2^{-7p} sum_{s+t=p} (a_s v_t)[i][j]
// keeping the 21 digit pairs with s + t <= 7.  Every (a_s v_t) is an exact
// int8 x int8 -> int32 dot product; pairs with equal s + t share one int32
// accumulator (at most 6 pairs x 127^2 x 16384 < 2^31 per K range, so the
// K range of one accumulation is capped at 16384).  The dropped pairs and
// the digit remainders are below 2^-42 of the row/column scales, about
// 2e-13 of |A||V| where FP32 accumulation gives 6e-8.  That margin matters:
// the basis of a converging subspace is ill-conditioned, and the Ritz
// values amplify per-column product errors by the cancellation in V z;
// five digits per side (2^-35) left Ritz values 1e-9 off.  Iterations whose
// residuals are still far above that level take fewer digits: five (15
// pairs) or four (10 pairs), the leading digit planes of the same slicing.
//
// MFMA v_mfma_i32_32x32x32_i8: lane l holds A[l%32][16(l/32)..+16] and
// B[16(l/32)..+16][l%32] (any consistent K order is exact for integers);
// accumulator register r is D[(r/4)*8 + 4(l/32) + r%4][l%32].
#include <string>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

constexpr int I8_S = 6;     // digit planes of A and of V
constexpr int I8_BM = 64;   // rows per workgroup tile
constexpr int I8_BK = 64;   // K bytes per LDS stage
constexpr int I8_LD = 80;   // LDS row stride in bytes (64 + 16: conflict-free 16-byte reads)
constexpr int I8_KMAX = 16384;  // K per int32 accumulation

// Digit planes are stored K-blocked: 64-deep K blocks, each holding all
// (padded) rows of the plane with their 64 digits contiguous.  A workgroup's
// 64-deep stage of 64 rows is then one contiguous 4 KiB span, so every
// 128-byte line it fetches is used whole (a row-major plane read 64 bytes at
// a time fetched each line twice).
__device__ __forceinline__ int64_t plane_off(int64_t row, int64_t k, int64_t rows_pad) {
    return ((k >> 6) * rows_pad + row) * 64 + (k & 63);
}

// exponent e with |x| < 2^e for the largest |x| (0 for an all-zero set)
__device__ __forceinline__ int exp_bound(double amax) {
    if (!(amax > 0.0)) return 0;
    int e;
    (void)frexp(amax, &e);  // amax = m 2^e, m in [0.5, 1)
    return e;
}

// I8_S signed 7-bit digits of x 2^-e, |x 2^-e| < 1, by truncation (exact)
__device__ __forceinline__ void digits_of(double x, int e, int8_t (&d)[I8_S]) {
    double r = ldexp(x, -e);
#pragma unroll
    for (int s = 0; s < I8_S; ++s) {
        r *= 128.0;
        const double q = trunc(r);
        d[s] = (int8_t)(int)q;
        r -= q;
    }
}

// Row slicing of op(A) (one workgroup per output row, rows past m zero).
// ATRANS: op(A)[i][k] = A[k + i*lda] (K-contiguous), else A[i + k*lda].
template <class TA, bool ATRANS>
__global__ __launch_bounds__(256) void k_slice_rows(const TA *__restrict__ A, int64_t lda, int64_t m,
                                                    int64_t mpad, int64_t kdim, int64_t kpad,
                                                    int8_t *__restrict__ planes, int64_t plane_stride,
                                                    int32_t *__restrict__ ex) {
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    const int t = threadIdx.x;
    // row i clamped into A, so every load is unconditional; eight loads in
    // flight per thread for the row maximum
    const int64_t ic = i < m ? i : m - 1;
    auto at = [&](int64_t k) -> double {
        return (double)(ATRANS ? A[k + ic * lda] : A[ic + k * lda]);
    };
    double amax = 0.0;
    if (i < m) {
        int64_t k = t;
        for (; k + 7 * 256 < kdim; k += 8 * 256) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = at(k + 256 * u);
#pragma unroll
            for (int u = 0; u < 8; ++u) amax = fmax(amax, fabs(v[u]));
        }
        for (; k < kdim; k += 256) amax = fmax(amax, fabs(at(k)));
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    if ((t & 63) == 0) red[t >> 6] = amax;
    __syncthreads();
    amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const int e = exp_bound(amax);
    if (t == 0) ex[i] = e;
    for (int64_t k0 = (int64_t)t * 16; k0 < kpad; k0 += 256 * 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = at(k0 + q < kdim ? k0 + q : kdim - 1);
        int8_t d[I8_S][16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int8_t dq[I8_S];
            digits_of((i < m && k0 + q < kdim) ? v[q] : 0.0, e, dq);
#pragma unroll
            for (int s = 0; s < I8_S; ++s) d[s][q] = dq[s];
        }
#pragma unroll
        for (int s = 0; s < I8_S; ++s)
            *(v4i_t *)(planes + s * plane_stride + plane_off(i, k0, mpad)) = __builtin_bit_cast(v4i_t, d[s]);
    }
}

// Row slicing of a column-major A (op(A) = A): one workgroup per 64 rows, a
// lane per row, so every load of a wavefront is 64 consecutive entries of one
// column (one row per workgroup would touch a cache line per entry).  The
// four wavefronts take interleaved 16-column chunks; the row maxima meet in
// LDS; the planes and exponents are those of k_slice_rows.
template <class TA>
__global__ __launch_bounds__(256) void k_slice_rows_cm(const TA *__restrict__ A, int64_t lda, int64_t m,
                                                       int64_t mpad, int64_t kdim, int64_t kpad,
                                                       int8_t *__restrict__ planes, int64_t plane_stride,
                                                       int32_t *__restrict__ ex) {
    __shared__ double red[4][64];
    const int t = threadIdx.x, r = t & 63, w = t >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + r;
    // row i clamped into A and columns clamped into [0, kdim): every load
    // is unconditional
    const TA *a = A + (i < m ? i : m - 1);
    auto at = [&](int64_t k) -> double { return (double)a[(k < kdim ? k : kdim - 1) * lda]; };
    double amax = 0.0;
    for (int64_t k0 = (int64_t)w * 16; k0 < kdim; k0 += 64) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = at(k0 + q);
#pragma unroll
        for (int q = 0; q < 16; ++q) amax = fmax(amax, fabs(v[q]));
    }
    red[w][r] = i < m ? amax : 0.0;
    __syncthreads();
    amax = fmax(fmax(red[0][r], red[1][r]), fmax(red[2][r], red[3][r]));
    const int e = exp_bound(amax);
    if (w == 0 && i < mpad) ex[i] = e;
    if (i >= mpad) return;
    for (int64_t k0 = (int64_t)w * 16; k0 < kpad; k0 += 64) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = at(k0 + q);
        int8_t d[I8_S][16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int8_t dq[I8_S];
            digits_of((i < m && k0 + q < kdim) ? v[q] : 0.0, e, dq);
#pragma unroll
            for (int s = 0; s < I8_S; ++s) d[s][q] = dq[s];
        }
#pragma unroll
        for (int s = 0; s < I8_S; ++s)
            *(v4i_t *)(planes + s * plane_stride + plane_off(i, k0, mpad)) = __builtin_bit_cast(v4i_t, d[s]);
    }
}

constexpr int VM_COPIES = 4;    // copies of the merged column maxima
constexpr int VM_STRIDE = 4096;  // entries per copy (b <= 4096)

__global__ void k_zero_u64(unsigned long long *__restrict__ p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

// Column maxima of an FP64 row-major block (rows x b, ld) over 64-row
// blocks, merged by atomic maximum of the (non-negative) FP64 bit patterns
// into cmax[c * VM_STRIDE + j], c = block index mod VM_COPIES (zero on
// entry; the maximum does not depend on the merge order).  For b <= 256 the 256 threads split
// into 256 / b row groups over the block's rows (consecutive threads read
// consecutive columns), loads unrolled by 8.
__global__ __launch_bounds__(256) void k_vmax_partial(const double *__restrict__ V, int64_t rows, int b,
                                                      int64_t ld, unsigned long long *__restrict__ cmax) {
    __shared__ double cm[256];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int64_t r1 = r0 + 64 < rows ? r0 + 64 : rows;
    for (int jb = 0; jb < b; jb += 256) {
        const int cols = (b - jb) < 256 ? (b - jb) : 256;
        const int groups = 256 / cols;
        const int j = jb + t % cols, g = t / cols;
        double m = 0.0;
        if (g < groups) {
            int64_t r = r0 + g;
            for (; r + 7 * groups < r1; r += 8 * groups) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = V[(r + u * groups) * ld + j];
#pragma unroll
                for (int u = 0; u < 8; ++u) m = fmax(m, fabs(v[u]));
            }
            for (; r < r1; r += groups) m = fmax(m, fabs(V[r * ld + j]));
        }
        cm[t] = m;
        __syncthreads();
        if (t < cols) {
            double mm = 0.0;
            for (int q = 0; q < groups; ++q) mm = fmax(mm, cm[q * cols + t]);
            atomicMax(cmax + (blockIdx.x % VM_COPIES) * VM_STRIDE + jb + t, (unsigned long long)__double_as_longlong(mm));
        }
        __syncthreads();
    }
}

// Digit planes of V, K-contiguous per column: planes[s][j][k], 16 rows of
// one column per thread (columns past b and rows past `rows` are zero).
__global__ __launch_bounds__(256) void k_vslice(const double *__restrict__ V, int64_t rows, int b,
                                                int64_t ld, int bpad, int64_t kpad,
                                                const unsigned long long *__restrict__ cmax,
                                                unsigned long long *__restrict__ clear,
                                                int32_t *__restrict__ fx,
                                                int8_t *__restrict__ planes, int64_t plane_stride) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gstride = (int64_t)gridDim.x * blockDim.x;
    // the other merge arrays, whole, for the next call (whatever its width)
    for (int64_t e = gid; e < (int64_t)VM_COPIES * VM_STRIDE; e += gstride) clear[e] = 0ull;
    const int64_t total = (int64_t)bpad * (kpad / 16);
    for (int64_t e = gid; e < total; e += gstride) {
        const int j = (int)(e % bpad);
        const int64_t k0 = (e / bpad) * 16;
        // the column's exponent bound from its merged maximum (columns past
        // b have none: 0); written out once for the product
        unsigned long long mb = 0ull;
#pragma unroll
        for (int c = 0; c < VM_COPIES; ++c) mb = max(mb, cmax[c * VM_STRIDE + j]);
        const int f = exp_bound(__longlong_as_double((long long)mb));
        if (k0 == 0) fx[j] = f;
        // the sixteen loads first (clamped into the block, unconditional),
        // the range test where the values are used
        const int jc = j < b ? j : b - 1;
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t k = k0 + q;
            v[q] = V[(k < rows ? k : rows - 1) * ld + jc];
        }
        int8_t d[I8_S][16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int8_t dq[I8_S];
            digits_of((j < b && k0 + q < rows) ? v[q] : 0.0, f, dq);
#pragma unroll
            for (int s = 0; s < I8_S; ++s) d[s][q] = dq[s];
        }
#pragma unroll
        for (int s = 0; s < I8_S; ++s)
            *(v4i_t *)(planes + s * plane_stride + plane_off(j, k0, bpad)) = __builtin_bit_cast(v4i_t, d[s]);
    }
}

// W slab z (rows x b FP64, ld) = the K range z of op(A) V from the digit
// planes.  Workgroup tile 64 rows x (64 NCT) columns with 4 NCT waves, one
// 32 x 32 output block each (six int32 accumulators = 96 registers), so two
// waves share each SIMD and hide each other's LDS and global latency;
// 64-byte K stages through LDS, the next stage prefetched into registers.
// (s, u) digit pairs with s + u < S (0-based) for S = 6, 5, 4 digits per
// side, ordered so that two pairs of equal s + u (one accumulator) are at
// least three apart, also cyclically across K steps (four digits: two, the
// most an order of ten pairs with a group of four allows)
constexpr int kPair6S[21] = {0, 5, 3, 2, 3, 0, 1, 1, 4, 0, 0, 2, 0, 2, 0, 1, 2, 1, 3, 1, 4};
constexpr int kPair6U[21] = {0, 0, 1, 1, 2, 1, 2, 3, 1, 2, 3, 2, 5, 0, 4, 0, 3, 1, 0, 4, 0};
constexpr int kPair5S[15] = {4, 1, 2, 1, 1, 2, 0, 0, 0, 2, 0, 1, 3, 3, 0};
constexpr int kPair5U[15] = {0, 2, 0, 3, 0, 1, 4, 1, 3, 2, 0, 1, 1, 0, 2};
constexpr int kPair4S[10] = {0, 1, 0, 2, 0, 1, 1, 0, 2, 3};
constexpr int kPair4U[10] = {1, 2, 0, 1, 2, 0, 1, 3, 0, 0};

template <int S>
__device__ __forceinline__ int pair_s(int q) {
    return S == 6 ? kPair6S[q] : (S == 5 ? kPair5S[q] : kPair4S[q]);
}
template <int S>
__device__ __forceinline__ int pair_u(int q) {
    return S == 6 ? kPair6U[q] : (S == 5 ? kPair5U[q] : kPair4U[q]);
}

template <int NCT, int S>
__global__ __launch_bounds__(256 * NCT) void k_gemm_i8s(const int8_t *__restrict__ Ap, int64_t a_stride,
                                                        const int32_t *__restrict__ ex,
                                                        const int8_t *__restrict__ Vp, int64_t v_stride,
                                                        const int32_t *__restrict__ fx, int64_t kpad,
                                                        int64_t mpad, int bpad, int64_t m, int b,
                                                        double *__restrict__ W, int64_t ldw,
                                                        int64_t k_per_split, int ntiles, int nsplit,
                                                        int xcd_map) {
    constexpr int BN = 64 * NCT;
    constexpr int NT = 256 * NCT;                  // threads
    constexpr int NG = S;                          // digit-pair groups p = s + u
    constexpr int NP = S * (S + 1) / 2;            // digit pairs
    constexpr int ATOT = S * I8_BM * 4, VTOT = S * BN * 4;  // 16-byte chunks per stage
    constexpr int ACH = (ATOT + NT - 1) / NT;      // A chunks per thread per stage
    constexpr int VCH = (VTOT + NT - 1) / NT;      // V chunks per thread per stage
    __shared__ __attribute__((aligned(16))) int8_t As[S][I8_BM][I8_LD];
    __shared__ __attribute__((aligned(16))) int8_t Vs[S][BN][I8_LD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave / (2 * NCT), wc = wave % (2 * NCT);
    int tile, z;
    const int L = blockIdx.x;
    if (xcd_map) {
        const int xcd = L & 7, slot = L >> 3, per = 8 / nsplit;
        z = xcd % nsplit;
        tile = slot * per + xcd / nsplit;
    } else {
        tile = L % ntiles;
        z = L / ntiles;
    }
    if (tile >= ntiles) return;
    const int gy = (b + BN - 1) / BN;
    const int64_t i0 = (int64_t)(tile / gy) * I8_BM;
    const int j0 = (tile % gy) * BN;
    const int64_t kbeg = (int64_t)z * k_per_split;
    const int64_t kend = kbeg + k_per_split < kpad ? kbeg + k_per_split : kpad;

    v16i_t acc[NG];
#pragma unroll
    for (int p = 0; p < NG; ++p) acc[p] = v16i_t{};

    // chunk c of a stage: plane c / (rows * 4), row (c / 4) % rows, 16 bytes at 16 (c % 4)
    v4i_t ra[ACH], rv[VCH];
    auto fetch = [&](int64_t k0) {
    // (a chunk index past the stage, possible when the chunks do not divide
    // evenly among the threads, is clamped to the last chunk for the load
    // and skipped for the store)
#pragma unroll
        for (int u = 0; u < ACH; ++u) {
            int c = t + NT * u;
            if (ATOT % NT != 0) c = c < ATOT ? c : ATOT - 1;
            const int pl = c / (I8_BM * 4), rem = c % (I8_BM * 4);
            ra[u] = *(const v4i_t *)(Ap + pl * a_stride + plane_off(i0 + (rem >> 2), k0 + (rem & 3) * 16, mpad));
        }
#pragma unroll
        for (int u = 0; u < VCH; ++u) {
            int c = t + NT * u;
            if (VTOT % NT != 0) c = c < VTOT ? c : VTOT - 1;
            const int pl = c / (BN * 4), rem = c % (BN * 4);
            rv[u] = *(const v4i_t *)(Vp + pl * v_stride + plane_off(j0 + (rem >> 2), k0 + (rem & 3) * 16, bpad));
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < ACH; ++u) {
            const int c = t + NT * u;
            if (ATOT % NT != 0 && c >= ATOT) continue;
            const int pl = c / (I8_BM * 4), rem = c % (I8_BM * 4);
            *(v4i_t *)&As[pl][rem >> 2][(rem & 3) * 16] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < VCH; ++u) {
            const int c = t + NT * u;
            if (VTOT % NT != 0 && c >= VTOT) continue;
            const int pl = c / (BN * 4), rem = c % (BN * 4);
            *(v4i_t *)&Vs[pl][rem >> 2][(rem & 3) * 16] = rv[u];
        }
    };

    fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += I8_BK) {
        stash();
        __syncthreads();
        if (k0 + I8_BK < kend) fetch(k0 + I8_BK);
#pragma unroll
        for (int ks = 0; ks < I8_BK; ks += 32) {
            const int kq = ks + 16 * (lane >> 5);
            v4i_t a[S], v[S];
#pragma unroll
            for (int s = 0; s < S; ++s) a[s] = *(const v4i_t *)&As[s][32 * wr + (lane & 31)][kq];
#pragma unroll
            for (int s = 0; s < S; ++s) v[s] = *(const v4i_t *)&Vs[s][32 * wc + (lane & 31)][kq];
            // the digit pairs in an order that keeps two MFMAs on the same
            // accumulator apart
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int s = pair_s<S>(q), u = pair_u<S>(q);
                acc[s + u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[s], v[u], acc[s + u], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double *Wz = W + (int64_t)z * m * ldw;
    const int gj = j0 + 32 * wc + (lane & 31);
    const int fj = gj < b ? fx[gj] : 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t gi = i0 + 32 * wr + (r >> 2) * 8 + 4 * (lane >> 5) + (r & 3);
        if (gi >= m || gj >= b) continue;
        double v = (double)acc[NG - 1][r];
#pragma unroll
        for (int p = NG - 2; p >= 0; --p) v = (double)acc[p][r] + v * 0.0078125;
        Wz[gi * ldw + gj] = ldexp(v, ex[gi] + fj - 14);
    }
}

__global__ void k_sum_slabs_f64(const double *__restrict__ P, int nsplit, int64_t m, int b, int64_t ld,
                                double *__restrict__ W) {
    const int64_t total = m * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / b;
        const int j = (int)(e - i * b);
        double s = 0.0;
        for (int zz = 0; zz < nsplit; ++zz) s += P[(int64_t)zz * m * ld + i * ld + j];
        W[i * ld + j] = s;
    }
}

inline int grid1(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

}  // namespace

SlicedA slice_matrix_i8(Context *ctx, const ofrr_matrix *A, int trans, const char *tag) {
    OFRR_CHECK_ARG(A->format == OFRR_DENSE_COLMAJOR, "sliced product: dense A");
    OFRR_CHECK_ARG(A->dtype == OFRR_F32 || A->dtype == OFRR_F64, "sliced product: A is F32 or F64");
    SlicedA s;
    s.m = trans ? A->cols : A->rows;
    s.kdim = trans ? A->rows : A->cols;
    s.mpad = (s.m + I8_BM - 1) / I8_BM * I8_BM;
    s.kpad = (s.kdim + I8_BK - 1) / I8_BK * I8_BK;
    s.plane_stride = s.mpad * s.kpad;
    s.planes = ctx->buf<int8_t>(std::string(tag) + "_planes", (size_t)I8_S * s.plane_stride);
    s.ex = ctx->buf<int32_t>(std::string(tag) + "_exp", (size_t)s.mpad);
    KTimer tm(ctx, "quantize");
    auto go = [&](auto kern, auto p) {
        hipLaunchKernelGGL(kern, dim3((unsigned)s.mpad), dim3(256), 0, ctx->stream, p, A->ld, s.m, s.mpad,
                           s.kdim, s.kpad, s.planes, s.plane_stride, s.ex);
    };
    const float *af = (const float *)A->values;
    const double *ad = (const double *)A->values;
    // A's rows (column-major A): 64 rows per workgroup, mpad a multiple of 64
    static_assert(I8_BM % 64 == 0, "row slicing assumes mpad is a multiple of 64");
    auto go_cm = [&](auto kern, auto p) {
        hipLaunchKernelGGL(kern, dim3((unsigned)(s.mpad / 64)), dim3(256), 0, ctx->stream, p, A->ld, s.m, s.mpad,
                           s.kdim, s.kpad, s.planes, s.plane_stride, s.ex);
    };
    if (A->dtype == OFRR_F32) {
        if (trans) go(k_slice_rows<float, true>, af); else go_cm(k_slice_rows_cm<float>, af);
    } else {
        if (trans) go(k_slice_rows<double, true>, ad); else go_cm(k_slice_rows_cm<double>, ad);
    }
    OFRR_HIP(hipGetLastError());
    return s;
}

void product_i8s(Context *ctx, const SlicedA &sa, int32_t b, const double *V, int64_t ldv, double *W,
                 int64_t ldw, SlabOut *defer, int digits) {
    OFRR_CHECK_ARG(b >= 1 && b <= 4096, "sliced product: 1 <= b <= 4096");
    OFRR_CHECK_ARG(digits >= 4 && digits <= I8_S, "sliced product: 4 to 6 digits per side");
    const int NCT = b > 64 ? 2 : 1;
    const int BN = 64 * NCT;
    const int bpad = (b + BN - 1) / BN * BN;
    const int64_t kpad = sa.kpad;
    // digit planes of V
    const int64_t v_stride = (int64_t)bpad * kpad;
    int8_t *vp = ctx->buf<int8_t>("i8_v_planes", (size_t)I8_S * v_stride);
    int32_t *fx = ctx->buf<int32_t>("i8_v_exp", (size_t)bpad);
    const int nblk = (int)((sa.kdim + 63) / 64);
    // column maxima merged into one of two alternating sets of arrays; the
    // slicing kernel clears the other set, which the next call merges into
    unsigned long long *vm = ctx->buf<unsigned long long>("i8_v_merge", (size_t)2 * VM_COPIES * VM_STRIDE);
    if (ctx->vmax_parity < 0) {
        hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, ctx->stream, vm, 2 * VM_COPIES * VM_STRIDE);
        ctx->vmax_parity = 0;
    }
    unsigned long long *cur = vm + (size_t)VM_COPIES * VM_STRIDE * ctx->vmax_parity;
    unsigned long long *nxt = vm + (size_t)VM_COPIES * VM_STRIDE * (1 - ctx->vmax_parity);
    {
        KTimer tm(ctx, "quantize");
        hipLaunchKernelGGL(k_vmax_partial, dim3(nblk), dim3(256), 0, ctx->stream, V, sa.kdim, b, ldv, cur);
        hipLaunchKernelGGL(k_vslice, dim3(grid1((int64_t)bpad * (kpad / 16))), dim3(256), 0, ctx->stream, V,
                           sa.kdim, b, ldv, bpad, kpad, (const unsigned long long *)cur, nxt, fx, vp, v_stride);
        OFRR_HIP(hipGetLastError());
    }
    ctx->vmax_parity ^= 1;
    // launch shape: enough workgroups for two per CU; K ranges <= I8_KMAX;
    // and K ranges short enough that one range of the basis planes
    // (I8_S x bpad x range bytes, re-read by every row tile) stays within
    // 2 MiB, so it is served from the XCD's L2 rather than refetched
    const int gx = (int)(sa.mpad / I8_BM), gy = bpad / BN;
    const int ntiles = gx * gy;
    int nsplit = 1;
    const int64_t want = 2LL * (ctx->cu_count > 0 ? ctx->cu_count : 256);
    auto vslab = [&](int ns) { return (int64_t)I8_S * bpad * ((kpad + ns - 1) / ns); };
    while ((((int64_t)ntiles * nsplit < want || vslab(nsplit) > (2LL << 20)) && kpad / (nsplit * 2) >= 1024 &&
            nsplit < 8) ||
           (kpad + nsplit - 1) / nsplit > I8_KMAX)
        nsplit *= 2;
    int64_t kps = (kpad + nsplit - 1) / nsplit;
    kps = (kps + I8_BK - 1) / I8_BK * I8_BK;
    nsplit = (int)((kpad + kps - 1) / kps);
    const int xcd_map = (nsplit >= 2 && 8 % nsplit == 0) ? 1 : 0;
    int64_t nwg = (int64_t)ntiles * nsplit;
    if (xcd_map) nwg = (int64_t)((ntiles + 8 / nsplit - 1) / (8 / nsplit)) * 8;
    double *dst = W;
    if (nsplit > 1) dst = ctx->buf<double>("i8_slabs", (size_t)nsplit * sa.m * ldw);
    {
        KTimer tm(ctx, digits == 6 ? "product_i8x_d6" : digits == 5 ? "product_i8x_d5" : "product_i8x_d4");
        auto go = [&](auto kern, int nt) {
            hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(nt), 0, ctx->stream, sa.planes, sa.plane_stride,
                               sa.ex, vp, v_stride, fx, kpad, sa.mpad, bpad, sa.m, b, dst, ldw, kps, ntiles, nsplit,
                               xcd_map);
        };
        if (NCT == 2) {
            if (digits == 6) go(k_gemm_i8s<2, 6>, 512);
            else if (digits == 5) go(k_gemm_i8s<2, 5>, 512);
            else go(k_gemm_i8s<2, 4>, 512);
        } else {
            if (digits == 6) go(k_gemm_i8s<1, 6>, 256);
            else if (digits == 5) go(k_gemm_i8s<1, 5>, 256);
            else go(k_gemm_i8s<1, 4>, 256);
        }
        OFRR_HIP(hipGetLastError());
    }
    if (defer) {
        defer->p = dst;
        defer->t = OFRR_F64;
        defer->nsplit = nsplit;
        defer->stride = sa.m * ldw;
        return;
    }
    if (nsplit > 1) {
        KTimer tm(ctx, "product_reduce");
        hipLaunchKernelGGL(k_sum_slabs_f64, dim3(grid1(sa.m * b)), dim3(256), 0, ctx->stream, dst, nsplit, sa.m,
                           b, ldw, W);
        OFRR_HIP(hipGetLastError());
    }
}

}  // namespace ofrr
