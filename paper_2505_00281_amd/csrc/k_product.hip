// k_product.hip -- the block products W = op(A) V of the subspace iteration
// (Sec. 2: X_{iter} = A^{iter} X_0; Sec. 4: products in reduced precision
// with FP32 accumulation).
//
//   product_f64   FP64 arithmetic, A dense FP64 or FP32 (promoted exactly).
//   (the BF16/F16 MFMA product is in k_gemm_lp.hip)
//   product_csr   CSR A (FP32/FP64 values), one wavefront per row.
//
// Blocks V and W are row-major (element (i, j) at i*ld + j); A is the
// caller's column-major matrix.
#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

// ------------------------------------------------------------------ FP64 --
// W (m x b) = op(A) (m x kdim) * V (kdim x b) on FP64 MFMA
// (v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and B[l/16][l%16];
// accumulator register r of lane l is D[4r + l/16][l%16]).
// Workgroup tile 64 rows x (64 NCT) columns (the whole basis for b <= 128,
// so A is streamed once), 2 x 2 waves of 32 x (32 NCT); 32-deep K stages in
// LDS, the next stage loaded into registers while the MFMAs run; split-K
// with the XCD-aware workgroup map when the tiles alone cannot fill the chip.
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4_t;

constexpr int F64_BM = 64;
constexpr int F64_BK = 32;

template <class TA, bool ATRANS, int NCT>
__global__ __launch_bounds__(256) void k_gemm_f64(const TA *__restrict__ A, int64_t lda, int64_t m,
                                                  int64_t kdim, int b, const double *__restrict__ V,
                                                  int64_t ldv, double *__restrict__ W, int64_t ldw,
                                                  int64_t k_per_split, int ntiles, int nsplit,
                                                  int xcd_map) {
    constexpr int BN = 64 * NCT;
    constexpr int VPT = BN / 8;  // V values per thread per stage
    __shared__ double As[F64_BK][F64_BM + 4];
    __shared__ double Vs[F64_BK][BN + 4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
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
    const int64_t i0 = (int64_t)(tile / gy) * F64_BM;
    const int j0 = (tile % gy) * BN;
    const int64_t kbeg = (int64_t)z * k_per_split;
    const int64_t kend = kbeg + k_per_split < kdim ? kbeg + k_per_split : kdim;

    f64x4_t acc[2][2 * NCT];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2 * NCT; ++q) acc[p][q] = f64x4_t{0.0, 0.0, 0.0, 0.0};

    // A: ATRANS -> thread owns row t/4 and 8 consecutive k; else k t/8 and
    // 8 consecutive rows.  V: k t/8 and VPT consecutive columns.  The loads
    // are unconditional (indices clamped into the operands) and keep the
    // stored values; the range test and the promotion to FP64 happen when
    // the stage is written to LDS, so no load waits before the next is issued.
    TA ra[8];
    double rv[VPT];
    int64_t kf = kbeg;  // first k of the stage held in ra / rv
    auto a_index = [&](int64_t k0, int q, int64_t &gi, int64_t &gk) {
        if (ATRANS) {
            gi = i0 + (t >> 2);
            gk = k0 + (t & 3) * 8 + q;
        } else {
            gk = k0 + (t >> 3);
            gi = i0 + (t & 7) * 8 + q;
        }
    };
    auto fetch = [&](int64_t k0) {
        kf = k0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int64_t gi, gk;
            a_index(k0, q, gi, gk);
            const int64_t ci = gi < m ? gi : m - 1, ck = gk < kend ? gk : kend - 1;
            ra[q] = ATRANS ? A[ck + ci * lda] : A[ci + ck * lda];
        }
        const int64_t vk = k0 + (t >> 3);
        const int64_t cvk = vk < kend ? vk : kend - 1;
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int jj = j0 + (t & 7) * VPT + q;
            rv[q] = V[cvk * ldv + (jj < b ? jj : b - 1)];
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int64_t gi, gk;
            a_index(kf, q, gi, gk);
            const double v = (gi < m && gk < kend) ? (double)ra[q] : 0.0;
            if (ATRANS)
                As[(t & 3) * 8 + q][t >> 2] = v;
            else
                As[t >> 3][(t & 7) * 8 + q] = v;
        }
        const int64_t vk = kf + (t >> 3);
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int jj = j0 + (t & 7) * VPT + q;
            Vs[t >> 3][(t & 7) * VPT + q] = (vk < kend && jj < b) ? rv[q] : 0.0;
        }
    };

    fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += F64_BK) {
        stash();
        __syncthreads();
        if (k0 + F64_BK < kend) fetch(k0 + F64_BK);
#pragma unroll
        for (int kk = 0; kk < F64_BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[2], bv[2 * NCT];
#pragma unroll
            for (int p = 0; p < 2; ++p) a[p] = As[kr][32 * wr + 16 * p + (lane & 15)];
#pragma unroll
            for (int q = 0; q < 2 * NCT; ++q) bv[q] = Vs[kr][32 * NCT * wc + 16 * q + (lane & 15)];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2 * NCT; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], bv[q], acc[p][q], 0, 0, 0);
        }
        __syncthreads();
    }
    double *Wz = W + (int64_t)z * m * ldw;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2 * NCT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = i0 + 32 * wr + 16 * p + 4 * r + (lane >> 4);
                const int gj = j0 + 32 * NCT * wc + 16 * q + (lane & 15);
                if (gi < m && gj < b) Wz[gi * ldw + gj] = acc[p][q][r];
            }
}

__global__ void k_sum_slabs_d(const double *__restrict__ P, int nsplit, int64_t m, int b, int64_t ld,
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

// -------------------------------------------------------------- CSR SpMM --
// One wavefront per row, lane j owns output columns j, j+64, ...  Entry and
// column indices are clamped to the arrays' bounds, so a malformed CSR can
// give wrong numbers but never an access outside them (the structure is
// validated before use by k_csr_check).
template <class TV, class TW, class TA>
__global__ __launch_bounds__(256) void k_spmm(const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci,
                                              const TA *__restrict__ val, int64_t n_rows,
                                              int64_t n_cols, int64_t nnz, int b,
                                              const TV *__restrict__ V, int64_t ldv,
                                              TW *__restrict__ W, int64_t ldw) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n_rows) return;
    int64_t e0 = rp[row], e1 = rp[row + 1];
    if (e0 < 0) e0 = 0;
    if (e1 > nnz) e1 = nnz;
    for (int j = lane; j < b; j += 64) {
        double acc = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t c = ci[e];
            if (c >= 0 && c < n_cols) acc = fma((double)val[e], load_as_f64(V + c * ldv + j), acc);
        }
        store_as<TW>(W + row * ldw + j, acc);
    }
}

// CSR SpMM, vector form (rows of V stored with an even leading dimension).
// A group of L lanes (a power of two, L <= 64) takes one row; every lane
// holds two adjacent columns, so each gathered row of V is read by one
// 4-, 8- or 16-byte load per lane and a 64-column FP64 row by 32 lanes.
// The entries of a row are visited in storage order, four index/value loads
// issued before their four gathers.  Accumulation: FP64 for FP64 vectors,
// FP32 otherwise (the method's reduced-precision products compute in FP32).
// RND rounds each gathered FP32 value to binary16 (1) or bfloat16 (2) on
// load: the product of a reduced-precision phase read straight from its
// FP32 master block, bit for bit the product of the rounded copy.
// With CHEB the Chebyshev three-term step is applied to the product, as
// rounded to its output type, before it is stored:
//   Yn = alpha (P - c Yc) - beta Yp
// with the same fused operations as the separate combine kernel.  Rows are
// handed to the XCDs in contiguous ranges (blockIdx modulo 8 picks the
// XCD), so the rows that share gathered neighbours share an L2.
template <class TG>
struct Pair;
template <>
struct Pair<double> {
    using T = double2;
    static __device__ __forceinline__ void get(const double *p, double &a, double &b) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        a = v.x;
        b = v.y;
    }
};
template <>
struct Pair<float> {
    static __device__ __forceinline__ void get(const float *p, float &a, float &b) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        a = v.x;
        b = v.y;
    }
};
template <>
struct Pair<f16_t> {
    static __device__ __forceinline__ void get(const f16_t *p, float &a, float &b) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
        a = f16_bits_to_f32((uint16_t)(v & 0xffffu));
        b = f16_bits_to_f32((uint16_t)(v >> 16));
    }
};
template <>
struct Pair<bf16_t> {
    static __device__ __forceinline__ void get(const bf16_t *p, float &a, float &b) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
        a = __builtin_bit_cast(float, v << 16);
        b = __builtin_bit_cast(float, v & 0xffff0000u);
    }
};

template <int RND>
__device__ __forceinline__ float spmm_round(float x) {
    if (RND == 1) return f16_bits_to_f32(f32_to_f16_bits(x));
    if (RND == 2) return bf16_bits_to_f32(f32_to_bf16_bits(x));
    return x;
}
template <int RND>
__device__ __forceinline__ double spmm_round(double x) {
    return x;
}

constexpr int SPMM_PASSES = 8;  // row groups per workgroup of the scaled Chebyshev step

__device__ __forceinline__ int64_t xcd_row_block(int64_t bid, int64_t G) {
    const int64_t q = G / 8, r = G % 8, x = bid % 8, k = bid / 8;
    return x * q + (x < r ? x : r) + k;
}

template <class TG, int RND, class TA, bool CHEB>
__global__ __launch_bounds__(256) void k_spmm_v(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const TA *__restrict__ val, int64_t n_rows, int64_t n_cols,
                                                int64_t nnz, int b, int lanes_log2, const TG *__restrict__ V,
                                                int64_t ld,
                                                typename std::conditional<std::is_same<TG, double>::value, double,
                                                                          float>::type *__restrict__ W,
                                                const typename std::conditional<std::is_same<TG, double>::value,
                                                                                double, float>::type *__restrict__ Yc,
                                                const typename std::conditional<std::is_same<TG, double>::value,
                                                                                double, float>::type *__restrict__ Yp,
                                                double alpha, double c, double beta) {
    using ACC = typename std::conditional<std::is_same<TG, double>::value, double, float>::type;
    const int L = 1 << lanes_log2;
    const int rows_per = 256 >> lanes_log2;
    const int64_t blk = xcd_row_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * rows_per + (threadIdx.x >> lanes_log2);
    const int li = threadIdx.x & (L - 1);
    if (row >= n_rows) return;
    int64_t e0 = rp[row], e1 = rp[row + 1];
    if (e0 < 0) e0 = 0;
    if (e1 > nnz) e1 = nnz;
    const int64_t cmax = n_cols - 1;
    for (int j = 2 * li; j < b; j += 2 * L) {
        ACC acc0 = (ACC)0, acc1 = (ACC)0;
        int64_t e = e0;
        for (; e + 4 <= e1; e += 4) {
            int64_t cc[4];
            ACC a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t q = ci[e + u];
                cc[u] = q < 0 ? 0 : (q > cmax ? cmax : q);
                a[u] = (ACC)val[e + u];
            }
            ACC x0[4], x1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) Pair<TG>::get(V + cc[u] * ld + j, x0[u], x1[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc0 = fma(a[u], spmm_round<RND>(x0[u]), acc0);
                acc1 = fma(a[u], spmm_round<RND>(x1[u]), acc1);
            }
        }
        for (; e < e1; ++e) {
            const int64_t q = ci[e];
            const int64_t cc = q < 0 ? 0 : (q > cmax ? cmax : q);
            const ACC a = (ACC)val[e];
            ACC x0, x1;
            Pair<TG>::get(V + cc * ld + j, x0, x1);
            acc0 = fma(a, spmm_round<RND>(x0), acc0);
            acc1 = fma(a, spmm_round<RND>(x1), acc1);
        }
        const int64_t o = row * ld + j;
        const bool two = j + 1 < b;
        if (CHEB) {
            double v0 = alpha * fma(-c, (double)Yc[o], (double)acc0);
            if (beta != 0.0) v0 = fma(-beta, (double)Yp[o], v0);
            W[o] = (ACC)v0;
            if (two) {
                double v1 = alpha * fma(-c, (double)Yc[o + 1], (double)acc1);
                if (beta != 0.0) v1 = fma(-beta, (double)Yp[o + 1], v1);
                W[o + 1] = (ACC)v1;
            }
        } else {
            W[o] = acc0;
            if (two) W[o + 1] = acc1;
        }
    }
}

// VW consecutive columns of a row-major block: one 16-byte load (two FP64
// or four FP32 values); the row's ld is a multiple of VW, so the load stays
// inside the row even past the last used column
template <class T, int VW>
struct VecLd;
template <>
struct VecLd<double, 2> {
    static __device__ __forceinline__ void get(const double *p, double *o) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct VecLd<float, 2> {
    static __device__ __forceinline__ void get(const float *p, float *o) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct VecLd<float, 4> {
    static __device__ __forceinline__ void get(const float *p, float *o) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};

// One Chebyshev step on CSR A with the recurrence's column scaling folded
// in.  The scaled iteration brings the newest block Y1 to infinity-norm
// (1/2, 1] per column by a power of two s (from the merged magnitude keys
// of its columns) and multiplies the older block Y0 by the same s before
// the step; here neither block is rewritten: Y1 is read as s Y1 (rounded
// to the phase's storage type for reduced phases, as the stored block
// would be) and Y0 as s p0 Y0, p0 being the factor still pending on Y0 from
// the step before (rounded when Y0 was that step's Y1).  Powers of two
// scale exactly, so the values are those of the scaled iteration.  The
// step's output Y2 = alpha (A Y1 - c Y1) - beta Y0 is written unscaled and
// its column keys are merged into cmax_out for the next step; workgroup 0
// records s for that step's p0 and clears the key array two steps ahead.
// A group of L lanes takes a row, each lane VW adjacent columns.
template <class T, int RND, class TA, int VW>
__global__ __launch_bounds__(256) void k_spmm_cheb_scaled(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const TA *__restrict__ val, int64_t n_rows,
    int64_t n_cols, int64_t nnz, int b, int lanes_log2, const T *__restrict__ Y1, const T *__restrict__ Y0,
    T *__restrict__ Y2, int64_t ld, double alpha, double c, double beta, const unsigned *__restrict__ cmax_in,
    const double *__restrict__ p0, int round_prev, double *__restrict__ s_out, unsigned *__restrict__ cmax_out,
    unsigned *__restrict__ clear) {
    using ACC = T;
    __shared__ ACC sc[512], pp[512];
    __shared__ unsigned km[512];
    const int t = threadIdx.x;
    for (int j = t; j < 512; j += 256) {
        double f = 1.0;
        if (j < b && cmax_in) {
            unsigned mb = cmax_in[j];
#pragma unroll
            for (int q = 1; q < CM_COPIES; ++q) mb = max(mb, cmax_in[q * 512 + j]);
            f = key_scale<T>(mb);
        }
        sc[j] = (ACC)f;
        pp[j] = (j < b && p0) ? (ACC)p0[j] : (ACC)1;
        km[j] = 0u;
        if (j < b && blockIdx.x == 0 && s_out) s_out[j] = f;
    }
    if (blockIdx.x == 0 && clear)
        for (int e = t; e < CM_COPIES * 512; e += 256) clear[e] = 0u;
    __syncthreads();
    const int L = 1 << lanes_log2;
    const int rows_per = 256 >> lanes_log2;
    const int64_t blk = xcd_row_block(blockIdx.x, gridDim.x);
    const int li = t & (L - 1);
    // SPMM_PASSES row groups per workgroup: the scale setup and the key
    // merge (one global atomic per column) are shared by all of them
    for (int pass = 0; pass < SPMM_PASSES; ++pass) {
        const int64_t row = (blk * SPMM_PASSES + pass) * rows_per + (t >> lanes_log2);
        if (row >= n_rows) break;
        int64_t e0 = rp[row], e1 = rp[row + 1];
        if (e0 < 0) e0 = 0;
        if (e1 > nnz) e1 = nnz;
        const int64_t cmx = n_cols - 1;
        for (int j = VW * li; j < b; j += VW * L) {
            // (the scale arrays hold 512 entries: j + VW - 1 < 512 since
            // b <= 512 and VW divides the row's ld)
            ACC s[VW], acc[VW];
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                s[v] = sc[j + v];
                acc[v] = (ACC)0;
            }
            int64_t e = e0;
            for (; e + 4 <= e1; e += 4) {
                int64_t cc[4];
                ACC a[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t q = ci[e + u];
                    cc[u] = q < 0 ? 0 : (q > cmx ? cmx : q);
                    a[u] = (ACC)val[e + u];
                }
                ACC x[4][VW];
#pragma unroll
                for (int u = 0; u < 4; ++u) VecLd<T, VW>::get(Y1 + cc[u] * ld + j, x[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < VW; ++v) acc[v] = fma(a[u], spmm_round<RND>(x[u][v] * s[v]), acc[v]);
            }
            for (; e < e1; ++e) {
                const int64_t q = ci[e];
                const int64_t cc = q < 0 ? 0 : (q > cmx ? cmx : q);
                const ACC a = (ACC)val[e];
                ACC x[VW];
                VecLd<T, VW>::get(Y1 + cc * ld + j, x);
#pragma unroll
                for (int v = 0; v < VW; ++v) acc[v] = fma(a, spmm_round<RND>(x[v] * s[v]), acc[v]);
            }
            const int64_t o = row * ld + j;
            ACC yc[VW], yp[VW];
            VecLd<T, VW>::get(Y1 + o, yc);
            if (beta != 0.0) VecLd<T, VW>::get(Y0 + o, yp);
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                if (j + v >= b) break;
                // a scaled step's Y1 is the stored (rounded) block; the first
                // step's combine reads its input as it is, only the product
                // reading it rounded
                ACC ycv = yc[v];
                if (cmax_in) ycv = spmm_round<RND>(ycv * s[v]);
                double val2 = alpha * fma(-c, (double)ycv, (double)acc[v]);
                if (beta != 0.0) {
                    const ACC q = yp[v] * pp[j + v];
                    const ACC ypv = (round_prev ? spmm_round<RND>(q) : q) * s[v];
                    val2 = fma(-beta, (double)ypv, val2);
                }
                const T w = (T)val2;
                Y2[o + v] = w;
                if (cmax_out) atomicMax(&km[j + v], mag_key<T>((double)w));
            }
        }
    }
    if (cmax_out) {
        __syncthreads();
        for (int j = t; j < b; j += 256)
            if (km[j]) atomicMax(cmax_out + (blockIdx.x % CM_COPIES) * 512 + j, km[j]);
    }
}



// CSR structure check: row_ptr[0] == 0, non-decreasing, row_ptr[n] == nnz,
// every column index in [0, n_cols).  Sets *bad to a nonzero code.
__global__ void k_csr_check(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            int64_t n_rows, int64_t n_cols, int64_t nnz, int *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0 && (rp[0] != 0 || rp[n_rows] != nnz)) atomicOr(bad, 1);
    for (int64_t i = t0; i < n_rows; i += stride)
        if (rp[i + 1] < rp[i]) atomicOr(bad, 2);
    for (int64_t e = t0; e < nnz; e += stride) {
        const int32_t c = ci[e];
        if (c < 0 || c >= n_cols) atomicOr(bad, 4);
    }
}

}  // namespace

void product_f64(Context *ctx, const ofrr_matrix *A, int trans, int32_t b, const double *V,
                 int64_t ldv, double *W, int64_t ldw) {
    OFRR_CHECK_ARG(A->dtype == OFRR_F64 || A->dtype == OFRR_F32, "product_f64: A must be F64 or F32");
    const int64_t m = trans ? A->cols : A->rows;
    const int64_t kdim = trans ? A->rows : A->cols;
    const int NCT = b > 64 ? 2 : 1;
    const int BN = 64 * NCT;
    const int gx = (int)((m + F64_BM - 1) / F64_BM), gy = (b + BN - 1) / BN;
    const int ntiles = gx * gy;
    int nsplit = 1;
    const int64_t want = 2LL * (ctx->cu_count > 0 ? ctx->cu_count : 256);
    while ((int64_t)ntiles * nsplit < want && kdim / (nsplit * 2) >= 1024 && nsplit < 8) nsplit *= 2;
    int64_t kps = (kdim + nsplit - 1) / nsplit;
    kps = (kps + F64_BK - 1) / F64_BK * F64_BK;
    nsplit = (int)((kdim + kps - 1) / kps);
    const int xcd_map = (nsplit >= 2 && 8 % nsplit == 0) ? 1 : 0;
    int64_t nwg = (int64_t)ntiles * nsplit;
    if (xcd_map) nwg = (int64_t)((ntiles + 8 / nsplit - 1) / (8 / nsplit)) * 8;
    double *dst = W;
    if (nsplit > 1) dst = ctx->buf<double>("f64_slabs", (size_t)nsplit * m * ldw);
    {
        KTimer t(ctx, "product_f64");
        auto go = [&](auto kern, auto ap) {
            hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(256), 0, ctx->stream, ap, A->ld, m, kdim, b, V,
                               ldv, dst, ldw, kps, ntiles, nsplit, xcd_map);
        };
        const float *af = (const float *)A->values;
        const double *ad = (const double *)A->values;
        if (A->dtype == OFRR_F32) {
            if (trans) {
                if (NCT == 2) go(k_gemm_f64<float, true, 2>, af); else go(k_gemm_f64<float, true, 1>, af);
            } else {
                if (NCT == 2) go(k_gemm_f64<float, false, 2>, af); else go(k_gemm_f64<float, false, 1>, af);
            }
        } else {
            if (trans) {
                if (NCT == 2) go(k_gemm_f64<double, true, 2>, ad); else go(k_gemm_f64<double, true, 1>, ad);
            } else {
                if (NCT == 2) go(k_gemm_f64<double, false, 2>, ad); else go(k_gemm_f64<double, false, 1>, ad);
            }
        }
        OFRR_HIP(hipGetLastError());
    }
    if (nsplit > 1) {
        KTimer t(ctx, "product_reduce");
        const int64_t total = m * b;
        const int g = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
        hipLaunchKernelGGL(k_sum_slabs_d, dim3(g), dim3(256), 0, ctx->stream, dst, nsplit, m, b, ldw, W);
        OFRR_HIP(hipGetLastError());
    }
}

namespace {

int spmm_lanes_log2(int b) {
    const int need = (b + 1) / 2;
    int lg = 0;
    while ((1 << lg) < need && lg < 6) ++lg;
    return lg;
}

template <class TG, int RND, bool CHEB, class TW>
void launch_spmm_v(Context *ctx, const ofrr_matrix *A, int32_t b, const TG *V, int64_t ld, TW *W, const TW *Yc,
                   const TW *Yp, double alpha, double c, double beta) {
    const int lg = spmm_lanes_log2(b);
    const int64_t rows_per = 256 >> lg;
    const int64_t G = (A->rows + rows_per - 1) / rows_per;
    OFRR_CHECK_ARG(G < ((int64_t)1 << 31), "spmm: too many rows");
    if (A->dtype == OFRR_F32)
        hipLaunchKernelGGL((k_spmm_v<TG, RND, float, CHEB>), dim3((unsigned)G), dim3(256), 0, ctx->stream,
                           A->row_ptr, A->col_idx, (const float *)A->values, A->rows, A->cols, A->nnz, b, lg, V, ld,
                           W, Yc, Yp, alpha, c, beta);
    else
        hipLaunchKernelGGL((k_spmm_v<TG, RND, double, CHEB>), dim3((unsigned)G), dim3(256), 0, ctx->stream,
                           A->row_ptr, A->col_idx, (const double *)A->values, A->rows, A->cols, A->nnz, b, lg, V,
                           ld, W, Yc, Yp, alpha, c, beta);
    OFRR_HIP(hipGetLastError());
}

bool pair_aligned(const void *p, int64_t ld, size_t es) {
    return ld % 2 == 0 && (reinterpret_cast<uintptr_t>(p) % (2 * es)) == 0;
}

}  // namespace

void product_csr(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype vt, const void *V,
                 int64_t ldv, void *W, int64_t ldw) {
    KTimer tm(ctx, "spmm");
    const int64_t n = A->rows;
    const size_t es = vt == OFRR_F64 ? 8 : (vt == OFRR_F32 ? 4 : 2);
    const size_t ws = vt == OFRR_F64 ? 8 : 4;
    if (ldv == ldw && pair_aligned(V, ldv, es) && pair_aligned(W, ldw, ws)) {
        switch (vt) {
            case OFRR_F64:
                launch_spmm_v<double, 0, false>(ctx, A, b, (const double *)V, ldv, (double *)W, (const double *)nullptr,
                                                (const double *)nullptr, 0.0, 0.0, 0.0);
                return;
            case OFRR_F32:
                launch_spmm_v<float, 0, false>(ctx, A, b, (const float *)V, ldv, (float *)W, (const float *)nullptr,
                                               (const float *)nullptr, 0.0, 0.0, 0.0);
                return;
            case OFRR_F16:
                launch_spmm_v<f16_t, 0, false>(ctx, A, b, (const f16_t *)V, ldv, (float *)W, (const float *)nullptr,
                                               (const float *)nullptr, 0.0, 0.0, 0.0);
                return;
            case OFRR_BF16:
                launch_spmm_v<bf16_t, 0, false>(ctx, A, b, (const bf16_t *)V, ldv, (float *)W,
                                                (const float *)nullptr, (const float *)nullptr, 0.0, 0.0, 0.0);
                return;
            default: fail(OFRR_ERR_UNSUPPORTED, "spmm: basis type");
        }
    }
    dim3 grid((unsigned)((n + 3) / 4));
    auto go = [&](auto *vtag, auto *wtag) {
        using TV = std::remove_pointer_t<decltype(vtag)>;
        using TW = std::remove_pointer_t<decltype(wtag)>;
        if (A->dtype == OFRR_F32)
            hipLaunchKernelGGL((k_spmm<TV, TW, float>), grid, dim3(256), 0, ctx->stream, A->row_ptr,
                               A->col_idx, (const float *)A->values, n, A->cols, A->nnz, b,
                               (const TV *)V, ldv, (TW *)W, ldw);
        else
            hipLaunchKernelGGL((k_spmm<TV, TW, double>), grid, dim3(256), 0, ctx->stream, A->row_ptr,
                               A->col_idx, (const double *)A->values, n, A->cols, A->nnz, b,
                               (const TV *)V, ldv, (TW *)W, ldw);
    };
    switch (vt) {
        case OFRR_F64: go((double *)nullptr, (double *)nullptr); break;
        case OFRR_F32: go((float *)nullptr, (float *)nullptr); break;
        case OFRR_F16: go((f16_t *)nullptr, (float *)nullptr); break;
        case OFRR_BF16: go((bf16_t *)nullptr, (float *)nullptr); break;
        default: fail(OFRR_ERR_UNSUPPORTED, "spmm: basis type");
    }
    OFRR_HIP(hipGetLastError());
}

bool product_csr_master(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype phase, const void *Vm, int64_t ld,
                        void *Out, const void *Yc, const void *Yp, bool cheb, double alpha, double c, double beta) {
    const size_t es = phase == OFRR_F64 ? 8 : 4;
    if (!pair_aligned(Vm, ld, es) || !pair_aligned(Out, ld, es)) return false;
    if (cheb && (!pair_aligned(Yc, ld, es) || (Yp && !pair_aligned(Yp, ld, es)))) return false;
    KTimer tm(ctx, phase == OFRR_F64 ? "spmm_f64" : phase == OFRR_F32 ? "spmm_f32" : "spmm_f16");
    auto go = [&](auto *tag, auto rnd) {
        using T = std::remove_pointer_t<decltype(tag)>;
        constexpr int R = decltype(rnd)::value;
        const T *v = static_cast<const T *>(Vm);
        T *o = static_cast<T *>(Out);
        const T *yc = static_cast<const T *>(Yc);
        const T *yp = static_cast<const T *>(Yp);
        if (cheb)
            launch_spmm_v<T, R, true>(ctx, A, b, v, ld, o, yc, yp, alpha, c, beta);
        else
            launch_spmm_v<T, R, false>(ctx, A, b, v, ld, o, yc, yp, 0.0, 0.0, 0.0);
    };
    switch (phase) {
        case OFRR_F64: go((double *)nullptr, std::integral_constant<int, 0>{}); break;
        case OFRR_F32: go((float *)nullptr, std::integral_constant<int, 0>{}); break;
        case OFRR_F16: go((float *)nullptr, std::integral_constant<int, 1>{}); break;
        case OFRR_BF16: go((float *)nullptr, std::integral_constant<int, 2>{}); break;
        default: return false;
    }
    return true;
}

bool spmm_cheb_scaled(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype phase, const void *Y1,
                      const void *Y0, void *Y2, int64_t ld, double alpha, double c, double beta,
                      const unsigned *cmax_in, const double *p0, bool round_prev, double *s_out, unsigned *cmax_out,
                      unsigned *clear) {
    const size_t es = phase == OFRR_F64 ? 8 : 4;
    if (!pair_aligned(Y1, ld, es) || !pair_aligned(Y2, ld, es) || (Y0 && !pair_aligned(Y0, ld, es))) return false;
    if (b > 512) return false;
    // FP32 blocks: four columns per lane (16-byte loads) when the rows allow it
    auto quad = [&](const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) % 16) == 0; };
    const bool vw4 = es == 4 && ld % 4 == 0 && quad(Y1) && quad(Y2) && quad(Y0);
    KTimer tm(ctx, phase == OFRR_F64 ? "spmm_f64" : phase == OFRR_F32 ? "spmm_f32" : "spmm_f16");
    const int lg = spmm_lanes_log2(vw4 ? (b + 1) / 2 : b);
    const int64_t rows_per = (int64_t)(256 >> lg) * SPMM_PASSES;
    const int64_t G = (A->rows + rows_per - 1) / rows_per;
    OFRR_CHECK_ARG(G < ((int64_t)1 << 31), "spmm: too many rows");
    const int rp = round_prev ? 1 : 0;
    auto go = [&](auto *tag, auto rnd, auto *atag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        using TA = std::remove_pointer_t<decltype(atag)>;
        constexpr int R = decltype(rnd)::value;
        auto launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(256), 0, ctx->stream, A->row_ptr, A->col_idx,
                               (const TA *)A->values, A->rows, A->cols, A->nnz, b, lg, (const T *)Y1, (const T *)Y0,
                               (T *)Y2, ld, alpha, c, beta, cmax_in, p0, rp, s_out, cmax_out, clear);
        };
        if constexpr (std::is_same<T, float>::value) {
            if (vw4) {
                launch(k_spmm_cheb_scaled<T, R, TA, 4>);
                return;
            }
        }
        launch(k_spmm_cheb_scaled<T, R, TA, 2>);
    };
    auto by_a = [&](auto *tag, auto rnd) {
        if (A->dtype == OFRR_F32) go(tag, rnd, (float *)nullptr);
        else go(tag, rnd, (double *)nullptr);
    };
    switch (phase) {
        case OFRR_F64: by_a((double *)nullptr, std::integral_constant<int, 0>{}); break;
        case OFRR_F32: by_a((float *)nullptr, std::integral_constant<int, 0>{}); break;
        case OFRR_F16: by_a((float *)nullptr, std::integral_constant<int, 1>{}); break;
        case OFRR_BF16: by_a((float *)nullptr, std::integral_constant<int, 2>{}); break;
        default: return false;
    }
    OFRR_HIP(hipGetLastError());
    return true;
}

}  // namespace ofrr

namespace ofrr {

void check_csr(Context *ctx, const ofrr_matrix *A) {
    int *bad = ctx->buf<int>("csr_bad", 4);
    zero_bytes(ctx, bad, 16);
    const int64_t work = std::max<int64_t>(A->rows, A->nnz);
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 4096));
    hipLaunchKernelGGL(k_csr_check, dim3(g), dim3(256), 0, ctx->stream, A->row_ptr, A->col_idx,
                       A->rows, A->cols, A->nnz, bad);
    OFRR_HIP(hipGetLastError());
    int host = 0;
    OFRR_HIP(hipMemcpyAsync(&host, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    if (host & 1) fail(OFRR_ERR_INVALID_ARG, "CSR: row_ptr[0] must be 0 and row_ptr[rows] == nnz");
    if (host & 2) fail(OFRR_ERR_INVALID_ARG, "CSR: row_ptr must be non-decreasing");
    if (host & 4) fail(OFRR_ERR_INVALID_ARG, "CSR: column index out of range");
}

}  // namespace ofrr
