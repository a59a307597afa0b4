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

void product_csr(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype vt, const void *V,
                 int64_t ldv, void *W, int64_t ldw) {
    KTimer tm(ctx, "spmm");
    const int64_t n = A->rows;
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
