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
// accumulator register r of lane l is D[4r + l/16][l%16]).  64 x 64
// output tile per 256-thread workgroup (2 x 2 waves, each 2 x 2 MFMA
// blocks), 16-deep K slices staged in LDS; the next slice is loaded into
// registers while the current one is multiplied.
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4_t;

template <class TA>
__device__ __forceinline__ void f64_tile_load(const TA *__restrict__ A, int64_t lda, int trans,
                                              int64_t m, int64_t kdim, int b,
                                              const double *__restrict__ V, int64_t ldv,
                                              int64_t i0, int j0, int64_t k0, int t, double (&ra)[4],
                                              double (&rv)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        int ii, kk;
        if (trans) {  // contiguous in k: 4 consecutive k per thread
            ii = t >> 2;
            kk = (t & 3) * 4 + s;
        } else {  // contiguous in i: 4 consecutive i per thread
            kk = t >> 4;
            ii = (t & 15) * 4 + s;
        }
        const int64_t gi = i0 + ii, gk = k0 + kk;
        ra[s] = (gi < m && gk < kdim) ? (double)(trans ? A[gk + gi * lda] : A[gi + gk * lda]) : 0.0;
        const int vk = t >> 4, vj = (t & 15) * 4 + s;
        const int64_t gvk = k0 + vk;
        rv[s] = (gvk < kdim && j0 + vj < b) ? V[gvk * ldv + j0 + vj] : 0.0;
    }
}

template <class TA>
__global__ __launch_bounds__(256) void k_gemm_f64(const TA *__restrict__ A, int64_t lda, int trans,
                                                  int64_t m, int64_t kdim, int b,
                                                  const double *__restrict__ V, int64_t ldv,
                                                  double *__restrict__ W, int64_t ldw) {
    __shared__ double As[16][64 + 2];
    __shared__ double Vs[16][64 + 2];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    f64x4_t acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    double ra[4], rv[4];
    f64_tile_load(A, lda, trans, m, kdim, b, V, ldv, i0, j0, 0, t, ra, rv);
    for (int64_t k0 = 0; k0 < kdim; k0 += 16) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (trans)
                As[(t & 3) * 4 + s][t >> 2] = ra[s];
            else
                As[t >> 4][(t & 15) * 4 + s] = ra[s];
            Vs[t >> 4][(t & 15) * 4 + s] = rv[s];
        }
        __syncthreads();
        if (k0 + 16 < kdim) f64_tile_load(A, lda, trans, m, kdim, b, V, ldv, i0, j0, k0 + 16, t, ra, rv);
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[2], bb[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) a[p] = As[kr][32 * wr + 16 * p + (lane & 15)];
#pragma unroll
            for (int q = 0; q < 2; ++q) bb[q] = Vs[kr][32 * wc + 16 * q + (lane & 15)];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], bb[q], acc[p][q], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = i0 + 32 * wr + 16 * p + 4 * r + (lane >> 4);
                const int gj = j0 + 32 * wc + 16 * q + (lane & 15);
                if (gi < m && gj < b) W[gi * ldw + gj] = acc[p][q][r];
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
    KTimer t(ctx, "product_f64");
    const int64_t m = trans ? A->cols : A->rows;
    const int64_t kdim = trans ? A->rows : A->cols;
    dim3 grid((unsigned)((m + 63) / 64), (unsigned)((b + 63) / 64));
    if (A->dtype == OFRR_F64)
        hipLaunchKernelGGL((k_gemm_f64<double>), grid, dim3(256), 0, ctx->stream,
                           (const double *)A->values, A->ld, trans, m, kdim, b, V, ldv, W, ldw);
    else if (A->dtype == OFRR_F32)
        hipLaunchKernelGGL((k_gemm_f64<float>), grid, dim3(256), 0, ctx->stream,
                           (const float *)A->values, A->ld, trans, m, kdim, b, V, ldv, W, ldw);
    else
        fail(OFRR_ERR_UNSUPPORTED, "product_f64: A must be F64 or F32");
    OFRR_HIP(hipGetLastError());
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
