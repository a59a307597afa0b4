// k_product.hip -- the block products W = op(A) V of the subspace iteration
// (Sec. 2: X_{iter} = A^{iter} X_0; Sec. 4: products in reduced precision
// with FP32 accumulation).
//
//   product_f64   FP64 arithmetic, A dense FP64 or FP32 (promoted exactly).
//   product_lowp  A and V in BF16 or F16, MFMA 32x32x16 with FP32
//                 accumulation; optional two-term split of V (V = Vhi + Vlo)
//                 carried through a second MFMA on the same A fragment.
//   product_csr   CSR A (FP32/FP64 values), one wavefront per row.
//
// Blocks V and W are row-major (element (i, j) at i*ld + j); A is the
// caller's column-major matrix.
#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

// ------------------------------------------------------------------ FP64 --
// W (m x b) = op(A) (m x kdim) * V (kdim x b).  64 x 64 output tile per
// 256-thread workgroup, 16-deep K slices staged in LDS, 4 x 4 outputs per
// thread.
template <class TA>
__global__ __launch_bounds__(256) void k_gemm_f64(const TA *__restrict__ A, int64_t lda, int trans,
                                                  int64_t m, int64_t kdim, int b,
                                                  const double *__restrict__ V, int64_t ldv,
                                                  double *__restrict__ W, int64_t ldw) {
    __shared__ double As[16][64 + 1];
    __shared__ double Vs[16][64 + 1];
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    double acc[4][4] = {};
    for (int64_t k0 = 0; k0 < kdim; k0 += 16) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = t + 256 * s;
            int ii, kk;
            if (!trans) {
                ii = e & 63;
                kk = e >> 6;
            } else {
                kk = e & 15;
                ii = e >> 4;
            }
            const int64_t gi = i0 + ii, gk = k0 + kk;
            double v = 0.0;
            if (gi < m && gk < kdim) v = (double)(trans ? A[gk + gi * lda] : A[gi + gk * lda]);
            As[kk][ii] = v;
            const int vk = e >> 6, vj = e & 63;
            const int64_t gvk = k0 + vk;
            Vs[vk][vj] = (gvk < kdim && j0 + vj < b) ? V[gvk * ldv + j0 + vj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = Vs[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], v[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + ty + 16 * r;
        if (gi >= m) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gj = j0 + tx + 16 * c;
            if (gj < b) W[gi * ldw + gj] = acc[r][c];
        }
    }
}

// ------------------------------------------------------- BF16 / F16 MFMA --
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4_t;

template <bool IS_BF16>
__device__ __forceinline__ f32x16_t mfma32x32x16(u32x4_t a, u32x4_t b, f32x16_t c) {
    if constexpr (IS_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                      __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
}

// Tile: 128 rows x 64 cols of W per 256-thread workgroup (each wave 32 rows x
// 64 cols = two 32x32 MFMA blocks), 32-deep K slices.  LDS rows are padded
// (40 halves = 80 B) to spread the 16-byte fragment reads over the banks.
// Operand layout of v_mfma_f32_32x32x16: lane l holds A[l%32][8(l/32)..+8]
// and B[8(l/32)..+8][l%32]; the accumulator register r of lane l is
// D[(r/4)*8 + 4(l/32) + r%4][l%32].
constexpr int LP_BM = 128, LP_BK = 32, LP_PAD = 40;

// NB 32-column blocks per wave: the workgroup tile is 128 x (32*NB).
template <bool IS_BF16, int NB>
__global__ __launch_bounds__(256) void k_gemm_lowp(const uint16_t *__restrict__ A, int64_t lda,
                                                   int trans, int64_t m, int64_t kdim, int b,
                                                   const uint16_t *__restrict__ V,
                                                   const uint16_t *__restrict__ Vlo, int64_t ldv,
                                                   float *__restrict__ W, int64_t ldw,
                                                   int64_t k_per_split) {
    constexpr int BN = 32 * NB;
    __shared__ __attribute__((aligned(16))) uint16_t As[LP_BM][LP_PAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LP_PAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bls[BN][LP_PAD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * LP_BM;
    const int j0 = blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * k_per_split;
    int64_t kend = kbeg + k_per_split;
    if (kend > kdim) kend = kdim;
    const bool split = Vlo != nullptr;
    f32x16_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x16_t{};

    for (int64_t k0 = kbeg; k0 < kend; k0 += LP_BK) {
        // ---- A tile: 128 rows x 32 k
        if (trans) {
            // op(A)[i][k] = A[k + i*lda]: contiguous in k; 4 threads per row
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int row = (t >> 2) + 64 * s, kc = (t & 3) * 8;
                const int64_t gi = i0 + row, gk = k0 + kc;
                u32x4_t v = {0u, 0u, 0u, 0u};
                if (gi < m) {
                    const uint16_t *p = A + gk + gi * lda;
                    if (gk + 8 <= kend && (((uintptr_t)p) & 15) == 0) {
                        v = *(const u32x4_t *)p;
                    } else {
                        uint16_t tmp[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) tmp[q] = (gk + q < kend) ? p[q] : (uint16_t)0;
                        v = __builtin_bit_cast(u32x4_t, tmp);
                    }
                }
                *(u32x4_t *)&As[row][kc] = v;
            }
        } else {
            // op(A)[i][k] = A[i + k*lda]: contiguous in i; 16 threads per k column
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int e = t + 256 * s;
                const int kk = e >> 4, rc = (e & 15) * 8;
                const int64_t gk = k0 + kk, gi = i0 + rc;
                uint16_t tmp[8];
                if (gk < kend) {
                    const uint16_t *p = A + gi + gk * lda;
                    if (gi + 8 <= m && (((uintptr_t)p) & 15) == 0) {
                        u32x4_t v = *(const u32x4_t *)p;
                        __builtin_memcpy(tmp, &v, 16);
                    } else {
#pragma unroll
                        for (int q = 0; q < 8; ++q) tmp[q] = (gi + q < m) ? p[q] : (uint16_t)0;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) tmp[q] = 0;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) As[rc + q][kk] = tmp[q];
            }
        }
        // ---- B tile: 32 k x (32*NB) n, V row-major -> Bs[n][k]
#pragma unroll
        for (int s = 0; s < NB / 2; ++s) {
            const int kk = t >> 3, nc = (t & 7) * 8 + 64 * s;
            const int64_t gk = k0 + kk;
            uint16_t tmp[8], tmpl[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool ok = gk < kend && j0 + nc + q < b;
                tmp[q] = ok ? V[gk * ldv + j0 + nc + q] : (uint16_t)0;
                tmpl[q] = (ok && split) ? Vlo[gk * ldv + j0 + nc + q] : (uint16_t)0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                Bs[nc + q][kk] = tmp[q];
                Bls[nc + q][kk] = tmpl[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < LP_BK; kk += 16) {
            const int kq = kk + 8 * (lane >> 5);
            const u32x4_t a = *(const u32x4_t *)&As[32 * wave + (lane & 31)][kq];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const u32x4_t bv = *(const u32x4_t *)&Bs[32 * nb + (lane & 31)][kq];
                acc[nb] = mfma32x32x16<IS_BF16>(a, bv, acc[nb]);
                if (split) {
                    const u32x4_t cv = *(const u32x4_t *)&Bls[32 * nb + (lane & 31)][kq];
                    acc[nb] = mfma32x32x16<IS_BF16>(a, cv, acc[nb]);
                }
            }
        }
        __syncthreads();
    }
    float *Wz = W + (int64_t)blockIdx.z * m * ldw;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = (r >> 2) * 8 + 4 * (lane >> 5) + (r & 3);
        const int64_t gi = i0 + 32 * wave + i;
        if (gi >= m) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int gj = j0 + 32 * nb + (lane & 31);
            if (gj < b) Wz[gi * ldw + gj] = acc[nb][r];
        }
    }
}

// Sum of split-K partial slabs in fixed order (deterministic).
__global__ void k_sum_slabs(const float *__restrict__ P, int nsplit, int64_t m, int b, int64_t ld,
                            float *__restrict__ W) {
    const int64_t total = m * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / b;
        const int j = (int)(e - i * b);
        float s = 0.f;
        for (int z = 0; z < nsplit; ++z) s += P[(int64_t)z * m * ld + i * ld + j];
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

void product_lowp(Context *ctx, ofrr_dtype t, int64_t m, int64_t kdim, const uint16_t *A,
                  int64_t lda, int trans, int32_t b, const uint16_t *V, const uint16_t *Vlo,
                  int64_t ldv, float *W, int64_t ldw) {
    // whole basis in one tile column when b > 64 (A is then streamed once)
    const int NB = b > 64 ? 4 : 2;
    const int BN = 32 * NB;
    const unsigned gx = (unsigned)((m + LP_BM - 1) / LP_BM), gy = (unsigned)((b + BN - 1) / BN);
    // split K so that the launch has at least ~2 workgroups per CU
    int nsplit = 1;
    const int64_t want = 2LL * (ctx->cu_count > 0 ? ctx->cu_count : 256);
    while ((int64_t)gx * gy * nsplit < want && kdim / (nsplit * 2) >= 1024) nsplit *= 2;
    int64_t kps = (kdim + nsplit - 1) / nsplit;
    kps = (kps + LP_BK - 1) / LP_BK * LP_BK;
    float *dst = W;
    if (nsplit > 1) dst = ctx->buf<float>("lowp_slabs", (size_t)nsplit * m * ldw);
    dim3 grid(gx, gy, nsplit);
    {
        KTimer tm(ctx, t == OFRR_BF16 ? "product_bf16" : "product_f16");
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(256), 0, ctx->stream, A, lda, trans, m, kdim, b, V,
                               Vlo, ldv, dst, ldw, kps);
        };
        if (t == OFRR_BF16)
            NB == 4 ? go(k_gemm_lowp<true, 4>) : go(k_gemm_lowp<true, 2>);
        else
            NB == 4 ? go(k_gemm_lowp<false, 4>) : go(k_gemm_lowp<false, 2>);
        OFRR_HIP(hipGetLastError());
    }
    if (nsplit > 1) {
        KTimer tm(ctx, "product_reduce");
        int64_t total = m * b;
        int g = (int)std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(k_sum_slabs, dim3(g), dim3(256), 0, ctx->stream, dst, nsplit, m, b, ldw, W);
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
