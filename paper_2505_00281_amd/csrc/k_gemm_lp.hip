// k_gemm_lp.hip -- the reduced-precision block product W = op(A) V of the
// basis build (Sec. 2: X_{iter} = A^{iter} X_0; Sec. 4: A and the basis in
// reduced precision, products accumulated in FP32), on BF16/F16 MFMA.
//
// The product is bound by streaming A from HBM (2 n^2 bytes against
// 2 n^2 b flops: about b flop per byte, below the BF16 ridge), so the kernel
// is organised around keeping HBM busy:
//   * the basis operand arrives K-contiguous per column (the split kernel
//     writes it that way), so both operands load as 16-byte vectors and are
//     stored to LDS without transposition (for K-contiguous A);
//   * 64-deep K slices, the next slice prefetched into registers while the
//     MFMAs consume the current one;
//   * one 128-row x (32 NB)-column tile per workgroup covers the whole basis
//     (NB = 4 for b <= 128), so A is read exactly once;
//   * split-K fills the chip; the workgroup -> (tile, split) map sends all
//     workgroups of one K range to the same XCD(s), so that range of the
//     basis stays in one L2; the FP32 partials are summed in a fixed order.
// MFMA v_mfma_f32_32x32x16: lane l holds A[l%32][8(l/32)..+8] and
// B[8(l/32)..+8][l%32]; accumulator register r of lane l is
// D[(r/4)*8 + 4(l/32) + r%4][l%32].
#include <cstdlib>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4_t;

template <bool IS_BF16>
__device__ __forceinline__ f32x16_t mfma_32x32x16(u32x4_t a, u32x4_t b, f32x16_t c) {
    if constexpr (IS_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                      __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
}

constexpr int GL_BM = 128;  // rows per workgroup tile

// 8 halves starting at p, zero beyond `valid` (and for misaligned p).
__device__ __forceinline__ u32x4_t load8(const uint16_t *p, int64_t valid) {
    if (valid >= 8 && (((uintptr_t)p) & 15) == 0) return *(const u32x4_t *)p;
    uint16_t tmp[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) tmp[q] = (q < valid) ? p[q] : (uint16_t)0;
    return __builtin_bit_cast(u32x4_t, tmp);
}

// ATRANS: op(A)[i][k] = A[k + i*lda] (K-contiguous); else A[i + k*lda].
// SPLITV: the basis is a two-term split Vhi + Vlo (two MFMAs per fragment).
// SPLITA: A is also a two-term split Ahi + Alo (same layout); the product is
// Ahi Vhi + Ahi Vlo + Alo Vhi, i.e. about 16 significant bits on each side.
// BK: K depth per slice (64 or 128); the LDS row stride is BK + 8 halves
// (16-byte aligned, and 16-byte reads of eight consecutive rows hit
// distinct banks).
template <bool IS_BF16, int NB, bool ATRANS, bool SPLITV, bool SPLITA, int BK>
__global__ __launch_bounds__(256) void k_gemm_lp(const uint16_t *__restrict__ A,
                                                 const uint16_t *__restrict__ Alo, int64_t lda,
                                                 int64_t m, int64_t kdim, int b,
                                                 const uint16_t *__restrict__ Vt,
                                                 const uint16_t *__restrict__ Vtlo, int64_t ldvt,
                                                 float *__restrict__ W, int64_t ldw,
                                                 int64_t k_per_split, int ntiles, int nsplit,
                                                 int xcd_map) {
    constexpr int BN = 32 * NB;
    constexpr int GL_BK = BK, GL_LD = BK + 8;
    constexpr int CPR = BK / 8;                // 16-byte chunks per tile row
    constexpr int ACH = GL_BM * CPR / 256;     // A chunks per thread per slice
    constexpr int BCH = BN * CPR / 256;        // basis chunks per thread per slice
    __shared__ __attribute__((aligned(16))) uint16_t As[GL_BM][GL_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Als[SPLITA ? GL_BM : 1][GL_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][GL_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Bls[SPLITV ? BN : 1][GL_LD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

    // workgroup -> (tile, split)
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
    const int64_t i0 = (int64_t)(tile / gy) * GL_BM;
    const int j0 = (tile % gy) * BN;
    const int64_t kbeg = (int64_t)z * k_per_split;
    const int64_t kend = kbeg + k_per_split < kdim ? kbeg + k_per_split : kdim;

    f32x16_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x16_t{};

    // register staging of one K slice: A ACH chunks, B BCH chunks (+ lo)
    u32x4_t ra[ACH], ral[SPLITA ? ACH : 1], rb[BCH], rl[SPLITV ? BCH : 1];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int s = 0; s < ACH; ++s) {
            const int c = t + 256 * s;
            if (ATRANS) {
                const int row = c / CPR, kc = (c % CPR) * 8;
                const int64_t gi = i0 + row, gk = k0 + kc;
                ra[s] = (gi < m) ? load8(A + gk + gi * lda, kend - gk) : u32x4_t{0u, 0u, 0u, 0u};
                if constexpr (SPLITA)
                    ral[s] = (gi < m) ? load8(Alo + gk + gi * lda, kend - gk) : u32x4_t{0u, 0u, 0u, 0u};
            } else {
                const int kk = c >> 4, rc = (c & 15) * 8;
                const int64_t gk = k0 + kk, gi = i0 + rc;
                ra[s] = (gk < kend) ? load8(A + gi + gk * lda, m - gi) : u32x4_t{0u, 0u, 0u, 0u};
                if constexpr (SPLITA)
                    ral[s] = (gk < kend) ? load8(Alo + gi + gk * lda, m - gi) : u32x4_t{0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int s = 0; s < BCH; ++s) {
            const int c = t + 256 * s;
            const int col = c / CPR, kc = (c % CPR) * 8;
            const int64_t gk = k0 + kc;
            const bool ok = j0 + col < b;
            rb[s] = ok ? load8(Vt + (int64_t)(j0 + col) * ldvt + gk, kend - gk) : u32x4_t{0u, 0u, 0u, 0u};
            if constexpr (SPLITV)
                rl[s] = ok ? load8(Vtlo + (int64_t)(j0 + col) * ldvt + gk, kend - gk) : u32x4_t{0u, 0u, 0u, 0u};
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int s = 0; s < ACH; ++s) {
            const int c = t + 256 * s;
            if (ATRANS) {
                *(u32x4_t *)&As[c / CPR][(c % CPR) * 8] = ra[s];
                if constexpr (SPLITA) *(u32x4_t *)&Als[c / CPR][(c % CPR) * 8] = ral[s];
            } else {
                const int kk = c >> 4, rc = (c & 15) * 8;
                uint16_t tmp[8];
                __builtin_memcpy(tmp, &ra[s], 16);
#pragma unroll
                for (int q = 0; q < 8; ++q) As[rc + q][kk] = tmp[q];
                if constexpr (SPLITA) {
                    __builtin_memcpy(tmp, &ral[s], 16);
#pragma unroll
                    for (int q = 0; q < 8; ++q) Als[rc + q][kk] = tmp[q];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < BCH; ++s) {
            const int c = t + 256 * s;
            *(u32x4_t *)&Bs[c / CPR][(c % CPR) * 8] = rb[s];
            if constexpr (SPLITV) *(u32x4_t *)&Bls[c / CPR][(c % CPR) * 8] = rl[s];
        }
    };

    if (kbeg < kend) fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += GL_BK) {
        stash();
        __syncthreads();
        if (k0 + GL_BK < kend) fetch(k0 + GL_BK);
#pragma unroll
        for (int kk = 0; kk < GL_BK; kk += 16) {
            const int kq = kk + 8 * (lane >> 5);
            const u32x4_t a = *(const u32x4_t *)&As[32 * wave + (lane & 31)][kq];
            u32x4_t al = a;
            if constexpr (SPLITA) al = *(const u32x4_t *)&Als[32 * wave + (lane & 31)][kq];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const u32x4_t bv = *(const u32x4_t *)&Bs[32 * nb + (lane & 31)][kq];
                acc[nb] = mfma_32x32x16<IS_BF16>(a, bv, acc[nb]);
                if constexpr (SPLITV) {
                    const u32x4_t cv = *(const u32x4_t *)&Bls[32 * nb + (lane & 31)][kq];
                    acc[nb] = mfma_32x32x16<IS_BF16>(a, cv, acc[nb]);
                }
                if constexpr (SPLITA) acc[nb] = mfma_32x32x16<IS_BF16>(al, bv, acc[nb]);
            }
        }
        __syncthreads();
    }
    float *Wz = W + (int64_t)z * m * ldw;
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
        for (int zz = 0; zz < nsplit; ++zz) s += P[(int64_t)zz * m * ld + i * ld + j];
        W[i * ld + j] = s;
    }
}

// row-major (rows x b, ld) 16-bit block -> column-major (b x rows, ldt)
__global__ void k_transpose_u16(const uint16_t *__restrict__ s, int64_t rows, int b, int64_t ld,
                                uint16_t *__restrict__ d, int64_t ldt) {
    const int64_t total = rows * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / rows);
        const int64_t i = e - (int64_t)j * rows;
        d[(int64_t)j * ldt + i] = s[i * ld + j];
    }
}

// FP32 row-major block (rows x b, ld) -> 16-bit hi (+ lo) K-contiguous per
// column (b x ldt), through a 64 x 64 LDS tile: rows are read coalesced, and
// each thread writes 8 consecutive rows of one column as one 16-byte store.
template <bool BF16>
__global__ __launch_bounds__(256) void k_split_t(const float *__restrict__ s, int64_t rows, int b, int64_t ld,
                                                 uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                 int64_t ldt) {
    __shared__ float tile[64][65];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    // sixteen unconditional loads (indices clamped into the block) in flight,
    // the range test when the tile is written
    {
        const int cc = t & 63;
        const int gj = j0 + cc;
        const int gjc = gj < b ? gj : b - 1;
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t gi = i0 + (t >> 6) + 4 * q;
            v[q] = s[(gi < rows ? gi : rows - 1) * ld + gjc];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int rr = (t >> 6) + 4 * q;
            tile[rr][cc] = (i0 + rr < rows && gj < b) ? v[q] : 0.f;
        }
    }
    __syncthreads();
    // thread -> column j0 + (t >> 3), rows i0 + 8 (t & 7) .. + 8
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int cc = (t >> 3) + 32 * half, r8 = (t & 7) * 8;
        const int gj = j0 + cc;
        const int64_t gi = i0 + r8;
        if (gj >= b || gi >= ldt) continue;
        uint16_t h[8], l[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float x = (gi + u < rows) ? tile[r8 + u][cc] : 0.f;
            h[u] = BF16 ? f32_to_bf16_bits(x) : f32_to_f16_bits(x);
            const float hv = BF16 ? bf16_bits_to_f32(h[u]) : f16_bits_to_f32(h[u]);
            l[u] = BF16 ? f32_to_bf16_bits(x - hv) : f32_to_f16_bits(x - hv);  // x - hv is exact
        }
        uint16_t *ph = hi + (int64_t)gj * ldt + gi;
        if (gi + 8 <= ldt) {
            *(u32x4_t *)ph = __builtin_bit_cast(u32x4_t, h);
            if (lo) *(u32x4_t *)(lo + (int64_t)gj * ldt + gi) = __builtin_bit_cast(u32x4_t, l);
        } else {
            for (int u = 0; gi + u < ldt; ++u) {
                ph[u] = h[u];
                if (lo) lo[(int64_t)gj * ldt + gi + u] = l[u];
            }
        }
    }
}

inline int grid1(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

}  // namespace

int64_t lowp_ldt(int64_t rows) { return (rows + 7) / 8 * 8; }

void split_block_t(Context *ctx, ofrr_dtype t, int64_t rows, int32_t b, const float *src,
                   int64_t ld, uint16_t *hi, uint16_t *lo, int64_t ldt) {
    // the tiles cover the padded length ldt, so its tail is written as zeros
    const dim3 grid((unsigned)((ldt + 63) / 64), (unsigned)((b + 63) / 64));
    if (t == OFRR_BF16)
        hipLaunchKernelGGL((k_split_t<true>), grid, dim3(256), 0, ctx->stream, src, rows, b, ld, hi, lo, ldt);
    else if (t == OFRR_F16)
        hipLaunchKernelGGL((k_split_t<false>), grid, dim3(256), 0, ctx->stream, src, rows, b, ld, hi, lo, ldt);
    else
        fail(OFRR_ERR_UNSUPPORTED, "split_block_t: BF16 or F16");
    OFRR_HIP(hipGetLastError());
}

void product_lowp_t(Context *ctx, ofrr_dtype t, int64_t m, int64_t kdim, const uint16_t *A,
                    int64_t lda, int trans, int32_t b, const uint16_t *Vt, const uint16_t *Vtlo,
                    int64_t ldvt, float *W, int64_t ldw, const uint16_t *Alo, SlabOut *defer) {
    OFRR_CHECK_ARG(b >= 1 && b <= 4096, "product: 1 <= b <= 4096");
    OFRR_CHECK_ARG(Alo == nullptr || (Vtlo != nullptr && t == OFRR_BF16),
                   "product: a split A needs a split BF16 basis");
    const int NB = b > 64 ? 4 : 2;
    const int BN = 32 * NB;
    const int gx = (int)((m + GL_BM - 1) / GL_BM), gy = (b + BN - 1) / BN;
    const int ntiles = gx * gy;
    // split K so that the launch has at least ~2 workgroups per CU
    int nsplit = 1;
    const int64_t want = 2LL * (ctx->cu_count > 0 ? ctx->cu_count : 256);
    while ((int64_t)ntiles * nsplit < want && kdim / (nsplit * 2) >= 2048 && nsplit < 8) nsplit *= 2;
    int64_t kps = (kdim + nsplit - 1) / nsplit;
    kps = (kps + 127) / 128 * 128;  // a whole number of slices for every depth
    nsplit = (int)((kdim + kps - 1) / kps);
    // XCD-aware map when the splits divide the 8 XCDs evenly
    const int xcd_map = (nsplit >= 2 && 8 % nsplit == 0) ? 1 : 0;
    int64_t nwg = (int64_t)ntiles * nsplit;
    if (xcd_map) {
        const int per = 8 / nsplit;
        nwg = (int64_t)((ntiles + per - 1) / per) * 8;
    }
    float *dst = W;
    if (nsplit > 1) dst = ctx->buf<float>("lowp_slabs", (size_t)nsplit * m * ldw);
    const bool splitv = Vtlo != nullptr;
    {
        KTimer tm(ctx, Alo ? "product_bf16x2" : (t == OFRR_BF16 ? "product_bf16" : "product_f16"));
        // K slice depth: 128 (256 contiguous bytes per row and slice) for
        // the unsplit products, 64 when A or the basis is split (the larger
        // LDS stage would drop to one workgroup per CU); measured on the
        // n = 16384 product.  OFRR_LP_BK=64|128 overrides, for tuning sweeps.
        int bk = (Alo || splitv) ? 64 : 128;
        if (const char *e = std::getenv("OFRR_LP_BK")) {
            const int v = std::atoi(e);
            if (v == 64 || v == 128) bk = v;
        }
        auto go2 = [&](auto k64, auto k128) {
            auto launch = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(256), 0, ctx->stream, A, Alo, lda, m, kdim,
                                   b, Vt, Vtlo, ldvt, dst, ldw, kps, ntiles, nsplit, xcd_map);
            };
            if (bk == 128) launch(k128); else launch(k64);
        };
#define OFRR_GO(BFV, NBV, TR, SP) go2(k_gemm_lp<BFV, NBV, TR, SP, false, 64>, k_gemm_lp<BFV, NBV, TR, SP, false, 128>)
#define OFRR_GO2(NBV, TR) go2(k_gemm_lp<true, NBV, TR, true, true, 64>, k_gemm_lp<true, NBV, TR, true, true, 128>)
        const bool bf = t == OFRR_BF16;
        const bool tr = trans != 0;
        if (Alo) {
            if (NB == 4) {
                if (tr) OFRR_GO2(4, true); else OFRR_GO2(4, false);
            } else {
                if (tr) OFRR_GO2(2, true); else OFRR_GO2(2, false);
            }
        } else if (bf) {
            if (NB == 4) {
                if (tr) { if (splitv) OFRR_GO(true, 4, true, true); else OFRR_GO(true, 4, true, false); }
                else { if (splitv) OFRR_GO(true, 4, false, true); else OFRR_GO(true, 4, false, false); }
            } else {
                if (tr) { if (splitv) OFRR_GO(true, 2, true, true); else OFRR_GO(true, 2, true, false); }
                else { if (splitv) OFRR_GO(true, 2, false, true); else OFRR_GO(true, 2, false, false); }
            }
        } else {
            if (NB == 4) {
                if (tr) { if (splitv) OFRR_GO(false, 4, true, true); else OFRR_GO(false, 4, true, false); }
                else { if (splitv) OFRR_GO(false, 4, false, true); else OFRR_GO(false, 4, false, false); }
            } else {
                if (tr) { if (splitv) OFRR_GO(false, 2, true, true); else OFRR_GO(false, 2, true, false); }
                else { if (splitv) OFRR_GO(false, 2, false, true); else OFRR_GO(false, 2, false, false); }
            }
        }
#undef OFRR_GO
#undef OFRR_GO2
        OFRR_HIP(hipGetLastError());
    }
    if (defer) {
        defer->p = dst;
        defer->t = OFRR_F32;
        defer->nsplit = nsplit;
        defer->stride = m * ldw;
        return;
    }
    if (nsplit > 1) {
        KTimer tm(ctx, "product_reduce");
        hipLaunchKernelGGL(k_sum_slabs, dim3(grid1(m * b)), dim3(256), 0, ctx->stream, dst, nsplit, m, b,
                           ldw, W);
        OFRR_HIP(hipGetLastError());
    }
}

void product_lowp(Context *ctx, ofrr_dtype t, int64_t m, int64_t kdim, const uint16_t *A,
                  int64_t lda, int trans, int32_t b, const uint16_t *V, const uint16_t *Vlo,
                  int64_t ldv, float *W, int64_t ldw) {
    // row-major basis -> the K-contiguous layout the kernel streams
    const int64_t ldt = lowp_ldt(kdim);
    uint16_t *Vt = ctx->buf<uint16_t>("lowp_vt", (size_t)b * ldt);
    uint16_t *Vtl = Vlo ? ctx->buf<uint16_t>("lowp_vtlo", (size_t)b * ldt) : nullptr;
    hipLaunchKernelGGL(k_transpose_u16, dim3(grid1(kdim * b)), dim3(256), 0, ctx->stream, V, kdim, b,
                       ldv, Vt, ldt);
    if (Vlo)
        hipLaunchKernelGGL(k_transpose_u16, dim3(grid1(kdim * b)), dim3(256), 0, ctx->stream, Vlo, kdim,
                           b, ldv, Vtl, ldt);
    OFRR_HIP(hipGetLastError());
    product_lowp_t(ctx, t, m, kdim, A, lda, trans, b, Vt, Vtl, ldt, W, ldw, nullptr);
}

namespace {
__global__ void k_f32_to_bf16x2(const float *__restrict__ s, int64_t rows, int64_t cols, int64_t lds,
                                uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / rows, r = e - c * rows;
        const float x = s[r + c * lds];
        const uint16_t h = f32_to_bf16_bits(x);
        hi[e] = h;
        lo[e] = f32_to_bf16_bits(x - bf16_bits_to_f32(h));  // the difference is exact
    }
}
}  // namespace

void cast_f32_to_bf16x2(Context *ctx, int64_t rows, int64_t cols, const float *src, int64_t lds,
                        uint16_t *hi, uint16_t *lo) {
    KTimer tm(ctx, "quantize");
    hipLaunchKernelGGL(k_f32_to_bf16x2, dim3(grid1(rows * cols)), dim3(256), 0, ctx->stream, src, rows,
                       cols, lds, hi, lo);
    OFRR_HIP(hipGetLastError());
}

}  // namespace ofrr
