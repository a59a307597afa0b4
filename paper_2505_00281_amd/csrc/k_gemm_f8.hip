// k_gemm_f8.hip -- FP8 (OCP e4m3fn) block product W = op(A) V for the
// reduced-precision basis build (Sec. 4 plan, taken one format lower), on the
// block-scaled MFMA of gfx950 (v_mfma_scale_f32_32x32x64_f8f6f4).
//
// Scaling.  A carries one power-of-two scale per 32 x 32 block (square, so
// the same copy serves A V and A^T U); the basis carries one per 32
// consecutive rows of each column.  The MFMA applies an E8M0 scale per lane
// per 32 K-values, which is exactly one block of each operand, so scales
// are applied inside the instruction and the FP32 accumulation sees the
// true products.
//
// Operand layout of the 32x32x64 FP8 MFMA (eight dwords per lane, row
// l%32 of A, column l%32 of B): bytes 0..15 of a lane belong to the first
// 32-deep K block and bytes 16..31 to the second; the two lane halves
// (l/32 = 0, 1) each supply 16 values of both blocks, and the E8M0 scale
// of lane l applies to K block l/32 of its row (column).  Lane half h
// therefore carries K = 16h..16h+15 and 32+16h..32+16h+15 of the 64-deep
// step, and its scale is that of block h.  The accumulator is laid out as
// for the other 32x32 MFMAs.
#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4_t;

constexpr int F8_BM = 128;   // rows per tile
constexpr int F8_BK = 128;   // K per slice (two MFMA K steps)
constexpr int F8_LD = 144;   // LDS row stride in bytes (16-byte aligned, skewed)

__device__ __forceinline__ u32x4_t load16(const uint8_t *p, int64_t valid) {
    if (valid >= 16 && (((uintptr_t)p) & 15) == 0) return *(const u32x4_t *)p;
    uint8_t tmp[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) tmp[q] = (q < valid) ? p[q] : (uint8_t)0;
    return __builtin_bit_cast(u32x4_t, tmp);
}

// E8M0 exponent byte of a power-of-two FP32 scale
__device__ __forceinline__ int e8m0_of(float s) { return (int)((__float_as_uint(s) >> 23) & 0xFF); }

template <int NB, bool ATRANS>
__global__ __launch_bounds__(256) void k_gemm_f8(const uint8_t *__restrict__ A, int64_t lda,
                                                 const float *__restrict__ Ascale, int64_t lds_blk,
                                                 int64_t m, int64_t kdim, int b,
                                                 const uint8_t *__restrict__ Vt, int64_t ldvt,
                                                 const uint8_t *__restrict__ Vsc, int64_t ldvs,
                                                 float *__restrict__ W, int64_t ldw,
                                                 int64_t k_per_split, int ntiles, int nsplit,
                                                 int xcd_map) {
    constexpr int BN = 32 * NB;
    __shared__ __attribute__((aligned(16))) uint8_t As[F8_BM][F8_LD];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[BN][F8_LD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
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
    const int64_t i0 = (int64_t)(tile / gy) * F8_BM;
    const int j0 = (tile % gy) * BN;
    const int64_t kbeg = (int64_t)z * k_per_split;
    const int64_t kend = kbeg + k_per_split < kdim ? kbeg + k_per_split : kdim;

    f32x16_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x16_t{};
    u32x4_t ra[4], rb[NB];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int c = t + 256 * s;
            if (ATRANS) {  // row i: 128 contiguous bytes of K
                const int row = c >> 3, kc = (c & 7) * 16;
                const int64_t gi = i0 + row, gk = k0 + kc;
                ra[s] = (gi < m) ? load16(A + gk + gi * lda, kend - gk) : u32x4_t{0u, 0u, 0u, 0u};
            } else {  // column k: 128 contiguous rows
                const int kk = c >> 3, rc = (c & 7) * 16;
                const int64_t gk = k0 + kk, gi = i0 + rc;
                ra[s] = (gk < kend) ? load16(A + gi + gk * lda, m - gi) : u32x4_t{0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            const int c = t + 256 * s;
            const int col = c >> 3, kc = (c & 7) * 16;
            const int64_t gk = k0 + kc;
            rb[s] = (j0 + col < b) ? load16(Vt + (int64_t)(j0 + col) * ldvt + gk, kend - gk)
                                   : u32x4_t{0u, 0u, 0u, 0u};
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int c = t + 256 * s;
            if (ATRANS) {
                *(u32x4_t *)&As[c >> 3][(c & 7) * 16] = ra[s];
            } else {
                const int kk = c >> 3, rc = (c & 7) * 16;
                uint8_t tmp[16];
                __builtin_memcpy(tmp, &ra[s], 16);
#pragma unroll
                for (int q = 0; q < 16; ++q) As[rc + q][kk] = tmp[q];
            }
        }
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            const int c = t + 256 * s;
            *(u32x4_t *)&Bs[c >> 3][(c & 7) * 16] = rb[s];
        }
    };
    // per-lane E8M0 scales of the current K step
    const int64_t arow = i0 + 32 * wave + (lane & 31);
    if (kbeg < kend) fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += F8_BK) {
        stash();
        __syncthreads();
        if (k0 + F8_BK < kend) fetch(k0 + F8_BK);
#pragma unroll
        for (int kk = 0; kk < F8_BK; kk += 64) {
            const int kq = kk + 32 * (lane >> 5);
            const int64_t kblk = (k0 + kq) >> 5;
            int sa = 127;  // scale 1 for rows/k past the end (their codes are 0)
            if (arow < m && k0 + kq < kend) {
                const int64_t rb_ = arow >> 5;
                const float s = ATRANS ? Ascale[kblk + rb_ * lds_blk] : Ascale[rb_ + kblk * lds_blk];
                sa = e8m0_of(s);
            }
            // this lane's 16 values of each 32-deep block of the step
            const int kb0 = kk + 16 * (lane >> 5), kb1 = kb0 + 32;
            i32x8_t a;
            {
                const u32x4_t lo = *(const u32x4_t *)&As[32 * wave + (lane & 31)][kb0];
                const u32x4_t hi = *(const u32x4_t *)&As[32 * wave + (lane & 31)][kb1];
                a = i32x8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                            (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int col = j0 + 32 * nb + (lane & 31);
                int sb = 127;
                if (col < b && k0 + kq < kend) sb = Vsc[(int64_t)col * ldvs + kblk];
                const u32x4_t lo = *(const u32x4_t *)&Bs[32 * nb + (lane & 31)][kb0];
                const u32x4_t hi = *(const u32x4_t *)&Bs[32 * nb + (lane & 31)][kb1];
                const i32x8_t bv = i32x8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                                           (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                acc[nb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, bv, acc[nb], 0, 0, 0, sa, 0,
                                                                          sb);
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

// FP32 row-major block (rows x b, ld) -> e4m3fn codes K-contiguous per column
// (b x ldt bytes) with one E8M0 scale byte per 32 rows of each column
// (b x ldt/32); scale = smallest power of two with amax / scale <= 448.
__global__ void k_quant_basis_f8(const float *__restrict__ s, int64_t rows, int b, int64_t ld,
                                 uint8_t *__restrict__ codes, int64_t ldt, uint8_t *__restrict__ sc,
                                 int64_t lds) {
    const int64_t nblk = (rows + 31) / 32;
    const int64_t total = nblk * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / nblk);
        const int64_t kb = e - (int64_t)j * nblk;
        float amax = 0.f;
        for (int q = 0; q < 32; ++q) {
            const int64_t i = kb * 32 + q;
            if (i < rows) amax = fmaxf(amax, fabsf(s[i * ld + j]));
        }
        int e8 = 127;
        if (amax > 0.f) {
            int ex;
            const float mm = frexpf(amax, &ex);
            e8 = 127 + (mm <= 0.875f ? ex - 9 : ex - 8);
            if (e8 < 1) e8 = 1;
            if (e8 > 254) e8 = 254;
        }
        const float inv = __uint_as_float((uint32_t)(254 - e8) << 23);  // 2^-(e8-127)
        sc[(int64_t)j * lds + kb] = (uint8_t)e8;
        for (int q = 0; q < 32; ++q) {
            const int64_t i = kb * 32 + q;
            if (i < ldt) codes[(int64_t)j * ldt + i] = (i < rows) ? f32_to_e4m3_bits(s[i * ld + j] * inv) : 0;
        }
    }
}

__global__ void k_sum_slabs_f8(const float *__restrict__ P, int nsplit, int64_t m, int b, int64_t ld,
                               float *__restrict__ W) {
    const int64_t total = m * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / b;
        const int j = (int)(e - i * b);
        float acc = 0.f;
        for (int zz = 0; zz < nsplit; ++zz) acc += P[(int64_t)zz * m * ld + i * ld + j];
        W[i * ld + j] = acc;
    }
}

inline int grid1(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

}  // namespace

int64_t f8_ldt(int64_t rows) { return (rows + 127) / 128 * 128; }

void quant_basis_f8(Context *ctx, int64_t rows, int32_t b, const float *src, int64_t ld,
                    uint8_t *codes, uint8_t *scales) {
    const int64_t ldt = f8_ldt(rows);
    const int64_t nblk = (rows + 31) / 32;
    hipLaunchKernelGGL(k_quant_basis_f8, dim3(grid1(nblk * b)), dim3(256), 0, ctx->stream, src, rows, b,
                       ld, codes, ldt, scales, ldt / 32);
    OFRR_HIP(hipGetLastError());
}

// A: e4m3fn codes (A->rows x A->cols, column-major, ld = rows) with block
// scales (ceil(rows/32) x ceil(cols/32), column-major).  W = op(A) V.
void product_f8(Context *ctx, int64_t arows, int64_t acols, const uint8_t *Acodes,
                const float *Ascale, int trans, int32_t b, const uint8_t *Vt,
                const uint8_t *Vsc, float *W, int64_t ldw) {
    OFRR_CHECK_ARG(b >= 1 && b <= 4096, "product_f8: 1 <= b <= 4096");
    const int64_t m = trans ? acols : arows, kdim = trans ? arows : acols;
    const int64_t ldvt = f8_ldt(kdim), ldvs = ldvt / 32;
    const int64_t lds_blk = (arows + 31) / 32;
    const int NB = b > 64 ? 4 : 2;
    const int BN = 32 * NB;
    const int gx = (int)((m + F8_BM - 1) / F8_BM), gy = (b + BN - 1) / BN;
    const int ntiles = gx * gy;
    int nsplit = 1;
    const int64_t want = 2LL * (ctx->cu_count > 0 ? ctx->cu_count : 256);
    while ((int64_t)ntiles * nsplit < want && kdim / (nsplit * 2) >= 2048 && nsplit < 8) nsplit *= 2;
    int64_t kps = (kdim + nsplit - 1) / nsplit;
    kps = (kps + F8_BK - 1) / F8_BK * F8_BK;
    nsplit = (int)((kdim + kps - 1) / kps);
    const int xcd_map = (nsplit >= 2 && 8 % nsplit == 0) ? 1 : 0;
    int64_t nwg = (int64_t)ntiles * nsplit;
    if (xcd_map) nwg = (int64_t)((ntiles + 8 / nsplit - 1) / (8 / nsplit)) * 8;
    float *dst = W;
    if (nsplit > 1) dst = ctx->buf<float>("f8_slabs", (size_t)nsplit * m * ldw);
    {
        KTimer tm(ctx, "product_f8");
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(256), 0, ctx->stream, Acodes, arows, Ascale,
                               lds_blk, m, kdim, b, Vt, ldvt, Vsc, ldvs, dst, ldw, kps, ntiles, nsplit,
                               xcd_map);
        };
        if (NB == 4)
            trans ? go(k_gemm_f8<4, true>) : go(k_gemm_f8<4, false>);
        else
            trans ? go(k_gemm_f8<2, true>) : go(k_gemm_f8<2, false>);
        OFRR_HIP(hipGetLastError());
    }
    if (nsplit > 1) {
        KTimer tm(ctx, "product_reduce");
        hipLaunchKernelGGL(k_sum_slabs_f8, dim3(grid1(m * b)), dim3(256), 0, ctx->stream, dst, nsplit, m,
                           b, ldw, W);
        OFRR_HIP(hipGetLastError());
    }
}

}  // namespace ofrr
