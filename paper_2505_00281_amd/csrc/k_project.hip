// k_project.hip -- the projections of the orthogonalization-free
// Rayleigh-Ritz step (Sec. 3.1, Alg. "Orthogonalization-Free Rayleigh-Ritz
// Projection": B = U^T A U and M = U^T U; here G = V^T V and H = V^T W with
// W = A V already formed).  Inputs are tall row-major n x b blocks in any
// storage type.  Three accumulation modes (the mixed-precision plan at the
// end of Sec. 4 forms these products in FP32 from reduced-precision data):
//   FP64         each product of two stored values is exact in FP64 (16 x
//                16, 16 x 24 and 24 x 24 significand bits all fit in 53), so
//                the only rounding is the FP64 accumulation (FP64 MFMA);
//   FP32         FP32 MFMA over a workgroup's whole row chunk, the chunk
//                partials summed in FP32;
//   compensated  FP32 MFMA over runs of PJ_RUN rows, each run's sums added
//                into FP64 accumulators, chunk partials summed in FP64: the
//                error per entry is that of a PJ_RUN-term FP32 sum (plus the
//                FP32 rounding of the products), independent of n.
// Row chunks are summed per workgroup, then the chunk partials are added in
// a fixed order (deterministic).
#include <cstdlib>
#include <type_traits>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

constexpr int PJ_T = 64;      // output tile (PJ_T x PJ_T) per workgroup
constexpr int PJ_D = 8;       // row steps (of four) in flight per wave
constexpr int PJ_RUN = 4 * PJ_D;  // rows per FP32 run of the compensated mode

enum { PJ_F64 = 0, PJ_F32C = 1, PJ_F32 = 2 };

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double pj_f64x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float pj_f32x4_t;

// grid (nchunks, ntiles_i, ntiles_j).  Partial sums over rows
// [c*rows_per, (c+1)*rows_per) of X^T Y for one 64 x 64 tile, written to
// part[c][tile] (row-major within the tile).  MFMA 16x16x4 (FP64, or FP32
// in the FP32 modes) with both operands read straight from the row-major
// blocks: for a 4-row step, lane l needs X[r + l/16][i + l%16] and
// Y[r + l/16][j + l%16], 16 consecutive values of a row per lane group, so
// no LDS staging is needed; the next step's operands are loaded while the
// current MFMAs run.  Each wave owns a 32 x 32 quarter of the tile (2 x 2
// MFMA blocks).
template <class TX, class TY, int MODE>
__global__ __launch_bounds__(256) void k_gram_partial(const TX *__restrict__ X, int64_t ldx,
                                                      const TY *__restrict__ Yb, int64_t ldy,
                                                      int64_t n, int b1, int b2, int64_t rows_per,
                                                      double *__restrict__ part) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int i0 = blockIdx.y * PJ_T + 32 * (wave >> 1), j0 = blockIdx.z * PJ_T + 32 * (wave & 1);
    const int64_t rbeg = (int64_t)blockIdx.x * rows_per;
    int64_t rend = rbeg + rows_per;
    if (rend > n) rend = n;
    const int kr = lane >> 4, cc = lane & 15;
    pj_f64x4_t acc[2][2];
    pj_f32x4_t acc32[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            acc[p][q] = pj_f64x4_t{0.0, 0.0, 0.0, 0.0};
            acc32[p][q] = pj_f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
    // PJ_D steps of four rows in flight: the loads of step s + PJ_D are
    // issued when step s is consumed.  Every load is unconditional (row and
    // column clamped into the block) and holds the stored value; the range
    // test and the conversion happen where the value is used, so no load
    // waits for its data before the next ones are issued.
    bool oki[2], okj[2];
    int64_t ci[2], cj[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int i = i0 + 16 * p + cc, j = j0 + 16 * p + cc;
        oki[p] = i < b1;
        okj[p] = j < b2;
        ci[p] = oki[p] ? i : b1 - 1;
        cj[p] = okj[p] ? j : b2 - 1;
    }
    TX xr[PJ_D][2];
    TY yr[PJ_D][2];
    auto fetch = [&](int64_t r0, TX (&xs)[2], TY (&ys)[2]) {
        const int64_t r = r0 + kr;
        const int64_t rc = r < rend ? r : rend - 1;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            xs[p] = X[rc * ldx + ci[p]];
            ys[p] = Yb[rc * ldy + cj[p]];
        }
    };
#pragma unroll
    for (int st = 0; st < PJ_D; ++st) fetch(rbeg + 4 * st, xr[st], yr[st]);
    for (int64_t r0 = rbeg; r0 < rend; r0 += 4 * PJ_D) {
#pragma unroll
        for (int st = 0; st < PJ_D; ++st) {
            const bool okr = r0 + 4 * st + kr < rend;
            const double a0 = (okr && oki[0]) ? load_as_f64(&xr[st][0]) : 0.0;
            const double a1 = (okr && oki[1]) ? load_as_f64(&xr[st][1]) : 0.0;
            const double b0 = (okr && okj[0]) ? load_as_f64(&yr[st][0]) : 0.0;
            const double b1v = (okr && okj[1]) ? load_as_f64(&yr[st][1]) : 0.0;
            fetch(r0 + 4 * (st + PJ_D), xr[st], yr[st]);
            if constexpr (MODE == PJ_F64) {
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1v, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1v, acc[1][1], 0, 0, 0);
            } else {
                // FP32 modes take FP32 or narrower inputs: the conversions are exact
                const float fa0 = (float)a0, fa1 = (float)a1, fb0 = (float)b0, fb1 = (float)b1v;
                acc32[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa0, fb0, acc32[0][0], 0, 0, 0);
                acc32[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa0, fb1, acc32[0][1], 0, 0, 0);
                acc32[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa1, fb0, acc32[1][0], 0, 0, 0);
                acc32[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa1, fb1, acc32[1][1], 0, 0, 0);
            }
        }
        if constexpr (MODE == PJ_F32C) {
            // end of a PJ_RUN-row run: its FP32 sums go into the FP64 accumulators
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        acc[p][q][r] += (double)acc32[p][q][r];
                        acc32[p][q][r] = 0.f;
                    }
        }
    }
    if constexpr (MODE == PJ_F32) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[p][q][r] = (double)acc32[p][q][r];
    }
    // accumulator register r of lane l is D[4r + l/16][l%16] for the FP64
    // MFMA and D[4(l/16) + r][l%16] for the FP32 one
    const int ntile = gridDim.y * gridDim.z;
    const int tile = blockIdx.y * gridDim.z + blockIdx.z;
    double *dst = part + ((int64_t)blockIdx.x * ntile + tile) * PJ_T * PJ_T;
    const int ti = 32 * (wave >> 1), tj = 32 * (wave & 1);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = MODE == PJ_F64 ? 4 * r + kr : 4 * kr + r;
                dst[(ti + 16 * p + row) * PJ_T + tj + 16 * q + cc] = acc[p][q][r];
            }
}

// Sum the chunk partials in chunk order and write C (b1 x b2, column-major,
// ld = b1).  Threads walk the partials in their memory order (tile, row,
// column), so a wave reads 64 consecutive doubles of every chunk; the
// scattered writes of C are 8 bytes each.
// F32SUM: the sums run in FP32 (the FP32 mode; its partials are FP32
// values held in doubles), else in FP64.
template <bool F32SUM>
__global__ void k_gram_reduce(const double *__restrict__ part, int nchunks, int ntj, int b1,
                              int b2, double *__restrict__ C) {
    const int nti = (b1 + PJ_T - 1) / PJ_T;
    const int64_t cstride = (int64_t)nti * ntj * PJ_T * PJ_T;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cstride;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int tile = (int)(e / (PJ_T * PJ_T)), rem = (int)(e % (PJ_T * PJ_T));
        const int i = (tile / ntj) * PJ_T + rem / PJ_T, j = (tile % ntj) * PJ_T + rem % PJ_T;
        // chunk order fixed (deterministic); 16 loads in flight
        const double *pp = part + e;
        using S = std::conditional_t<F32SUM, float, double>;
        S s = 0;
        int c = 0;
        for (; c + 16 <= nchunks; c += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = pp[(int64_t)(c + u) * cstride];
#pragma unroll
            for (int u = 0; u < 16; ++u) s += (S)v[u];
        }
        for (; c < nchunks; ++c) s += (S)pp[(int64_t)c * cstride];
        if (i < b1 && j < b2) C[(int64_t)j * b1 + i] = (double)s;
    }
}

// t = sum_i G_ii sum_j Y_ij^2 / b (one workgroup; G and Y column-major b x b)
__global__ __launch_bounds__(256) void k_gram_condition(const double *__restrict__ G,
                                                        const double *__restrict__ Y, int b,
                                                        const int32_t *__restrict__ rank,
                                                        double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < b; i += 256) {
        double r = 0.0;
        for (int j = 0; j < b; ++j) {
            const double y = Y[i + (int64_t)j * b];
            r = fma(y, y, r);
        }
        s = fma(G[i + (int64_t)i * b], r, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (rank && rank[0] < b) ? __builtin_inf() : red[0] / b;
}

template <class F>
void dispatch_store(ofrr_dtype t, F &&f) {
    switch (t) {
        case OFRR_F64: f((double *)nullptr); break;
        case OFRR_F32: f((float *)nullptr); break;
        case OFRR_BF16: f((bf16_t *)nullptr); break;
        case OFRR_F16: f((f16_t *)nullptr); break;
        default: fail(OFRR_ERR_UNSUPPORTED, "projection: element type");
    }
}

}  // namespace

void gram_rect(Context *ctx, int64_t n, int32_t b1, int32_t b2, ofrr_dtype xt, const void *X,
               int64_t ldx, ofrr_dtype yt, const void *Y, int64_t ldy, double *C, ofrr_accum acc) {
    KTimer tm(ctx, "gram");
    if (acc != OFRR_ACC_F64 && (xt == OFRR_F64 || yt == OFRR_F64))
        fail(OFRR_ERR_UNSUPPORTED, "projection: FP32 accumulation takes FP32, BF16 or F16 blocks");
    const int nti = (b1 + PJ_T - 1) / PJ_T, ntj = (b2 + PJ_T - 1) / PJ_T;
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    // enough chunks to fill the chip, each at least min_rows rows
    // (OFRR_GRAM_ROWS overrides, for tuning sweeps)
    int64_t min_rows = 256;
    if (const char *e = std::getenv("OFRR_GRAM_ROWS")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 32 && v <= 4096) min_rows = v;
    }
    int64_t nchunks = std::max<int64_t>(
        1, std::min<int64_t>((n + min_rows - 1) / min_rows, (8 * cus + nti * ntj - 1) / (nti * ntj)));
    int64_t rows_per = (n + nchunks - 1) / nchunks;
    // whole passes of PJ_RUN rows (the compensated mode's FP32 runs)
    rows_per = (rows_per + PJ_RUN - 1) / PJ_RUN * PJ_RUN;
    nchunks = (n + rows_per - 1) / rows_per;
    double *part = ctx->buf<double>("gram_part", (size_t)nchunks * nti * ntj * PJ_T * PJ_T);
    dim3 grid((unsigned)nchunks, nti, ntj);
    auto launch = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        dispatch_store(xt, [&](auto *xp) {
            using TX = std::remove_pointer_t<decltype(xp)>;
            dispatch_store(yt, [&](auto *yp) {
                using TY = std::remove_pointer_t<decltype(yp)>;
                hipLaunchKernelGGL((k_gram_partial<TX, TY, M>), grid, dim3(256), 0, ctx->stream,
                                   (const TX *)X, ldx, (const TY *)Y, ldy, n, b1, b2, rows_per, part);
            });
        });
    };
    if (acc == OFRR_ACC_F64)
        launch(std::integral_constant<int, PJ_F64>{});
    else if (acc == OFRR_ACC_F32_COMPENSATED)
        launch(std::integral_constant<int, PJ_F32C>{});
    else
        launch(std::integral_constant<int, PJ_F32>{});
    OFRR_HIP(hipGetLastError());
    const int64_t total = (int64_t)nti * ntj * PJ_T * PJ_T;
    const dim3 rg((unsigned)std::min<int64_t>((total + 255) / 256, 4096));
    if (acc == OFRR_ACC_F32)
        hipLaunchKernelGGL(k_gram_reduce<true>, rg, dim3(256), 0, ctx->stream, part, (int)nchunks, ntj, b1, b2, C);
    else
        hipLaunchKernelGGL(k_gram_reduce<false>, rg, dim3(256), 0, ctx->stream, part, (int)nchunks, ntj, b1, b2, C);
    OFRR_HIP(hipGetLastError());
}

void gram_condition(Context *ctx, int32_t b, const double *G, const double *Y, const int32_t *rank,
                    double *out) {
    hipLaunchKernelGGL(k_gram_condition, dim3(1), dim3(256), 0, ctx->stream, G, Y, b, rank, out);
    OFRR_HIP(hipGetLastError());
}

void project(Context *ctx, int64_t n, int32_t b, ofrr_dtype vt, const void *V, int64_t ldv,
             ofrr_dtype wt, const void *W, int64_t ldw, ofrr_accum acc, double *G, double *H) {
    gram_rect(ctx, n, b, b, vt, V, ldv, vt, V, ldv, G, acc);
    gram_rect(ctx, n, b, b, vt, V, ldv, wt, W, ldw, H, acc);
}

}  // namespace ofrr
