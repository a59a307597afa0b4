// k_misc.hip -- elementwise and column-wise kernels: fills, precision
// conversions (storage formats of the mixed-precision plan, end of Sec. 4),
// FP8 block quantisation, the U(0,1) start block (Sec. 5.2) and the
// per-column scaling that follows each product (Sec. 2, Alg. "Multiple Step
// Subspace Iteration": column scaling after every multiplication).
#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

__global__ void k_zero(uint32_t *p, int64_t words) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

__global__ void k_f32_to_bf16(const float *__restrict__ s, uint16_t *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = f32_to_bf16_bits(s[i]);
}

__global__ void k_f32_to_f16(const float *__restrict__ s, uint16_t *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = f32_to_f16_bits(s[i]);
}

__global__ void k_f64_to_f32(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = (float)s[i];
}

template <class S, class D>
__global__ void k_cast_matrix(const S *__restrict__ s, int64_t lds, D *__restrict__ d,
                              int64_t ldd, int64_t rows, int64_t cols, double scale) {
    int64_t total = rows * cols;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        int64_t c = i / rows, r = i - c * rows;
        store_as<D>(d + r + c * ldd, load_as_f64(s + r + c * lds) * scale);
    }
}

// dst[c + r * ldd] = src[r * lds + c] (a row-major rows x cols block into a
// column-major one, or back with the roles swapped), converting the type
template <class S, class D>
__global__ void k_transpose_cast(const S *__restrict__ s, int64_t lds, D *__restrict__ d, int64_t ldd,
                                 int64_t rows, int64_t cols) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e - r * cols;
        store_as<D>(d + c * ldd + r, load_as_f64(s + r * lds + c));
    }
}

// Largest magnitude of an FP64 array (dense column-major rows x cols with
// leading dimension ld, or a flat array: rows = count, cols = 1), merged as
// the FP64 bit pattern by atomic maximum (non-negative doubles order as
// their bits); NaN or infinity merges all ones.
__global__ __launch_bounds__(256) void k_absmax_f64(const double *__restrict__ a, int64_t ld, int64_t rows,
                                                    int64_t cols, unsigned long long *__restrict__ out) {
    const int64_t total = rows * cols;
    unsigned long long m = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / rows, r = i - c * rows;
        const double v = a[r + c * ld];
        const unsigned long long key =
            (v == v && !isinf(v)) ? (unsigned long long)__double_as_longlong(fabs(v)) : ~0ull;
        m = key > m ? key : m;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long q = __shfl_xor(m, o);
        m = q > m ? q : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// One 32 x 32 block per 256-thread workgroup: amax, power-of-two scale,
// e4m3fn codes.
__global__ void k_fp8_blocks(const float *__restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                             uint8_t *__restrict__ codes, float *__restrict__ scales,
                             int64_t brows) {
    const int64_t bi = blockIdx.x, bj = blockIdx.y;
    const int tid = threadIdx.x;
    __shared__ float red[256];
    float amax = 0.f;
    for (int e = tid; e < 1024; e += 256) {
        int64_t r = bi * 32 + (e & 31), c = bj * 32 + (e >> 5);
        if (r < rows && c < cols) amax = fmaxf(amax, fabsf(A[r + c * lda]));
    }
    red[tid] = amax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    amax = red[0];
    // scale = smallest power of two 2^k, k >= -126, with amax / 2^k <= 448
    // (448 = 0.875 * 2^9), decided exactly from amax = m 2^e, m in [0.5, 1);
    // 1 for an all-zero block.  The floor keeps 2^k and 2^-k normal FP32
    // numbers and 2^k an E8M0 scale byte.
    float scale = 1.f;
    if (amax > 0.f) {
        int e;
        const float m = frexpf(amax, &e);
        scale = ldexpf(1.f, max(m <= 0.875f ? e - 9 : e - 8, -126));
    }
    if (tid == 0) scales[bi + bj * brows] = scale;
    const float inv = 1.f / scale;  // exact: scale is a power of two
    for (int e = tid; e < 1024; e += 256) {
        int64_t r = bi * 32 + (e & 31), c = bj * 32 + (e >> 5);
        if (r < rows && c < cols) codes[r + c * rows] = f32_to_e4m3_bits(A[r + c * lda] * inv);
    }
}

// Counter-based U(0,1): SplitMix64 of (seed, index), top 53 bits.
__global__ void k_uniform(double *X, int64_t count, uint64_t seed) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        X[i] = (double)(z >> 11) * 0x1.0p-53;
    }
}

// Block x reduces rows [x*rows_per_block, ...) over all b columns and merges
// its maxima into cmax[c * 512 + j] (c = block index mod CM_COPIES, zero on
// entry) by atomic maximum: the maximum of keys does not depend on the
// merge order, and the copies spread the atomics of many blocks.

template <class T>
__global__ __launch_bounds__(256) void k_colmax_partial(const T *__restrict__ Y, int64_t ldy,
                                                        int64_t n, int b, int64_t rows_per_block,
                                                        unsigned *__restrict__ cmax) {
    // for b <= 256 the block is split into 256 / b row groups, thread t takes
    // column t % b of group t / b (consecutive threads read consecutive
    // columns); wider blocks loop over columns
    __shared__ unsigned cm[256];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
    if (b <= 256) {
        const int groups = 256 / b;
        const int j = t % b, g = t / b;
        unsigned m = 0u;
        if (g < groups) {
            int64_t r = r0 + g;
            for (; r + 7 * groups < r1; r += 8 * groups) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = load_as_f64(Y + (r + u * groups) * ldy + j);
#pragma unroll
                for (int u = 0; u < 8; ++u) m = max(m, mag_key<T>(v[u]));
            }
            for (; r < r1; r += groups) m = max(m, mag_key<T>(load_as_f64(Y + r * ldy + j)));
        }
        cm[t] = m;
        __syncthreads();
        if (t < b) {
            unsigned mm = 0u;
            for (int q = 0; q < groups; ++q) mm = max(mm, cm[q * b + t]);
            atomicMax(cmax + (blockIdx.x % CM_COPIES) * 512 + t, mm);
        }
    } else {
        for (int j = t; j < b; j += 256) {
            unsigned m = 0u;
            for (int64_t r = r0; r < r1; ++r) m = max(m, mag_key<T>(load_as_f64(Y + r * ldy + j)));
            atomicMax(cmax + (blockIdx.x % CM_COPIES) * 512 + j, m);
        }
    }
}

// Power-of-two column scales (key_scale of the merged maxima, the largest of
// CM_COPIES copies) applied to Y and, when given, Z; workgroup 0 also zeroes
// all copies of `clear` for the next merge.
template <class T>
__global__ __launch_bounds__(256) void k_scale_apply2(T *__restrict__ Y, int64_t ldy, T *__restrict__ Z,
                                                      int64_t ldz, int64_t n, int b,
                                                      const unsigned *__restrict__ cmax,
                                                      unsigned *__restrict__ clear) {
    __shared__ double sc[512];
    const int t = threadIdx.x;
    for (int j = t; j < b; j += 256) {
        unsigned mb = cmax[j];
#pragma unroll
        for (int c = 1; c < CM_COPIES; ++c) mb = max(mb, cmax[c * 512 + j]);
        sc[j] = key_scale<T>(mb);
    }
    // the other merge arrays, whole, for the next call (whatever its width)
    if (blockIdx.x == 0)
        for (int e = t; e < CM_COPIES * 512; e += 256) clear[e] = 0u;
    __syncthreads();
    const int cols = b < 256 ? b : 256;
    const int groups = 256 / cols;
    const int j0 = t % cols, g = t / cols;
    if (g >= groups) return;
    for (int64_t r = (int64_t)blockIdx.x * groups + g; r < n; r += (int64_t)gridDim.x * groups)
        for (int j = j0; j < b; j += cols) {
            const double f = sc[j];
            T *p = Y + r * ldy + j;
            const double yv = load_as_f64(p);
            if (Z) {
                T *q = Z + r * ldz + j;
                const double zv = load_as_f64(q);
                store_as<T>(q, zv * f);
            }
            store_as<T>(p, yv * f);
        }
}

__global__ void k_zero_u32(unsigned *__restrict__ p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// row-major compaction: d[i, dest[j]] = s[i, j] for kept j
template <class T>
__global__ void k_compact_rm(const T *__restrict__ s, int64_t lds, T *__restrict__ d, int64_t ldd,
                             int64_t n, const int32_t *__restrict__ dest_col, int b) {
    const int64_t total = n * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / b;
        const int j = (int)(e - i * b);
        const int dj = dest_col[j];
        if (dj >= 0) d[i * ldd + dj] = s[i * lds + j];
    }
}

template <class D>
__global__ void k_cm_to_rm(const double *__restrict__ s, int64_t lds, int64_t n, int b,
                           D *__restrict__ d, int64_t ldd) {
    const int64_t total = n * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / b;
        const int j = (int)(e - i * b);
        store_as<D>(d + i * ldd + j, s[i + (int64_t)j * lds]);
    }
}

template <bool BF16>
__global__ void k_split(const float *__restrict__ s, int64_t n, uint16_t *__restrict__ hi,
                        uint16_t *__restrict__ lo) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float x = s[e];
        const uint16_t h = BF16 ? f32_to_bf16_bits(x) : f32_to_f16_bits(x);
        hi[e] = h;
        if (lo) {
            const float hv = BF16 ? bf16_bits_to_f32(h) : f16_bits_to_f32(h);
            const float r = x - hv;  // exact: x and hv share the leading bits
            lo[e] = BF16 ? f32_to_bf16_bits(r) : f32_to_f16_bits(r);
        }
    }
}

template <bool BF16>
__global__ void k_round(float *__restrict__ x, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        x[e] = BF16 ? bf16_bits_to_f32(f32_to_bf16_bits(x[e])) : f16_bits_to_f32(f32_to_f16_bits(x[e]));
}

__global__ void k_f32_to_f64_copy(const float *__restrict__ s, double *__restrict__ d, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        d[e] = (double)s[e];
}

__global__ void k_keep_to_dest(const int32_t *keep, int b, int32_t *dest) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int c = 0;
        for (int j = 0; j < b; ++j) dest[j] = keep[j] ? c++ : -1;
    }
}

inline int grid_for(int64_t count, int block = 256) {
    int64_t g = (count + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

template <class F>
void dispatch_type(ofrr_dtype t, F &&f) {
    switch (t) {
        case OFRR_F64: f((double *)nullptr); break;
        case OFRR_F32: f((float *)nullptr); break;
        case OFRR_BF16: f((bf16_t *)nullptr); break;
        case OFRR_F16: f((f16_t *)nullptr); break;
        default: fail(OFRR_ERR_UNSUPPORTED, "element type not supported here");
    }
}

}  // namespace

void zero_bytes(Context *ctx, void *p, size_t bytes) {
    if (!bytes) return;
    int64_t words = (int64_t)((bytes + 3) / 4);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(words)), dim3(256), 0, ctx->stream, (uint32_t *)p, words);
    OFRR_HIP(hipGetLastError());
}

void cast_f32_to_bf16(Context *ctx, int64_t count, const float *src, uint16_t *dst) {
    KTimer t(ctx, "quantize");
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for(count)), dim3(256), 0, ctx->stream, src, dst, count);
    OFRR_HIP(hipGetLastError());
}

void cast_f32_to_f16(Context *ctx, int64_t count, const float *src, uint16_t *dst) {
    KTimer t(ctx, "quantize");
    hipLaunchKernelGGL(k_f32_to_f16, dim3(grid_for(count)), dim3(256), 0, ctx->stream, src, dst, count);
    OFRR_HIP(hipGetLastError());
}

void cast_f64_to_f32(Context *ctx, int64_t count, const double *src, float *dst) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(count)), dim3(256), 0, ctx->stream, src, dst, count);
    OFRR_HIP(hipGetLastError());
}

void cast_matrix(Context *ctx, ofrr_dtype st, ofrr_dtype dt, int64_t rows, int64_t cols,
                 const void *src, int64_t lds, void *dst, int64_t ldd, double scale) {
    if (rows <= 0 || cols <= 0) return;
    int g = grid_for(rows * cols);
    dispatch_type(st, [&](auto *sp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        dispatch_type(dt, [&](auto *dp) {
            using D = std::remove_pointer_t<decltype(dp)>;
            hipLaunchKernelGGL((k_cast_matrix<S, D>), dim3(g), dim3(256), 0, ctx->stream,
                               (const S *)src, lds, (D *)dst, ldd, rows, cols, scale);
        });
    });
    OFRR_HIP(hipGetLastError());
}

__global__ void k_pair(int32_t *d, int32_t a, int32_t b) {
    if (threadIdx.x == 0) {
        d[0] = a;
        d[1] = b;
    }
}

__global__ void k_identity(double *G, int b) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < b * b; e += gridDim.x * blockDim.x)
        G[e] = (e % b == e / b) ? 1.0 : 0.0;
}

const int32_t *status_pair(Context *ctx, int32_t a, int32_t b) {
    int32_t *d = ctx->buf<int32_t>("status_pair", 2);
    hipLaunchKernelGGL(k_pair, dim3(1), dim3(64), 0, ctx->stream, d, a, b);
    OFRR_HIP(hipGetLastError());
    return d;
}

void set_identity(Context *ctx, int32_t b, double *G) {
    hipLaunchKernelGGL(k_identity, dim3((b * b + 255) / 256), dim3(256), 0, ctx->stream, G, b);
    OFRR_HIP(hipGetLastError());
}

void transpose_cast(Context *ctx, ofrr_dtype st, ofrr_dtype dt, int64_t rows, int64_t cols, const void *src,
                    int64_t lds, void *dst, int64_t ldd) {
    if (rows <= 0 || cols <= 0) return;
    dispatch_type(st, [&](auto *sp) {
        using S = std::remove_pointer_t<decltype(sp)>;
        dispatch_type(dt, [&](auto *dp) {
            using D = std::remove_pointer_t<decltype(dp)>;
            hipLaunchKernelGGL((k_transpose_cast<S, D>), dim3(grid_for(rows * cols)), dim3(256), 0, ctx->stream,
                               (const S *)src, lds, (D *)dst, ldd, rows, cols);
        });
    });
    OFRR_HIP(hipGetLastError());
}

double absmax_values(Context *ctx, const ofrr_matrix *A) {
    OFRR_CHECK_ARG(A->dtype == OFRR_F64, "absmax_values: FP64 values");
    int64_t rows = A->rows, cols = A->cols, ld = A->ld;
    if (A->format == OFRR_CSR) {
        rows = A->nnz;
        cols = 1;
        ld = rows;
    }
    if (rows <= 0 || cols <= 0) return 0.0;
    unsigned long long *d = ctx->buf<unsigned long long>("absmax", 1);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, ctx->stream, (uint32_t *)d, (int64_t)2);
    const int g = (int)std::min<int64_t>(2048, (rows * cols + 255) / 256);
    hipLaunchKernelGGL(k_absmax_f64, dim3(g), dim3(256), 0, ctx->stream, (const double *)A->values, ld, rows,
                       cols, d);
    OFRR_HIP(hipGetLastError());
    unsigned long long h = 0;
    OFRR_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    OFRR_HIP(hipStreamSynchronize(ctx->stream));
    if (h == ~0ull) return INFINITY;
    double v;
    std::memcpy(&v, &h, sizeof(v));
    return v;
}

void quantize_fp8_blocks(Context *ctx, int64_t rows, int64_t cols, const float *A, int64_t lda,
                         uint8_t *codes, float *scales) {
    KTimer t(ctx, "quantize");
    int64_t br = (rows + 31) / 32, bc = (cols + 31) / 32;
    OFRR_CHECK_ARG(br <= 0x7fffffff && bc <= 65535, "matrix too large for FP8 block grid");
    hipLaunchKernelGGL(k_fp8_blocks, dim3((unsigned)br, (unsigned)bc), dim3(256), 0, ctx->stream, A,
                       lda, rows, cols, codes, scales, br);
    OFRR_HIP(hipGetLastError());
}

void uniform_start(Context *ctx, int64_t n, int32_t b, uint64_t seed, double *X) {
    int64_t count = n * b;
    hipLaunchKernelGGL(k_uniform, dim3(grid_for(count)), dim3(256), 0, ctx->stream, X, count, seed);
    OFRR_HIP(hipGetLastError());
}

void scale_columns_reset(Context *ctx) {
    unsigned *cm2 = ctx->buf<unsigned>("colmax_merge", 2 * CM_COPIES * 512);
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, ctx->stream, cm2, 2 * CM_COPIES * 512);
    OFRR_HIP(hipGetLastError());
    ctx->colmax_parity = 0;
    ctx->vmax_parity = -1;  // the digit-plane slicing clears its own on next use
}

void scale_columns_pow2(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                        ofrr_dtype tz, void *Z, int64_t ldz, float *work) {
    KTimer tm(ctx, "scale");
    (void)work;
    OFRR_CHECK_ARG(b <= 512, "scale_columns_pow2: b <= 512");
    OFRR_CHECK_ARG(Z == nullptr || tz == t, "scale_columns_pow2: both blocks of one type");
    const int64_t rpb = 64;
    const int nblk = (int)((n + rpb - 1) / rpb);
    // two maxima arrays used alternately: each call merges into one and its
    // apply kernel clears the other, which the next call merges into
    if (ctx->colmax_parity < 0) scale_columns_reset(ctx);
    unsigned *cm2 = ctx->buf<unsigned>("colmax_merge", 2 * CM_COPIES * 512);
    unsigned *cur = cm2 + CM_COPIES * 512 * ctx->colmax_parity;
    unsigned *nxt = cm2 + CM_COPIES * 512 * (1 - ctx->colmax_parity);
    dispatch_type(t, [&](auto *p) {
        using T = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_colmax_partial<T>), dim3(nblk), dim3(256), 0, ctx->stream,
                           (const T *)Y, ldy, n, b, rpb, cur);
    });
    // at most 1024 workgroups (each reads the merged maxima once)
    const int rows_per_wg = 256 / (b < 256 ? b : 256);
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + rows_per_wg - 1) / rows_per_wg, 1024));
    dispatch_type(t, [&](auto *p) {
        using T = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_scale_apply2<T>), dim3(g), dim3(256), 0, ctx->stream, (T *)Y, ldy, (T *)Z, ldz, n,
                           b, (const unsigned *)cur, nxt);
    });
    OFRR_HIP(hipGetLastError());
    ctx->colmax_parity ^= 1;
}

void column_keys(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, const void *Y, int64_t ldy, unsigned *keys) {
    KTimer tm(ctx, "scale");
    OFRR_CHECK_ARG(b <= 512, "column_keys: b <= 512");
    const int64_t rpb = 64;
    const int nblk = (int)((n + rpb - 1) / rpb);
    dispatch_type(t, [&](auto *p) {
        using T = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_colmax_partial<T>), dim3(nblk), dim3(256), 0, ctx->stream, (const T *)Y, ldy, n, b,
                           rpb, keys);
    });
    OFRR_HIP(hipGetLastError());
}

void scale_apply_keys(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy, const unsigned *keys,
                      unsigned *clear) {
    KTimer tm(ctx, "scale");
    OFRR_CHECK_ARG(b <= 512, "scale_apply_keys: b <= 512");
    const int rows_per_wg = 256 / (b < 256 ? b : 256);
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + rows_per_wg - 1) / rows_per_wg, 1024));
    dispatch_type(t, [&](auto *p) {
        using T = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_scale_apply2<T>), dim3(g), dim3(256), 0, ctx->stream, (T *)Y, ldy, (T *)nullptr, ldy,
                           n, b, keys, clear);
    });
    OFRR_HIP(hipGetLastError());
}

void zero_keys(Context *ctx, unsigned *keys, int count) {
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::max(1, std::min(64, (count + 255) / 256))), dim3(256), 0,
                       ctx->stream, keys, count);
    OFRR_HIP(hipGetLastError());
}

void compact_columns_rm(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, const void *src,
                        int64_t lds, const int32_t *keep, void *dst, int64_t ldd) {
    OFRR_CHECK_ARG(src != dst, "compact_columns_rm: src and dst must differ");
    int32_t *dest = ctx->buf<int32_t>("compact_dest", b);
    hipLaunchKernelGGL(k_keep_to_dest, dim3(1), dim3(64), 0, ctx->stream, keep, b, dest);
    dispatch_type(t, [&](auto *p) {
        using T = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_compact_rm<T>), dim3(grid_for(n * b)), dim3(256), 0, ctx->stream,
                           (const T *)src, lds, (T *)dst, ldd, n, dest, b);
    });
    OFRR_HIP(hipGetLastError());
}

void colmajor_to_rowmajor(Context *ctx, int64_t n, int32_t b, const double *src, int64_t lds,
                          ofrr_dtype dt, void *dst, int64_t ldd) {
    dispatch_type(dt, [&](auto *p) {
        using D = std::remove_pointer_t<decltype(p)>;
        hipLaunchKernelGGL((k_cm_to_rm<D>), dim3(grid_for(n * b)), dim3(256), 0, ctx->stream, src,
                           lds, n, b, (D *)dst, ldd);
    });
    OFRR_HIP(hipGetLastError());
}

void split_block(Context *ctx, ofrr_dtype t, int64_t count, const float *src, uint16_t *hi,
                 uint16_t *lo) {
    if (t == OFRR_BF16)
        hipLaunchKernelGGL((k_split<true>), dim3(grid_for(count)), dim3(256), 0, ctx->stream, src,
                           count, hi, lo);
    else if (t == OFRR_F16)
        hipLaunchKernelGGL((k_split<false>), dim3(grid_for(count)), dim3(256), 0, ctx->stream, src,
                           count, hi, lo);
    else
        fail(OFRR_ERR_UNSUPPORTED, "split_block: BF16 or F16");
    OFRR_HIP(hipGetLastError());
}

void round_block(Context *ctx, ofrr_dtype t, int64_t count, float *x) {
    if (t == OFRR_F32) return;  // already the storage type
    if (t == OFRR_BF16)
        hipLaunchKernelGGL((k_round<true>), dim3(grid_for(count)), dim3(256), 0, ctx->stream, x, count);
    else if (t == OFRR_F16)
        hipLaunchKernelGGL((k_round<false>), dim3(grid_for(count)), dim3(256), 0, ctx->stream, x, count);
    else
        fail(OFRR_ERR_UNSUPPORTED, "round_block: BF16 or F16");
    OFRR_HIP(hipGetLastError());
}

void promote_block(Context *ctx, int64_t count, void *buf) {
    double *tmp = ctx->buf<double>("promote_tmp", (size_t)count);
    hipLaunchKernelGGL(k_f32_to_f64_copy, dim3(grid_for(count)), dim3(256), 0, ctx->stream,
                       (const float *)buf, tmp, count);
    OFRR_HIP(hipGetLastError());
    OFRR_HIP(hipMemcpyAsync(buf, tmp, (size_t)count * 8, hipMemcpyDeviceToDevice, ctx->stream));
}

}  // namespace ofrr
