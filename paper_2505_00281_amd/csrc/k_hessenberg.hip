// k_hessenberg.hip -- the right-looking Hessenberg process on an n x b block
// (Sec. 4.2, Algorithm "Computing non-orthogonal bases from the Hessenberg
// Process"): for each column j, the first row r of largest magnitude is the
// pivot; if |Y_rj| < tol the column is dropped, otherwise it is divided by
// Y_rj and Y_:i -= Y_ri * Y_:j eliminates row r from every later column i.
// The output equals P^T L of the row-pivoted LU factorisation (Sec. 4.2).
//
// MI355X design.  One cooperative launch; workgroup g owns a contiguous
// slice of rows for the whole sweep (in LDS when the slice fits, otherwise
// in place in HBM/L2).  Per column there is exactly one grid-wide exchange:
//   1. every workgroup publishes its local pivot candidate (value, row) and
//      a copy of that candidate row's trailing entries into a double-
//      buffered slot, then raises the slot's sequence flag to j+1;
//   2. every workgroup waits for all G flags (one thread per flag, polled in
//      parallel: the barrier and the candidate exchange are one round trip,
//      with no contended atomic counter);
//   3. every workgroup picks the global winner (largest magnitude, smallest
//      row on ties -- the same rule in every workgroup, so no broadcast is
//      needed), reads the winner's published row as the multipliers, and
//      runs the elimination over its rows.  That pass also produces the
//      local candidate of column j+1, so the pivot search never needs a
//      pass of its own.
// The slot copy is what makes one barrier enough: the pivot row's owner may
// already be overwriting that row while others still need its old values.
// Each update is one fused multiply-add, as in the reference process.
#include <cstdlib>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

struct Cand {
    float mag;  // magnitude used for the comparison (the element type's |.|)
    int idx;
};

template <class T>
__device__ __forceinline__ float mag_of(T v) {
    return (float)fabs((double)v);
}

// (mag, idx) comparison: larger magnitude wins, smaller row on ties; NaN
// magnitudes never win.
__device__ __forceinline__ bool better(float m1, int i1, float m2, int i2) {
    if (m1 > m2) return true;
    if (m1 == m2 && i1 < i2) return true;
    return false;
}

// For T = double the magnitudes are compared in FP64: keep a double copy.
template <class T>
struct MagT {
    using type = float;
};
template <>
struct MagT<double> {
    using type = double;
};

template <class M>
__device__ __forceinline__ void wave_argmax(M &m, int &i) {
    for (int o = 32; o > 0; o >>= 1) {
        M m2 = __shfl_xor(m, o, 64);
        int i2 = __shfl_xor(i, o, 64);
        if (m2 > m || (m2 == m && i2 < i)) {
            m = m2;
            i = i2;
        }
    }
}

template <class T, bool RESIDENT>
__global__ __launch_bounds__(256) void k_hessenberg(T *__restrict__ Y, int64_t ldy, int64_t n,
                                                    int b, double tol, int32_t *__restrict__ piv,
                                                    int32_t *__restrict__ keep, int64_t rows_per,
                                                    T *__restrict__ slot_rows,
                                                    typename MagT<T>::type *__restrict__ slot_mag,
                                                    int32_t *__restrict__ slot_idx,
                                                    int32_t *__restrict__ slot_seq,
                                                    int *__restrict__ err,
                                                    int32_t *__restrict__ kept_out) {
    using M = typename MagT<T>::type;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ T w_sh[512];  // multipliers of the current column (b <= 512)
    __shared__ M red_m[4];
    __shared__ int red_i[4];
    __shared__ int s_win_idx, s_win_g;
    __shared__ M s_win_mag;

    const int G = gridDim.x, g = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t r0 = (int64_t)g * rows_per;
    const int64_t r1 = (r0 + rows_per < n) ? r0 + rows_per : n;
    const int64_t nrows = r1 > r0 ? r1 - r0 : 0;
    const int ldl = b;  // leading dimension of the LDS copy
    T *rows = RESIDENT ? reinterpret_cast<T *>(smem_raw) : Y + r0 * ldy;
    const int64_t ldr = RESIDENT ? ldl : ldy;

    if (RESIDENT) {
        for (int64_t e = t; e < nrows * b; e += 256) {
            const int64_t rr = e / b, c = e - rr * b;
            rows[rr * ldl + c] = Y[(r0 + rr) * ldy + c];
        }
        __syncthreads();
    }

    // local candidate of column 0
    auto local_argmax = [&](int col, M &bm, int &bi) {
        bm = (M)-1;
        bi = 0x7fffffff;
        for (int64_t rr = t; rr < nrows; rr += 256) {
            const M v = (M)fabs((double)rows[rr * ldr + col]);
            if (v > bm) {  // rows visited in increasing order per thread
                bm = v;
                bi = (int)(r0 + rr);
            }
        }
    };
    auto block_argmax = [&](M &bm, int &bi) {
        wave_argmax(bm, bi);
        if (lane == 0) {
            red_m[wave] = bm;
            red_i[wave] = bi;
        }
        __syncthreads();
        bm = red_m[0];
        bi = red_i[0];
        for (int w = 1; w < 4; ++w)
            if (red_m[w] > bm || (red_m[w] == bm && red_i[w] < bi)) {
                bm = red_m[w];
                bi = red_i[w];
            }
        __syncthreads();
    };

    M cm;
    int ci;
    local_argmax(0, cm, ci);
    block_argmax(cm, ci);

    int kept = 0;
    for (int j = 0; j < b; ++j) {
        const int buf = j & 1;
        // 1. publish the local candidate and a copy of its row (columns j..b-1)
        T *my_slot = slot_rows + ((int64_t)buf * G + g) * b;
        if (ci != 0x7fffffff) {
            const int64_t rr = ci - r0;
            for (int c = j + t; c < b; c += 256)
                __hip_atomic_store(my_slot + c, rows[rr * ldr + c], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (t == 0) {
            __hip_atomic_store(slot_mag + buf * G + g, cm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(slot_idx + buf * G + g, ci, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        __syncthreads();
        // 2. the slot's sequence flag (column j+1) is the only grid-wide signal:
        // readers poll every workgroup's flag in parallel (one thread each), so
        // the barrier and the candidate exchange are one round trip and there
        // is no contended counter
        if (t == 0)
            __hip_atomic_store(slot_seq + buf * G + g, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // 3. global winner, same rule everywhere
        {
            M bm = (M)-1;
            int bi = 0x7fffffff, bg = -1;
            int ok = 1;
            for (int h = t; h < G; h += 256) {
                unsigned long long spins = 0;
                while (__hip_atomic_load(slot_seq + buf * G + h, __ATOMIC_ACQUIRE,
                                         __HIP_MEMORY_SCOPE_AGENT) < j + 1) {
                    if (++spins > (1ull << 24) ||
                        __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (!ok) break;
                const M m2 = __hip_atomic_load(slot_mag + buf * G + h, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                const int i2 = __hip_atomic_load(slot_idx + buf * G + h, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                if (m2 > bm || (m2 == bm && i2 < bi)) {
                    bm = m2;
                    bi = i2;
                    bg = h;
                }
            }
            if (!__syncthreads_and(ok)) break;
            // reduce (bm, bi) and carry the owning workgroup along with the row
            for (int o = 32; o > 0; o >>= 1) {
                M m2 = __shfl_xor(bm, o, 64);
                int i2 = __shfl_xor(bi, o, 64);
                int g2 = __shfl_xor(bg, o, 64);
                if (m2 > bm || (m2 == bm && i2 < bi)) {
                    bm = m2;
                    bi = i2;
                    bg = g2;
                }
            }
            __shared__ int red_g[4];
            if (lane == 0) {
                red_m[wave] = bm;
                red_i[wave] = bi;
                red_g[wave] = bg;
            }
            __syncthreads();
            if (t == 0) {
                M m = red_m[0];
                int i = red_i[0], gg = red_g[0];
                for (int w = 1; w < 4; ++w)
                    if (red_m[w] > m || (red_m[w] == m && red_i[w] < i)) {
                        m = red_m[w];
                        i = red_i[w];
                        gg = red_g[w];
                    }
                s_win_mag = m;
                s_win_idx = i;
                s_win_g = gg;
            }
            __syncthreads();
        }
        const M wmag = s_win_mag;
        const int wrow = s_win_idx, wg = s_win_g;
        const bool take = (wmag >= (M)tol) && (wmag > (M)0) && wg >= 0;
        if (g == 0 && t == 0) {
            piv[j] = take ? wrow : -1;
            keep[j] = take ? 1 : 0;
        }
        if (!take) {
            // dropped: nothing changes; the next candidate is a plain search
            if (j + 1 < b) {
                local_argmax(j + 1, cm, ci);
                block_argmax(cm, ci);
            }
            continue;
        }
        ++kept;
        // multipliers: the winner's published row (columns j..b-1)
        const T *win_slot = slot_rows + ((int64_t)buf * G + wg) * b;
        for (int c = j + t; c < b; c += 256)
            w_sh[c] = __hip_atomic_load(win_slot + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const T pivot = w_sh[j];
        // elimination over own rows, one wavefront per row, lanes over columns;
        // lane 0..63 also track the next column's candidate
        M nm = (M)-1;
        int ni = 0x7fffffff;
        for (int64_t rr = wave; rr < nrows; rr += 4) {
            T *row = rows + rr * ldr;
            const T q = row[j] / pivot;
            for (int c = j + 1 + lane; c < b; c += 64) {
                const T y = fma(-w_sh[c], q, row[c]);
                row[c] = y;
                if (c == j + 1) {
                    const M v = (M)fabs((double)y);
                    if (v > nm) {
                        nm = v;
                        ni = (int)(r0 + rr);
                    }
                }
            }
            if (lane == 0) row[j] = q;
        }
        // the candidate sits in lane 0 of each wave (column j+1 is handled by
        // lane 0 since c = j+1 is the first column of the lane loop)
        if (j + 1 < b) {
            cm = nm;
            ci = ni;
            if (lane != 0) {
                cm = (M)-1;
                ci = 0x7fffffff;
            }
            __syncthreads();
            block_argmax(cm, ci);
        }
        __syncthreads();
    }

    if (RESIDENT) {
        __syncthreads();
        for (int64_t e = t; e < nrows * b; e += 256) {
            const int64_t rr = e / b, c = e - rr * b;
            Y[(r0 + rr) * ldy + c] = rows[rr * ldl + c];
        }
    }
    if (g == 0 && t == 0 && kept_out) *kept_out = kept;
}

// clears the error flag, the kept count and the 2*G sequence flags (a
// kernel, not a memset, so the sweep can be captured in a graph)
__global__ void k_hess_reset(int *flags, int nflags) {
    for (int i = threadIdx.x; i < nflags; i += blockDim.x) flags[i] = 0;
}

template <class T>
int32_t run(Context *ctx, int64_t n, int32_t b, T *Y, int64_t ldy, double tol, int32_t *piv,
            int32_t *keep, bool want_count) {
    OFRR_CHECK_ARG(b >= 1 && b <= 512, "hessenberg: 1 <= b <= 512");
    OFRR_CHECK_ARG(n >= 1 && n < (int64_t)0x7fffffff, "hessenberg: 1 <= n < 2^31");
    OFRR_CHECK_ARG(ldy >= b, "hessenberg: ld >= b");
    using M = typename MagT<T>::type;
    // rows per workgroup: LDS-resident when the slice fits in 64 KiB
    // LDS per workgroup for its row slice (OFRR_HESS_LDS_KB overrides, for
    // tuning sweeps): a bigger slice means fewer workgroups meeting at each
    // per-column grid barrier
    size_t lds_budget = 64 * 1024;
    if (const char *s = std::getenv("OFRR_HESS_LDS_KB")) {
        const long kb = std::strtol(s, nullptr, 10);
        if (kb >= 8 && kb <= 150) lds_budget = (size_t)kb * 1024;
    }
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    int64_t rows_res = (int64_t)(lds_budget / ((size_t)b * sizeof(T)));
    bool resident = false;
    int64_t rows_per;
    int G;
    if (rows_res >= 16 && (n + rows_res - 1) / rows_res <= cus) {
        resident = true;
        // as many rows per workgroup as fit: the sweep is barrier-bound, and
        // fewer participants make each grid barrier cheaper
        rows_per = std::min<int64_t>(rows_res, n);
        G = (int)((n + rows_per - 1) / rows_per);
    } else {
        int64_t want_g = std::min<int64_t>(cus, (n + 255) / 256);
        if (want_g < 1) want_g = 1;
        rows_per = (n + want_g - 1) / want_g;
        G = (int)((n + rows_per - 1) / rows_per);
    }
    const size_t shmem = resident ? (size_t)rows_per * b * sizeof(T) : 0;

    T *slot_rows = ctx->buf<T>("hess_slot_rows", (size_t)2 * G * b);
    M *slot_mag = ctx->buf<M>("hess_slot_mag", (size_t)2 * G);
    int32_t *slot_idx = ctx->buf<int32_t>("hess_slot_idx", (size_t)2 * G);
    // flags: [0] error, [1] kept count, [2..2+2G) per-slot sequence numbers
    int *flags = ctx->buf<int>("hess_flags", 2 + (size_t)2 * G);
    int *err = flags;
    int32_t *kept_d = flags + 1;
    int32_t *slot_seq = flags + 2;
    hipLaunchKernelGGL(k_hess_reset, dim3(1), dim3(256), 0, ctx->stream, flags, 2 + 2 * G);
    OFRR_HIP(hipGetLastError());

    auto kern = resident ? (void *)k_hessenberg<T, true> : (void *)k_hessenberg<T, false>;
    if (shmem > 0) OFRR_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    int per_cu = 0;
    OFRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, shmem));
    if ((int64_t)per_cu * cus < G)
        fail(OFRR_ERR_UNSUPPORTED, "hessenberg: grid cannot be co-resident");
    void *args[] = {&Y, &ldy, &n, &b, &tol, &piv, &keep, &rows_per, &slot_rows, &slot_mag,
                    &slot_idx, &slot_seq, &err, &kept_d};
    {
        KTimer tm(ctx, "hessenberg");
        OFRR_HIP(hipLaunchCooperativeKernel(kern, dim3(G), dim3(256), args, (unsigned)shmem, ctx->stream));
    }
    int32_t host[2] = {0, 0};
    OFRR_HIP(hipMemcpyAsync(host, err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    if (host[0] != 0) fail(OFRR_ERR_HIP, "hessenberg: wait for the column candidates timed out");
    (void)want_count;
    return host[1];
}

}  // namespace

int32_t hessenberg(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                   double tol, int32_t *piv, int32_t *keep, bool want_count) {
    if (t == OFRR_F64) return run<double>(ctx, n, b, (double *)Y, ldy, tol, piv, keep, want_count);
    if (t == OFRR_F32) return run<float>(ctx, n, b, (float *)Y, ldy, tol, piv, keep, want_count);
    fail(OFRR_ERR_UNSUPPORTED, "hessenberg: element type must be F64 or F32");
}

}  // namespace ofrr
