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
//      buffered slot;
//   2. every workgroup reads all G candidates (one thread per workgroup,
//      in parallel), picks the global winner (largest magnitude, smallest
//      row on ties -- the same rule everywhere, so no broadcast is needed),
//      reads the winner's published row as the multipliers, and runs the
//      elimination over its rows.  That pass also produces the local
//      candidate of column j+1, so the pivot search never needs a pass of
//      its own.
// The exchange uses no fences and no flags: every published 32-bit word is
// stored together with the column's sequence number as one 64-bit relaxed
// device-scope atomic, and a reader polls each word it needs until the tag
// matches.  A 64-bit atomic is single-copy atomic, so a matching tag proves
// the payload beside it is the current one; cache write-backs and
// invalidations (what release/acquire ordering costs across the XCDs) are
// never needed.  The slot copy is what makes one exchange per column
// enough: the pivot row's owner may already be overwriting that row while
// others still read its old values.  The slots are cleared (tag 0) before
// the sweep; column j uses tag j + 1.
// Each update is one fused multiply-add, as in the reference process.
#include <cstdlib>
#include <map>
#include <tuple>
#include <utility>
#include <type_traits>

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

// Cross-lane moves through the DPP lane patterns (all lanes active).
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_val(float v) {
    return __builtin_bit_cast(float, dpp_i32<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_val(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)dpp_i32<CTRL>((int)(uint32_t)u), hi = (uint32_t)dpp_i32<CTRL>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float lane_val(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_val(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One exchange step of the (magnitude, row, tag) maximum: larger magnitude,
// then smaller row.  The lane patterns pair lanes symmetrically, so both
// lanes of a pair keep the same winner.
template <int CTRL, class M>
__device__ __forceinline__ void argmax_step(M &m, int &i, int &g) {
    const M m2 = dpp_val<CTRL>(m);
    const int i2 = dpp_i32<CTRL>(i), g2 = dpp_i32<CTRL>(g);
    if (m2 > m || (m2 == m && i2 < i)) {
        m = m2;
        i = i2;
        g = g2;
    }
}
// Wave maximum: within each row of 16 lanes (swap neighbours, swap pairs,
// mirror each 8, mirror the 16), then the four row winners in a fixed order.
// Magnitudes are never NaN here (the local searches skip NaN).
template <class M>
__device__ __forceinline__ void wave_argmax(M &m, int &i, int &g) {
    argmax_step<0xB1>(m, i, g);
    argmax_step<0x4E>(m, i, g);
    argmax_step<0x141>(m, i, g);
    argmax_step<0x140>(m, i, g);
    M bm = lane_val(m, 0);
    int bi = __builtin_amdgcn_readlane(i, 0), bg = __builtin_amdgcn_readlane(g, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16) {
        const M m2 = lane_val(m, r);
        const int i2 = __builtin_amdgcn_readlane(i, r), g2 = __builtin_amdgcn_readlane(g, r);
        if (m2 > bm || (m2 == bm && i2 < bi)) {
            bm = m2;
            bi = i2;
            bg = g2;
        }
    }
    m = bm;
    i = bi;
    g = bg;
}

// Tagged words: payload in the high 32 bits, sequence tag in the low 32.
__device__ __forceinline__ void put_word(uint64_t *dst, uint32_t w, uint32_t tag) {
    __hip_atomic_store(dst, ((uint64_t)w << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Loads N consecutive tagged words, all in flight at once, until every tag
// is `tag`; false after the spin budget or once another workgroup has
// raised the error flag.
template <int N>
__device__ __forceinline__ bool get_words(const uint64_t *src, uint32_t tag, uint32_t (&w)[N], int *err) {
    unsigned long long spins = 0;
    for (;;) {
        uint64_t v[N];
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = __hip_atomic_load(src + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool ok = true;
#pragma unroll
        for (int q = 0; q < N; ++q) ok = ok && ((uint32_t)v[q] == tag);
        if (ok) {
#pragma unroll
            for (int q = 0; q < N; ++q) w[q] = (uint32_t)(v[q] >> 32);
            return true;
        }
        if (++spins > (1ull << 22) ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Polls N tagged words at independent addresses, all loads in flight at
// once, until every word with use[q] set carries `tag`; false after the
// spin budget or once another workgroup has raised the error flag.
template <int N>
__device__ __forceinline__ bool get_words_at(const uint64_t *const (&src)[N], const bool (&use)[N], uint32_t tag,
                                             uint32_t (&w)[N], int *err) {
    unsigned long long spins = 0;
    for (;;) {
        uint64_t v[N];
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = __hip_atomic_load(src[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool ok = true;
#pragma unroll
        for (int q = 0; q < N; ++q) ok = ok && (!use[q] || (uint32_t)v[q] == tag);
        if (ok) {
#pragma unroll
            for (int q = 0; q < N; ++q) w[q] = (uint32_t)(v[q] >> 32);
            return true;
        }
        if (++spins > (1ull << 22) ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// 32-bit words of a value
template <class V>
struct NWords {
    static constexpr int value = sizeof(V) / 4;
};
template <class V>
__device__ __forceinline__ void put_value(uint64_t *dst, V v, uint32_t tag) {
    uint32_t w[NWords<V>::value];
    __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
    for (int q = 0; q < NWords<V>::value; ++q) put_word(dst + q, w[q], tag);
}
template <class V>
__device__ __forceinline__ bool get_value(const uint64_t *src, uint32_t tag, V &v, int *err) {
    uint32_t w[NWords<V>::value];
    const bool ok = get_words<NWords<V>::value>(src, tag, w, err);
    __builtin_memcpy(&v, w, sizeof(V));
    return ok;
}

template <class T, bool RESIDENT, int NT>
__global__ __launch_bounds__(NT) void k_hessenberg(T *__restrict__ Y, int64_t ldy, int64_t n,
                                                    int b, double tol, int32_t *__restrict__ piv,
                                                    int32_t *__restrict__ keep, int64_t rows_per,
                                                    uint64_t *__restrict__ slot_rows,
                                                    uint64_t *__restrict__ slot_cand,
                                                    int *__restrict__ err,
                                                    int32_t *__restrict__ kept_out) {
    using M = typename MagT<T>::type;
    constexpr int TW = NWords<T>::value;      // words per row entry
    constexpr int CW = NWords<M>::value + 1;  // words per candidate (magnitude, row)
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ __attribute__((aligned(16))) T w_sh[512];  // multipliers of the current column (b <= 512)
    constexpr int NW = NT / 64;
    __shared__ M red_m[NW];
    __shared__ int red_i[NW], red_g[NW];
    __shared__ int s_win_idx, s_win_g;
    __shared__ M s_win_mag;

    const int G = gridDim.x, g = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t r0 = (int64_t)g * rows_per;
    const int64_t r1 = (r0 + rows_per < n) ? r0 + rows_per : n;
    const int64_t nrows = r1 > r0 ? r1 - r0 : 0;
    // element (rr, c) of the slice: row-major in both cases; in LDS each row
    // is padded to a whole number of 16-byte chunks plus one more, so that a
    // thread-per-row pass reading 16 bytes per lane touches every bank once
    // per eight lanes (row stride = 4 banks modulo 32)
    constexpr int VEC = 16 / (int)sizeof(T);
    const int ldr = RESIDENT ? ((b + VEC - 1) / VEC + 1) * VEC : 0;
    T *rows = RESIDENT ? reinterpret_cast<T *>(smem_raw) : Y + r0 * ldy;
    auto at = [&](int64_t rr, int c) -> T & { return RESIDENT ? rows[rr * ldr + c] : rows[rr * ldy + c]; };

    if (RESIDENT) {
        for (int64_t e = t; e < nrows * b; e += NT) {
            const int64_t rr = e / b, c = e - rr * b;
            rows[rr * ldr + c] = Y[(r0 + rr) * ldy + c];
        }
    }
    // multipliers beyond column b stay zero (the vector pass below runs over
    // whole chunks)
    for (int c = b + t; c < 512; c += NT) w_sh[c] = (T)0;
    __syncthreads();
    // elimination mapping: tpr threads per row (so that all NT threads work
    // when the slice has fewer than NT rows), each taking every tpr-th
    // trailing column
    int tpr = 1;
    while (tpr < 16 && nrows * tpr * 2 <= NT) tpr *= 2;
    const int sub = t % tpr, rstep = NT / tpr;
    const bool one_row = nrows <= rstep;

    auto local_argmax = [&](int col, M &bm, int &bi) {
        bm = (M)-1;
        bi = 0x7fffffff;
        for (int64_t rr = t; rr < nrows; rr += NT) {
            const M v = (M)fabs((double)at(rr, col));
            if (v > bm) {  // rows visited in increasing order per thread
                bm = v;
                bi = (int)(r0 + rr);
            }
        }
    };
    auto block_argmax = [&](M &bm, int &bi) {
        int unused = 0;
        wave_argmax(bm, bi, unused);
        if (lane == 0) {
            red_m[wave] = bm;
            red_i[wave] = bi;
        }
        __syncthreads();
        bm = red_m[0];
        bi = red_i[0];
        for (int w = 1; w < NW; ++w)
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

    // publish the candidate of column jj (its row's entries jj..b-1 must be
    // final for the columns before jj); every thread must see the same (cm, ci)
    auto publish = [&](int jj) {
        const int bufp = jj & 1;
        const uint32_t tagp = (uint32_t)jj + 1u;
        uint64_t *my_row = slot_rows + ((int64_t)bufp * G + g) * b * TW;
        if (ci != 0x7fffffff) {
            const int64_t rr = ci - r0;
            for (int c = jj + t; c < b; c += NT) put_value<T>(my_row + (int64_t)c * TW, at(rr, c), tagp);
        }
        if (t == 0) {
            uint64_t *my_cand = slot_cand + ((int64_t)bufp * G + g) * CW;
            put_value<M>(my_cand, cm, tagp);
            put_word(my_cand + CW - 1, (uint32_t)ci, tagp);
        }
    };
    publish(0);

    // Look-ahead: once column j's multipliers are known, column j+1 and the
    // next candidate row are finished first and the candidate of column j+1
    // is published; the rest of the slice is eliminated while the other
    // workgroups' candidates are in flight.
    int kept = 0;
    for (int j = 0; j < b; ++j) {
        const int buf = j & 1;
        const uint32_t tag = (uint32_t)j + 1u;
        // 1. every candidate of column j (CPL per thread and round, all
        // words of a round polled at once)
        {
            constexpr int CPL = (256 + NT - 1) / NT;
            M bm = (M)-1;
            int bi = 0x7fffffff, bg = -1;
            bool ok = true;
            for (int h0 = 0; h0 < G; h0 += CPL * NT) {
                const uint64_t *src[CPL * CW];
                bool use[CPL * CW];
                uint32_t cw[CPL * CW];
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int h = h0 + t + q * NT;
                    const bool u = h < G;
                    const uint64_t *base = slot_cand + ((int64_t)buf * G + (u ? h : 0)) * CW;
#pragma unroll
                    for (int w = 0; w < CW; ++w) {
                        src[q * CW + w] = base + w;
                        use[q * CW + w] = u;
                    }
                }
                if (!get_words_at<CPL * CW>(src, use, tag, cw, err)) {
                    ok = false;
                    break;
                }
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    M m2;
                    __builtin_memcpy(&m2, &cw[q * CW], sizeof(M));
                    const int i2 = (int)cw[q * CW + CW - 1];
                    if (use[q * CW] && (m2 > bm || (m2 == bm && i2 < bi))) {
                        bm = m2;
                        bi = i2;
                        bg = h0 + t + q * NT;
                    }
                }
            }
            if (!__syncthreads_and(ok)) break;
            wave_argmax(bm, bi, bg);
            if (lane == 0) {
                red_m[wave] = bm;
                red_i[wave] = bi;
                red_g[wave] = bg;
            }
            __syncthreads();
            if (t == 0) {
                M m = red_m[0];
                int i = red_i[0], gg = red_g[0];
                for (int w = 1; w < NW; ++w)
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
                publish(j + 1);
            }
            continue;
        }
        ++kept;
        // 2. multipliers: the winner's published row (columns j..b-1, all of
        // a thread's words polled at once; b <= 512)
        {
            constexpr int CPR = (512 + NT - 1) / NT;
            const uint64_t *win_row = slot_rows + ((int64_t)buf * G + wg) * b * TW;
            const uint64_t *src[CPR * TW];
            bool use[CPR * TW];
            uint32_t rw[CPR * TW];
#pragma unroll
            for (int q = 0; q < CPR; ++q) {
                const int c = j + t + q * NT;
                const bool u = c < b;
#pragma unroll
                for (int w = 0; w < TW; ++w) {
                    src[q * TW + w] = win_row + (int64_t)(u ? c : j) * TW + w;
                    use[q * TW + w] = u;
                }
            }
            const bool ok = get_words_at<CPR * TW>(src, use, tag, rw, err);
#pragma unroll
            for (int q = 0; q < CPR; ++q)
                if (use[q * TW]) __builtin_memcpy(&w_sh[j + t + q * NT], &rw[q * TW], sizeof(T));
            if (!__syncthreads_and(ok)) break;
        }
        const T pivot = w_sh[j];
        // with at most one row per thread, that row's multiplier once per
        // column (the same IEEE quotient everywhere it is used)
        const T qm = (one_row && t / tpr < nrows) ? at(t / tpr, j) / pivot : (T)0;
        if (j + 1 < b) {
            // 3. column j+1 of every row (one fused multiply-add each) and the
            // local candidate of column j+1
            M nm = (M)-1;
            int ni = 0x7fffffff;
            if (sub == 0)
                for (int64_t rr = t / tpr; rr < nrows; rr += rstep) {
                    const T q = one_row ? qm : at(rr, j) / pivot;
                    const T y = fma(-w_sh[j + 1], q, at(rr, j + 1));
                    at(rr, j + 1) = y;
                    const M v = (M)fabs((double)y);
                    if (v > nm) {  // rows visited in increasing order per thread
                        nm = v;
                        ni = (int)(r0 + rr);
                    }
                }
            cm = nm;
            ci = ni;
            __syncthreads();
            block_argmax(cm, ci);
            // 4. finish the candidate row (columns j+2..b-1), then publish it
            if (ci != 0x7fffffff) {
                const int64_t rr = ci - r0;
                const T q = at(rr, j) / pivot;
                for (int c = j + 2 + t; c < b; c += NT) at(rr, c) = fma(-w_sh[c], q, at(rr, c));
            }
            __syncthreads();
            publish(j + 1);
        }
        // 5. the rest: columns j+2..b-1 of every other row, then the
        // multipliers into column j
        for (int64_t rr = t / tpr; rr < nrows; rr += rstep) {
            const T q = one_row ? qm : at(rr, j) / pivot;
            if (RESIDENT && r0 + rr != ci) {
                // scalar head up to a chunk boundary, then 16-byte chunks
                // (chunk u of the row to sub-thread u % tpr)
                const int ca = (j + 2 + VEC - 1) / VEC * VEC;
                if (sub == 0)
                    for (int c = j + 2; c < ca && c < b; ++c) at(rr, c) = fma(-w_sh[c], q, at(rr, c));
                typedef T vec_t __attribute__((ext_vector_type(VEC)));
                T *row = &at(rr, 0);
                int c = ca + sub * VEC;
                for (; c + 3 * tpr * VEC < b; c += 4 * tpr * VEC) {
                    vec_t y[4], w[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        y[u] = *reinterpret_cast<const vec_t *>(row + c + u * tpr * VEC);
                        w[u] = *reinterpret_cast<const vec_t *>(w_sh + c + u * tpr * VEC);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int e = 0; e < VEC; ++e) y[u][e] = fma(-w[u][e], q, y[u][e]);
#pragma unroll
                    for (int u = 0; u < 4; ++u) *reinterpret_cast<vec_t *>(row + c + u * tpr * VEC) = y[u];
                }
                for (; c < b; c += tpr * VEC) {
                    vec_t y = *reinterpret_cast<const vec_t *>(row + c);
                    const vec_t w = *reinterpret_cast<const vec_t *>(w_sh + c);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) y[e] = fma(-w[e], q, y[e]);
                    *reinterpret_cast<vec_t *>(row + c) = y;
                }
            } else if (r0 + rr != ci) {
                int c = j + 2 + sub;
                for (; c + 7 * tpr < b; c += 8 * tpr) {
                    T y[8], w[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        y[u] = at(rr, c + u * tpr);
                        w[u] = w_sh[c + u * tpr];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) y[u] = fma(-w[u], q, y[u]);
#pragma unroll
                    for (int u = 0; u < 8; ++u) at(rr, c + u * tpr) = y[u];
                }
                for (; c < b; c += tpr) at(rr, c) = fma(-w_sh[c], q, at(rr, c));
            }
        }
        __syncthreads();
        if (sub == 0)
            for (int64_t rr = t / tpr; rr < nrows; rr += rstep) at(rr, j) = one_row ? qm : at(rr, j) / pivot;
        __syncthreads();
    }

    if (RESIDENT) {
        __syncthreads();
        for (int64_t e = t; e < nrows * b; e += NT) {
            const int64_t rr = e / b, c = e - rr * b;
            Y[(r0 + rr) * ldy + c] = rows[rr * ldr + c];
        }
    }
    if (g == 0 && t == 0 && kept_out) *kept_out = kept;
}

// ---------------------------------------------------------------------------
// Register-resident sweep for blocks of at most 128 columns (FP32, and FP64
// with one-wave workgroups): each of the NT threads (64, 128 or 256) holds
// one whole row of its workgroup's slice in registers, so the eliminations are register fused multiply-adds on
// multipliers read from LDS, and only the pivot-candidate row passes through
// LDS (to be published).  The column loop runs as eight sweeps of sixteen
// columns with the sweep index a template parameter: the registers of the
// finished columns are left alone and every register index is static (a
// column picked by the loop index is read through a select tree).  The
// exchange between workgroups and every arithmetic operation are those of
// k_hessenberg, so the result is bit-identical.
constexpr int HR_B = 128;     // columns held per thread
constexpr int HR_GMAX = 256;  // workgroups (one candidate each per column) at most

// r[base + i] for i in [0, 16): the sixteen values are passed as values and
// picked by a select tree on the bits of i, so the register array is never
// indexed (which would send it to scratch memory)
template <class V>
__device__ __forceinline__ V hr_sel16(V x0, V x1, V x2, V x3, V x4, V x5, V x6, V x7, V x8, V x9, V x10, V x11,
                                      V x12, V x13, V x14, V x15, int i) {
    const bool b0 = (i & 1) != 0, b1 = (i & 2) != 0, b2 = (i & 4) != 0, b3 = (i & 8) != 0;
    const V a0 = b0 ? x1 : x0, a1 = b0 ? x3 : x2, a2 = b0 ? x5 : x4, a3 = b0 ? x7 : x6;
    const V a4 = b0 ? x9 : x8, a5 = b0 ? x11 : x10, a6 = b0 ? x13 : x12, a7 = b0 ? x15 : x14;
    const V c0 = b1 ? a1 : a0, c1 = b1 ? a3 : a2, c2 = b1 ? a5 : a4, c3 = b1 ? a7 : a6;
    const V d0 = b2 ? c1 : c0, d1 = b2 ? c3 : c2;
    return b3 ? d1 : d0;
}
#define hr_pick16(r, base, i)                                                                               \
    hr_sel16((r)[(base) + 0], (r)[(base) + 1], (r)[(base) + 2], (r)[(base) + 3], (r)[(base) + 4],             \
             (r)[(base) + 5], (r)[(base) + 6], (r)[(base) + 7], (r)[(base) + 8], (r)[(base) + 9],             \
             (r)[(base) + 10], (r)[(base) + 11], (r)[(base) + 12], (r)[(base) + 13], (r)[(base) + 14],        \
             (r)[(base) + 15], (i))

template <class T>
struct HRShared {
    using M = typename MagT<T>::type;
    T *w_sh;    // multipliers of the current column (HR_B + 16, zero beyond b)
    T *cand;    // the candidate row being published (HR_B)
    M *red_m;   // per-wave partials
    int *red_i, *red_g;
    int *s_win;  // [0] row, [1] workgroup
    M *s_wmag;
    T *s_qown;  // the candidate row's multiplier of the current column
};

struct HRArgs {
    int b, G, g, t, lane, wave;
    int64_t r0, nrows;
    double tol;
    int32_t *piv, *keep;
    uint64_t *slot_rows, *slot_cand;
    int *err;
};

// every thread's `ok`, at a barrier (one wave: a ballot after the barrier)
template <int NT>
__device__ __forceinline__ bool hr_block_all(bool ok) {
    if constexpr (NT == 64) {
        __syncthreads();
        return __builtin_amdgcn_ballot_w64(!ok) == 0;
    } else {
        return __syncthreads_and(ok) != 0;
    }
}

// block-wide (magnitude, row) maximum; the same winner in every thread
template <int NT, class T>
__device__ __forceinline__ void hr_block_argmax(const HRArgs &a, const HRShared<T> &sh,
                                                typename MagT<T>::type &bm, int &bi) {
    int unused = 0;
    wave_argmax(bm, bi, unused);
    if constexpr (NT == 64) return;
    if (a.lane == 0) {
        sh.red_m[a.wave] = bm;
        sh.red_i[a.wave] = bi;
    }
    __syncthreads();
    bm = sh.red_m[0];
    bi = sh.red_i[0];
    for (int w = 1; w < NT / 64; ++w)
        if (sh.red_m[w] > bm || (sh.red_m[w] == bm && sh.red_i[w] < bi)) {
            bm = sh.red_m[w];
            bi = sh.red_i[w];
        }
    __syncthreads();
}

// publish the candidate (cm, ci) of column jj and its row's entries jj..b-1
// (in sh.cand); all threads.  With `pending` the row in sh.cand still lacks
// the elimination of column jj - 1 in its entries past jj, which is applied
// here (multipliers sh.w_sh, the row's multiplier *sh.s_qown), one fused
// multiply-add per entry exactly as the row update itself does it.
template <int NT, class T>
__device__ __forceinline__ void hr_publish(const HRArgs &a, const HRShared<T> &sh, int jj,
                                           typename MagT<T>::type cm, int ci, bool pending) {
    using M = typename MagT<T>::type;
    constexpr int TW = NWords<T>::value, CW = NWords<M>::value + 1;
    const int bufp = jj & 1;
    const uint32_t tagp = (uint32_t)jj + 1u;
    uint64_t *my_row = a.slot_rows + ((int64_t)bufp * a.G + a.g) * a.b * TW;
    if (ci != 0x7fffffff) {
        const T qo = pending ? *sh.s_qown : (T)0;
        for (int c = jj + a.t; c < a.b; c += NT) {
            T v = sh.cand[c];
            if (pending && c > jj) v = fma(-sh.w_sh[c], qo, v);
            put_value<T>(my_row + (int64_t)c * TW, v, tagp);
        }
    }
    if (a.t == 0) {
        uint64_t *my_cand = a.slot_cand + ((int64_t)bufp * a.G + a.g) * CW;
        put_value<M>(my_cand, cm, tagp);
        put_word(my_cand + CW - 1, (uint32_t)ci, tagp);
    }
}

// local candidate of column c0 + i (my row's value x): magnitude -1 and
// row 0x7fffffff when there is no (finite, non-NaN-compared) candidate
template <class T>
__device__ __forceinline__ void hr_local_cand(const HRArgs &a, T x, typename MagT<T>::type &cm, int &ci) {
    using M = typename MagT<T>::type;
    const M v = (M)fabs(x);
    const bool ok = a.t < a.nrows && v > (M)-1;
    cm = ok ? v : (M)-1;
    ci = ok ? (int)(a.r0 + a.t) : 0x7fffffff;
}

template <class T, int NT, int JV>
__device__ __forceinline__ bool hr_sweep(T (&row)[HR_B], const HRArgs &a, const HRShared<T> &sh,
                                         typename MagT<T>::type &cm, int &ci, int &kept) {
    using M = typename MagT<T>::type;
    constexpr int TW = NWords<T>::value, CW = NWords<M>::value + 1;
    const bool valid = a.t < a.nrows;
    const int myrow = (int)(a.r0 + a.t);
    for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * JV + jj;
        if (j >= a.b) return true;
        const int buf = j & 1;
        const uint32_t tag = (uint32_t)j + 1u;
        // 1. every candidate of column j (CPL per thread, all polled at once)
        M wmag;
        int wrow, wg;
        {
            constexpr int CPL = (HR_GMAX + NT - 1) / NT;
            const uint64_t *src[CW * CPL];
            bool use[CW * CPL];
            uint32_t cw[CW * CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int h = a.t + q * NT;
                const bool u = h < a.G;
                const uint64_t *base = a.slot_cand + ((int64_t)buf * a.G + (u ? h : 0)) * CW;
#pragma unroll
                for (int w = 0; w < CW; ++w) {
                    src[CW * q + w] = base + w;
                    use[CW * q + w] = u;
                }
            }
            const bool ok = get_words_at<CW * CPL>(src, use, tag, cw, a.err);
            if (!hr_block_all<NT>(ok)) return false;
            M bm = (M)-1;
            int bi = 0x7fffffff, bg = -1;
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                M m2;
                __builtin_memcpy(&m2, &cw[CW * q], sizeof(M));
                const int i2 = (int)cw[CW * q + CW - 1];
                if (use[CW * q] && (m2 > bm || (m2 == bm && i2 < bi))) {
                    bm = m2;
                    bi = i2;
                    bg = a.t + q * NT;
                }
            }
            wave_argmax(bm, bi, bg);
            if constexpr (NT == 64) {
                wmag = bm;
                wrow = bi;
                wg = bg;
            } else {
                if (a.lane == 0) {
                    sh.red_m[a.wave] = bm;
                    sh.red_i[a.wave] = bi;
                    sh.red_g[a.wave] = bg;
                }
                __syncthreads();
                if (a.t == 0) {
                    M m = sh.red_m[0];
                    int i = sh.red_i[0], gg = sh.red_g[0];
                    for (int w = 1; w < NT / 64; ++w)
                        if (sh.red_m[w] > m || (sh.red_m[w] == m && sh.red_i[w] < i)) {
                            m = sh.red_m[w];
                            i = sh.red_i[w];
                            gg = sh.red_g[w];
                        }
                    *sh.s_wmag = m;
                    sh.s_win[0] = i;
                    sh.s_win[1] = gg;
                }
                __syncthreads();
                wmag = *sh.s_wmag;
                wrow = sh.s_win[0];
                wg = sh.s_win[1];
            }
        }
        const bool take = (wmag >= (M)a.tol) && (wmag > (M)0) && wg >= 0;
        if (a.g == 0 && a.t == 0) {
            a.piv[j] = take ? wrow : -1;
            a.keep[j] = take ? 1 : 0;
        }
        // column j + 1 of my row (static index through the select tree)
        auto col_next = [&]() -> T {
            if constexpr (JV < 7) return (jj == 15) ? row[16 * JV + 16] : hr_pick16(row, 16 * JV, (jj + 1) & 15);
            else return hr_pick16(row, 16 * JV, (jj + 1) & 15);
        };
        if (!take) {
            // dropped: nothing changes; the next candidate is a plain search
            if (j + 1 < a.b) {
                hr_local_cand(a, col_next(), cm, ci);
                hr_block_argmax<NT>(a, sh, cm, ci);
                if (valid && myrow == ci) {
#pragma unroll
                    for (int c = 16 * JV; c < HR_B; ++c) sh.cand[c] = row[c];
                }
                __syncthreads();
                hr_publish<NT>(a, sh, j + 1, cm, ci, false);
            }
            continue;
        }
        ++kept;
        // 2. multipliers: the winner's published row (columns j..b-1, all
        // of a thread's words polled at once)
        {
            constexpr int CPR = (HR_B + NT - 1) / NT;
            const uint64_t *win_row = a.slot_rows + ((int64_t)buf * a.G + wg) * a.b * TW;
            const uint64_t *src[CPR * TW];
            bool use[CPR * TW];
            uint32_t rw[CPR * TW];
#pragma unroll
            for (int q = 0; q < CPR; ++q) {
                const int c = j + a.t + q * NT;
                const bool u = c < a.b;
#pragma unroll
                for (int w = 0; w < TW; ++w) {
                    src[TW * q + w] = win_row + (int64_t)(u ? c : j) * TW + w;
                    use[TW * q + w] = u;
                }
            }
            const bool ok = get_words_at<CPR * TW>(src, use, tag, rw, a.err);
#pragma unroll
            for (int q = 0; q < CPR; ++q)
                if (use[TW * q]) __builtin_memcpy(&sh.w_sh[j + a.t + q * NT], &rw[TW * q], sizeof(T));
            if (!hr_block_all<NT>(ok)) return false;
        }
        const T pivot = sh.w_sh[j];
        const T q = valid ? hr_pick16(row, 16 * JV, jj) / pivot : (T)0;
        // columns j + 2 .. b - 1 of a row (the finished columns of this
        // sweep are kept by a select; from column 16 JV + 17 on every column
        // is past j + 1)
        auto eliminate = [&]() {
#pragma unroll
            for (int c = 16 * JV; c < HR_B; ++c) {
                const T r = fma(-sh.w_sh[c], q, row[c]);
                if (c < 16 * JV + 17) row[c] = (c > j + 1) ? r : row[c];
                else row[c] = r;
            }
        };
        if (j + 1 < a.b) {
            // 3. column j+1 of every row and the local candidate of column j+1
            const T y = fma(-sh.w_sh[j + 1], q, col_next());
#pragma unroll
            for (int c = 16 * JV; c < HR_B && c < 16 * JV + 17; ++c) row[c] = (c == j + 1) ? y : row[c];
            hr_local_cand(a, y, cm, ci);
            hr_block_argmax<NT>(a, sh, cm, ci);
            // 4. the candidate row goes out first: its owner stages the row
            // (column j + 1 already updated) and its multiplier, and the
            // publishing threads apply the elimination of column j on the fly
            if (valid && myrow == ci) {
#pragma unroll
                for (int c = 16 * JV; c < HR_B; ++c) sh.cand[c] = row[c];
                *sh.s_qown = q;
            }
            __syncthreads();
            hr_publish<NT>(a, sh, j + 1, cm, ci, true);
        }
        // 5. every row of the slice, then the multiplier into column j
        if (valid) eliminate();
#pragma unroll
        for (int c = 16 * JV; c < 16 * JV + 16; ++c) row[c] = (valid && c == j) ? q : row[c];
        __syncthreads();
    }
    return true;
}

template <class T, int NT>
__global__ __launch_bounds__(NT) void k_hessenberg_reg(T *__restrict__ Y, int64_t ldy, int64_t n, int b,
                                                          double tol, int32_t *__restrict__ piv,
                                                          int32_t *__restrict__ keep,
                                                          uint64_t *__restrict__ slot_rows,
                                                          uint64_t *__restrict__ slot_cand, int *__restrict__ err,
                                                          int32_t *__restrict__ kept_out) {
    using M = typename MagT<T>::type;
    __shared__ __attribute__((aligned(16))) T w_sh[HR_B + 16];
    __shared__ T cand[HR_B];
    __shared__ M red_m[NT / 64];
    __shared__ int red_i[NT / 64], red_g[NT / 64];
    __shared__ int s_win[2];
    __shared__ M s_wmag;
    HRArgs a;
    a.b = b;
    a.G = gridDim.x;
    a.g = blockIdx.x;
    a.t = threadIdx.x;
    a.lane = a.t & 63;
    a.wave = a.t >> 6;
    a.r0 = (int64_t)a.g * NT;
    const int64_t r1 = (a.r0 + NT < n) ? a.r0 + NT : n;
    a.nrows = r1 > a.r0 ? r1 - a.r0 : 0;
    a.tol = tol;
    a.piv = piv;
    a.keep = keep;
    a.slot_rows = slot_rows;
    a.slot_cand = slot_cand;
    a.err = err;
    __shared__ T s_qown;
    HRShared<T> sh{w_sh, cand, red_m, red_i, red_g, s_win, &s_wmag, &s_qown};

    const bool valid = a.t < a.nrows;
    T row[HR_B];
    {
        const T *src = Y + (a.r0 + (valid ? a.t : 0)) * ldy;
#pragma unroll
        for (int c = 0; c < HR_B; ++c) row[c] = (valid && c < b) ? src[c < b ? c : 0] : (T)0;
    }
    for (int c = b + a.t; c < HR_B + 16; c += NT) w_sh[c] = (T)0;
    M cm;
    int ci;
    hr_local_cand(a, row[0], cm, ci);
    hr_block_argmax<NT>(a, sh, cm, ci);
    if (valid && (int)(a.r0 + a.t) == ci) {
#pragma unroll
        for (int c = 0; c < HR_B; ++c) cand[c] = row[c];
    }
    __syncthreads();
    hr_publish<NT>(a, sh, 0, cm, ci, false);

    int kept = 0;
    const bool ok = hr_sweep<T, NT, 0>(row, a, sh, cm, ci, kept) && hr_sweep<T, NT, 1>(row, a, sh, cm, ci, kept) &&
                    hr_sweep<T, NT, 2>(row, a, sh, cm, ci, kept) && hr_sweep<T, NT, 3>(row, a, sh, cm, ci, kept) &&
                    hr_sweep<T, NT, 4>(row, a, sh, cm, ci, kept) && hr_sweep<T, NT, 5>(row, a, sh, cm, ci, kept) &&
                    hr_sweep<T, NT, 6>(row, a, sh, cm, ci, kept) && hr_sweep<T, NT, 7>(row, a, sh, cm, ci, kept);
    (void)ok;
    if (valid) {
        T *dst = Y + (a.r0 + a.t) * ldy;
#pragma unroll
        for (int c = 0; c < HR_B; ++c)
            if (c < b) dst[c] = row[c];
    }
    if (a.g == 0 && a.t == 0 && kept_out) *kept_out = kept;
}

// Exchange words of the allocation-free entry point: one fixed array per
// GPU, held until the process ends.  Host code never names it directly (in
// host code the name is a stand-in, not a device address): the library's
// set-up asks for its address on each device (hess_scratch_address) and
// kernels get that pointer.  Sized for the largest sweep the launchers
// build: 256 workgroups, 512 FP64 columns (1 + 2*256*3 + 2*256*512*2 words).
constexpr int64_t HESS_SCRATCH_WORDS = 526336;
__device__ __align__(256) uint64_t scratch[HESS_SCRATCH_WORDS];

// The sweeps exchange data between all workgroups of the grid, so every
// workgroup must be resident: a cooperative launch guarantees it.
// OFRR_HESS_COOP=0 launches plainly instead, for comparisons (the grid is
// sized to the occupancy either way, and every wait is bounded and ends in
// an error rather than a hang); measured, the plain launch saved nothing on
// the whole call.
inline hipError_t launch_resident(const void *kern, dim3 grid, dim3 block, void **args, size_t shmem,
                                  hipStream_t stream) {
    static const bool coop = [] {
        const char *e = std::getenv("OFRR_HESS_COOP");
        return !(e && std::atoi(e) == 0);
    }();
    return coop ? hipLaunchCooperativeKernel(kern, grid, block, args, (unsigned)shmem, stream)
                : hipLaunchKernel(kern, grid, block, args, shmem, stream);
}

// Waits for the sweep and returns its kept count (a timed-out wait raises).
// The allocation-free path reads into host stack memory and waits with a
// plain stream synchronisation (no pinned staging, no event).
int32_t read_status(Context *ctx, const int *err, bool no_alloc) {
    int32_t local[2] = {0, 0};
    int32_t *host = no_alloc ? local : ctx->host_stage<int32_t>(2);
    OFRR_HIP(hipMemcpyAsync(host, err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    if (no_alloc)
        OFRR_HIP(hipStreamSynchronize(ctx->stream));
    else
        ctx->sync();
    if (host[0] != 0) fail(OFRR_ERR_HIP, "hessenberg: wait for the column candidates timed out");
    return host[1];
}

// Clears the error flag, the kept count and every tagged slot word (a
// kernel, not a memset, so the sweep can be captured in a graph).
__global__ void k_hess_reset(uint64_t *words, int64_t nwords) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x)
        words[i] = 0;
}

// Exchange words: the context's workspace, or (ext != null) a caller-given
// array of ext_cap words that the launch must fit in.
struct WordsBuf {
    uint64_t *ext = nullptr;
    int64_t ext_cap = 0;
    uint64_t *get(Context *ctx, int64_t nwords) const {
        if (!ext) return ctx->buf<uint64_t>("hess_words", (size_t)nwords);
        if (nwords > ext_cap)
            fail(OFRR_ERR_INVALID_ARG, "hessenberg: the sweep needs " + std::to_string(nwords) +
                                           " exchange words, the fixed array holds " + std::to_string(ext_cap));
        return ext;
    }
};

// Occupancy answers (workgroups per CU) cached in fixed tables, so the
// steady state allocates nothing on the host either.
struct OccEntry {
    int dev;
    const void *kern;
    size_t shmem;
    int value;
};
constexpr int OCC_SLOTS = 128;

template <class Q>
int occupancy_cached(OccEntry (&tab)[OCC_SLOTS], int dev, const void *kern, size_t shmem, Q query) {
    for (int i = 0; i < OCC_SLOTS; ++i) {
        if (tab[i].kern == nullptr) {
            tab[i] = OccEntry{dev, kern, shmem, query()};
            return tab[i].value;
        }
        if (tab[i].dev == dev && tab[i].kern == kern && tab[i].shmem == shmem) return tab[i].value;
    }
    return query();  // table full: ask again
}

template <class T, int NT>
int32_t run_reg(Context *ctx, int64_t n, int32_t b, T *Y, int64_t ldy, double tol, int32_t *piv,
                int32_t *keep, const int32_t **status, const WordsBuf &wb) {
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    const int64_t G64 = (n + NT - 1) / NT;
    if (G64 > HR_GMAX) fail(OFRR_ERR_UNSUPPORTED, "hessenberg: too many row slices for the register kernel");
    // same word buffer layout as the LDS kernel: [0] error flag and kept
    // count, candidate slots (2 x G x 2 words), row slots (2 x G x b words)
    const int G = (int)G64;
    constexpr int TW = NWords<T>::value, CW = NWords<typename MagT<T>::type>::value + 1;
    const int64_t ncand = (int64_t)2 * G * CW, nrow = (int64_t)2 * G * b * TW;
    const int64_t nwords = 1 + ncand + nrow;
    uint64_t *words = wb.get(ctx, nwords);
    int *err = reinterpret_cast<int *>(words);
    int32_t *kept_d = err + 1;
    uint64_t *slot_cand = words + 1;
    uint64_t *slot_rows = words + 1 + ncand;
    static OccEntry occ[OCC_SLOTS] = {};
    const int per_cu = occupancy_cached(occ, ctx->device, (const void *)k_hessenberg_reg<T, NT>, 0, [&] {
        int pc = 0;
        OFRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, (const void *)k_hessenberg_reg<T, NT>, NT, 0));
        return pc;
    });
    if (G64 > (int64_t)per_cu * cus) fail(OFRR_ERR_UNSUPPORTED, "hessenberg: grid cannot be co-resident");
    hipLaunchKernelGGL(k_hess_reset, dim3((unsigned)std::min<int64_t>(256, (nwords + 255) / 256)), dim3(256), 0,
                       ctx->stream, words, nwords);
    OFRR_HIP(hipGetLastError());
    void *args[] = {&Y, &ldy, &n, &b, &tol, &piv, &keep, &slot_rows, &slot_cand, &err, &kept_d};
    {
        KTimer tm(ctx, "hessenberg");
        OFRR_HIP(launch_resident((const void *)k_hessenberg_reg<T, NT>, dim3(G), dim3(NT), args, 0, ctx->stream));
    }
    if (status) {
        *status = err;
        return 0;
    }
    return read_status(ctx, err, wb.ext != nullptr);
}

// ---------------------------------------------------------------------------
// Panel form of the sweep for blocks too tall for the row slices to stay in
// LDS or registers across all b columns (rows per CU x b x element size well
// above the CU's storage).  The per-column form then streams every trailing
// column of every row through HBM once per column (n b^2 element reads and
// writes).  Here the columns are taken P at a time:
//   1. the panel's P columns of the workgroup's rows are loaded into
//      registers (R rows per thread) and swept column by column as above:
//      one grid barrier per column, every workgroup publishing its candidate
//      (magnitude, row, value) and that row's panel entries, every workgroup
//      taking the same winner (largest magnitude, first row on ties);
//   2. the multipliers of the trailing columns, U[l][i] = entry i of pivot
//      row l at the time column l is processed, come from the pivot rows'
//      trailing entries at the start of the panel by the small triangular
//      chain over the panel's earlier pivots (each workgroup computes it);
//   3. after one more grid barrier every row's trailing entries receive the
//      panel's eliminations, in column order, one fused multiply-add each:
//      Y[r][i] = fma(-U[l][i], Y[r][l], Y[r][i]).
// Every entry therefore goes through the same operations in the same order
// as in the per-column process (pivots, drops and bits unchanged), and the
// trailing block is read and written once per panel instead of once per
// column: about n b^2 / P element reads and writes.
constexpr int HP_NT = 512;  // threads per workgroup of the panel sweep

// value of lane l of the wave, in every lane (l a compile-time lane)
__device__ __forceinline__ double wave_bcast(double v, int l) {
    return lane_val(v, l);
}
__device__ __forceinline__ float wave_bcast(float v, int l) {
    return lane_val(v, l);
}

// one column of the panel sweep (JJ: the column within the panel, a
// compile-time index so the panel stays in registers).  The exchange is the
// per-column sweeps' tagged words: every workgroup publishes its candidate
// (magnitude, row) and that row's entries (the panel's, then the trailing
// ones as they stand at the start of the panel) beside the column's tag;
// readers poll the words they need.  No fence and no grid barrier: a
// reader waits only for the words of the current column, and the slot
// copy of the pivot row is what the trailing multipliers are built from,
// so its owner may overwrite the row itself later.
template <class T, int R, int P, int JJ>
__device__ __forceinline__ bool hp_column(T (&v)[R][P], int j0, int pw, int b, int64_t r0, int64_t r1, double tol,
                                          const T *__restrict__ Y, int64_t ldy, int32_t *__restrict__ piv,
                                          int32_t *__restrict__ keep, uint64_t *__restrict__ slots, int64_t slot_w,
                                          int *__restrict__ err, int &kept, double *s_cm, int *s_cr, T *s_pan,
                                          T *s_Lp, T *s_Tr, int *s_keep, int *s_flag) {
    using M = typename MagT<T>::type;
    constexpr int NT = HP_NT, NW = NT / 64;
    constexpr int TW = NWords<T>::value, MW = NWords<M>::value, CW = MW + 1;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int G = gridDim.x, g = blockIdx.x;
    const int j = j0 + JJ;
    const uint32_t tag = (uint32_t)j + 1u;
    const int buf = j & 1;
    const int c0 = j0 + pw, ntr = b - c0;
    // local candidate: largest magnitude, first row on ties
    M bm = (M)-1;
    int br = INT32_MAX, bq = -1;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t row = r0 + t + (int64_t)NT * q;
        const M m = (M)(v[q][JJ] < (T)0 ? -v[q][JJ] : v[q][JJ]);
        if (row < r1 && m > bm) {
            bm = m;
            br = (int)row;
            bq = q;
        }
    }
    M cm = bm;
    int cr = br;
    for (int o = 32; o > 0; o >>= 1) {
        const M qm = __shfl_xor(cm, o, 64);
        const int qr = __shfl_xor(cr, o, 64);
        if (qm > cm || (qm == cm && qr < cr)) {
            cm = qm;
            cr = qr;
        }
    }
    if (lane == 0) {
        s_cm[wave] = (double)cm;
        s_cr[wave] = cr;
    }
    if (t == 0) *s_flag = 0;
    __syncthreads();
    M wm = (M)s_cm[0];
    int wr = s_cr[0];
    for (int w = 1; w < NW; ++w)
        if ((M)s_cm[w] > wm || ((M)s_cm[w] == wm && s_cr[w] < wr)) {
            wm = (M)s_cm[w];
            wr = s_cr[w];
        }
    // the candidate row's panel entries staged in LDS by its owner (a select
    // over the compile-time indices keeps the panel in registers)
    if (bq >= 0 && br == wr) {
        T e[P];
#pragma unroll
        for (int ii = 0; ii < P; ++ii) e[ii] = v[0][ii];
#pragma unroll
        for (int q = 1; q < R; ++q)
#pragma unroll
            for (int ii = 0; ii < P; ++ii) e[ii] = q == bq ? v[q][ii] : e[ii];
#pragma unroll
        for (int ii = 0; ii < P; ++ii) s_pan[ii] = e[ii];
    }
    __syncthreads();
    // publish: candidate words, then the row (panel entries, trailing entries)
    uint64_t *my = slots + ((int64_t)buf * G + g) * slot_w;
    if (t == 0) {
        put_value<M>(my, wm, tag);
        put_word(my + MW, (uint32_t)wr, tag);
    }
    if (wm >= (M)0)
        for (int i = t; i < pw + ntr; i += NT) {
            const T x = i < pw ? s_pan[i] : Y[(int64_t)wr * ldy + c0 + (i - pw)];
            put_value<T>(my + CW + (int64_t)i * TW, x, tag);
        }
    // the winner: thread h reads workgroup h's candidate
    M hm = (M)-2;
    int hr = INT32_MAX, hg = 0;
    for (int h = t; h < G; h += NT) {
        uint32_t w[CW];
        if (!get_words<CW>(slots + ((int64_t)buf * G + h) * slot_w, tag, w, err)) {
            *s_flag = 1;
            break;
        }
        M qm;
        __builtin_memcpy(&qm, w, sizeof(M));
        const int qr = (int)w[MW];
        if (qm > hm || (qm == hm && qr < hr)) {
            hm = qm;
            hr = qr;
            hg = h;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const M qm = __shfl_xor(hm, o, 64);
        const int qr = __shfl_xor(hr, o, 64), qg = __shfl_xor(hg, o, 64);
        if (qm > hm || (qm == hm && qr < hr)) {
            hm = qm;
            hr = qr;
            hg = qg;
        }
    }
    __syncthreads();
    if (lane == 0) {
        s_cm[wave] = (double)hm;
        s_cr[wave] = hr;
        s_cr[NW + wave] = hg;
    }
    __syncthreads();
    if (*s_flag) return false;
    M xm = (M)s_cm[0];
    int xr = s_cr[0], xg = s_cr[NW];
    for (int w = 1; w < NW; ++w)
        if ((M)s_cm[w] > xm || ((M)s_cm[w] == xm && s_cr[w] < xr)) {
            xm = (M)s_cm[w];
            xr = s_cr[w];
            xg = s_cr[NW + w];
        }
    const bool take = (double)xm >= tol && xm > (M)0;
    // the pivot row: panel entries and trailing entries at the panel start
    if (take) {
        const uint64_t *wp = slots + ((int64_t)buf * G + xg) * slot_w + CW;
        for (int i = t; i < pw + ntr; i += NT) {
            T x;
            if (!get_value<T>(wp + (int64_t)i * TW, tag, x, err)) {
                *s_flag = 1;
                break;
            }
            if (i < pw)
                s_Lp[JJ * P + i] = x;
            else
                s_Tr[JJ * 512 + (i - pw)] = x;
        }
    }
    if (t == 0) {
        s_keep[JJ] = take ? 1 : 0;
        if (g == 0) {
            piv[j] = take ? xr : -1;
            keep[j] = take ? 1 : 0;
        }
    }
    __syncthreads();
    if (*s_flag) return false;
    if (take) {
        ++kept;
        const T pv = s_Lp[JJ * P + JJ];
        T w[P];
#pragma unroll
        for (int ii = 0; ii < P; ++ii) w[ii] = s_Lp[JJ * P + ii];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const T x = v[q][JJ] / pv;
            v[q][JJ] = x;
#pragma unroll
            for (int ii = JJ + 1; ii < P; ++ii)
                if (ii < pw) v[q][ii] = fma(-w[ii], x, v[q][ii]);
        }
    }
    return true;
}

template <class T, int R, int P>
__global__ __launch_bounds__(HP_NT) void k_hess_panel(T *__restrict__ Y, int64_t ldy, int64_t n, int b, double tol,
                                                      int32_t *__restrict__ piv, int32_t *__restrict__ keep,
                                                      int64_t per, uint64_t *__restrict__ slots, int64_t slot_w,
                                                      int *__restrict__ err, int32_t *__restrict__ kept_d) {
    constexpr int NT = HP_NT, NW = NT / 64;
    __shared__ T s_Tr[P * 512]; // pivot rows' trailing entries, then the multipliers
    __shared__ T s_Lp[P * P];   // pivot rows' panel entries
    __shared__ T s_pan[P];      // the local candidate row's panel entries
    __shared__ int s_keep[P];
    __shared__ double s_cm[NW];
    __shared__ int s_cr[2 * NW];
    __shared__ int s_flag;
    const int t = threadIdx.x;
    const int g = blockIdx.x;
    const int64_t r0 = (int64_t)g * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    int kept = 0;
    T v[R][P];
    for (int j0 = 0; j0 < b; j0 += P) {
        const int pw = b - j0 < P ? b - j0 : P;
        // 1. the panel, swept column by column
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int64_t row = r0 + t + (int64_t)NT * q;
#pragma unroll
            for (int jj = 0; jj < P; ++jj) v[q][jj] = (row < r1 && jj < pw) ? Y[row * ldy + j0 + jj] : (T)0;
        }
#define OFRR_HP_COL(JJ)                                                                                          \
        if constexpr (JJ < P) {                                                                                 \
            if (JJ < pw && !hp_column<T, R, P, JJ>(v, j0, pw, b, r0, r1, tol, Y, ldy, piv, keep, slots, slot_w, \
                                                   err, kept, s_cm, s_cr, s_pan, s_Lp, s_Tr, s_keep, &s_flag))  \
                return;                                                                                         \
        }
        OFRR_HP_COL(0)
        OFRR_HP_COL(1)
        OFRR_HP_COL(2)
        OFRR_HP_COL(3)
        OFRR_HP_COL(4)
        OFRR_HP_COL(5)
        OFRR_HP_COL(6)
        OFRR_HP_COL(7)
#undef OFRR_HP_COL
        const int c0 = j0 + pw;
        const int nt_ = b - c0;  // trailing columns
        if (nt_ > 0) {
            // 2. multipliers, in place: entry i of pivot row jj once the
            // panel's earlier pivots have been eliminated from it
            for (int i = t; i < nt_; i += NT)
                for (int jj = 0; jj < pw; ++jj) {
                    if (!s_keep[jj]) continue;
                    T x = s_Tr[jj * 512 + i];
                    for (int l = 0; l < jj; ++l)
                        if (s_keep[l]) x = fma(-s_Tr[l * 512 + i], s_Lp[jj * P + l], x);
                    s_Tr[jj * 512 + i] = x;
                }
            __syncthreads();
            // 3. the panel's columns are final: stored first, so the trailing
            // update reads each row's panel entries with the row and the
            // panel registers are free for loads in flight.  A wave takes
            // rows, its lanes 64 consecutive trailing columns (one coalesced
            // access per row segment); a lane keeps its columns' multipliers
            // in registers, and the row's panel entries are read by the
            // first lanes and broadcast across the wave.
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int64_t row = r0 + t + (int64_t)NT * q;
                if (row < r1)
#pragma unroll
                    for (int jj = 0; jj < P; ++jj)
                        if (jj < pw) Y[row * ldy + j0 + jj] = v[q][jj];
            }
            __syncthreads();
            int kk[P];
#pragma unroll
            for (int l = 0; l < P; ++l) kk[l] = l < pw ? s_keep[l] : 0;
            const int lane = t & 63, wave = t >> 6;
            const int nrows = (int)(r1 - r0 > 0 ? r1 - r0 : 0);
            constexpr int UR = 4;  // rows in flight per lane
            for (int cb = 0; cb < nt_; cb += 64) {
                const int i = cb + lane;
                const bool on = i < nt_;
                T u[P];
#pragma unroll
                for (int l = 0; l < P; ++l) u[l] = on && kk[l] ? s_Tr[l * 512 + i] : (T)0;
                T *col = Y + c0 + (on ? i : 0);
                const T *pan = Y + j0 + (lane < pw ? lane : 0);
                int rr = wave;
                for (; rr + (UR - 1) * NW < nrows; rr += UR * NW) {
                    T x[UR], lv[UR];
#pragma unroll
                    for (int z = 0; z < UR; ++z) {
                        const int64_t row = r0 + rr + z * NW;
                        x[z] = on ? col[row * ldy] : (T)0;
                        lv[z] = pan[row * ldy];
                    }
#pragma unroll
                    for (int z = 0; z < UR; ++z)
#pragma unroll
                        for (int l = 0; l < P; ++l)
                            if (kk[l]) x[z] = fma(-u[l], wave_bcast(lv[z], l), x[z]);
                    if (on)
#pragma unroll
                        for (int z = 0; z < UR; ++z) col[(r0 + rr + z * NW) * ldy] = x[z];
                }
                for (; rr < nrows; rr += NW) {
                    const int64_t row = r0 + rr;
                    T x = on ? col[row * ldy] : (T)0;
                    const T lv = pan[row * ldy];
#pragma unroll
                    for (int l = 0; l < P; ++l)
                        if (kk[l]) x = fma(-u[l], wave_bcast(lv, l), x);
                    if (on) col[row * ldy] = x;
                }
            }
            __syncthreads();
        } else {
            // the panel's columns are final
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int64_t row = r0 + t + (int64_t)NT * q;
                if (row < r1)
#pragma unroll
                    for (int jj = 0; jj < P; ++jj)
                        if (jj < pw) Y[row * ldy + j0 + jj] = v[q][jj];
            }
            __syncthreads();
        }
    }
    if (g == 0 && t == 0) *kept_d = kept;
}

template <class T>
int32_t run_panel(Context *ctx, int64_t n, int32_t b, T *Y, int64_t ldy, double tol, int32_t *piv, int32_t *keep,
                  const int32_t **status, const WordsBuf &wb) {
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    // every CU takes a slice once there are 256 rows per CU (more slices
    // stream the trailing block with more of the chip's memory paths)
    const int G = (int)std::min<int64_t>(cus, (n + HP_NT / 2 - 1) / (HP_NT / 2));
    const int64_t per = (n + G - 1) / G;
    const int R = (int)((per + HP_NT - 1) / HP_NT);
    // word buffer: [0] error flag and kept count, then per column parity and
    // workgroup one slot: the candidate (magnitude words, row) and a row of
    // up to b entries
    constexpr int TW = NWords<T>::value, CW = NWords<typename MagT<T>::type>::value + 1;
    const int64_t slot_w = CW + (int64_t)b * TW;
    const int64_t nwords = 1 + (int64_t)2 * G * slot_w;
    uint64_t *words = wb.get(ctx, nwords);
    int *err = reinterpret_cast<int *>(words);
    int32_t *kept_d = err + 1;
    uint64_t *slots = words + 1;
    // panel width eight (eight FP64 rows per thread: the 8 x 8 panel takes
    // the whole register budget of two waves per SIMD, with no spill)
    const void *kern = R <= 1   ? (const void *)k_hess_panel<T, 1, 8>
                       : R <= 2 ? (const void *)k_hess_panel<T, 2, 8>
                       : R <= 4 ? (const void *)k_hess_panel<T, 4, 8>
                                : (const void *)k_hess_panel<T, 8, 8>;
    static OccEntry occ[OCC_SLOTS] = {};
    const int per_cu = occupancy_cached(occ, ctx->device, kern, 0, [&] {
        int pc = 0;
        OFRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, HP_NT, 0));
        return pc;
    });
    if ((int64_t)per_cu * cus < G) fail(OFRR_ERR_UNSUPPORTED, "hessenberg: panel grid cannot be co-resident");
    hipLaunchKernelGGL(k_hess_reset, dim3((unsigned)std::min<int64_t>(256, (nwords + 255) / 256)), dim3(256), 0,
                       ctx->stream, words, nwords);
    OFRR_HIP(hipGetLastError());
    void *args[] = {&Y, &ldy, &n, &b, &tol, &piv, &keep, (void *)&per, &slots, (void *)&slot_w, &err, &kept_d};
    {
        KTimer tm(ctx, "hessenberg");
        OFRR_HIP(launch_resident(kern, dim3(G), dim3(HP_NT), args, 0, ctx->stream));
    }
    if (status) {
        *status = err;
        return 0;
    }
    return read_status(ctx, err, wb.ext != nullptr);
}

template <class T>
int32_t run(Context *ctx, int64_t n, int32_t b, T *Y, int64_t ldy, double tol, int32_t *piv,
            int32_t *keep, const int32_t **status, const WordsBuf &wb) {
    OFRR_CHECK_ARG(b >= 1 && b <= 512, "hessenberg: 1 <= b <= 512");
    OFRR_CHECK_ARG(n >= 1 && n < (int64_t)0x7fffffff, "hessenberg: 1 <= n < 2^31");
    OFRR_CHECK_ARG(ldy >= b, "hessenberg: ld >= b");
    using M = typename MagT<T>::type;
    // LDS per workgroup for its row slice (OFRR_HESS_LDS_KB overrides, for
    // tuning sweeps): the rows stay resident when the slices of all
    // workgroups fit one per CU; fewer, larger slices mean fewer candidates
    // to read per column
    size_t lds_budget = 128 * 1024;
    if (const char *s = std::getenv("OFRR_HESS_LDS_KB")) {
        const long kb = std::strtol(s, nullptr, 10);
        if (kb >= 8 && kb <= 150) lds_budget = (size_t)kb * 1024;
    }
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    // blocks of at most 128 columns: one row per thread in registers
    // (OFRR_HESS_REG=0 selects the LDS kernel, for comparisons)
    // rows per workgroup: the smallest of 64, 128, 256 (at least
    // OFRR_HESS_REG_NT, for comparisons) that keeps the slices within
    // HR_GMAX.  One wave per workgroup is fastest (n = 16384, b = 128:
    // 0.51 ms against 0.60 ms at 128 and 0.68 ms at 256 rows, measured): its
    // argmax is a DPP reduction with no LDS round trip or barrier, and the
    // 256 workgroups spread the row updates over every CU.
    int rnt = 64;
    if (const char *s = std::getenv("OFRR_HESS_REG_NT")) {
        const int v = std::atoi(s);
        if (v == 64 || v == 128 || v == 256) rnt = v;
    }
    while (rnt < 256 && (n + rnt - 1) / rnt > HR_GMAX) rnt *= 2;
    // FP64 rows take 256 registers per thread (plus accumulation registers
    // for the rest): faster than the LDS kernel only with one-wave
    // workgroups (n = 16384, b = 128: 0.60 ms against 0.72 ms; 0.67 and
    // 0.77 ms at 128 and 256 rows, measured).  OFRR_HESS_REG64=0|1 forces
    // the choice, for comparisons.
    bool reg_type = std::is_same<T, float>::value || rnt == 64;
    if (const char *s = std::getenv("OFRR_HESS_REG64"))
        reg_type = std::is_same<T, float>::value || std::atoi(s) != 0;
    bool use_reg = reg_type && b <= HR_B && (n + rnt - 1) / rnt <= HR_GMAX;
    if (const char *s = std::getenv("OFRR_HESS_REG")) use_reg = use_reg && std::atoi(s) != 0;
    if (use_reg) {
        if (rnt == 64) return run_reg<T, 64>(ctx, n, b, Y, ldy, tol, piv, keep, status, wb);
        if (rnt == 128) return run_reg<T, 128>(ctx, n, b, Y, ldy, tol, piv, keep, status, wb);
        return run_reg<T, 256>(ctx, n, b, Y, ldy, tol, piv, keep, status, wb);
    }
    const int vec = 16 / (int)sizeof(T);
    const int64_t ldr = ((b + vec - 1) / vec + 1) * vec;  // padded row length in LDS
    int64_t rows_res = (int64_t)(lds_budget / ((size_t)ldr * sizeof(T)));
    bool resident = false;
    int64_t rows_per;
    int G;
    // workgroup size (OFRR_HESS_THREADS overrides, for tuning sweeps): 256
    // measured fastest for this kernel (FP64, n = 16384, b = 128: 0.72 ms
    // against 0.74 ms at 128 and 0.76 ms at 64 threads with one row each)
    int nt = 256;
    if (const char *s = std::getenv("OFRR_HESS_THREADS")) {
        const long v = std::strtol(s, nullptr, 10);
        if (v == 64 || v == 128 || v == 256 || v == 512 || v == 1024) nt = (int)v;
    }
    if (rows_res >= 16 && (n + rows_res - 1) / rows_res <= cus) {
        resident = true;
        rows_per = std::min<int64_t>(rows_res, n);
        // narrow workgroups take one row per thread where the CUs allow it
        if (nt <= 128) rows_per = std::min<int64_t>(rows_per, std::max<int64_t>(nt, (n + cus - 1) / cus));
        G = (int)((n + rows_per - 1) / rows_per);
    } else {
        int64_t want_g = std::min<int64_t>(cus, (n + 255) / 256);
        if (want_g < 1) want_g = 1;
        rows_per = (n + want_g - 1) / want_g;
        G = (int)((n + rows_per - 1) / rows_per);
    }
    // too tall for the slices to stay on chip: the panel form (trailing
    // block streamed once per panel of columns instead of once per column),
    // up to eight rows per thread (OFRR_HESS_PANEL=0 selects the in-place
    // per-column kernel, for comparisons)
    bool panel = !resident && n <= (int64_t)cus * HP_NT * 8;
    if (const char *s = std::getenv("OFRR_HESS_PANEL")) panel = panel && std::atoi(s) != 0;
    if (panel) return run_panel<T>(ctx, n, b, Y, ldy, tol, piv, keep, status, wb);
    const size_t shmem = resident ? (size_t)rows_per * ldr * sizeof(T) : 0;

    // one word buffer: [0] error flag and kept count (two ints), then the
    // candidate slots (2 x G x CW words), then the row slots (2 x G x b x TW)
    constexpr int TW = (int)(sizeof(T) / 4);
    constexpr int CW = (int)(sizeof(M) / 4) + 1;
    const int64_t ncand = (int64_t)2 * G * CW, nrow = (int64_t)2 * G * b * TW;
    const int64_t nwords = 1 + ncand + nrow;
    uint64_t *words = wb.get(ctx, nwords);
    int *err = reinterpret_cast<int *>(words);
    int32_t *kept_d = err + 1;
    uint64_t *slot_cand = words + 1;
    uint64_t *slot_rows = words + 1 + ncand;
    hipLaunchKernelGGL(k_hess_reset, dim3((unsigned)std::min<int64_t>(256, (nwords + 255) / 256)), dim3(256), 0,
                       ctx->stream, words, nwords);
    OFRR_HIP(hipGetLastError());

    void *kern = nullptr;
    if (nt == 64) kern = resident ? (void *)k_hessenberg<T, true, 64> : (void *)k_hessenberg<T, false, 64>;
    else if (nt == 128) kern = resident ? (void *)k_hessenberg<T, true, 128> : (void *)k_hessenberg<T, false, 128>;
    else if (nt == 256) kern = resident ? (void *)k_hessenberg<T, true, 256> : (void *)k_hessenberg<T, false, 256>;
    else if (nt == 512) kern = resident ? (void *)k_hessenberg<T, true, 512> : (void *)k_hessenberg<T, false, 512>;
    else kern = resident ? (void *)k_hessenberg<T, true, 1024> : (void *)k_hessenberg<T, false, 1024>;
    // the dynamic-LDS limit and the occupancy answer depend only on the
    // kernel variant, its LDS size and the device: asked once, then reused
    // (the sweep runs every iteration)
    // (the dynamic-LDS limit of a kernel only ever grows: lds_set holds the
    // largest size set so far per device and kernel)
    static OccEntry occ[OCC_SLOTS] = {};
    static OccEntry lds_set[OCC_SLOTS] = {};
    const int per_cu = occupancy_cached(occ, ctx->device, (const void *)kern, shmem, [&] {
        OccEntry *cur = nullptr;
        for (int i = 0; i < OCC_SLOTS && !cur; ++i)
            if (lds_set[i].kern == nullptr || (lds_set[i].dev == ctx->device && lds_set[i].kern == kern)) {
                if (lds_set[i].kern == nullptr) lds_set[i] = OccEntry{ctx->device, kern, 0, 0};
                cur = &lds_set[i];
            }
        if (!cur || shmem > cur->shmem) {
            OFRR_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
            if (cur) cur->shmem = shmem;
        }
        int pc = 0;
        OFRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, nt, shmem));
        return pc;
    });
    if ((int64_t)per_cu * cus < G)
        fail(OFRR_ERR_UNSUPPORTED, "hessenberg: grid cannot be co-resident");
    void *args[] = {&Y, &ldy, &n, &b, &tol, &piv, &keep, &rows_per, &slot_rows, &slot_cand, &err,
                    &kept_d};
    {
        KTimer tm(ctx, "hessenberg");
        OFRR_HIP(launch_resident(kern, dim3(G), dim3(nt), args, shmem, ctx->stream));
    }
    if (status) {
        *status = err;
        return 0;
    }
    return read_status(ctx, err, wb.ext != nullptr);
}

}  // namespace

int32_t hessenberg(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                   double tol, int32_t *piv, int32_t *keep, const int32_t **status) {
    const WordsBuf wb;
    if (t == OFRR_F64) return run<double>(ctx, n, b, (double *)Y, ldy, tol, piv, keep, status, wb);
    if (t == OFRR_F32) return run<float>(ctx, n, b, (float *)Y, ldy, tol, piv, keep, status, wb);
    fail(OFRR_ERR_UNSUPPORTED, "hessenberg: element type must be F64 or F32");
}

void hess_scratch_address(Context *ctx) {
    void *p = nullptr;
    OFRR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ctx->hess_scratch = static_cast<uint64_t *>(p);
}

int32_t hessenberg_noalloc(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                           double tol, int32_t *piv, int32_t *keep) {
    if (!ctx->hess_scratch) fail(OFRR_ERR_HIP, "hessenberg_noalloc: the fixed exchange array has no address");
    WordsBuf wb;
    wb.ext = ctx->hess_scratch;
    wb.ext_cap = HESS_SCRATCH_WORDS;
    if (t == OFRR_F64) return run<double>(ctx, n, b, (double *)Y, ldy, tol, piv, keep, nullptr, wb);
    if (t == OFRR_F32) return run<float>(ctx, n, b, (float *)Y, ldy, tol, piv, keep, nullptr, wb);
    fail(OFRR_ERR_UNSUPPORTED, "hessenberg: element type must be F64 or F32");
}

}  // namespace ofrr
