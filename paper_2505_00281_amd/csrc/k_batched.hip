// k_batched.hip -- many independent symmetric eigenproblems of uneven size
// solved together by the same method (Sec. 2 subspace iteration with
// restart from all Ritz vectors, Sec. 4.2 Hessenberg process in place of
// QR, Sec. 3.1 orthogonalization-free projection, the mixed-precision plan
// at the end of Sec. 4).
//
// Every step of an outer iteration is one grouped launch over the
// unconverged problems, so hundreds of small problems fill the chip
// together instead of one after another:
//   kb_stabilise   one workgroup per problem: filter step from A X, per-
//                  column power-of-two scaling and the Hessenberg process,
//                  left-looking (column j receives the eliminations of the
//                  kept columns before it, in order: per element the same
//                  fused multiply-adds as the right-looking sweep), dropped
//                  columns compacted on the fly, the basis rounded to its
//                  storage type;
//   kb_product_*   W = A V over a work list of (problem, row tile): the
//                  reduced copy of A on BF16/F16 MFMA (FP32 accumulation)
//                  for problems in the first phase, A as stored on FP64
//                  MFMA for problems in the FP64 phase; the tile height is
//                  picked by a timing autotuner;
//   kb_psl         one workgroup per problem: G = V^T V and H = V^T W in
//                  FP64, the pencil H y = theta G y (Cholesky, Jacobi in
//                  parallel order, G-eigen truncation when G is not
//                  positive definite), the lift X = V Y, A X = W Y, the
//                  residual estimates and the phase / convergence
//                  bookkeeping;
//   kb_lists       rebuilds the work lists of the unconverged problems.
// The launches of an iteration read their work counts from device memory,
// so one iteration is captured once in a HIP graph and replayed; the host
// reads back the number of unconverged problems every few replays.
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

constexpr int KB_BMAX = 32;  // basis columns per problem
constexpr int KB_WIN = 16;   // longest stall window
constexpr int KB_NT = 256;   // threads of the per-problem kernels

// Blocks of a problem: row-major n x ld (XF, AXF: n x k), 8 bytes per entry
// reserved (an FP32 block uses the first half).
enum { BLK_X = 0, BLK_AX = 1, BLK_Y = 2, BLK_V = 3, BLK_W = 4, BLK_XF = 5, BLK_AXF = 6, BLK_N = 7 };

struct BProb {
    const void *A;        // caller's A, column-major
    int64_t lda;
    int32_t n;
    int32_t a_f64;        // A holds FP64 values (else FP32)
    int64_t ldr;          // n rounded up to 16: rows of the reduced copy and of Vt columns
    const uint16_t *Alo;  // reduced copy of A (BF16/F16 bits), column c at Alo + c*ldr, zero-padded
    uint16_t *Vt;         // reduced basis operand, column c at Vt + c*ldr, zero-padded
    void *blk[BLK_N];
    double *theta;        // Ritz values of the last projection (sorted)
    double *evals, *evecs, *resid;  // the caller's outputs
};

struct BState {
    int32_t phase;     // 0 first, 1 FP64 tail, 2 finished
    int32_t xf64;      // X and A X are stored in FP64 (else FP32)
    int32_t bc;        // current basis size
    int32_t iters, iters_low, products;
    int32_t status;    // 0 or a negative ofrr_status
    int32_t nhist;     // values pushed to the stall detector in this phase
    double min_before; // smallest value that has left the window
    double ring[KB_WIN];
    double anorm;
    double emax;
};

struct BParams {
    int32_t nprob, k, ld, smallest;
    int32_t max_iters, window, has_tail, first_f64;
    int32_t red_bf16;  // reduced type of the first phase: 1 BF16, 0 F16
    int32_t pad;
    double alpha, cshift;  // filter step Y = alpha (A X - cshift X)
    double tol, switch_resid, anorm_fixed, drop_red, drop_f64;
};

// ------------------------------------------------------------------ utils

__device__ __forceinline__ double load_blk(const void *p, int64_t i, int f64) {
    return f64 ? static_cast<const double *>(p)[i] : (double)static_cast<const float *>(p)[i];
}
__device__ __forceinline__ void store_blk(void *p, int64_t i, int f64, double v) {
    if (f64)
        static_cast<double *>(p)[i] = v;
    else
        static_cast<float *>(p)[i] = (float)v;
}

__device__ __forceinline__ float round_red(float x, int bf16) {
    return bf16 ? bf16_bits_to_f32(f32_to_bf16_bits(x)) : f16_bits_to_f32(f32_to_f16_bits(x));
}
__device__ __forceinline__ uint16_t bits_red(float x, int bf16) {
    return bf16 ? f32_to_bf16_bits(x) : f32_to_f16_bits(x);
}

__device__ __forceinline__ bool isnan_d(double v) { return !(v == v); }

// block-wide (KB_NT threads) maximum of non-negative values; NaN wins
__device__ double kb_block_max(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) {
        const double q = __shfl_xor(v, o, 64);
        v = (q > v || isnan_d(q)) ? q : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < KB_NT / 64; ++i) r = (red[i] > r || isnan_d(red[i])) ? red[i] : r;
    __syncthreads();
    return r;
}

// block-wide argmax of (mag, row): larger magnitude first, then the smaller
// row; a NaN magnitude wins (the caller reports it)
__device__ __forceinline__ bool argmax_take(double qm, int qr, double m, int r) {
    if (isnan_d(m)) return false;
    if (isnan_d(qm)) return true;
    return qm > m || (qm == m && qr < r);
}
__device__ void kb_block_argmax(double &mag, int &row, double *redv, int *redi) {
    for (int o = 32; o > 0; o >>= 1) {
        const double qm = __shfl_xor(mag, o, 64);
        const int qr = __shfl_xor(row, o, 64);
        if (argmax_take(qm, qr, mag, row)) {
            mag = qm;
            row = qr;
        }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        redv[threadIdx.x >> 6] = mag;
        redi[threadIdx.x >> 6] = row;
    }
    __syncthreads();
    double m = redv[0];
    int r = redi[0];
    for (int i = 1; i < KB_NT / 64; ++i)
        if (argmax_take(redv[i], redi[i], m, r)) {
            m = redv[i];
            r = redi[i];
        }
    __syncthreads();
    mag = m;
    row = r;
}

// ------------------------------------------------------------ stabilise

// Filter step, scaling and Hessenberg process for one problem in the
// arithmetic T of its phase.  Y (row-major, ld) receives the eliminated
// columns in place (the multipliers later columns need); the kept columns
// go to V (compacted; rounded to the storage type in the reduced phase)
// and, in the reduced phase, to the K-contiguous operand Vt.
template <class T>
__device__ void stab_problem(const BProb &P, BState &S, const BParams &prm, int reduced) {
    __shared__ double s_red[KB_NT / 64];
    __shared__ int s_redi[KB_NT / 64];
    __shared__ int s_piv[KB_BMAX];                  // pivot rows of the kept columns
    __shared__ int s_col[KB_BMAX];                  // their column indices in Y
    __shared__ double s_sub[KB_BMAX][KB_BMAX + 1];  // s_sub[i][l] = Y[piv_i][col_l]
    __shared__ double s_cur[KB_BMAX];               // Y[piv_i][j] scaled, before elimination
    __shared__ double s_u[KB_BMAX];                 // the same after elimination
    const int t = threadIdx.x;
    const int n = P.n, ld = prm.ld, bc = S.bc;
    const int xf = S.xf64;
    const void *X = P.blk[BLK_X];
    const void *AX = P.blk[BLK_AX];
    T *Y = static_cast<T *>(P.blk[BLK_Y]);
    T *V = static_cast<T *>(P.blk[BLK_V]);
    const double alpha = prm.alpha, csh = prm.cshift;
    const double tol = reduced ? prm.drop_red : prm.drop_f64;
    bool bad = false;
    int m = 0;  // columns kept so far (the same in every thread)
    for (int j = 0; j < bc; ++j) {
        // 1. filter step into Y (type T) and the column maximum
        double cm = 0.0;
        for (int r = t; r < n; r += KB_NT) {
            const int64_t e = (int64_t)r * ld + j;
            double y = load_blk(AX, e, xf);
            if (csh != 0.0)
                y = alpha * (y - csh * load_blk(X, e, xf));
            else if (alpha != 1.0)
                y = alpha * y;
            const T yt = (T)y;
            Y[e] = yt;
            const double a = fabs((double)yt);
            cm = (a > cm || isnan_d(a)) ? a : cm;
        }
        cm = kb_block_max(cm, s_red);
        if (isnan_d(cm) || isinf(cm)) {
            bad = true;
            break;
        }
        // power-of-two scale bringing the column to infinity-norm (1/2, 1]
        double sc = 1.0;
        if (cm > 0.0) {
            int e2;
            (void)frexp(cm, &e2);
            sc = ldexp(1.0, -e2);
        }
        // 2. the multipliers at the kept pivot rows and this column there
        for (int q = t; q < m * (m + 1); q += KB_NT) {
            const int i = q / (m + 1), l = q - i * (m + 1);
            const int64_t e = (int64_t)s_piv[i] * ld;
            if (l < m)
                s_sub[i][l] = (double)Y[e + s_col[l]];
            else
                s_cur[i] = (double)(T)((double)Y[e + j] * sc);
        }
        __syncthreads();
        // eliminations of the kept columns, in order, at the pivot rows
        if (t == 0) {
            for (int i = 0; i < m; ++i) {
                T u = (T)s_cur[i];
                for (int l = 0; l < i; ++l) u = fma(-(T)s_u[l], (T)s_sub[i][l], u);
                s_u[i] = (double)u;
            }
        }
        __syncthreads();
        // 3. scale and eliminate every row; argmax of the result
        double best = -1.0;
        int brow = 0x7fffffff;
        for (int r = t; r < n; r += KB_NT) {
            const int64_t e = (int64_t)r * ld;
            T y = (T)((double)Y[e + j] * sc);
            for (int l = 0; l < m; ++l) y = fma(-(T)s_u[l], Y[e + s_col[l]], y);
            Y[e + j] = y;
            const double a = fabs((double)y);
            if (isnan_d(a)) {
                best = a;
                brow = r;
            } else if (!isnan_d(best) && a > best) {
                best = a;
                brow = r;
            }
        }
        kb_block_argmax(best, brow, s_red, s_redi);
        if (isnan_d(best)) {
            bad = true;
            break;
        }
        if (best >= tol && best > 0.0) {
            // 4. divide by the pivot; multipliers stay in Y, the column goes to V
            const T piv = Y[(int64_t)brow * ld + j];
            for (int r = t; r < n; r += KB_NT) {
                const int64_t e = (int64_t)r * ld;
                const T y = Y[e + j] / piv;
                Y[e + j] = y;
                if (reduced) {
                    const float yf = (float)y;
                    V[e + m] = (T)round_red(yf, prm.red_bf16);
                    P.Vt[(int64_t)m * P.ldr + r] = bits_red(yf, prm.red_bf16);
                } else {
                    V[e + m] = y;
                }
            }
            if (t == 0) {
                s_piv[m] = brow;
                s_col[m] = j;
            }
            ++m;
        }
        __syncthreads();
    }
    if (t == 0) {
        if (bad || m < prm.k) {
            S.status = OFRR_ERR_NUMERIC;
            S.phase = 2;
        } else {
            S.bc = m;
        }
    }
}

__global__ __launch_bounds__(KB_NT) void kb_stabilise(const BProb *probs, BState *states, BParams prm,
                                                      const int32_t *active, const int32_t *counts) {
    const int na = counts[0];
    for (int w = blockIdx.x; w < na; w += gridDim.x) {
        const int p = active[w];
        const int phase = states[p].phase;
        if (phase == 2) continue;  // uniform: one value per workgroup
        if (phase == 1 || prm.first_f64)
            stab_problem<double>(probs[p], states[p], prm, 0);
        else
            stab_problem<float>(probs[p], states[p], prm, 1);
        __syncthreads();
    }
}

// ------------------------------------------------------------- products

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 kb_bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 kb_f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float kb_f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t kb_u32x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double kb_f64x4_t;

template <bool IS_BF16>
__device__ __forceinline__ kb_f32x16_t kb_mfma(kb_u32x4_t a, kb_u32x4_t b, kb_f32x16_t c) {
    if constexpr (IS_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(kb_bf16x8_t, a),
                                                       __builtin_bit_cast(kb_bf16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(kb_f16x8_t, a),
                                                      __builtin_bit_cast(kb_f16x8_t, b), c, 0, 0, 0);
}

constexpr int KB_KU = 4;  // K steps of 16 whose loads are in flight together

// W (FP32, row-major, ldw) = A V for problems in the reduced phase; one
// work item = 32*WAVES rows of one problem, all basis columns (<= 32).  A
// is symmetric, so row i of A is column i of the reduced copy (K-
// contiguous); the basis is the K-contiguous operand Vt.  Both are zero-
// padded to ldr rows (a multiple of 16), so the K loop needs no test.
// MFMA 32x32x16: lane l holds A[l%32][8(l/32)..+8] and V[8(l/32)..+8][l%32];
// accumulator r of lane l is D[(r/4)*8 + 4(l/32) + r%4][l%32].
template <bool IS_BF16, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void kb_product_lp(const BProb *probs, const BState *states,
                                                            const int2 *items, const int32_t *counts,
                                                            int count_slot, int out_blk, int64_t ldw) {
    const int nitems = counts[count_slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int2 it = items[w];
        const BProb &P = probs[it.x];
        const int n = P.n;
        const int bc = states[it.x].bc;
        const int64_t ldr = P.ldr;
        const int row0 = it.y * (32 * WAVES) + 32 * wave;
        const int arow = min(row0 + l32, n - 1);  // rows past n read row n - 1, not stored
        const int vcol = min(l32, bc - 1);
        const bool vok = l32 < bc;
        const uint16_t *ap = P.Alo + (int64_t)arow * ldr + 8 * h;
        const uint16_t *vp = P.Vt + (int64_t)vcol * ldr + 8 * h;
        kb_f32x16_t acc = kb_f32x16_t{};
        kb_u32x4_t ra[KB_KU], rb[KB_KU];
#pragma unroll
        for (int u = 0; u < KB_KU; ++u) {
            const int64_t kk = 16 * u < ldr ? 16 * u : 0;
            ra[u] = *reinterpret_cast<const kb_u32x4_t *>(ap + kk);
            rb[u] = *reinterpret_cast<const kb_u32x4_t *>(vp + kk);
        }
        for (int64_t k0 = 0; k0 < ldr; k0 += 16 * KB_KU) {
            kb_u32x4_t na[KB_KU], nb[KB_KU];
#pragma unroll
            for (int u = 0; u < KB_KU; ++u) {
                const int64_t k1 = k0 + 16 * (KB_KU + u);
                const int64_t kk = k1 < ldr ? k1 : 0;
                na[u] = *reinterpret_cast<const kb_u32x4_t *>(ap + kk);
                nb[u] = *reinterpret_cast<const kb_u32x4_t *>(vp + kk);
            }
#pragma unroll
            for (int u = 0; u < KB_KU; ++u)
                if (k0 + 16 * u < ldr)
                    acc = kb_mfma<IS_BF16>(ra[u], vok ? rb[u] : kb_u32x4_t{0u, 0u, 0u, 0u}, acc);
#pragma unroll
            for (int u = 0; u < KB_KU; ++u) {
                ra[u] = na[u];
                rb[u] = nb[u];
            }
        }
        float *Wp = static_cast<float *>(P.blk[out_blk]);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = row0 + (r >> 2) * 8 + 4 * h + (r & 3);
            if (row < n && vok) Wp[(int64_t)row * ldw + l32] = acc[r];
        }
    }
}

// W (FP64, row-major, ldw) = A V on FP64 MFMA with A as stored (FP32 values
// promoted exactly, or FP64) and V FP64 (row-major, ldv); one work item =
// 32*WAVES rows of one problem, ncols (or the problem's basis size) columns
// <= 32.  v_mfma_f64_16x16x4: lane l holds A[l%16][l/16] and V[l/16][l%16];
// accumulator r of lane l is D[4r + l/16][l%16].  Lane group g supplies
// k = k0 + 8g + s at step s, so each lane reads eight consecutive entries
// of its row of A (symmetric: a column of the stored matrix).
template <class TA, int WAVES>
__device__ void kb_f64_item(const BProb &P, int n, int bc, int tile, int wave, int lane, const double *Vp,
                            int64_t ldv, double *Wp, int64_t ldw) {
    const int r16 = lane & 15, g = lane >> 4;
    const int row0 = tile * (32 * WAVES) + 32 * wave;
    const TA *A = static_cast<const TA *>(P.A);
    const int64_t lda = P.lda;
    const TA *arow[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) arow[rb] = A + (int64_t)min(row0 + 16 * rb + r16, n - 1) * lda;
    const bool two = bc > 16;
    int vcol[2];
    bool vok[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int c = 16 * cb + r16;
        vok[cb] = c < bc;
        vcol[cb] = min(c, bc - 1);
    }
    kb_f64x4_t acc[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = kb_f64x4_t{0.0, 0.0, 0.0, 0.0};
    TA ra[2][8];
    double rv[2][8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int k = k0 + 8 * g + s;
            const int kc = k < n ? k : n - 1;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) ra[rb][s] = arow[rb][kc];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) rv[cb][s] = Vp[(int64_t)kc * ldv + vcol[cb]];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < n; k0 += 32) {
        double a[2][8], v[2][8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bool kin = k0 + 8 * g + s < n;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) a[rb][s] = kin ? (double)ra[rb][s] : 0.0;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) v[cb][s] = (kin && vok[cb]) ? rv[cb][s] : 0.0;
        }
        if (k0 + 32 < n) fetch(k0 + 32);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                acc[rb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][s], v[0][s], acc[rb][0], 0, 0, 0);
                if (two) acc[rb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][s], v[1][s], acc[rb][1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 16 * rb + 4 * r + g;
                if (row < n && vok[cb] && (cb == 0 || two)) Wp[(int64_t)row * ldw + 16 * cb + r16] = acc[rb][cb][r];
            }
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void kb_product_f64(const BProb *probs, const BState *states,
                                                             const int2 *items, const int32_t *counts,
                                                             int count_slot, int in_blk, int out_blk,
                                                             int64_t ldv, int64_t ldw, int ncols) {
    const int nitems = counts[count_slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int2 it = items[w];
        const BProb &P = probs[it.x];
        const int bc = ncols > 0 ? ncols : states[it.x].bc;
        const double *Vp = static_cast<const double *>(P.blk[in_blk]);
        double *Wp = static_cast<double *>(P.blk[out_blk]);
        if (P.a_f64)
            kb_f64_item<double, WAVES>(P, P.n, bc, it.y, wave, lane, Vp, ldv, Wp, ldw);
        else
            kb_f64_item<float, WAVES>(P, P.n, bc, it.y, wave, lane, Vp, ldv, Wp, ldw);
    }
}

// ------------------------------------------------- project, solve, lift

// Jacobi rotation of the pair (p, q) annihilating C_pq (the oracle's
// convention: columns p, q become c col_p - s col_q and s col_p + c col_q).
__device__ __forceinline__ void jacobi_cs(double cpp, double cqq, double cpq, double &c, double &s) {
    if (cpq == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    const double tau = (cqq - cpp) / (2.0 * cpq);
    double t;
    if (fabs(tau) > 1e150)
        t = 0.5 / tau;
    else
        t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
}

// Symmetric eigen-decomposition of C (m x m, LDS, leading dimension 33) by
// Jacobi rotations in round-robin parallel order (m/2 disjoint pairs per
// round, all threads of the block apply them), until the off-diagonal
// Frobenius norm is at most 1e-15 of the whole (or 40 sweeps).  Z receives
// the eigenvectors; the eigenvalues are left on the diagonal of C.
__device__ void kb_jacobi(double (*C)[KB_BMAX + 1], double (*Z)[KB_BMAX + 1], int m, double *cs_c,
                          double *cs_s, int *pp, int *pq, double *red, int *s_go) {
    const int t = threadIdx.x;
    for (int e = t; e < m * m; e += KB_NT) {
        const int i = e / m, j = e - i * m;
        Z[i][j] = (i == j) ? 1.0 : 0.0;
    }
    const int mm = m + (m & 1);  // players (one dummy when m is odd)
    const int np = mm / 2;
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        // convergence test on the off-diagonal part
        double off = 0.0, all = 0.0;
        for (int e = t; e < m * m; e += KB_NT) {
            const int i = e / m, j = e - i * m;
            const double v = C[i][j] * C[i][j];
            all += v;
            if (i != j) off += v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, 64);
            all += __shfl_xor(all, o, 64);
        }
        if ((t & 63) == 0) {
            red[t >> 6] = off;
            red[KB_NT / 64 + (t >> 6)] = all;
        }
        __syncthreads();
        if (t == 0) {
            double so = 0.0, sa = 0.0;
            for (int i = 0; i < KB_NT / 64; ++i) {
                so += red[i];
                sa += red[KB_NT / 64 + i];
            }
            *s_go = (so > 1e-30 * sa) ? 1 : 0;
        }
        __syncthreads();
        if (!*s_go) break;
        for (int round = 0; round < mm - 1; ++round) {
            // pairs of this round: player 0 fixed, the others rotate
            if (t < np) {
                auto player = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + round) % (mm - 1); };
                int a = player(t), b = player(mm - 1 - t);
                if (a > b) {
                    const int x = a;
                    a = b;
                    b = x;
                }
                pp[t] = a;
                pq[t] = b;
                double c = 1.0, s = 0.0;
                if (b < m) jacobi_cs(C[a][a], C[b][b], C[a][b], c, s);
                cs_c[t] = c;
                cs_s[t] = s;
            }
            __syncthreads();
            // columns: C <- C J, Z <- Z J
            for (int e = t; e < 2 * m * np; e += KB_NT) {
                const int which = e / (m * np);
                const int rem = e - which * m * np;
                const int r = rem / np, k = rem - (rem / np) * np;
                const int p = pp[k], q = pq[k];
                if (q >= m) continue;
                const double c = cs_c[k], s = cs_s[k];
                double (*M)[KB_BMAX + 1] = which ? Z : C;
                const double xp = M[r][p], xq = M[r][q];
                M[r][p] = c * xp - s * xq;
                M[r][q] = s * xp + c * xq;
            }
            __syncthreads();
            // rows: C <- J^T C
            for (int e = t; e < m * np; e += KB_NT) {
                const int r = e / np, k = e - (e / np) * np;
                const int p = pp[k], q = pq[k];
                if (q >= m) continue;
                const double c = cs_c[k], s = cs_s[k];
                const double xp = C[p][r], xq = C[q][r];
                C[p][r] = c * xp - s * xq;
                C[q][r] = s * xp + c * xq;
            }
            __syncthreads();
        }
    }
}

// G = V^T V and H = V^T W (bc <= 32 columns, FP64 blocks or FP32 blocks
// whose products are exact in FP64) on FP64 MFMA 16x16x4: per step of four
// rows, lane l supplies V[r0 + l/16][l%16] as both the A operand (V^T) and
// the B operand, and W[r0 + l/16][l%16] as the B operand of H.  The four
// waves take every fourth step; their partial sums are added in a fixed
// order.
__device__ void kb_gram(const void *V, const void *W, int f64, int n, int ld, int bc,
                        double (*G)[KB_BMAX + 1], double (*H)[KB_BMAX + 1]) {
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int c16 = lane & 15, kg = lane >> 4;
    const bool two = bc > 16;
    kb_f64x4_t g[2][2], h[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            g[a][b] = kb_f64x4_t{0.0, 0.0, 0.0, 0.0};
            h[a][b] = kb_f64x4_t{0.0, 0.0, 0.0, 0.0};
        }
    const bool c0 = c16 < bc, c1 = 16 + c16 < bc;
    const int cc0 = min(c16, bc - 1), cc1 = min(16 + c16, bc - 1);
    for (int r0 = 4 * wave; r0 < n; r0 += 16) {
        const int r = r0 + kg;
        const bool rin = r < n;
        const int64_t o = (int64_t)min(r, n - 1) * ld;
        const double v0 = load_blk(V, o + cc0, f64), w0 = load_blk(W, o + cc0, f64);
        const double v1 = load_blk(V, o + cc1, f64), w1 = load_blk(W, o + cc1, f64);
        const double a0 = (rin && c0) ? v0 : 0.0, b0 = (rin && c0) ? w0 : 0.0;
        const double a1 = (rin && c1) ? v1 : 0.0, b1 = (rin && c1) ? w1 : 0.0;
        g[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, g[0][0], 0, 0, 0);
        h[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, h[0][0], 0, 0, 0);
        if (two) {
            g[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a1, g[0][1], 0, 0, 0);
            g[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a0, g[1][0], 0, 0, 0);
            g[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, g[1][1], 0, 0, 0);
            h[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, h[0][1], 0, 0, 0);
            h[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, h[1][0], 0, 0, 0);
            h[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, h[1][1], 0, 0, 0);
        }
    }
    // accumulator r of lane l is D[4r + l/16][l%16]; waves add in order
    for (int wv = 0; wv < 4; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if ((a || b) && !two) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * a + 4 * r + kg, j = 16 * b + c16;
                        if (i < bc && j < bc) {
                            G[i][j] = (wv == 0 ? 0.0 : G[i][j]) + g[a][b][r];
                            H[i][j] = (wv == 0 ? 0.0 : H[i][j]) + h[a][b][r];
                        }
                    }
                }
        }
        __syncthreads();
    }
}

// X = V Y and A X = W Y for rows of one problem (Y: bc x rank in LDS),
// stored in the phase's type; BM is the static bound of bc.
template <int BM>
__device__ void kb_lift_rows(const void *V, const void *W, void *Xo, void *AXo, int f64, int n, int ld, int bc,
                             int rank, double (*Y)[KB_BMAX + 1]) {
    for (int r = threadIdx.x; r < n; r += KB_NT) {
        const int64_t o = (int64_t)r * ld;
        double vr[BM], wr[BM];
#pragma unroll
        for (int i = 0; i < BM; ++i) {
            const int ic = i < bc ? i : bc - 1;
            const double v = load_blk(V, o + ic, f64), w = load_blk(W, o + ic, f64);
            vr[i] = i < bc ? v : 0.0;
            wr[i] = i < bc ? w : 0.0;
        }
#pragma unroll
        for (int c = 0; c < BM; ++c) {
            if (c < rank) {
                double x = 0.0, ax = 0.0;
#pragma unroll
                for (int i = 0; i < BM; ++i) {
                    const double y = i < bc ? Y[i][c] : 0.0;
                    x = fma(vr[i], y, x);
                    ax = fma(wr[i], y, ax);
                }
                store_blk(Xo, o + c, f64, x);
                store_blk(AXo, o + c, f64, ax);
            }
        }
    }
}

// Sums over the rows of ||A x_c - theta_c x_c||^2 and ||x_c||^2 for the
// wanted columns c0 <= c < min(c0 + 16, k) (from the stored X and A X),
// per wave into LDS.
__device__ void kb_resid_rows(const void *Xo, const void *AXo, int f64, int n, int ld, int k, int c0,
                              const double *th, double (*s_res2)[KB_BMAX], double (*s_xn2)[KB_BMAX]) {
    const int t = threadIdx.x;
    double r2[16], x2[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        r2[c] = 0.0;
        x2[c] = 0.0;
    }
    for (int r = t; r < n; r += KB_NT) {
        const int64_t o = (int64_t)r * ld + c0;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (c0 + c < k) {
                const double x = load_blk(Xo, o + c, f64), ax = load_blk(AXo, o + c, f64);
                const double d = ax - th[c0 + c] * x;
                r2[c] = fma(d, d, r2[c]);
                x2[c] = fma(x, x, x2[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        if (c0 + c < k) {
            double a = r2[c], b = x2[c];
            for (int o = 32; o > 0; o >>= 1) {
                a += __shfl_xor(a, o, 64);
                b += __shfl_xor(b, o, 64);
            }
            if ((t & 63) == 0) {
                s_res2[t >> 6][c0 + c] = a;
                s_xn2[t >> 6][c0 + c] = b;
            }
        }
    }
}

// Per problem: projections, pencil, lift, residual estimates, bookkeeping.
__global__ __launch_bounds__(KB_NT) void kb_psl(const BProb *probs, BState *states, BParams prm,
                                                const int32_t *active, const int32_t *counts) {
    __shared__ double sG[KB_BMAX][KB_BMAX + 1];
    __shared__ double sH[KB_BMAX][KB_BMAX + 1];
    __shared__ double sL[KB_BMAX][KB_BMAX + 1];
    __shared__ double sC[KB_BMAX][KB_BMAX + 1];
    __shared__ double sZ[KB_BMAX][KB_BMAX + 1];
    __shared__ double sY[KB_BMAX][KB_BMAX + 1];
    __shared__ double s_th[KB_BMAX], s_ths[KB_BMAX];
    __shared__ int s_perm[KB_BMAX];
    __shared__ double cs_c[KB_BMAX / 2 + 1], cs_s[KB_BMAX / 2 + 1];
    __shared__ int pp[KB_BMAX / 2 + 1], pq[KB_BMAX / 2 + 1];
    __shared__ double red[2 * KB_NT / 64];
    __shared__ double s_res2[KB_NT / 64][KB_BMAX], s_xn2[KB_NT / 64][KB_BMAX];
    __shared__ int s_go, s_chol_ok, s_rank;
    const int t = threadIdx.x;
    const int na = counts[0];
    for (int w = blockIdx.x; w < na; w += gridDim.x) {
        const int p = active[w];
        BState &S = states[p];
        if (S.phase == 2) continue;  // uniform: one value per workgroup
        const BProb &P = probs[p];
        const int n = P.n, ld = prm.ld, bc = S.bc, k = prm.k;
        const int f64 = (S.phase == 1 || prm.first_f64) ? 1 : 0;  // type of V and W in this phase
        const void *V = P.blk[BLK_V];
        const void *W = P.blk[BLK_W];
        // 1. G = V^T V, H = V^T W and their symmetric parts
        kb_gram(V, W, f64, n, ld, bc, sG, sH);
        for (int e = t; e < bc * bc; e += KB_NT) {
            const int i = e / bc, j = e - i * bc;
            if (i < j) {
                const double g = 0.5 * (sG[i][j] + sG[j][i]), hh = 0.5 * (sH[i][j] + sH[j][i]);
                sG[i][j] = g;
                sG[j][i] = g;
                sH[i][j] = hh;
                sH[j][i] = hh;
            }
        }
        __syncthreads();
        // 2. Cholesky G = L L^T (lane i of wave 0 owns row i)
        if (t < 64) {
            double dmax = 0.0;
            for (int i = 0; i < bc; ++i) dmax = fmax(dmax, sG[i][i]);
            const double floor_ = 1e-12 * dmax;
            bool ok = dmax > 0.0;
            for (int j = 0; j < bc && ok; ++j) {
                double d = sG[j][j];
                for (int l = 0; l < j; ++l) d = fma(-sL[j][l], sL[j][l], d);
                if (!(d > floor_)) {
                    ok = false;
                    break;
                }
                const double ljj = sqrt(d);
                if (t == j) sL[j][j] = ljj;
                if (t > j && t < bc) {
                    double v = sG[t][j];
                    for (int l = 0; l < j; ++l) v = fma(-sL[t][l], sL[j][l], v);
                    sL[t][j] = v / ljj;
                }
                if (t < j) sL[t][j] = 0.0;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (t == 0) s_chol_ok = ok ? 1 : 0;
        }
        __syncthreads();
        int rank = bc;
        if (s_chol_ok) {
            // C = L^{-1} H L^{-T}: column c of T = L^{-1} H (thread c) into
            // sC, then column c of C = L^{-1} (row c of T) into sZ
            if (t < bc) {
                const int c = t;
                for (int i = 0; i < bc; ++i) {
                    double v = sH[i][c];
                    for (int l = 0; l < i; ++l) v = fma(-sL[i][l], sC[l][c], v);
                    sC[i][c] = v / sL[i][i];
                }
            }
            __syncthreads();
            if (t < bc) {
                const int c = t;
                for (int i = 0; i < bc; ++i) {
                    double v = sC[c][i];
                    for (int l = 0; l < i; ++l) v = fma(-sL[i][l], sZ[l][c], v);
                    sZ[i][c] = v / sL[i][i];
                }
            }
            __syncthreads();
            for (int e = t; e < bc * bc; e += KB_NT) {
                const int i = e / bc, j = e - i * bc;
                sC[i][j] = 0.5 * (sZ[i][j] + sZ[j][i]);
            }
            __syncthreads();
            kb_jacobi(sC, sZ, bc, cs_c, cs_s, pp, pq, red, &s_go);
            // Y = L^{-T} Z (thread c: back substitution on column c)
            if (t < bc) {
                const int c = t;
                for (int i = bc - 1; i >= 0; --i) {
                    double v = sZ[i][c];
                    for (int l = i + 1; l < bc; ++l) v = fma(-sL[l][i], sY[l][c], v);
                    sY[i][c] = v / sL[i][i];
                }
            }
            if (t < bc) s_th[t] = sC[t][t];
            __syncthreads();
        } else {
            // G-eigen truncation: G = U D U^T, keep d_i > 1e-14 d_max,
            // S = U_r D_r^{-1/2}, C = S^T H S, Y = S Z
            for (int e = t; e < bc * bc; e += KB_NT) {
                const int i = e / bc, j = e - i * bc;
                sC[i][j] = sG[i][j];
            }
            __syncthreads();
            kb_jacobi(sC, sZ, bc, cs_c, cs_s, pp, pq, red, &s_go);
            if (t == 0) {
                double dmax = 0.0;
                for (int i = 0; i < bc; ++i) dmax = fmax(dmax, sC[i][i]);
                int r = 0;
                for (int i = 0; i < bc; ++i)
                    if (sC[i][i] > 1e-14 * dmax) s_perm[r++] = i;
                s_rank = r;
            }
            __syncthreads();
            rank = s_rank;
            for (int e = t; e < bc * rank; e += KB_NT) {
                const int i = e / rank, c = e - i * rank;
                const int src = s_perm[c];
                sL[i][c] = sZ[i][src] / sqrt(sC[src][src]);
            }
            __syncthreads();
            for (int e = t; e < bc * rank; e += KB_NT) {
                const int i = e / rank, c = e - i * rank;
                double v = 0.0;
                for (int l = 0; l < bc; ++l) v = fma(sH[i][l], sL[l][c], v);
                sY[i][c] = v;
            }
            __syncthreads();
            for (int e = t; e < rank * rank; e += KB_NT) {
                const int i = e / rank, c = e - i * rank;
                double v = 0.0;
                for (int l = 0; l < bc; ++l) v = fma(sL[l][i], sY[l][c], v);
                sZ[i][c] = v;
            }
            __syncthreads();
            for (int e = t; e < rank * rank; e += KB_NT) {
                const int i = e / rank, j = e - i * rank;
                sC[i][j] = 0.5 * (sZ[i][j] + sZ[j][i]);
            }
            __syncthreads();
            kb_jacobi(sC, sZ, rank, cs_c, cs_s, pp, pq, red, &s_go);
            for (int e = t; e < bc * rank; e += KB_NT) {
                const int i = e / rank, c = e - i * rank;
                double v = 0.0;
                for (int l = 0; l < rank; ++l) v = fma(sL[i][l], sZ[l][c], v);
                sY[i][c] = v;
            }
            if (t < rank) s_th[t] = sC[t][t];
            __syncthreads();
        }
        // order: descending (largest) or ascending (smallest), ties by index
        if (t < rank) {
            const double v = s_th[t];
            int pos = 0;
            for (int j = 0; j < rank; ++j) {
                const double u = s_th[j];
                const bool before = prm.smallest ? (u < v || (u == v && j < t)) : (u > v || (u == v && j < t));
                pos += before ? 1 : 0;
            }
            s_perm[pos] = t;
        }
        __syncthreads();
        for (int e = t; e < bc * rank; e += KB_NT) {
            const int i = e / rank, c = e - i * rank;
            sZ[i][c] = sY[i][s_perm[c]];
        }
        if (t < rank) {
            P.theta[t] = s_th[s_perm[t]];
            s_ths[t] = s_th[s_perm[t]];
        }
        __syncthreads();
        double anorm = prm.anorm_fixed;
        if (!(anorm > 0.0)) {
            anorm = 0.0;
            for (int i = 0; i < rank; ++i) anorm = fmax(anorm, fabs(s_th[i]));
            if (!(anorm > 0.0)) anorm = 1.0;
        }
        // 3. lift X = V Y, A X = W Y (every Ritz vector, the restart block),
        // then the residual sums of the k wanted pairs
        void *Xo = P.blk[BLK_X];
        void *AXo = P.blk[BLK_AX];
        if (bc <= 16)
            kb_lift_rows<16>(V, W, Xo, AXo, f64, n, ld, bc, rank, sZ);
        else
            kb_lift_rows<KB_BMAX>(V, W, Xo, AXo, f64, n, ld, bc, rank, sZ);
        __syncthreads();
        kb_resid_rows(Xo, AXo, f64, n, ld, k, 0, s_ths, s_res2, s_xn2);
        if (k > 16) kb_resid_rows(Xo, AXo, f64, n, ld, k, 16, s_ths, s_res2, s_xn2);
        __syncthreads();
        // 4. bookkeeping (one thread)
        if (t == 0) {
            S.xf64 = f64;
            S.products += 1;
            S.anorm = anorm;
            double emax = 0.0;
            bool finite = true;
            for (int c = 0; c < k; ++c) {
                double a = 0.0, b = 0.0;
                for (int i = 0; i < KB_NT / 64; ++i) {
                    a += s_res2[i][c];
                    b += s_xn2[i][c];
                }
                const double est = sqrt(a) / (b > 0.0 ? sqrt(b) : 1.0) / anorm;
                if (!(est == est) || isinf(est)) finite = false;
                emax = fmax(emax, est);
            }
            S.emax = emax;
            S.iters += 1;
            if (S.phase == 0) S.iters_low += 1;
            S.bc = rank;
            const bool last = S.phase == 1 || !prm.has_tail;
            if (!finite || rank < k) {
                S.status = OFRR_ERR_NUMERIC;
                S.phase = 2;
            } else if (last && prm.tol > 0.0 && emax <= prm.tol) {
                S.phase = 2;
            } else if (S.iters >= prm.max_iters) {
                S.phase = 2;
            } else if (!last) {
                // stall test: the smallest of the last `window` values is not
                // 10% below the smallest before them
                const int wdw = prm.window;
                if (S.nhist >= wdw) S.min_before = fmin(S.min_before, S.ring[S.nhist % wdw]);
                S.ring[S.nhist % wdw] = emax;
                S.nhist += 1;
                bool stalled = false;
                if (S.nhist > wdw) {
                    double recent = INFINITY;
                    for (int i = 0; i < wdw; ++i) recent = fmin(recent, S.ring[i]);
                    stalled = !(recent < 0.9 * S.min_before);
                }
                const bool by_value = prm.switch_resid > 0.0 && emax <= prm.switch_resid;
                if (stalled || by_value) {
                    S.phase = 1;
                    S.nhist = 0;
                    S.min_before = INFINITY;
                }
            }
        }
        __syncthreads();
    }
}

// Work lists of the unconverged problems (one workgroup): the active list
// and the (problem, row tile) items of the reduced and the FP64 products.
// counts: [0] active problems, [1] reduced items, [2] FP64 items,
// [3] all-problem items (final product), [4] problems with an error.
__global__ __launch_bounds__(KB_NT) void kb_lists(const BProb *probs, const BState *states, int nprob,
                                                  int rows_red, int rows_f64, int first_f64, int32_t *active,
                                                  int2 *items_red, int2 *items_f64, int32_t *counts) {
    __shared__ int s_tot[3];
    __shared__ int s_scan[3][KB_NT];
    const int t = threadIdx.x;
    if (t < 3) s_tot[t] = 0;
    __syncthreads();
    for (int base = 0; base < nprob; base += KB_NT) {
        const int p = base + t;
        int act = 0, tr = 0, tf = 0;
        if (p < nprob) {
            const int ph = states[p].phase;
            if (ph != 2) {
                act = 1;
                const int n = probs[p].n;
                if (ph == 1 || first_f64)
                    tf = (n + rows_f64 - 1) / rows_f64;
                else
                    tr = (n + rows_red - 1) / rows_red;
            }
        }
        s_scan[0][t] = act;
        s_scan[1][t] = tr;
        s_scan[2][t] = tf;
        __syncthreads();
        // inclusive scans (Hillis-Steele)
        for (int o = 1; o < KB_NT; o <<= 1) {
            int v0 = 0, v1 = 0, v2 = 0;
            if (t >= o) {
                v0 = s_scan[0][t - o];
                v1 = s_scan[1][t - o];
                v2 = s_scan[2][t - o];
            }
            __syncthreads();
            s_scan[0][t] += v0;
            s_scan[1][t] += v1;
            s_scan[2][t] += v2;
            __syncthreads();
        }
        const int o0 = s_tot[0] + s_scan[0][t] - act;
        const int o1 = s_tot[1] + s_scan[1][t] - tr;
        const int o2 = s_tot[2] + s_scan[2][t] - tf;
        if (act) active[o0] = p;
        for (int i = 0; i < tr; ++i) items_red[o1 + i] = make_int2(p, i);
        for (int i = 0; i < tf; ++i) items_f64[o2 + i] = make_int2(p, i);
        __syncthreads();
        if (t == KB_NT - 1) {
            s_tot[0] += s_scan[0][t];
            s_tot[1] += s_scan[1][t];
            s_tot[2] += s_scan[2][t];
        }
        __syncthreads();
    }
    if (t == 0) {
        counts[0] = s_tot[0];
        counts[1] = s_tot[1];
        counts[2] = s_tot[2];
        int bad = 0;
        for (int p = 0; p < nprob; ++p) bad += states[p].status != 0 ? 1 : 0;
        counts[4] = bad;
    }
}

// ------------------------------------------------------------ set-up / end

// Reduced copy of every problem's A (BF16/F16, column-major, zero-padded
// to ldr rows); one workgroup per (problem, 8 columns).
__global__ __launch_bounds__(KB_NT) void kb_cast_a(const BProb *probs, const int64_t *col_start, int nprob,
                                                   int64_t total_groups, int bf16) {
    for (int64_t gi = blockIdx.x; gi < total_groups; gi += gridDim.x) {
        // problem of this group: the last p with col_start[p] <= gi
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (col_start[mid] <= gi) lo = mid;
            else hi = mid - 1;
        }
        const BProb &P = probs[lo];
        const int64_t c0 = (gi - col_start[lo]) * 8;
        uint16_t *dst = const_cast<uint16_t *>(P.Alo);
        for (int cc = 0; cc < 8; ++cc) {
            const int64_t c = c0 + cc;
            if (c >= P.n) break;
            for (int64_t r = threadIdx.x; r < P.ldr; r += KB_NT) {
                float v = 0.f;
                if (r < P.n)
                    v = P.a_f64 ? (float)static_cast<const double *>(P.A)[r + c * P.lda]
                                : static_cast<const float *>(P.A)[r + c * P.lda];
                dst[r + c * P.ldr] = bits_red(v, bf16);
            }
        }
    }
}

// X (row-major master of the first phase) and, for a reduced first phase,
// the operand Vt from the caller's start block (column-major FP64, ld n);
// the padded rows of Vt are cleared.  One workgroup per problem.
__global__ __launch_bounds__(KB_NT) void kb_init_x(const BProb *probs, const double *const *x0, int nprob,
                                                   int b, int ld, int first_f64, int bf16) {
    for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
        const BProb &P = probs[p];
        const double *src = x0[p];
        for (int64_t e = threadIdx.x; e < (int64_t)P.n * b; e += KB_NT) {
            const int64_t r = e / b;
            const int c = (int)(e - r * b);
            const double v = src[r + (int64_t)c * P.n];
            store_blk(P.blk[BLK_X], r * ld + c, first_f64, v);
            if (!first_f64) P.Vt[(int64_t)c * P.ldr + r] = bits_red((float)v, bf16);
        }
        if (!first_f64)
            for (int64_t e = threadIdx.x; e < (int64_t)ld * (P.ldr - P.n); e += KB_NT) {
                const int64_t c = e / (P.ldr - P.n), r = P.n + (e - c * (P.ldr - P.n));
                P.Vt[c * P.ldr + r] = 0;
            }
    }
}

// Initial states: phase 0, basis b, stall detector empty.
__global__ void kb_init_states(BState *states, int nprob, int b) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nprob; p += gridDim.x * blockDim.x) {
        BState s;
        s.phase = 0;
        s.xf64 = 0;
        s.bc = b;
        s.iters = s.iters_low = s.products = 0;
        s.status = 0;
        s.nhist = 0;
        s.min_before = INFINITY;
        for (int i = 0; i < KB_WIN; ++i) s.ring[i] = 0.0;
        s.anorm = 0.0;
        s.emax = 0.0;
        states[p] = s;
    }
}

// The first product's output type: A X of the first phase is the master
// type (FP32 reduced, FP64 for the FP64 form); the state records it.
__global__ void kb_set_xf64(BState *states, int nprob, int f64) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nprob; p += gridDim.x * blockDim.x)
        states[p].xf64 = f64;
}

// Xf (FP64, row-major n x k) from X in its stored type; every problem.
__global__ __launch_bounds__(KB_NT) void kb_final_prep(const BProb *probs, const BState *states, int nprob,
                                                       int k, int ld) {
    for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
        const BProb &P = probs[p];
        const int xf = states[p].xf64;
        double *Xf = static_cast<double *>(P.blk[BLK_XF]);
        for (int64_t e = threadIdx.x; e < (int64_t)P.n * k; e += KB_NT) {
            const int64_t r = e / k;
            const int c = (int)(e - r * k);
            Xf[e] = load_blk(P.blk[BLK_X], r * ld + c, xf);
        }
    }
}

// Final FP64 residuals from A as stored: per column the norm of X, of
// A X - theta X and the sign rule (largest |x|, first index on ties, made
// positive); outputs are unit columns (column-major), eigenvalues and
// ||A x - theta x|| / (||x|| anorm).  One workgroup per problem.
__global__ __launch_bounds__(KB_NT) void kb_finalize(const BProb *probs, const BState *states, int nprob,
                                                     int k, double anorm_fixed) {
    __shared__ double red[KB_NT / 64];
    __shared__ int redi[KB_NT / 64];
    for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
        const BProb &P = probs[p];
        const int n = P.n;
        const double *Xf = static_cast<const double *>(P.blk[BLK_XF]);
        const double *AXf = static_cast<const double *>(P.blk[BLK_AXF]);
        double anorm = anorm_fixed > 0.0 ? anorm_fixed : states[p].anorm;
        if (!(anorm > 0.0)) anorm = 1.0;
        for (int c = 0; c < k; ++c) {
            const double th = P.theta[c];
            double sx = 0.0, sr = 0.0, best = -1.0;
            int bi = 0x7fffffff;
            for (int r = threadIdx.x; r < n; r += KB_NT) {
                const double x = Xf[(int64_t)r * k + c];
                const double d = AXf[(int64_t)r * k + c] - th * x;
                sx = fma(x, x, sx);
                sr = fma(d, d, sr);
                if (fabs(x) > best) {
                    best = fabs(x);
                    bi = r;
                }
            }
            kb_block_argmax(best, bi, red, redi);
            double tx = sx, tr = sr;
            for (int o = 32; o > 0; o >>= 1) {
                tx += __shfl_xor(tx, o, 64);
                tr += __shfl_xor(tr, o, 64);
            }
            __shared__ double s_tx[KB_NT / 64], s_tr[KB_NT / 64];
            if ((threadIdx.x & 63) == 0) {
                s_tx[threadIdx.x >> 6] = tx;
                s_tr[threadIdx.x >> 6] = tr;
            }
            __syncthreads();
            double ax = 0.0, ar = 0.0;
            for (int i = 0; i < KB_NT / 64; ++i) {
                ax += s_tx[i];
                ar += s_tr[i];
            }
            const double nx = ax > 0.0 ? sqrt(ax) : 1.0;
            const double sgn = (bi < n && Xf[(int64_t)bi * k + c] < 0.0) ? -1.0 : 1.0;
            for (int r = threadIdx.x; r < n; r += KB_NT)
                P.evecs[(int64_t)r + (int64_t)c * n] = Xf[(int64_t)r * k + c] * (sgn / nx);
            if (threadIdx.x == 0) {
                P.evals[c] = th;
                P.resid[c] = sqrt(ar) / nx / anorm;
            }
            __syncthreads();
        }
    }
}

}  // namespace

// ======================================================================
// Host orchestration
// ======================================================================

namespace {

struct Tuned {
    int waves_red = 4;
    int waves_f64 = 4;
};

// the product launchers by variant
void launch_lp(int waves, bool bf16, hipStream_t st, int grid, const BProb *probs, const BState *states,
               const int2 *items, const int32_t *counts, int slot, int out_blk, int64_t ldw) {
#define KB_LP(W)                                                                                       \
    if (bf16)                                                                                          \
        hipLaunchKernelGGL((kb_product_lp<true, W>), dim3(grid), dim3(64 * W), 0, st, probs, states, items, \
                           counts, slot, out_blk, ldw);                                                \
    else                                                                                               \
        hipLaunchKernelGGL((kb_product_lp<false, W>), dim3(grid), dim3(64 * W), 0, st, probs, states, items, \
                           counts, slot, out_blk, ldw);
    if (waves == 2) {
        KB_LP(2)
    } else if (waves == 8) {
        KB_LP(8)
    } else {
        KB_LP(4)
    }
#undef KB_LP
}

void launch_f64(int waves, hipStream_t st, int grid, const BProb *probs, const BState *states, const int2 *items,
                const int32_t *counts, int slot, int in_blk, int out_blk, int64_t ldv, int64_t ldw, int ncols) {
    if (waves == 2)
        hipLaunchKernelGGL((kb_product_f64<2>), dim3(grid), dim3(128), 0, st, probs, states, items, counts, slot,
                           in_blk, out_blk, ldv, ldw, ncols);
    else if (waves == 8)
        hipLaunchKernelGGL((kb_product_f64<8>), dim3(grid), dim3(512), 0, st, probs, states, items, counts, slot,
                           in_blk, out_blk, ldv, ldw, ncols);
    else
        hipLaunchKernelGGL((kb_product_f64<4>), dim3(grid), dim3(256), 0, st, probs, states, items, counts, slot,
                           in_blk, out_blk, ldv, ldw, ncols);
}

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

}  // namespace

bool batched_grouped_supported(const ofrr_plan *plan, int32_t nprob, const ofrr_matrix *As, int32_t k,
                               int32_t basis) {
    if (basis > KB_BMAX || k > basis) return false;
    if (plan->stab != 0 || plan->projection != 0) return false;
    if (plan->degree != 1) return false;
    if (plan->refine > 1) return false;
    if (!(plan->basis_dtype == OFRR_BF16 || plan->basis_dtype == OFRR_F16 || plan->basis_dtype == OFRR_F64))
        return false;
    if (plan->gram_accum != OFRR_ACC_F64) return false;
    if (plan->refine && (plan->stall_iters < 1 || plan->stall_iters > KB_WIN)) return false;
    for (int32_t p = 0; p < nprob; ++p) {
        if (As[p].format != OFRR_DENSE_COLMAJOR) return false;
        if (As[p].rows > 0x3fffffff) return false;
    }
    return true;
}

ofrr_status batched_grouped_impl(Context *ctx, int32_t nprob, const ofrr_matrix *As, int32_t k, int32_t basis,
                                 ofrr_which which, const ofrr_plan *plan, const double *const *X0s,
                                 double *const *evals, double *const *evecs, double *const *resid,
                                 ofrr_info *infos) {
    const int ld = basis;
    const bool first_f64 = plan->basis_dtype == OFRR_F64;
    const bool bf16 = plan->basis_dtype != OFRR_F16;
    const hipStream_t st = ctx->stream;
    hipEvent_t ev0, ev1;
    OFRR_HIP(hipEventCreate(&ev0));
    OFRR_HIP(hipEventCreate(&ev1));
    OFRR_HIP(hipEventRecord(ev0, st));

    // ---- layout of the per-problem arena
    std::vector<BProb> hp((size_t)nprob);
    std::vector<int64_t> off_alo(nprob), off_vt(nprob), off_blk(nprob), off_th(nprob), off_x0(nprob);
    int64_t bytes = 0, nmax = 0;
    for (int p = 0; p < nprob; ++p) {
        const int64_t n = As[p].rows;
        nmax = std::max(nmax, n);
        const int64_t ldr = align_up(n, 16);
        if (!first_f64) {
            off_alo[p] = bytes;
            bytes += align_up(ldr * n * 2, 256);
            off_vt[p] = bytes;
            bytes += align_up(ldr * ld * 2, 256);
        }
        off_blk[p] = bytes;
        bytes += 5 * align_up(n * ld * 8, 256) + 2 * align_up(n * k * 8, 256);
        off_th[p] = bytes;
        bytes += align_up((int64_t)ld * 8, 256);
        if (!X0s || !X0s[p]) {
            off_x0[p] = bytes;
            bytes += align_up(n * ld * 8, 256);
        } else {
            off_x0[p] = -1;
        }
    }
    char *arena = ctx->buf<char>("batched_arena", (size_t)bytes);
    std::vector<const double *> x0p((size_t)nprob);
    for (int p = 0; p < nprob; ++p) {
        BProb &P = hp[p];
        const int64_t n = As[p].rows;
        P.A = As[p].values;
        P.lda = As[p].ld;
        P.n = (int32_t)n;
        P.a_f64 = As[p].dtype == OFRR_F64 ? 1 : 0;
        P.ldr = align_up(n, 16);
        P.Alo = first_f64 ? nullptr : reinterpret_cast<const uint16_t *>(arena + off_alo[p]);
        P.Vt = first_f64 ? nullptr : reinterpret_cast<uint16_t *>(arena + off_vt[p]);
        char *b = arena + off_blk[p];
        for (int i = 0; i < 5; ++i) P.blk[i] = b + i * align_up(n * ld * 8, 256);
        P.blk[BLK_XF] = b + 5 * align_up(n * ld * 8, 256);
        P.blk[BLK_AXF] = b + 5 * align_up(n * ld * 8, 256) + align_up(n * k * 8, 256);
        P.theta = reinterpret_cast<double *>(arena + off_th[p]);
        P.evals = evals[p];
        P.evecs = evecs[p];
        P.resid = resid[p];
        if (off_x0[p] >= 0) {
            double *g = reinterpret_cast<double *>(arena + off_x0[p]);
            uniform_start(ctx, n, basis, 0x5EEDull, g);
            x0p[p] = g;
        } else {
            x0p[p] = X0s[p];
        }
    }
    // device copies of the descriptors, states, lists
    int64_t total_red_items = 0, total_f64_items = 0;
    // tile heights are at least 64 rows: item lists sized for that
    for (int p = 0; p < nprob; ++p) {
        total_red_items += (hp[p].n + 63) / 64;
        total_f64_items += (hp[p].n + 63) / 64;
    }
    BProb *d_probs = ctx->buf<BProb>("batched_probs", (size_t)nprob);
    BState *d_states = ctx->buf<BState>("batched_states", (size_t)nprob);
    int32_t *d_active = ctx->buf<int32_t>("batched_active", (size_t)nprob);
    int2 *d_items_red = ctx->buf<int2>("batched_items_red", (size_t)total_red_items + 1);
    int2 *d_items_f64 = ctx->buf<int2>("batched_items_f64", (size_t)total_f64_items + 1);
    int32_t *d_counts = ctx->buf<int32_t>("batched_counts", 8);
    const double **d_x0 = ctx->buf<const double *>("batched_x0", (size_t)nprob);
    int64_t *d_colstart = ctx->buf<int64_t>("batched_colstart", (size_t)nprob + 1);
    std::vector<int64_t> colstart((size_t)nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) colstart[p + 1] = colstart[p] + (hp[p].n + 7) / 8;
    OFRR_HIP(hipMemcpyAsync(d_probs, hp.data(), sizeof(BProb) * nprob, hipMemcpyHostToDevice, st));
    OFRR_HIP(hipMemcpyAsync(d_x0, x0p.data(), sizeof(double *) * nprob, hipMemcpyHostToDevice, st));
    OFRR_HIP(hipMemcpyAsync(d_colstart, colstart.data(), sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice, st));

    BParams prm{};
    prm.nprob = nprob;
    prm.k = k;
    prm.ld = ld;
    prm.smallest = which == OFRR_SMALLEST ? 1 : 0;
    prm.max_iters = plan->max_iters;
    prm.window = std::max(1, std::min(plan->stall_iters, KB_WIN));
    prm.has_tail = (plan->refine && !first_f64) ? 1 : 0;
    prm.first_f64 = first_f64 ? 1 : 0;
    prm.red_bf16 = bf16 ? 1 : 0;
    if (plan->filter == OFRR_CHEBYSHEV) {
        const double c = 0.5 * (plan->hi + plan->lo), e = 0.5 * (plan->hi - plan->lo);
        prm.alpha = 1.0 / e;
        prm.cshift = c;
    } else {
        prm.alpha = 1.0;
        prm.cshift = 0.0;
    }
    prm.tol = plan->tol;
    prm.switch_resid = plan->switch_resid;
    prm.anorm_fixed = plan->anorm;
    prm.drop_red = plan->drop_tol > 0 ? plan->drop_tol : std::ldexp(1.0, -23);
    prm.drop_f64 = plan->drop_tol > 0 ? plan->drop_tol : std::ldexp(1.0, -52);

    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    const int grid_prob = std::min(nprob, 2 * cus);
    const int grid_prod = 4 * cus;

    // ---- set-up: reduced copies of A, start blocks, states
    hipLaunchKernelGGL(kb_init_states, dim3((nprob + 255) / 256), dim3(256), 0, st, d_states, nprob, basis);
    if (!first_f64)
        hipLaunchKernelGGL(kb_cast_a, dim3((unsigned)std::min<int64_t>(colstart[nprob], 16 * cus)), dim3(KB_NT), 0,
                           st, d_probs, d_colstart, nprob, colstart[nprob], bf16 ? 1 : 0);
    hipLaunchKernelGGL(kb_init_x, dim3(grid_prob), dim3(KB_NT), 0, st, d_probs, d_x0, nprob, basis, ld,
                       first_f64 ? 1 : 0, bf16 ? 1 : 0);
    OFRR_HIP(hipGetLastError());

    // ---- autotuned tile heights (per context, keyed by the product kind,
    // basis width and the size mix): every candidate runs the first
    // product A X once, timed with events; the product is idempotent and
    // every candidate computes the same sums in the same order
    auto lists = [&](int rows_red, int rows_f64, hipStream_t s) {
        hipLaunchKernelGGL(kb_lists, dim3(1), dim3(KB_NT), 0, s, d_probs, d_states, nprob, rows_red, rows_f64,
                           first_f64 ? 1 : 0, d_active, d_items_red, d_items_f64, d_counts);
    };
    auto &tune_cache = ctx->batched_tune;
    char keybuf[128];
    std::snprintf(keybuf, sizeof keybuf, "%s:b%d:p%d:n%lld", first_f64 ? "f64" : (bf16 ? "bf16" : "f16"), ld,
                  nprob, (long long)nmax);
    const std::string key(keybuf);
    Tuned tuned;
    auto it = tune_cache.find(key);
    const int cand[3] = {2, 4, 8};
    if (it == tune_cache.end()) {
        hipEvent_t a, b;
        OFRR_HIP(hipEventCreate(&a));
        OFRR_HIP(hipEventCreate(&b));
        float best_red = 1e30f, best_f64 = 1e30f;
        for (int c : cand) {
            lists(32 * c, 32 * c, st);
            if (!first_f64) {
                OFRR_HIP(hipEventRecord(a, st));
                launch_lp(c, bf16, st, grid_prod, d_probs, d_states, d_items_red, d_counts, 1, BLK_AX, ld);
                OFRR_HIP(hipEventRecord(b, st));
                OFRR_HIP(hipEventSynchronize(b));
                float ms = 0.f;
                OFRR_HIP(hipEventElapsedTime(&ms, a, b));
                if (ms < best_red) {
                    best_red = ms;
                    tuned.waves_red = c;
                }
            }
            // the FP64 product on every problem (a scratch output: Y)
            hipLaunchKernelGGL(kb_lists, dim3(1), dim3(KB_NT), 0, st, d_probs, d_states, nprob, 32 * c, 32 * c, 1,
                               d_active, d_items_red, d_items_f64, d_counts);
            OFRR_HIP(hipEventRecord(a, st));
            launch_f64(c, st, grid_prod, d_probs, d_states, d_items_f64, d_counts, 2, first_f64 ? BLK_X : BLK_W,
                       first_f64 ? BLK_AX : BLK_Y, ld, ld, 0);
            OFRR_HIP(hipEventRecord(b, st));
            OFRR_HIP(hipEventSynchronize(b));
            float ms = 0.f;
            OFRR_HIP(hipEventElapsedTime(&ms, a, b));
            if (ms < best_f64) {
                best_f64 = ms;
                tuned.waves_f64 = c;
            }
        }
        OFRR_HIP(hipGetLastError());
        OFRR_HIP(hipEventDestroy(a));
        OFRR_HIP(hipEventDestroy(b));
        tune_cache[key] = std::make_pair(tuned.waves_red, tuned.waves_f64);
    } else {
        tuned.waves_red = it->second.first;
        tuned.waves_f64 = it->second.second;
    }
    const int rows_red = 32 * tuned.waves_red, rows_f64 = 32 * tuned.waves_f64;

    // ---- first product A X (the first filter step of iteration 1), timed
    // with events on the stream (every problem in the first phase: the
    // grouped product's rate over the whole set)
    lists(rows_red, rows_f64, st);
    hipEvent_t pa, pb;
    OFRR_HIP(hipEventCreate(&pa));
    OFRR_HIP(hipEventCreate(&pb));
    OFRR_HIP(hipEventRecord(pa, st));
    if (first_f64)
        launch_f64(tuned.waves_f64, st, grid_prod, d_probs, d_states, d_items_f64, d_counts, 2, BLK_X, BLK_AX, ld, ld,
                   0);
    else
        launch_lp(tuned.waves_red, bf16, st, grid_prod, d_probs, d_states, d_items_red, d_counts, 1, BLK_AX, ld);
    OFRR_HIP(hipEventRecord(pb, st));
    hipLaunchKernelGGL(kb_set_xf64, dim3((nprob + 255) / 256), dim3(256), 0, st, d_states, nprob, first_f64 ? 1 : 0);
    OFRR_HIP(hipGetLastError());

    // ---- one outer iteration, captured once and replayed
    if (!ctx->graph_stream) OFRR_HIP(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
    const hipStream_t gs = ctx->graph_stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    OFRR_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(kb_stabilise, dim3(grid_prob), dim3(KB_NT), 0, gs, d_probs, d_states, prm, d_active, d_counts);
    if (!first_f64)
        launch_lp(tuned.waves_red, bf16, gs, grid_prod, d_probs, d_states, d_items_red, d_counts, 1, BLK_W, ld);
    launch_f64(tuned.waves_f64, gs, grid_prod, d_probs, d_states, d_items_f64, d_counts, 2, BLK_V, BLK_W, ld, ld, 0);
    hipLaunchKernelGGL(kb_psl, dim3(grid_prob), dim3(KB_NT), 0, gs, d_probs, d_states, prm, d_active, d_counts);
    hipLaunchKernelGGL(kb_lists, dim3(1), dim3(KB_NT), 0, gs, d_probs, d_states, nprob, rows_red, rows_f64,
                       first_f64 ? 1 : 0, d_active, d_items_red, d_items_f64, d_counts);
    const hipError_t cap_err = hipGetLastError();
    const hipError_t end_err = hipStreamEndCapture(gs, &graph);
    OFRR_HIP(cap_err);
    OFRR_HIP(end_err);
    {
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            OFRR_HIP(e);
        }
    }
    // replays until every problem has finished (each problem stops at its own
    // iteration cap); the host looks every `per_check` replays
    int32_t *hc = ctx->host_stage<int32_t>(8);
    const int per_check = 2;
    int replays = 0;
    hipError_t loop_err = hipSuccess;
    for (;;) {
        for (int r = 0; r < per_check; ++r) {
            loop_err = hipGraphLaunch(exec, st);
            if (loop_err != hipSuccess) break;
            ++replays;
        }
        if (loop_err != hipSuccess) break;
        loop_err = hipMemcpyAsync(hc, d_counts, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (loop_err != hipSuccess) break;
        loop_err = hipStreamSynchronize(st);
        if (loop_err != hipSuccess) break;
        if (hc[0] == 0 || replays > plan->max_iters + per_check) break;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    OFRR_HIP(loop_err);

    // ---- final FP64 residuals from A as stored
    hipLaunchKernelGGL(kb_final_prep, dim3(grid_prob), dim3(KB_NT), 0, st, d_probs, d_states, nprob, k, ld);
    // every problem's FP64 items: lists built as if all were in the FP64 phase
    {
        // all problems: reuse kb_lists on a state copy marked FP64 is not
        // possible (states are final), so build the items on the host
        std::vector<int2> items;
        for (int p = 0; p < nprob; ++p)
            for (int i = 0; i < (hp[p].n + rows_f64 - 1) / rows_f64; ++i) items.push_back(make_int2(p, i));
        int2 *d_items_all = ctx->buf<int2>("batched_items_all", items.size() + 1);
        OFRR_HIP(hipMemcpyAsync(d_items_all, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, st));
        hc[3] = (int32_t)items.size();
        OFRR_HIP(hipMemcpyAsync(d_counts + 3, hc + 3, sizeof(int32_t), hipMemcpyHostToDevice, st));
        launch_f64(tuned.waves_f64, st, grid_prod, d_probs, d_states, d_items_all, d_counts, 3, BLK_XF, BLK_AXF, k, k,
                   k);
        OFRR_HIP(hipStreamSynchronize(st));  // the host items must outlive the copy
    }
    hipLaunchKernelGGL(kb_finalize, dim3(grid_prob), dim3(KB_NT), 0, st, d_probs, d_states, nprob, k, plan->anorm);
    OFRR_HIP(hipGetLastError());
    OFRR_HIP(hipEventRecord(ev1, st));
    std::vector<BState> hs((size_t)nprob);
    OFRR_HIP(hipMemcpyAsync(hs.data(), d_states, sizeof(BState) * nprob, hipMemcpyDeviceToHost, st));
    OFRR_HIP(hipStreamSynchronize(st));
    float ms = 0.f, pms = 0.f;
    OFRR_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    OFRR_HIP(hipEventElapsedTime(&pms, pa, pb));
    OFRR_HIP(hipEventDestroy(ev0));
    OFRR_HIP(hipEventDestroy(ev1));
    OFRR_HIP(hipEventDestroy(pa));
    OFRR_HIP(hipEventDestroy(pb));
    ctx->batched_last_first_ms = pms;
    ctx->batched_last_replays = replays;
    ctx->batched_last_waves[0] = tuned.waves_red;
    ctx->batched_last_waves[1] = tuned.waves_f64;

    // per-problem results
    ofrr_status worst = OFRR_OK;
    std::vector<double> rr((size_t)k);
    for (int p = 0; p < nprob; ++p) {
        if (hs[p].status != 0) {
            worst = (ofrr_status)hs[p].status;
            continue;
        }
        OFRR_HIP(hipMemcpy(rr.data(), resid[p], sizeof(double) * k, hipMemcpyDeviceToHost));
        int nconv = 0;
        double rmax = 0.0;
        for (double v : rr) {
            rmax = std::max(rmax, v);
            if (plan->tol > 0 ? v <= plan->tol : true) ++nconv;
        }
        if (infos) {
            ofrr_info &I = infos[p];
            I.iters = hs[p].iters;
            I.iters_low = first_f64 ? 0 : hs[p].iters_low;
            I.n_converged = nconv;
            I.basis_eff = hs[p].bc;
            I.products = hs[p].products + 2;  // + the first and the final product
            I.max_resid = rmax;
            I.seconds = ms * 1e-3;
            I.gram_t_max = 0.0;
            I.grams_f64 = 0;
        }
        if (plan->tol > 0 && nconv < k && worst == OFRR_OK) worst = OFRR_NOT_CONVERGED;
    }
    if (worst < 0) fail(worst, "batched: a problem failed (non-finite values or the basis lost rank below k)");
    return worst;
}

}  // namespace ofrr
