// k_basis.hip -- the basis-generation processes compared in Sec. 4.2 (the
// comparison table of MGS, CGS and the Hessenberg process) and timed in
// Sec. 5.3 (Table 3): left- and right-looking modified Gram-Schmidt
// without re-orthogonalisation, classical Gram-Schmidt, CGS with one re-
// orthogonalisation, and the left- and right-looking Hessenberg process,
// on a dense column-major m x n block in FP64, FP32, or binary16 storage
// with FP32 arithmetic (the paper's FP16 runs).
//
// Each process is one cooperative launch: every workgroup owns a
// contiguous slice of rows and keeps it for the whole process, so column
// updates never leave the workgroup; the steps that need a value from the
// whole column (an inner product, a pivot search, a pivot row) exchange
// per-workgroup partials through global memory across a grid barrier.
// The number of barriers is the method's own: one per inner product for
// left-looking MGS, one per projection for left-looking Hessenberg, two or
// three per column for the right-looking and classical forms.
// In binary16 storage every stored result is rounded to binary16 (as the
// oracle's FP16 Hessenberg rounds every quotient and every update); inner
// products accumulate in FP32.
#include <cmath>
#include <string>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

constexpr int BG_NT = 256;
constexpr int BG_NMAX = 512;

// storage policies: S the stored type, C the arithmetic type
template <class S>
struct Sto;
template <>
struct Sto<double> {
    using C = double;
    static __device__ __forceinline__ C ld(const double *p) { return *p; }
    static __device__ __forceinline__ void st(double *p, C v) { *p = v; }
    static __device__ __forceinline__ C rnd(C v) { return v; }
};
template <>
struct Sto<float> {
    using C = float;
    static __device__ __forceinline__ C ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, C v) { *p = v; }
    static __device__ __forceinline__ C rnd(C v) { return v; }
};
template <>
struct Sto<f16_t> {
    using C = float;
    static __device__ __forceinline__ C ld(const f16_t *p) { return f16_bits_to_f32(p->bits); }
    static __device__ __forceinline__ void st(f16_t *p, C v) { p->bits = f32_to_f16_bits(v); }
    static __device__ __forceinline__ C rnd(C v) { return f16_bits_to_f32(f32_to_f16_bits(v)); }
};

enum { BM_MGS_L = 0, BM_MGS_R = 1, BM_CGS = 2, BM_CGS2 = 3, BM_HESS_L = 4, BM_HESS_R = 5, BM_MGS2 = 6 };

struct BGArgs {
    int64_t m, lda;
    int n;
    double tol;
    double *R;       // n x n column-major (upper triangle), may be null
    int32_t *piv, *keep, *kept;
    double *part;    // 2 x G x (n + 4) partials
    double *prow;    // published pivot-row entries (Hessenberg), 2 x G x (n + 4)
    unsigned *bar;   // barrier counter
    int *err;
};

struct BGShared {
    double red[BG_NT / 64];
    double vals[BG_NMAX];
    int ii[BG_NT / 64];
    double cand[3];
    int flag;
};

// block-wide sum (fixed order), the same value in every thread
__device__ double bg_block_sum(double v, BGShared &sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < BG_NT / 64; ++i) r += sh.red[i];
    __syncthreads();
    return r;
}

// sum over workgroups of the partial at slot `idx` of buffer `buf`, fixed
// order; every thread gets it (thread 0 reads, LDS broadcast)
__device__ double bg_total(const BGArgs &a, int buf, int idx, BGShared &sh) {
    const int G = gridDim.x, stride = a.n + 4;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += a.part[((int64_t)buf * G + g) * stride + idx];
        sh.vals[0] = s;
    }
    __syncthreads();
    const double r = sh.vals[0];
    __syncthreads();
    return r;
}

// totals of slots [lo, hi) into sh.vals (thread-strided), then a barrier
__device__ void bg_totals(const BGArgs &a, int buf, int lo, int hi, BGShared &sh) {
    const int G = gridDim.x, stride = a.n + 4;
    __syncthreads();
    for (int i = lo + (int)threadIdx.x; i < hi; i += BG_NT) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += a.part[((int64_t)buf * G + g) * stride + i];
        sh.vals[i] = s;
    }
    __syncthreads();
}

template <class S>
__global__ __launch_bounds__(BG_NT) void k_basis(S *A, BGArgs a, int method) {
    using P = Sto<S>;
    using C = typename P::C;
    __shared__ BGShared sh;
    const int t = threadIdx.x, G = gridDim.x, g = blockIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int64_t per = (a.m + G - 1) / G;
    const int64_t r0 = (int64_t)g * per;
    const int64_t r1 = r0 + per < a.m ? r0 + per : a.m;
    const int n = a.n, stride = n + 4;
    unsigned epoch = 0;
    int step = 0;
    auto col = [&](int j) { return A + (int64_t)j * a.lda; };
    auto part = [&](int buf) { return a.part + ((int64_t)buf * G + g) * stride; };
    auto barrier = [&]() -> bool { return grid_barrier(a.bar, (unsigned)G, epoch, a.err); };
    // this workgroup's share of x . y over its rows (C arithmetic)
    auto wg_dot = [&](const S *x, const S *y) -> double {
        C s = (C)0;
        for (int64_t r = r0 + t; r < r1; r += BG_NT) s = fma(P::ld(x + r), P::ld(y + r), s);
        return bg_block_sum((double)s, sh);
    };
    if (method == BM_MGS_L) {
        for (int j = 0; j < n; ++j) {
            S *v = col(j);
            for (int i = 0; i <= j; ++i) {
                // i < j: coefficient of q_i; i == j: the norm
                const S *q = i < j ? col(i) : v;
                const double p = wg_dot(q, v);
                const int buf = step & 1;
                if (t == 0) part(buf)[0] = p;
                if (!barrier()) return;
                ++step;
                const double tot = bg_total(a, buf, 0, sh);
                if (i < j) {
                    const C r = (C)tot;
                    for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, fma(-r, P::ld(q + e), P::ld(v + e)));
                    if (g == 0 && t == 0 && a.R) a.R[i + (int64_t)j * n] = (double)r;
                } else {
                    const C nr = (C)sqrt(tot);
                    for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, P::ld(v + e) / nr);
                    if (g == 0 && t == 0 && a.R) a.R[j + (int64_t)j * n] = (double)nr;
                }
                __syncthreads();
            }
        }
        return;
    }
    if (method == BM_MGS2) {
        // left-looking MGS with one more projection pass when the first
        // one reduced the column's norm below sqrt(2)/2 of its value before
        // (the re-orthogonalisation test of Sec. 5.1); the coefficients of
        // the second pass are added to R.  With tol > 0 a column whose norm
        // after the projections is at most tol times its norm before them is
        // excluded (keep = 0, left unnormalised, not projected out of later
        // columns): the exclusion of numerically dependent columns the
        // comparison of Sec. 5.4 applies to the QR bases as well
        __shared__ int s_kq[BG_NMAX];
        int kept = 0;
        auto norm_of = [&](const S *v) -> double {
            const double p = wg_dot(v, v);
            const int buf = step & 1;
            if (t == 0) part(buf)[0] = p;
            if (!barrier()) return -1.0;
            ++step;
            return sqrt(bg_total(a, buf, 0, sh));
        };
        for (int j = 0; j < n; ++j) {
            S *v = col(j);
            double before = norm_of(v);
            if (before < 0) return;
            const double orig = before;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i < j; ++i) {
                    if (!s_kq[i]) continue;  // the same decision in every workgroup
                    const S *q = col(i);
                    const double p = wg_dot(q, v);
                    const int buf = step & 1;
                    if (t == 0) part(buf)[0] = p;
                    if (!barrier()) return;
                    ++step;
                    const C r = (C)bg_total(a, buf, 0, sh);
                    for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, fma(-r, P::ld(q + e), P::ld(v + e)));
                    if (g == 0 && t == 0 && a.R) a.R[i + (int64_t)j * n] += (double)r;
                    __syncthreads();
                }
                const double after = norm_of(v);
                if (after < 0) return;
                if (pass == 0 && after < 0.70710678118654752440 * before) {
                    before = after;
                    continue;
                }
                const bool take = !(a.tol > 0.0) || after > a.tol * orig;
                if (t == 0) s_kq[j] = take ? 1 : 0;
                if (g == 0 && t == 0) {
                    a.keep[j] = take ? 1 : 0;
                    a.piv[j] = take ? j : -1;
                }
                if (take) {
                    ++kept;
                    const C nr = (C)after;
                    for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, P::ld(v + e) / nr);
                    if (g == 0 && t == 0 && a.R) a.R[j + (int64_t)j * n] = (double)nr;
                }
                __syncthreads();
                break;
            }
        }
        if (g == 0 && t == 0 && a.kept) *a.kept = kept;
        return;
    }
    if (method == BM_MGS_R) {
        for (int i = 0; i < n; ++i) {
            S *q = col(i);
            // norm of column i (every projection before it already applied)
            {
                const double p = wg_dot(q, q);
                const int buf = step & 1;
                if (t == 0) part(buf)[0] = p;
                if (!barrier()) return;
                ++step;
                const C nr = (C)sqrt(bg_total(a, buf, 0, sh));
                for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(q + e, P::ld(q + e) / nr);
                if (g == 0 && t == 0 && a.R) a.R[i + (int64_t)i * n] = (double)nr;
                __syncthreads();
            }
            if (i + 1 == n) break;
            // coefficients q_i . a_j of every later column: wave w takes
            // columns j = i + 1 + w, i + 1 + w + 4, ...; lanes split the rows
            const int buf = step & 1;
            for (int j = i + 1 + wave; j < n; j += BG_NT / 64) {
                const S *aj = col(j);
                C s = (C)0;
                for (int64_t r = r0 + lane; r < r1; r += 64) s = fma(P::ld(q + r), P::ld(aj + r), s);
                double d = (double)s;
                for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
                if (lane == 0) part(buf)[j] = d;
            }
            if (!barrier()) return;
            ++step;
            bg_totals(a, buf, i + 1, n, sh);
            for (int j = i + 1; j < n; ++j) {
                const C r = (C)sh.vals[j];
                S *aj = col(j);
                for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(aj + e, fma(-r, P::ld(q + e), P::ld(aj + e)));
                if (g == 0 && t == 0 && a.R) a.R[i + (int64_t)j * n] = (double)r;
            }
            __syncthreads();
        }
        return;
    }
    if (method == BM_CGS || method == BM_CGS2) {
        const int passes = method == BM_CGS2 ? 2 : 1;
        for (int j = 0; j < n; ++j) {
            S *v = col(j);
            for (int ps = 0; ps < passes && j > 0; ++ps) {
                // coefficients Q_{:, <j}^T v (wave per column, lanes over rows)
                const int buf = step & 1;
                for (int i = wave; i < j; i += BG_NT / 64) {
                    const S *q = col(i);
                    C s = (C)0;
                    for (int64_t r = r0 + lane; r < r1; r += 64) s = fma(P::ld(q + r), P::ld(v + r), s);
                    double d = (double)s;
                    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
                    if (lane == 0) part(buf)[i] = d;
                }
                if (!barrier()) return;
                ++step;
                bg_totals(a, buf, 0, j, sh);
                // v = v - Q r, accumulated per row in C, stored once
                for (int64_t e = r0 + t; e < r1; e += BG_NT) {
                    C acc = P::ld(v + e);
                    for (int i = 0; i < j; ++i) acc = fma(-(C)sh.vals[i], P::ld(col(i) + e), acc);
                    P::st(v + e, acc);
                }
                if (g == 0 && t == 0 && a.R)
                    for (int i = 0; i < j; ++i)
                        a.R[i + (int64_t)j * n] = (ps == 0 ? 0.0 : a.R[i + (int64_t)j * n]) + (double)(C)sh.vals[i];
                __syncthreads();
            }
            const double p = wg_dot(v, v);
            const int buf = step & 1;
            if (t == 0) part(buf)[0] = p;
            if (!barrier()) return;
            ++step;
            const C nr = (C)sqrt(bg_total(a, buf, 0, sh));
            for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, P::ld(v + e) / nr);
            if (g == 0 && t == 0 && a.R) a.R[j + (int64_t)j * n] = (double)nr;
            __syncthreads();
        }
        return;
    }
    // ---- Hessenberg process (Sec. 4.2): pivot = first row of largest
    // magnitude, column divided by it, its multiple removed from later
    // columns with one fused multiply-add per element (rounded to the
    // storage type), dropped when |pivot| < tol
    int kept = 0;
    const bool left = method == BM_HESS_L;
    // every workgroup takes the same pivot decisions from the same
    // candidates, so each keeps its own copy of them (the keep and pivot
    // arrays in global memory are written by workgroup 0 for the caller and
    // are not read back here: no barrier orders them)
    __shared__ int s_keep[BG_NMAX];
    __shared__ int64_t s_pivr[BG_NMAX];
    // pivot search over the WG's rows of column j: candidate (mag, row, value)
    auto search = [&](const S *v, double &bm, int64_t &bi, double &bv) {
        double m = -1.0, val = 0.0;
        int64_t ri = 0x7fffffff;
        for (int64_t e = r0 + t; e < r1; e += BG_NT) {
            const C x = P::ld(v + e);
            const double mg = fabs((double)x);
            if (mg > m) {
                m = mg;
                ri = e;
                val = (double)x;
            }
        }
        // wave then block argmax (larger magnitude, then smaller row)
        for (int o = 32; o > 0; o >>= 1) {
            const double qm = __shfl_xor(m, o, 64);
            const int64_t qr = __shfl_xor(ri, o, 64);
            const double qv = __shfl_xor(val, o, 64);
            if (qm > m || (qm == m && qr < ri)) {
                m = qm;
                ri = qr;
                val = qv;
            }
        }
        __syncthreads();
        if (lane == 0) {
            sh.red[wave] = m;
            sh.vals[2 * wave] = (double)ri;
            sh.vals[2 * wave + 1] = val;
        }
        __syncthreads();
        bm = sh.red[0];
        bi = (int64_t)sh.vals[0];
        bv = sh.vals[1];
        for (int w = 1; w < BG_NT / 64; ++w) {
            const double qm = sh.red[w];
            const int64_t qr = (int64_t)sh.vals[2 * w];
            if (qm > bm || (qm == bm && qr < bi)) {
                bm = qm;
                bi = qr;
                bv = sh.vals[2 * w + 1];
            }
        }
        __syncthreads();
    };
    for (int j = 0; j < n; ++j) {
        S *v = col(j);
        if (left) {
            // the eliminations of the kept columns before j, one at a time:
            // the owner of pivot row piv_i publishes v[piv_i] (after the
            // earlier eliminations), every workgroup applies it
            for (int i = 0; i < j; ++i) {
                if (!s_keep[i]) continue;  // the same decision in every workgroup
                const int64_t pr = s_pivr[i];
                const int buf = step & 1;
                if (pr >= r0 && pr < r1 && t == 0) part(buf)[0] = (double)P::ld(v + pr);
                // the publisher's workgroup holds index g_pub; all read it
                if (!barrier()) return;
                ++step;
                const int gp = (int)(pr / per);
                const C u = (C)a.part[((int64_t)buf * G + gp) * stride];
                const S *q = col(i);
                for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, P::rnd(fma(-u, P::ld(q + e), P::ld(v + e))));
                __syncthreads();
            }
        }
        // pivot search: every workgroup publishes its candidate and (right-
        // looking) the candidate row's entries of the later columns
        double bm, bv;
        int64_t bi;
        search(v, bm, bi, bv);
        const int buf = step & 1;
        if (t == 0) {
            part(buf)[0] = bm;
            part(buf)[1] = (double)bi;
            part(buf)[2] = bv;
        }
        if (!left && bi != 0x7fffffff)
            for (int c = j + 1 + t; c < n; c += BG_NT)
                a.prow[((int64_t)buf * G + g) * stride + c] = (double)P::ld(col(c) + bi);
        if (!barrier()) return;
        ++step;
        // the winner: largest magnitude, then smallest row (fixed order)
        __syncthreads();
        if (t == 0) {
            double wm = -1.0, wv = 0.0;
            int64_t wi = 0x7fffffff;
            int wg = -1;
            for (int h = 0; h < G; ++h) {
                const double *pp = a.part + ((int64_t)buf * G + h) * stride;
                const double qm = pp[0];
                const int64_t qr = (int64_t)pp[1];
                if (qm > wm || (qm == wm && qr < wi)) {
                    wm = qm;
                    wi = qr;
                    wv = pp[2];
                    wg = h;
                }
            }
            sh.cand[0] = wm;
            sh.cand[1] = (double)wi;
            sh.cand[2] = wv;
            sh.ii[0] = wg;
        }
        __syncthreads();
        const double wm = sh.cand[0];
        const int64_t wi = (int64_t)sh.cand[1];
        const C pv = (C)sh.cand[2];
        const int wg = sh.ii[0];
        const bool take = wm >= a.tol && wm > 0.0;
        if (t == 0) {
            s_keep[j] = take ? 1 : 0;
            s_pivr[j] = wi;
        }
        if (g == 0 && t == 0) {
            a.piv[j] = take ? (int32_t)wi : -1;
            a.keep[j] = take ? 1 : 0;
        }
        if (take) {
            ++kept;
            for (int64_t e = r0 + t; e < r1; e += BG_NT) P::st(v + e, P::rnd(P::ld(v + e) / pv));
            if (!left) {
                // every later column loses its pivot-row entry times the column
                const double *wrow = a.prow + ((int64_t)buf * G + wg) * stride;
                for (int c = j + 1; c < n; ++c) {
                    const C w = (C)wrow[c];
                    S *vc = col(c);
                    for (int64_t e = r0 + t; e < r1; e += BG_NT)
                        P::st(vc + e, P::rnd(fma(-w, P::ld(v + e), P::ld(vc + e))));
                }
            }
        }
        __syncthreads();
    }
    if (g == 0 && t == 0 && a.kept) *a.kept = kept;
}

}  // namespace

void basis_generate(Context *ctx, int method, ofrr_dtype st, int64_t m, int32_t n, void *A, int64_t lda,
                    double tol, double *R, int32_t *piv, int32_t *keep, int32_t *kept_out, double *kernel_ms) {
    OFRR_CHECK_ARG(method >= 0 && method <= 6, "basis: unknown method");
    OFRR_CHECK_ARG(n >= 1 && n <= BG_NMAX && m >= n && lda >= m && m < 0x7fffffff,
                   "basis: 1 <= n <= 512, n <= m <= lda, m < 2^31");
    OFRR_CHECK_ARG(st == OFRR_F64 || st == OFRR_F32 || st == OFRR_F16, "basis: storage F64, F32 or F16");
    const bool hess = method == BM_HESS_L || method == BM_HESS_R;
    // methods that can exclude columns: the Hessenberg forms, and MGS2 with tol > 0
    const bool drops = hess || (method == BM_MGS2 && tol > 0.0);
    OFRR_CHECK_ARG(!hess || (piv && keep), "basis: the Hessenberg methods need piv and keep");
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    // workgroups: at least 256 rows each, at most one per CU
    int G = (int)std::min<int64_t>(cus, std::max<int64_t>(1, (m + 255) / 256));
    const int stride = n + 4;
    double *part = ctx->buf<double>("basis_part", (size_t)2 * G * stride);
    double *prow = ctx->buf<double>("basis_prow", (size_t)2 * G * stride);
    unsigned *bar = ctx->buf<unsigned>("basis_bar", 4);
    int *err = reinterpret_cast<int *>(bar + 2);
    int32_t *kept_d = ctx->buf<int32_t>("basis_kept", 4);
    int32_t *piv_d = piv, *keep_d = keep;
    if (!piv_d) piv_d = ctx->buf<int32_t>("basis_piv", (size_t)n);
    if (!keep_d) keep_d = ctx->buf<int32_t>("basis_keep", (size_t)n);
    zero_bytes(ctx, bar, 16);
    zero_bytes(ctx, keep_d, (size_t)n * 4);
    BGArgs a;
    a.m = m;
    a.lda = lda;
    a.n = n;
    a.tol = tol;
    a.R = R;
    a.piv = piv_d;
    a.keep = keep_d;
    a.kept = kept_d;
    a.part = part;
    a.prow = prow;
    a.bar = bar;
    a.err = err;
    if (R) zero_bytes(ctx, R, (size_t)n * n * 8);
    auto launch = [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        const void *kern = (const void *)k_basis<S>;
        int pc = 0;
        OFRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, BG_NT, 0));
        if ((int64_t)pc * cus < G) fail(OFRR_ERR_UNSUPPORTED, "basis: grid cannot be co-resident");
        S *Ap = static_cast<S *>(A);
        int meth = method;
        void *args[] = {&Ap, &a, &meth};
        OFRR_HIP(hipLaunchCooperativeKernel(kern, dim3(G), dim3(BG_NT), args, 0, ctx->stream));
    };
    hipEvent_t e0, e1;
    OFRR_HIP(hipEventCreate(&e0));
    OFRR_HIP(hipEventCreate(&e1));
    OFRR_HIP(hipEventRecord(e0, ctx->stream));
    if (st == OFRR_F64)
        launch((double *)nullptr);
    else if (st == OFRR_F32)
        launch((float *)nullptr);
    else
        launch((f16_t *)nullptr);
    OFRR_HIP(hipEventRecord(e1, ctx->stream));
    int32_t host[4] = {0, 0, 0, 0};
    OFRR_HIP(hipMemcpyAsync(host, bar, 16, hipMemcpyDeviceToHost, ctx->stream));
    OFRR_HIP(hipMemcpyAsync(host + 3, kept_d, 4, hipMemcpyDeviceToHost, ctx->stream));
    OFRR_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    OFRR_HIP(hipEventElapsedTime(&ms, e0, e1));
    OFRR_HIP(hipEventDestroy(e0));
    OFRR_HIP(hipEventDestroy(e1));
    if (host[2] != 0) fail(OFRR_ERR_HIP, "basis: a grid barrier wait timed out");
    if (kernel_ms) *kernel_ms = ms;
    if (kept_out) *kept_out = drops ? host[3] : n;
}

}  // namespace ofrr
