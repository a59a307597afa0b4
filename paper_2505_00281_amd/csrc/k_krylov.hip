// k_krylov.hip -- the Krylov-Hessenberg process (Sec. 4.1, Alg.
// "Computing non-orthogonal bases from the Krylov-Hessenberg Process")
// with the orthogonalization-free projection (Sec. 3.1) and single-vector
// restart from the Ritz vector of the largest Ritz value (Sec. 5.2, sparse
// experiments), for a symmetric A in CSR or dense storage.
//
// Step j of the process removes from w = A v_j, for i = 0..j in order, its
// entry at pivot row pi_i times v_i.  The entries that step i reads are
// those of the pivot rows, so all of them follow from the pivot rows
// alone: u_i = w[pi_i] minus sum_{l < i} u_l v_l[pi_i] (the same chain of
// fused multiply-adds, each rounded to the storage type, that row pi_i
// itself goes through).  One workgroup solves that small triangular chain,
// then every row applies all j + 1 removals in one pass, in the same order,
// and the pass also finds the new pivot: per step four launches, no inner
// products, one grid-wide argmax.  A cycle of k steps is captured once in
// a HIP graph and replayed for every restart.
//
// Storage types: FP64, FP32, or binary16 with FP32 arithmetic (every
// stored result rounded to binary16, the paper's FP16 runs).  The
// projection G = V^T V, H = V^T (A V) is formed in FP64 from the stored
// basis and the products kept during the process; the pencil is solved in
// FP64 on the GPU.
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "device_util.hpp"

namespace ofrr {

namespace {

constexpr int KR_NT = 256;

template <class S>
struct KSto;
template <>
struct KSto<double> {
    using C = double;
    static __device__ __forceinline__ C ld(const double *p) { return *p; }
    static __device__ __forceinline__ void st(double *p, C v) { *p = v; }
    static __device__ __forceinline__ C rnd(C v) { return v; }
};
template <>
struct KSto<float> {
    using C = float;
    static __device__ __forceinline__ C ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, C v) { *p = v; }
    static __device__ __forceinline__ C rnd(C v) { return v; }
};
template <>
struct KSto<f16_t> {
    using C = float;
    static __device__ __forceinline__ C ld(const f16_t *p) { return f16_bits_to_f32(p->bits); }
    static __device__ __forceinline__ void st(f16_t *p, C v) { p->bits = f32_to_f16_bits(v); }
    static __device__ __forceinline__ C rnd(C v) { return f16_bits_to_f32(f32_to_f16_bits(v)); }
};

struct KrState {
    const int32_t *rp;  // CSR structure (null: dense)
    const int32_t *ci;
    const void *val;    // CSR values or dense column-major A
    int a_f64;
    int64_t n, lda;
    int k;              // basis size (columns of V)
    void *V;            // n x k row-major, storage type
    double *W;          // n x k row-major: A v_j in the arithmetic type (FP64 slots)
    void *xs;           // v_j contiguous (storage type), the product's input
    double *xt;         // the step's result before scaling (arithmetic type, FP64 slots)
    double *u;          // k removal weights of the current step
    double *P;          // k x k: P[i*k + l] = v_l[pi_i]
    double *H;          // k x (k-1) column-major: the process's upper Hessenberg matrix
    int32_t *piv;       // k pivot rows
    double *part;       // per-workgroup candidates (3 doubles each)
    double *amax;       // per-workgroup max |A v_j| of the step's product
    int namax;          // workgroups of the product launch
    double brk;         // breakdown: max |w| after the removals <= brk (max |A v_j| + sum |u_i|)
    int32_t *stop;      // [0] set when w vanished; [1] columns built
};

template <class TA>
__device__ __forceinline__ double a_val(const void *p, int64_t i) {
    return (double)static_cast<const TA *>(p)[i];
}

// w = A v_j (arithmetic type, rounded to the storage type), into W[:, j] and
// xt; CSR: one thread per row; dense: one wave per row.
template <class S>
__global__ __launch_bounds__(KR_NT) void k_kr_product(KrState s, int j) {
    using P = KSto<S>;
    using C = typename P::C;
    if (s.stop[0]) return;
    __shared__ double s_m[KR_NT / 64];
    const S *x = static_cast<const S *>(s.xs);
    double bm = 0.0;
    if (s.rp) {
        for (int64_t r = (int64_t)blockIdx.x * KR_NT + threadIdx.x; r < s.n; r += (int64_t)gridDim.x * KR_NT) {
            C acc = (C)0;
            for (int32_t e = s.rp[r]; e < s.rp[r + 1]; ++e) {
                const C a = s.a_f64 ? (C)a_val<double>(s.val, e) : (C)a_val<float>(s.val, e);
                acc = fma(a, P::ld(x + s.ci[e]), acc);
            }
            const C w = P::rnd(acc);
            s.W[r * s.k + j] = (double)w;
            s.xt[r] = (double)w;
            { const double a = fabs((double)w); bm = (a > bm || a != a) ? a : bm; }
        }
    } else {
        const int lane = threadIdx.x & 63;
        const int64_t wv = ((int64_t)blockIdx.x * KR_NT + threadIdx.x) >> 6;
        const int64_t nw = ((int64_t)gridDim.x * KR_NT) >> 6;
        for (int64_t r = wv; r < s.n; r += nw) {
            C acc = (C)0;
            for (int64_t c = lane; c < s.n; c += 64) {
                const C a = s.a_f64 ? (C)a_val<double>(s.val, c + r * s.lda) : (C)a_val<float>(s.val, c + r * s.lda);
                acc = fma(a, P::ld(x + c), acc);
            }
            double d = (double)acc;
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
            if (lane == 0) {
                const C w = P::rnd((C)d);
                s.W[r * s.k + j] = (double)w;
                s.xt[r] = (double)w;
                { const double a = fabs((double)w); bm = (a > bm || a != a) ? a : bm; }
            }
        }
    }
    // this workgroup's max |A v_j| (the breakdown test's scale)
    // (a NaN wins every maximum here, so the scaling step can report it)
    for (int o = 32; o > 0; o >>= 1) {
        const double q = __shfl_xor(bm, o, 64);
        bm = (q > bm || q != q) ? q : bm;
    }
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = bm;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_m[0];
        for (int w = 1; w < KR_NT / 64; ++w) m = (s_m[w] > m || s_m[w] != s_m[w]) ? s_m[w] : m;
        s.amax[blockIdx.x] = m;
    }
}

// the removal weights of step j: u_i = w[pi_i] after the removals l < i
template <class S>
__global__ void k_kr_weights(KrState s, int j) {
    using P = KSto<S>;
    using C = typename P::C;
    if (s.stop[0] || threadIdx.x != 0) return;
    for (int i = 0; i <= j; ++i) {
        C x = (C)s.xt[s.piv[i]];
        for (int l = 0; l < i; ++l) x = P::rnd(fma(-(C)s.u[l], (C)s.P[(int64_t)i * s.k + l], x));
        s.u[i] = (double)x;
        s.H[i + (int64_t)j * s.k] = (double)x;
    }
}

// every row: the j + 1 removals in order (first = -1: no removal, the start
// vector), then the workgroup's pivot candidate (largest magnitude, first
// row on ties)
template <class S>
__global__ __launch_bounds__(KR_NT) void k_kr_update(KrState s, int j) {
    using P = KSto<S>;
    using C = typename P::C;
    __shared__ double rm[KR_NT / 64];
    __shared__ int64_t ri[KR_NT / 64];
    if (s.stop[0]) return;
    const S *V = static_cast<const S *>(s.V);
    double bm = -1.0;
    int64_t bi = 0x7fffffff;
    for (int64_t r = (int64_t)blockIdx.x * KR_NT + threadIdx.x; r < s.n; r += (int64_t)gridDim.x * KR_NT) {
        C x = (C)s.xt[r];
        for (int i = 0; i <= j; ++i) x = P::rnd(fma(-(C)s.u[i], P::ld(V + r * s.k + i), x));
        s.xt[r] = (double)x;
        const double m = fabs((double)x);
        if (m > bm) {
            bm = m;
            bi = r;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double qm = __shfl_xor(bm, o, 64);
        const int64_t qi = __shfl_xor(bi, o, 64);
        if (qm > bm || (qm == bm && qi < bi)) {
            bm = qm;
            bi = qi;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        rm[threadIdx.x >> 6] = bm;
        ri[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < KR_NT / 64; ++w)
            if (rm[w] > rm[0] || (rm[w] == rm[0] && ri[w] < ri[0])) {
                rm[0] = rm[w];
                ri[0] = ri[w];
            }
        s.part[3 * blockIdx.x] = rm[0];
        s.part[3 * blockIdx.x + 1] = (double)ri[0];
    }
}

// the pivot (every workgroup reduces the candidates in the same order) and
// column j + 1 = x / x[pivot]; workgroup 0 records the pivot, its row of
// the basis and the scaling
template <class S>
__global__ __launch_bounds__(KR_NT) void k_kr_scale(KrState s, int j, int ncand) {
    using P = KSto<S>;
    using C = typename P::C;
    __shared__ double s_p;
    __shared__ int64_t s_r;
    if (s.stop[0]) return;
    if (threadIdx.x == 0) {
        double bm = -1.0;
        int64_t bi = 0x7fffffff;
        for (int g = 0; g < ncand; ++g) {
            const double m = s.part[3 * g];
            const int64_t i = (int64_t)s.part[3 * g + 1];
            if (m > bm || (m == bm && i < bi)) {
                bm = m;
                bi = i;
            }
        }
        s_r = bi;
        s_p = (bm > 0.0 && bi < s.n) ? s.xt[bi] : 0.0;
        // breakdown: what is left of A v_j after the removals is at the
        // rounding level of A v_j and the removed multiples (an invariant
        // subspace)
        if (j >= 0) {
            double am = 0.0;
            for (int g = 0; g < s.namax; ++g) am = (s.amax[g] > am || s.amax[g] != s.amax[g]) ? s.amax[g] : am;
            for (int i = 0; i <= j; ++i) am += fabs(s.u[i]);
            if (am != am)
                s_p = am;  // not finite: reported below
            else if (!(bm > s.brk * am))
                s_p = 0.0;
        }
    }
    __syncthreads();
    const double pv = s_p;
    const int64_t pr = s_r;
    if (pv == 0.0 || !(pv == pv)) {
        // w vanished (an invariant subspace) or is not finite: stop here
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            s.stop[0] = pv == 0.0 ? 1 : 2;
            s.stop[1] = j + 1;
        }
        return;
    }
    S *V = static_cast<S *>(s.V);
    S *xs = static_cast<S *>(s.xs);
    const C p = (C)pv;
    for (int64_t r = (int64_t)blockIdx.x * KR_NT + threadIdx.x; r < s.n; r += (int64_t)gridDim.x * KR_NT) {
        const C y = P::rnd((C)s.xt[r] / p);
        P::st(V + r * s.k + (j + 1), y);
        P::st(xs + r, y);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.piv[j + 1] = (int32_t)pr;
        if (j >= 0) s.H[(j + 1) + (int64_t)j * s.k] = pv;
        s.stop[1] = j + 2;
    }
    // the new pivot row of the basis (entries l <= j are final; l = j + 1 is 1)
    if (blockIdx.x == 0)
        for (int l = threadIdx.x; l <= j + 1; l += KR_NT)
            s.P[(int64_t)(j + 1) * s.k + l] = l == j + 1 ? 1.0 : (double)P::ld(V + pr * s.k + l);
}

// start vector of a cycle: xt = rounded v (FP64 input), stop flags cleared
template <class S>
__global__ void k_kr_start(KrState s, const double *v) {
    using P = KSto<S>;
    using C = typename P::C;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.stop[0] = 0;
        s.stop[1] = 0;
    }
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < s.n; r += (int64_t)gridDim.x * blockDim.x)
        s.xt[r] = (double)P::rnd((C)v[r]);
}

// FP64 copy of a block of the storage type (row-major n x k)
template <class S>
__global__ void k_kr_to_f64(const S *V, int64_t count, double *out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (double)KSto<S>::ld(V + e);
}

// columns of the basis past the columns built are cleared (a stopped
// process leaves them unwritten)
template <class S>
__global__ void k_kr_clear_tail(S *V, double *W, int64_t n, int k, const int32_t *stop) {
    const int built = stop[1];
    if (built >= k) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * k; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % k);
        if (c >= built) {
            KSto<S>::st(V + e, 0.0f);
            W[e] = 0.0;
        }
    }
}

__global__ void k_kr_div_abs(double *resid, const double *theta, int count) {
    const int i = threadIdx.x;
    if (i < count) resid[i] = resid[i] / fabs(theta[i]);
}

}  // namespace

ofrr_status krylov_eig_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t nev, int32_t restarts,
                            ofrr_dtype bt, const double *v0, double tol, double *evals, double *evecs,
                            double *resid, ofrr_info *info) {
    const int64_t n = A->rows;
    const hipStream_t st = ctx->stream;
    hipEvent_t ev0, ev1;
    OFRR_HIP(hipEventCreate(&ev0));
    OFRR_HIP(hipEventCreate(&ev1));
    OFRR_HIP(hipEventRecord(ev0, st));
    const size_t es = bt == OFRR_F64 ? 8 : (bt == OFRR_F32 ? 4 : 2);
    KrState s;
    s.rp = A->format == OFRR_CSR ? A->row_ptr : nullptr;
    s.ci = A->format == OFRR_CSR ? A->col_idx : nullptr;
    s.val = A->values;
    s.a_f64 = A->dtype == OFRR_F64 ? 1 : 0;
    s.n = n;
    s.lda = A->ld;
    s.k = k;
    s.V = ctx->buf<char>("kr_V", (size_t)n * k * es);
    s.W = ctx->buf<double>("kr_W", (size_t)n * k);
    s.xs = ctx->buf<char>("kr_xs", (size_t)n * es);
    s.xt = ctx->buf<double>("kr_xt", (size_t)n);
    s.u = ctx->buf<double>("kr_u", (size_t)k);
    s.P = ctx->buf<double>("kr_P", (size_t)k * k);
    s.H = ctx->buf<double>("kr_H", (size_t)k * k);
    s.piv = ctx->buf<int32_t>("kr_piv", (size_t)k);
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    const int gu = (int)std::max<int64_t>(1, std::min<int64_t>(4 * cus, (n + KR_NT - 1) / KR_NT));
    s.part = ctx->buf<double>("kr_part", (size_t)3 * gu);
    s.stop = ctx->buf<int32_t>("kr_stop", 4);
    const int gprod = s.rp ? gu : (int)std::max<int64_t>(1, std::min<int64_t>(4 * cus, (n + 3) / 4));
    s.amax = ctx->buf<double>("kr_amax", (size_t)gprod);
    s.namax = gprod;
    // breakdown threshold per unit of (max |A v_j| + sum_i |u_i|): 64 units
    // of FP64 rounding (the process's own rounding noise at an invariant
    // subspace measured a few tens of units), the working-precision epsilon
    // for FP32 and FP16 storage
    s.brk = bt == OFRR_F64 ? 64.0 * std::ldexp(1.0, -52)
                           : (bt == OFRR_F32 ? std::ldexp(1.0, -23) : std::ldexp(1.0, -10));
    double *vstart = ctx->buf<double>("kr_v0", (size_t)n);
    if (v0)
        OFRR_HIP(hipMemcpyAsync(vstart, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    else
        uniform_start(ctx, n, 1, 0x5EEDull, vstart);
    zero_bytes(ctx, s.P, sizeof(double) * k * k);
    zero_bytes(ctx, s.H, sizeof(double) * k * k);
    double *G = ctx->buf<double>("kr_G", (size_t)k * k);
    double *Hp = ctx->buf<double>("kr_Hp", (size_t)k * k);
    double *Yr = ctx->buf<double>("kr_Y", (size_t)k * k);
    double *theta = ctx->buf<double>("kr_theta", (size_t)k + 8);
    double *X1 = ctx->buf<double>("kr_X1", (size_t)n);
    double *AX1 = ctx->buf<double>("kr_AX1", (size_t)n);
    double *Vd = bt == OFRR_F64 ? static_cast<double *>(s.V) : ctx->buf<double>("kr_Vd", (size_t)n * k);

    // one cycle of the process, captured once
    if (!ctx->graph_stream) OFRR_HIP(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
    const hipStream_t gs = ctx->graph_stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto capture = [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        OFRR_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(k_kr_start<S>, dim3(gu), dim3(KR_NT), 0, gs, s, (const double *)vstart);
        hipLaunchKernelGGL(k_kr_weights<S>, dim3(1), dim3(64), 0, gs, s, -1);
        hipLaunchKernelGGL(k_kr_update<S>, dim3(gu), dim3(KR_NT), 0, gs, s, -1);
        hipLaunchKernelGGL(k_kr_scale<S>, dim3(gu), dim3(KR_NT), 0, gs, s, -1, gu);
        for (int j = 0; j + 1 < k; ++j) {
            hipLaunchKernelGGL(k_kr_product<S>, dim3(gprod), dim3(KR_NT), 0, gs, s, j);
            hipLaunchKernelGGL(k_kr_weights<S>, dim3(1), dim3(64), 0, gs, s, j);
            hipLaunchKernelGGL(k_kr_update<S>, dim3(gu), dim3(KR_NT), 0, gs, s, j);
            hipLaunchKernelGGL(k_kr_scale<S>, dim3(gu), dim3(KR_NT), 0, gs, s, j, gu);
        }
        // the last column's product (A V needs every column)
        hipLaunchKernelGGL(k_kr_product<S>, dim3(gprod), dim3(KR_NT), 0, gs, s, k - 1);
        hipLaunchKernelGGL(k_kr_clear_tail<S>, dim3(gu), dim3(KR_NT), 0, gs, static_cast<S *>(s.V), s.W, n, k,
                           (const int32_t *)s.stop);
        if (bt != OFRR_F64)
            hipLaunchKernelGGL(k_kr_to_f64<S>, dim3(gu), dim3(KR_NT), 0, gs, static_cast<const S *>(s.V),
                               n * k, Vd);
        const hipError_t le = hipGetLastError();
        const hipError_t ee = hipStreamEndCapture(gs, &graph);
        OFRR_HIP(le);
        OFRR_HIP(ee);
    };
    if (bt == OFRR_F64)
        capture((double *)nullptr);
    else if (bt == OFRR_F32)
        capture((float *)nullptr);
    else
        capture((f16_t *)nullptr);
    {
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            OFRR_HIP(e);
        }
    }
    hipError_t run_err = hipSuccess;
    int products = 0;
    for (int cyc = 0; cyc <= restarts && run_err == hipSuccess; ++cyc) {
        run_err = hipGraphLaunch(exec, st);
        if (run_err != hipSuccess) break;
        products += k;
        // projection in FP64: G = V^T V, H = V^T (A V)
        try {
            project(ctx, n, k, OFRR_F64, Vd, k, OFRR_F64, s.W, k, OFRR_ACC_F64, G, Hp);
            pencil_eig_async(ctx, k, Hp, G, OFRR_LARGEST, theta, Yr);
            // restart vector: the Ritz vector of the largest Ritz value
            if (cyc < restarts) {
                lift(ctx, n, k, 1, OFRR_F64, Vd, k, OFRR_F64, s.W, k, Yr, k, theta, OFRR_F64, X1, AX1, 1, nullptr,
                     nullptr);
                OFRR_HIP(hipMemcpyAsync(vstart, X1, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            }
        } catch (...) {
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            throw;
        }
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    OFRR_HIP(run_err);
    int32_t hstop[2] = {0, 0};
    OFRR_HIP(hipMemcpyAsync(hstop, s.stop, sizeof(hstop), hipMemcpyDeviceToHost, st));
    // the nev largest pairs: X = V Y[:, :nev] (FP64), A X in FP64 from A as
    // stored, residual ||A x - theta x|| / (||x|| |theta|) with the sign rule
    double *Xf = ctx->buf<double>("kr_Xf", (size_t)n * nev + 8);
    double *AXf = ctx->buf<double>("kr_AXf", (size_t)n * nev + 8);
    double *AXl = ctx->buf<double>("kr_AXl", (size_t)n * nev + 8);
    lift(ctx, n, k, nev, OFRR_F64, Vd, k, OFRR_F64, s.W, k, Yr, k, theta, OFRR_F64, Xf, AXl, nev, nullptr, nullptr);
    if (A->format == OFRR_CSR)
        product_csr(ctx, A, nev, OFRR_F64, Xf, nev, AXf, nev);
    else
        product_f64(ctx, A, 1, nev, Xf, nev, AXf, nev);
    ++products;
    finalize_eig(ctx, n, nev, Xf, nev, AXf, nev, theta, 1.0, evals, evecs, resid);
    hipLaunchKernelGGL(k_kr_div_abs, dim3(1), dim3(256), 0, st, resid, evals, nev);
    OFRR_HIP(hipGetLastError());
    OFRR_HIP(hipEventRecord(ev1, st));
    std::vector<double> rr((size_t)nev);
    OFRR_HIP(hipMemcpyAsync(rr.data(), resid, sizeof(double) * nev, hipMemcpyDeviceToHost, st));
    OFRR_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    OFRR_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    OFRR_HIP(hipEventDestroy(ev0));
    OFRR_HIP(hipEventDestroy(ev1));
    if (hstop[0] == 2) fail(OFRR_ERR_NUMERIC, "krylov: non-finite values in the process");
    int nconv = 0;
    double rmax = 0.0;
    for (double v : rr) {
        rmax = std::max(rmax, v);
        if (tol > 0 ? v <= tol : true) ++nconv;
    }
    if (info) {
        info->iters = restarts + 1;
        info->iters_low = bt == OFRR_F64 ? 0 : restarts + 1;
        info->n_converged = nconv;
        info->basis_eff = hstop[1];
        info->products = products;
        info->max_resid = rmax;
        info->seconds = ms * 1e-3;
        info->gram_t_max = 0.0;
        info->grams_f64 = 0;
    }
    return (tol > 0 && nconv < nev) ? OFRR_NOT_CONVERGED : OFRR_OK;
}

}  // namespace ofrr
