// internal.hpp -- host-side internals shared by the library's translation
// units: context, workspace, error handling, kernel timing and the kernel
// launcher declarations.  Not part of the public ABI (include/ofrr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <cstdlib>
#include <string>
#include <algorithm>
#include <cmath>
#include <vector>

#include "ofrr.h"

namespace ofrr {

struct Error {
    ofrr_status status;
    std::string msg;
};

[[noreturn]] inline void fail(ofrr_status st, const std::string &msg) { throw Error{st, msg}; }

#define OFRR_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::ofrr::fail(OFRR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define OFRR_CHECK_ARG(cond, msg)                                   \
    do {                                                            \
        if (!(cond)) ::ofrr::fail(OFRR_ERR_INVALID_ARG, (msg));     \
    } while (0)

// Phase switch test of the refined plans: a phase has stalled when its
// residual estimate has not halved over the last `window` outer iterations.
// A precision phase has stalled when the smallest residual estimate seen in
// the last `window` outer iterations is not 10% below the smallest one seen
// before them: slow but steady convergence keeps setting new minima, while
// an estimate that has reached the phase's rounding floor only fluctuates.
struct StallDetector {
    int window;
    std::vector<double> h;
    bool push(double e) {
        h.push_back(e);
        const size_t w = (size_t)(window > 0 ? window : 1);
        if (h.size() <= w) return false;
        double before = INFINITY, recent = INFINITY;
        for (size_t i = 0; i + w < h.size(); ++i) before = std::min(before, h[i]);
        for (size_t i = h.size() - w; i < h.size(); ++i) recent = std::min(recent, h[i]);
        return !(recent < 0.9 * before);
    }
    void reset() { h.clear(); }
};

// Per-family launch timing with HIP events recorded on the context stream
// around each launch.  Events are resolved at the end of an API call.
struct KernelTimer {
    struct Pending {
        int family;
        hipEvent_t a, b;
    };
    std::vector<std::string> names;
    std::vector<int64_t> launches;
    std::vector<double> total_ms;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int family(const char *name) const {
        for (size_t i = 0; i < names.size(); ++i)
            if (names[i] == name) return (int)i;
        return -1;
    }
};

struct Context;

// RAII scope that times one kernel launch when profiling is on.
struct KTimer {
    Context *ctx;
    int fam;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(Context *c, const char *family);
    ~KTimer() noexcept(false);
};

// Device workspace: named buffers that grow on demand and are reused.
struct Workspace {
    struct Buf {
        void *ptr = nullptr;
        size_t bytes = 0;
    };
    std::map<std::string, Buf> bufs;
    void *get(const std::string &name, size_t bytes);
    void release_all();
};

struct Context {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    Workspace ws;
    bool profile = false;
    KernelTimer timer;
    int cu_count = 0;
    int max_lds = 0;
    // which of the two column-maximum merge arrays the next column scaling
    // uses (-1: not cleared yet)
    int colmax_parity = -1;
    // the same for the merged column maxima of the digit-plane slicing
    int vmax_parity = -1;
    // this device's address of the Hessenberg sweep's fixed exchange array
    // (allocation-free entry point)
    uint64_t *hess_scratch = nullptr;
    // batched solver: tile heights picked by its autotuner (waves per
    // workgroup of the reduced and the FP64 grouped product) per problem-set
    // key, the stream its iteration graph is captured on, and what the last
    // call used
    std::map<std::string, std::pair<int, int>> batched_tune;
    hipStream_t graph_stream = nullptr;
    int batched_last_grouped = 0;
    double batched_last_first_ms = 0.0;
    int batched_last_replays = 0;
    int batched_last_waves[2] = {0, 0};

    template <class T>
    T *buf(const std::string &name, size_t count) {
        return static_cast<T *>(ws.get(name, count * sizeof(T) + 256));
    }
    // Waits for the stream by polling an event: a spinning host thread sees
    // the completion sooner than a blocking wait, which matters for the one
    // small readback per outer iteration (OFRR_SYNC_BLOCKING=1 restores
    // hipStreamSynchronize, for comparisons).
    hipEvent_t sync_ev = nullptr;
    int sync_blocking = -1;
    void sync() {
        if (sync_blocking < 0) {
            const char *e = std::getenv("OFRR_SYNC_BLOCKING");
            sync_blocking = (e && std::atoi(e) != 0) ? 1 : 0;
        }
        if (sync_blocking) {
            OFRR_HIP(hipStreamSynchronize(stream));
            return;
        }
        if (!sync_ev) OFRR_HIP(hipEventCreateWithFlags(&sync_ev, hipEventDisableTiming));
        OFRR_HIP(hipEventRecord(sync_ev, stream));
        for (;;) {
            const hipError_t e = hipEventQuery(sync_ev);
            if (e == hipSuccess) return;
            if (e != hipErrorNotReady) OFRR_HIP(e);
        }
    }
    // pinned host staging for small per-iteration readbacks (grows on demand,
    // freed with the context)
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    template <class T>
    T *host_stage(size_t count) {
        const size_t need = count * sizeof(T);
        if (need > pinned_bytes) {
            if (pinned) OFRR_HIP(hipHostFree(pinned));
            pinned = nullptr;
            OFRR_HIP(hipHostMalloc(&pinned, need < 4096 ? 4096 : need, hipHostMallocDefault));
            pinned_bytes = need < 4096 ? 4096 : need;
        }
        return static_cast<T *>(pinned);
    }
    void resolve_timers();
};

// ------------------------------------------------------------------------
// Kernel launchers (defined in the .hip translation units).
// All pointers are device pointers; all launches go to ctx->stream.
// ------------------------------------------------------------------------

// k_misc.hip
void zero_bytes(Context *ctx, void *p, size_t bytes);
void cast_f32_to_bf16(Context *ctx, int64_t count, const float *src, uint16_t *dst);
void cast_f32_to_f16(Context *ctx, int64_t count, const float *src, uint16_t *dst);
void cast_f64_to_f32(Context *ctx, int64_t count, const double *src, float *dst);
// dst = scale * src elementwise (column-major, any element types)
void cast_matrix(Context *ctx, ofrr_dtype src_t, ofrr_dtype dst_t, int64_t rows, int64_t cols,
                 const void *src, int64_t lds, void *dst, int64_t ldd, double scale = 1.0);
// a device pair {a, b} (written by a kernel on the stream; valid until the
// next call)
const int32_t *status_pair(Context *ctx, int32_t a, int32_t b);
// G = I (b x b)
void set_identity(Context *ctx, int32_t b, double *G);
// dst[c + r * ldd] = (dt) src[r * lds + c] for r < rows, c < cols
void transpose_cast(Context *ctx, ofrr_dtype st, ofrr_dtype dt, int64_t rows, int64_t cols, const void *src,
                    int64_t lds, void *dst, int64_t ldd);
// max |a| over the FP64 values of a dense or CSR descriptor (one readback;
// +inf when a value is NaN or infinite)
double absmax_values(Context *ctx, const ofrr_matrix *A);
void quantize_fp8_blocks(Context *ctx, int64_t rows, int64_t cols, const float *A, int64_t lda,
                         uint8_t *codes, float *scales);
void uniform_start(Context *ctx, int64_t n, int32_t b, uint64_t seed, double *X);
// colmax[j] = max_i |Y_ij| for the n x b block (element type t, ld), then
// Y (and Z if not null, same layout and type tz) are multiplied per column
// by 2^-ceil(log2(colmax)); returns nothing; scale factors stay on device.
// Clears the column-maximum merge arrays (at the start of a solve, so a
// failed call cannot leave stale maxima behind).
void scale_columns_reset(Context *ctx);
void scale_columns_pow2(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                        ofrr_dtype tz, void *Z, int64_t ldz, float *work);
// Row-major block helpers (element (i, j) at i*ld + j).
// dst[:, dest(j)] = src[:, j] for every kept column j (src != dst).
void compact_columns_rm(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, const void *src,
                        int64_t lds, const int32_t *keep, void *dst, int64_t ldd);
// column-major FP64 (n x b, ld) -> row-major block of type dt (ld_dst)
void colmajor_to_rowmajor(Context *ctx, int64_t n, int32_t b, const double *src, int64_t lds,
                          ofrr_dtype dt, void *dst, int64_t ldd);
// FP32 values -> hi (and lo = value - hi when lo != null) in BF16/F16 bits
void split_block(Context *ctx, ofrr_dtype t, int64_t count, const float *src, uint16_t *hi,
                 uint16_t *lo);
// round FP32 values in place to the nearest BF16/F16 value
void round_block(Context *ctx, ofrr_dtype t, int64_t count, float *x);
// FP32 array of `count` values stored at the start of buf -> FP64 in place
void promote_block(Context *ctx, int64_t count, void *buf);

// k_product.hip
void product_f64(Context *ctx, const ofrr_matrix *A, int trans, int32_t b, const double *V,
                 int64_t ldv, double *W, int64_t ldw);
// k_gemm_lp.hip.  A BF16/F16 (dense, uint16 bits, column-major, lda), W FP32
// row-major.  product_lowp takes a row-major basis V (vlo, may be null: low
// halves of a two-term split); product_lowp_t takes it K-contiguous per
// column (Vt[j*ldvt + k]) as written by split_block_t.
void product_lowp(Context *ctx, ofrr_dtype t, int64_t m, int64_t kdim, const uint16_t *A,
                  int64_t lda, int trans, int32_t b, const uint16_t *V, const uint16_t *Vlo,
                  int64_t ldv, float *W, int64_t ldw);
// Split-K partial slabs of a product left unreduced for a consumer that sums
// them itself (in slab order, in the slab type: the same result as the
// reduction kernel).  nsplit = 1: the single slab is W.
struct SlabOut {
    const void *p = nullptr;
    ofrr_dtype t = OFRR_F32;
    int nsplit = 0;      // 0: not deferred (W written)
    int64_t stride = 0;  // elements between slabs
};
// Alo (may be null): low halves of a two-term BF16 split of A (then Vtlo is
// required): W = Ahi Vhi + Ahi Vlo + Alo Vhi.  With defer, the split-K
// partials are left in the workspace and described there instead.
void product_lowp_t(Context *ctx, ofrr_dtype t, int64_t m, int64_t kdim, const uint16_t *A,
                    int64_t lda, int trans, int32_t b, const uint16_t *Vt, const uint16_t *Vtlo,
                    int64_t ldvt, float *W, int64_t ldw, const uint16_t *Alo, SlabOut *defer = nullptr);
// k_gemm_f8.hip.  FP8 e4m3fn product with 32 x 32 block scales on A and
// per-(column, 32 rows) E8M0 scales on the basis.
int64_t f8_ldt(int64_t rows);
void quant_basis_f8(Context *ctx, int64_t rows, int32_t b, const float *src, int64_t ld,
                    uint8_t *codes, uint8_t *scales);
void product_f8(Context *ctx, int64_t arows, int64_t acols, const uint8_t *Acodes,
                const float *Ascale, int trans, int32_t b, const uint8_t *Vt, const uint8_t *Vsc,
                float *W, int64_t ldw);
// FP32 column-major (rows x cols, lds) -> hi = bf16(x), lo = bf16(x - hi),
// both column-major with ld = rows
void cast_f32_to_bf16x2(Context *ctx, int64_t rows, int64_t cols, const float *src, int64_t lds,
                        uint16_t *hi, uint16_t *lo);
// leading dimension of the K-contiguous basis copy for `rows` rows
int64_t lowp_ldt(int64_t rows);
// FP32 row-major block (rows x b, ld) -> hi (and lo) BF16/F16 bits in the
// K-contiguous layout (b x rows, ldt)
void split_block_t(Context *ctx, ofrr_dtype t, int64_t rows, int32_t b, const float *src,
                   int64_t ld, uint16_t *hi, uint16_t *lo, int64_t ldt);
// Validates a CSR descriptor's structure on the device (row_ptr[0] == 0,
// non-decreasing, row_ptr[rows] == nnz, column indices in range); fails
// with OFRR_ERR_INVALID_ARG otherwise.
void check_csr(Context *ctx, const ofrr_matrix *A);
void product_csr(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype vt, const void *V,
                 int64_t ldv, void *W, int64_t ldw);
// W = A V for CSR A read from a phase's master block (FP64, or FP32 holding
// the FP32/binary16/bfloat16 basis, rounded to the phase's type on load);
// with cheb, Out = alpha (A V - c Yc) - beta Yp (Yp may be null when beta = 0).
// Returns false (nothing launched) when the blocks are not pair-aligned.
// Column magnitude keys of a row-major block merged into keys (CM_COPIES x
// 512, zero on entry); the power-of-two column scaling from such keys
// applied to Y (clear, CM_COPIES x 512, is zeroed); a key array cleared.
void column_keys(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, const void *Y, int64_t ldy, unsigned *keys);
void scale_apply_keys(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy, const unsigned *keys,
                      unsigned *clear);
void zero_keys(Context *ctx, unsigned *keys, int count);
constexpr int CM_KEYS = 4 * 512;  // one key array: CM_COPIES copies of 512 columns
// One Chebyshev step on CSR A with the column scaling folded in (see the
// kernel); false (nothing launched) when the blocks are not pair-aligned.
bool spmm_cheb_scaled(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype phase, const void *Y1,
                      const void *Y0, void *Y2, int64_t ld, double alpha, double c, double beta,
                      const unsigned *cmax_in, const double *p0, bool round_prev, double *s_out, unsigned *cmax_out,
                      unsigned *clear);
bool product_csr_master(Context *ctx, const ofrr_matrix *A, int32_t b, ofrr_dtype phase, const void *Vm, int64_t ld,
                        void *Out, const void *Yc, const void *Yp, bool cheb, double alpha, double c, double beta);

// k_gemm_i8.hip: FP64-class product from exact INT8 digit-plane products
struct SlicedA {
    int8_t *planes = nullptr;  // 5 planes of mpad x kpad digits (K-contiguous rows of op(A))
    int32_t *ex = nullptr;     // per-row exponent bounds (mpad)
    int64_t m = 0, kdim = 0, mpad = 0, kpad = 0, plane_stride = 0;
};
// tag names the workspace buffers of the planes (two slicings of one A,
// e.g. its rows and its columns, need two tags)
SlicedA slice_matrix_i8(Context *ctx, const ofrr_matrix *A, int trans, const char *tag = "i8_a");
// digits: signed 7-bit digits per side (6: 21 digit pairs, exact to about
// 2^-42 of the row and column scales; 5: 15 pairs, 2^-35; 4: 10 pairs, 2^-28)
void product_i8s(Context *ctx, const SlicedA &sa, int32_t b, const double *V, int64_t ldv, double *W,
                 int64_t ldw, SlabOut *defer = nullptr, int digits = 6);
// digits per side for a sliced FP64 iteration from the largest residual
// estimate of the iteration before it (solver.cpp)
int i8_digits_for(double emax);

// k_hessenberg.hip
// Returns the kept count (after waiting for the sweep; a timed-out wait
// raises).  With `status` given it returns 0 at once instead and sets
// *status to the device pair {error flag, kept count}, valid on the stream
// until the next sweep on this context.
int32_t hessenberg(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                   double tol, int32_t *piv, int32_t *keep, const int32_t **status = nullptr);
// The same sweep with its exchange words in the library's fixed device
// array (ctx->hess_scratch, set by hess_scratch_address at context
// creation) instead of the workspace; allocates nothing.
void hess_scratch_address(Context *ctx);
int32_t hessenberg_noalloc(Context *ctx, ofrr_dtype t, int64_t n, int32_t b, void *Y, int64_t ldy,
                           double tol, int32_t *piv, int32_t *keep);

// k_batched.hip: many problems per grouped launch, iterations replayed from
// a HIP graph (plans with one product per iteration, basis <= 32, BF16/F16
// or FP64 first phase, FP64 projections)
bool batched_grouped_supported(const ofrr_plan *plan, int32_t nprob, const ofrr_matrix *As, int32_t k,
                               int32_t basis);
ofrr_status batched_grouped_impl(Context *ctx, int32_t nprob, const ofrr_matrix *As, int32_t k, int32_t basis,
                                 ofrr_which which, const ofrr_plan *plan, const double *const *X0s,
                                 double *const *evals, double *const *evecs, double *const *resid,
                                 ofrr_info *infos);

// k_basis.hip: the basis-generation processes of the comparison (method:
// 0 MGS-L, 1 MGS-R, 2 CGS, 3 CGS-2, 4 Hess-L, 5 Hess-R) on a column-major
// m x n block of storage type st (F64, F32, F16 = binary16 storage with
// FP32 arithmetic), in place; one cooperative launch, timed with events.
void basis_generate(Context *ctx, int method, ofrr_dtype st, int64_t m, int32_t n, void *A, int64_t lda,
                    double tol, double *R, int32_t *piv, int32_t *keep, int32_t *kept_out, double *kernel_ms);

// k_krylov.hip: restarted Krylov-Hessenberg + OFRR (arguments as
// ofrr_krylov_eig, validated by the caller)
ofrr_status krylov_eig_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t nev, int32_t restarts,
                            ofrr_dtype bt, const double *v0, double tol, double *evals, double *evecs,
                            double *resid, ofrr_info *info);

// k_project.hip
// G = V^T V, H = V^T W (b x b FP64, column-major) accumulated per `acc`
// (FP32 modes take FP32, BF16 or F16 blocks only).
void project(Context *ctx, int64_t n, int32_t b, ofrr_dtype vt, const void *V, int64_t ldv,
             ofrr_dtype wt, const void *W, int64_t ldw, ofrr_accum acc, double *G, double *H);
void gram_rect(Context *ctx, int64_t n, int32_t b1, int32_t b2, ofrr_dtype xt, const void *X,
               int64_t ldx, ofrr_dtype yt, const void *Y, int64_t ldy, double *C,
               ofrr_accum acc = OFRR_ACC_F64);
// Conditioning statistic of the projected mass matrix after a pencil solve
// with Y^T G Y = I: t = sum_i G_ii (Y Y^T)_ii / b (Y Y^T = G^{-1} when G has
// full rank; t = 1 for a diagonal G, t <= kappa(D^-1 G D^-1), D = diag(G)^(1/2)),
// written to *out on the device; +inf when the pencil's rank (device
// pointer) is below b.
void gram_condition(Context *ctx, int32_t b, const double *G, const double *Y, const int32_t *rank,
                    double *out);

// k_smalleig.hip
// Pencil H y = theta G y; returns rank of G used.
int32_t pencil_eig(Context *ctx, int32_t b, const double *H, const double *G, ofrr_which which,
                   double *theta, double *Y, bool want_rank);
// The same solve with no host synchronisation: returns a device pointer
// that holds the rank once the stream reaches it.  theta and the columns of
// Y beyond the rank come out zero.
const int32_t *pencil_eig_async(Context *ctx, int32_t b, const double *H, const double *G,
                                ofrr_which which, double *theta, double *Y);
void svd_pencil(Context *ctx, int32_t k1, int32_t k2, const double *B, const double *MU,
                const double *MV, double *sigma, double *Y, double *Z);
// Non-symmetric pencil H y = theta G y (G symmetric positive definite):
// theta_re/theta_im (b) ordered by modulus, real part, imaginary part
// (descending; a conjugate pair adjacent, + member first), Y (b x b) packed
// real: a real value's column is y, a pair's two columns Re y and Im y of
// the + member; y^H G y = 1.  The async form returns a device pointer to
// {status (0 ok, 1 G not positive definite, 2 no convergence), QR
// iterations}; pencil_general raises on a nonzero status.
const int32_t *pencil_general_async(Context *ctx, int32_t b, const double *H, const double *G, double *theta_re,
                                    double *theta_im, double *Y);
void pencil_general(Context *ctx, int32_t b, const double *H, const double *G, double *theta_re, double *theta_im,
                    double *Y);

// k_lift.hip
// X = V Y[:, :nc], AX = W Y[:, :nc] (n x nc outputs, element type per xt),
// optional residual partial sums ||AX_i - theta_i X_i||^2, ||X_i||^2:
// returns the number of partial rows written (row stride nc; at most
// ceil(n / 64)), for residual_reduce.
int64_t lift(Context *ctx, int64_t n, int32_t b, int32_t nc, ofrr_dtype vt, const void *V,
             int64_t ldv, ofrr_dtype wt, const void *W, int64_t ldw, const double *Y, int32_t ldy,
             const double *theta, ofrr_dtype xt, void *X, void *AX, int64_t ldx, double *res2,
             double *xn2);
// Chebyshev first step from X and AX: Y1 = alpha*(AX - c*X); or Y1 = AX
// (power); output in type yt.
void axpby_block(Context *ctx, int64_t n, int32_t b, ofrr_dtype it, const void *AX,
                 const void *X, int64_t ld, double alpha, double beta, ofrr_dtype yt, void *Y,
                 int64_t ldy);
// Chebyshev recurrence Ynext = alpha*(P - c*Ycur) - Yprev (P FP32/FP64
// product output, Ycur/Yprev in storage type st, Ynext in type nt).
void cheb_combine(Context *ctx, int64_t n, int32_t b, ofrr_dtype pt, const void *P,
                  ofrr_dtype st, const void *Ycur, const void *Yprev, int64_t ld, double alpha,
                  double c, double beta, ofrr_dtype nt, void *Ynext);
// The same with P the sum of deferred split-K slabs.
void cheb_combine_slabs(Context *ctx, int64_t n, int32_t b, const SlabOut &P, ofrr_dtype st,
                        const void *Ycur, const void *Yprev, int64_t ld, double alpha, double c,
                        double beta, ofrr_dtype nt, void *Ynext);
void scale_array(Context *ctx, int64_t count, double *x, double f);
// out[c] = ||X1_c - s_c X2_c|| / ||X2_c|| / anorm for row-major blocks
void col_resid(Context *ctx, ofrr_dtype t, int64_t n, int32_t count, const void *X1, const void *X2,
               int64_t ld, const double *s, double anorm, double *out);
// Final residual: R = AX - X theta, norms -> resid[i] = ||R_i|| / (||X_i|| anorm);
// normalises X to unit columns with the sign rule and writes FP64 outputs.
void finalize_eig(Context *ctx, int64_t n, int32_t k, const double *X, int64_t ldx,
                  const double *AX, int64_t ldax, const double *theta, double anorm,
                  double *evals, double *evecs, double *resid);
// out[c] = sqrt(sum res2[blk][c]) / sqrt(sum xn2[blk][c]) / anorm for
// c < count; partial arrays have row stride `stride`.  out[count] =
// extra[0] and out[count + 1 + i] = extra2[i] (i < 2) when given, so one
// copy brings back device-side counts with the estimates.
void residual_reduce(Context *ctx, const double *res2, const double *xn2, int nblk, int stride,
                     int count, double anorm, double *out, const int32_t *extra = nullptr,
                     const int32_t *extra2 = nullptr);
// k_general.hip: complex Ritz pairs held packed real (a pair = Re, Im of
// its + member in adjacent columns; th_im > 0 first member, < 0 second).
// Residual partials per 64-row block for slots c < nc (layout of lift's).
void residual_partials_general(Context *ctx, ofrr_dtype t, int64_t n, int32_t nc, const void *X, const void *AX,
                               int64_t ld, const double *th_re, const double *th_im, double *res2, double *xn2);
// Final outputs of the k wanted slots from FP64 row-major X, AX (ld, the
// columns of a pair cut at k included): evals, complex unit vectors with
// the largest-modulus entry real positive (column-major n x k, re and im
// parts), resid = ||A x - lambda x|| / (||x|| anorm).
void finalize_general(Context *ctx, int64_t n, int32_t k, const double *X, const double *AX, int64_t ld,
                      const double *th_re, const double *th_im, double anorm, double *evals_re,
                      double *evals_im, double *evecs_re, double *evecs_im, double *resid);
// SVD final step: resid[c] = sqrt(|A v - s u|^2 + |A^T u - s v|^2)/anorm,
// normalisation and sign rule (sign fixed on v, u follows); outputs
// column-major FP64.
void finalize_svd(Context *ctx, int64_t m, int64_t n, int32_t k, const double *U, const double *AV,
                  const double *Vv, const double *ATU, int64_t ld, const double *sigma,
                  double anorm, double *sig_out, double *Uo, double *Vo, double *resid);

}  // namespace ofrr
