// api.cpp -- the extern "C" entry points of include/ofrr.h: context
// lifetime, argument validation (before any device work), error capture (no
// C++ exception crosses the boundary) and kernel timing.
#include <initializer_list>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace ofrr {

ofrr_status eig_partial_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             ofrr_which which, const ofrr_plan *plan, const double *X0,
                             double *evals, double *evecs, double *resid, ofrr_info *info,
                             bool normal = false);
ofrr_status svd_normal_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                            const ofrr_plan *plan, const double *V0, double *sigma, double *U,
                            double *V, double *resid, ofrr_info *info);
ofrr_status svd_partial_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             const ofrr_plan *plan, const double *V0, double *sigma, double *U,
                             double *V, double *resid, ofrr_info *info);
ofrr_status eig_general_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis, const ofrr_plan *plan,
                             const double *X0, double *evals_re, double *evals_im, double *evecs_re,
                             double *evecs_im, double *resid, ofrr_info *info);

static const char *kFamilies[] = {"quantize", "product_bf16", "product_bf16x2", "product_f16", "product_f8",
                                  "product_f64", "product_f32", "product_i8x", "product_reduce", "spmm", "scale",
                                  "hessenberg", "gram", "small_eig", "lift", "residual", "spmm_f16", "spmm_f32",
                                  "spmm_f64", "product_i8x_d4", "product_i8x_d5", "product_i8x_d6"};

void *Workspace::get(const std::string &name, size_t bytes) {
    Buf &b = bufs[name];
    if (b.bytes >= bytes && b.ptr) return b.ptr;
    if (b.ptr) {
        // the stream may still use the old buffer
        (void)hipDeviceSynchronize();
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        fail(OFRR_ERR_OOM, "workspace allocation of " + std::to_string(want) + " bytes for " + name +
                               " failed: " + hipGetErrorString(e));
    }
    b.bytes = want;
    return b.ptr;
}

void Workspace::release_all() {
    for (auto &kv : bufs)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    bufs.clear();
}

KTimer::KTimer(Context *c, const char *family) : ctx(c), fam(-1) {
    if (!ctx->profile) return;
    fam = ctx->timer.family(family);
    if (fam < 0) return;
    auto take = [&]() {
        hipEvent_t e;
        if (!ctx->timer.pool.empty()) {
            e = ctx->timer.pool.back();
            ctx->timer.pool.pop_back();
        } else {
            OFRR_HIP(hipEventCreate(&e));
        }
        return e;
    };
    a = take();
    b = take();
    OFRR_HIP(hipEventRecord(a, ctx->stream));
}

KTimer::~KTimer() noexcept(false) {
    if (fam < 0 || !a) return;
    if (hipEventRecord(b, ctx->stream) == hipSuccess)
        ctx->timer.pending.push_back(KernelTimer::Pending{fam, a, b});
}

void Context::resolve_timers() {
    if (timer.pending.empty()) return;
    (void)hipStreamSynchronize(stream);
    for (auto &p : timer.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            timer.launches[p.family] += 1;
            timer.total_ms[p.family] += ms;
        }
        timer.pool.push_back(p.a);
        timer.pool.push_back(p.b);
    }
    timer.pending.clear();
}

}  // namespace ofrr

using namespace ofrr;

struct ofrr_ctx_s {
    Context c;
};

static thread_local std::string g_create_error;

template <class F>
static ofrr_status guarded(ofrr_ctx ctx, F &&f) {
    if (!ctx) return OFRR_ERR_INVALID_ARG;
    try {
        ctx->c.last_error.clear();
        ofrr_status st = f(&ctx->c);
        ctx->c.resolve_timers();
        return st;
    } catch (const Error &e) {
        ctx->c.last_error = e.msg;
        try {
            ctx->c.timer.pending.clear();
        } catch (...) {
        }
        return e.status;
    } catch (const std::exception &e) {
        ctx->c.last_error = std::string("internal error: ") + e.what();
        return OFRR_ERR_HIP;
    } catch (...) {
        ctx->c.last_error = "internal error";
        return OFRR_ERR_HIP;
    }
}

static void validate_matrix(const ofrr_matrix *A, bool square) {
    OFRR_CHECK_ARG(A != nullptr, "A is NULL");
    OFRR_CHECK_ARG(A->rows >= 1 && A->cols >= 1, "A must have rows >= 1 and cols >= 1");
    OFRR_CHECK_ARG(A->values != nullptr, "A->values is NULL");
    OFRR_CHECK_ARG(A->dtype == OFRR_F64 || A->dtype == OFRR_F32, "A values must be F64 or F32");
    if (square) OFRR_CHECK_ARG(A->rows == A->cols, "A must be square for an eigenproblem");
    if (A->format == OFRR_DENSE_COLMAJOR) {
        OFRR_CHECK_ARG(A->ld >= A->rows, "ld must be >= rows");
    } else if (A->format == OFRR_CSR) {
        OFRR_CHECK_ARG(A->row_ptr && A->col_idx, "CSR row_ptr/col_idx are NULL");
        OFRR_CHECK_ARG(A->nnz >= 0 && A->nnz < (int64_t)0x7fffffff, "CSR nnz out of range");
        OFRR_CHECK_ARG(A->rows < (int64_t)0x7fffffff, "CSR rows must fit int32");
    } else {
        fail(OFRR_ERR_INVALID_ARG, "unknown matrix format");
    }
}

static void validate_plan(const ofrr_plan *p) {
    OFRR_CHECK_ARG(p != nullptr, "plan is NULL");
    OFRR_CHECK_ARG(p->stab == 0 || p->stab == 1, "plan.stab must be 0 or 1");
    OFRR_CHECK_ARG(p->projection == 0 || p->projection == 1, "plan.projection must be 0 or 1");
    OFRR_CHECK_ARG(p->qr_dtype == -1 || p->qr_dtype == OFRR_F64 || p->qr_dtype == OFRR_F32 || p->qr_dtype == OFRR_F16,
                   "plan.qr_dtype must be -1, F64, F32 or F16");
    OFRR_CHECK_ARG(p->matvec_round == -1 || p->matvec_round == OFRR_F16 || p->matvec_round == OFRR_BF16,
                   "plan.matvec_round must be -1, F16 or BF16");
    OFRR_CHECK_ARG(p->tail_digits == 0 || (p->tail_digits >= 4 && p->tail_digits <= 6),
                   "plan.tail_digits must be 0, 4, 5 or 6");
    OFRR_CHECK_ARG(p->basis_dtype == OFRR_F64 || p->basis_dtype == OFRR_BF16 ||
                       p->basis_dtype == OFRR_F16 || p->basis_dtype == OFRR_F32 ||
                       p->basis_dtype == OFRR_F8E4M3,
                   "unknown basis_dtype");
    OFRR_CHECK_ARG(p->gram_accum >= OFRR_ACC_F32 && p->gram_accum <= OFRR_ACC_F64, "unknown gram_accum");
    OFRR_CHECK_ARG(p->filter == OFRR_POWER || p->filter == OFRR_CHEBYSHEV, "unknown filter");
    OFRR_CHECK_ARG(p->degree >= 1 && p->degree <= 1000, "degree must be in [1, 1000]");
    if (p->filter == OFRR_CHEBYSHEV)
        OFRR_CHECK_ARG(std::isfinite(p->lo) && std::isfinite(p->hi) && p->lo < p->hi,
                       "Chebyshev interval needs finite lo < hi");
    OFRR_CHECK_ARG(p->drop_tol >= 0 && p->tol >= 0 && p->anorm >= 0, "tolerances must be >= 0");
    OFRR_CHECK_ARG(p->max_iters >= 1, "max_iters must be >= 1");
    OFRR_CHECK_ARG(p->stall_iters >= 1, "stall_iters must be >= 1");
    OFRR_CHECK_ARG(p->b_split == 1 || p->b_split == 2, "b_split must be 1 or 2");
    OFRR_CHECK_ARG(p->tail_product == OFRR_TAIL_F64 || p->tail_product == OFRR_TAIL_I8_SLICED,
                   "tail_product must be OFRR_TAIL_F64 or OFRR_TAIL_I8_SLICED");
}

extern "C" {

void ofrr_plan_default(ofrr_plan *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->basis_dtype = OFRR_F64;
    p->gram_accum = OFRR_ACC_F64;
    p->refine = 0;
    p->filter = OFRR_POWER;
    p->degree = 1;
    p->lo = 0.0;
    p->hi = 0.0;
    p->drop_tol = 0.0;
    p->tol = 0.0;
    p->anorm = 0.0;
    p->max_iters = 20;
    p->stall_iters = 3;
    p->switch_resid = 0.0;
    p->b_split = 1;
    p->profile = 0;
    p->tail_product = OFRR_TAIL_F64;
    p->gram_switch_t = 0.0;
    p->svd_form = 0;
    p->stab = 0;
    p->projection = 0;
    p->qr_dtype = -1;
    p->matvec_round = -1;
    p->tail_digits = 0;
}

ofrr_status ofrr_create(ofrr_ctx *out, int device, void *hip_stream) {
    if (!out) return OFRR_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        g_create_error = "no HIP device visible";
        return OFRR_ERR_NO_DEVICE;
    }
    if (device < 0 || device >= count) {
        g_create_error = "device index out of range";
        return OFRR_ERR_NO_DEVICE;
    }
    ofrr_ctx ctx = new (std::nothrow) ofrr_ctx_s;
    if (!ctx) return OFRR_ERR_OOM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        g_create_error = "hipSetDevice failed";
        return OFRR_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->c.cu_count = prop.multiProcessorCount;
        ctx->c.max_lds = (int)prop.sharedMemPerBlock;
    }
    for (const char *f : kFamilies) {
        ctx->c.timer.names.push_back(f);
        ctx->c.timer.launches.push_back(0);
        ctx->c.timer.total_ms.push_back(0.0);
    }
    // this device's address of the fixed array the allocation-free
    // Hessenberg entry point uses (one copy per GPU)
    try {
        hess_scratch_address(&ctx->c);
    } catch (const Error &e) {
        g_create_error = e.msg;
        delete ctx;
        return e.status;
    }
    *out = ctx;
    return OFRR_OK;
}

ofrr_status ofrr_destroy(ofrr_ctx ctx) {
    if (!ctx) return OFRR_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    ctx->c.ws.release_all();
    if (ctx->c.pinned) (void)hipHostFree(ctx->c.pinned);
    if (ctx->c.sync_ev) (void)hipEventDestroy(ctx->c.sync_ev);
    if (ctx->c.graph_stream) (void)hipStreamDestroy(ctx->c.graph_stream);
    for (auto e : ctx->c.timer.pool) (void)hipEventDestroy(e);
    for (auto &p : ctx->c.timer.pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    delete ctx;
    return OFRR_OK;
}

const char *ofrr_last_error(ofrr_ctx ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->c.last_error.c_str();
}

ofrr_status ofrr_kernel_stats(ofrr_ctx ctx, const char *name, int64_t *launches, double *total_ms) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(name && launches && total_ms, "NULL argument");
        const int f = c->timer.family(name);
        OFRR_CHECK_ARG(f >= 0, std::string("unknown kernel family: ") + name);
        c->resolve_timers();
        *launches = c->timer.launches[f];
        *total_ms = c->timer.total_ms[f];
        // "spmm" is every CSR product: also the per-storage families;
        // "product_i8x" every digit-plane product: also the per-digit ones
        auto add = [&](std::initializer_list<const char *> subs) {
            for (const char *sub : subs) {
                const int g = c->timer.family(sub);
                *launches += c->timer.launches[g];
                *total_ms += c->timer.total_ms[g];
            }
        };
        if (std::string(name) == "spmm") add({"spmm_f16", "spmm_f32", "spmm_f64"});
        if (std::string(name) == "product_i8x") add({"product_i8x_d4", "product_i8x_d5", "product_i8x_d6"});
        return OFRR_OK;
    });
}

ofrr_status ofrr_kernel_stats_reset(ofrr_ctx ctx) {
    return guarded(ctx, [&](Context *c) {
        c->resolve_timers();
        for (auto &v : c->timer.launches) v = 0;
        for (auto &v : c->timer.total_ms) v = 0.0;
        return OFRR_OK;
    });
}

ofrr_status ofrr_eig_partial(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             ofrr_which which, const ofrr_plan *plan, const double *X0,
                             double *evals, double *evecs, double *resid, ofrr_info *info) {
    return guarded(ctx, [&](Context *c) {
        validate_matrix(A, true);
        validate_plan(plan);
        OFRR_CHECK_ARG(which == OFRR_LARGEST || which == OFRR_SMALLEST, "unknown which");
        OFRR_CHECK_ARG(k >= 1 && k <= basis && basis <= A->rows, "need 1 <= k <= basis <= n");
        OFRR_CHECK_ARG(basis <= 512, "basis must be <= 512");
        OFRR_CHECK_ARG(evals && evecs && resid, "output pointers must not be NULL");
        if (plan->basis_dtype == OFRR_F8E4M3)
            fail(OFRR_ERR_UNSUPPORTED, "eig_partial: basis_dtype F8E4M3 (the SVD path) not supported");
        if (plan->basis_dtype == OFRR_F32 && plan->refine >= 2)
            fail(OFRR_ERR_UNSUPPORTED, "eig_partial: the split middle phase needs a BF16 basis");
        if (plan->stab == 1) OFRR_CHECK_ARG(basis <= 512, "QR stabilisation: basis <= 512");
        if (A->format == OFRR_DENSE_COLMAJOR && plan->basis_dtype != OFRR_F64)
            OFRR_CHECK_ARG(A->rows < (int64_t)1 << 31, "dense reduced-precision path needs n < 2^31");
        OFRR_HIP(hipSetDevice(c->device));
        c->profile = plan->profile != 0;
        if (A->format == OFRR_CSR) check_csr(c, A);
        return eig_partial_impl(c, A, k, basis, which, plan, X0, evals, evecs, resid, info);
    });
}

ofrr_status ofrr_eig_general(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t basis, const ofrr_plan *plan,
                             const double *X0, double *evals_re, double *evals_im, double *evecs_re,
                             double *evecs_im, double *resid, ofrr_info *info) {
    return guarded(ctx, [&](Context *c) {
        validate_matrix(A, true);
        validate_plan(plan);
        OFRR_CHECK_ARG(k >= 1 && k <= basis && basis <= A->rows, "need 1 <= k <= basis <= n");
        OFRR_CHECK_ARG(basis <= 512, "basis must be <= 512");
        OFRR_CHECK_ARG(evals_re && evals_im && evecs_re && evecs_im && resid, "output pointers must not be NULL");
        OFRR_CHECK_ARG(plan->basis_dtype == OFRR_F64 || plan->basis_dtype == OFRR_BF16 ||
                           plan->basis_dtype == OFRR_F16,
                       "eig_general: basis F64, BF16 or F16");
        if (plan->filter != OFRR_POWER) fail(OFRR_ERR_UNSUPPORTED, "eig_general: power filter only");
        if (plan->stab != 0 || plan->projection != 0)
            fail(OFRR_ERR_UNSUPPORTED, "eig_general: Hessenberg stabilisation and the OFRR projection only");
        if (plan->gram_accum != OFRR_ACC_F64)
            fail(OFRR_ERR_UNSUPPORTED, "eig_general: the projections are accumulated in FP64 (gram_accum F64)");
        if (plan->qr_dtype >= 0 || plan->matvec_round >= 0)
            fail(OFRR_ERR_UNSUPPORTED, "eig_general: qr_dtype and matvec_round are not used");
        if (A->format == OFRR_DENSE_COLMAJOR && plan->basis_dtype != OFRR_F64)
            OFRR_CHECK_ARG(A->rows < (int64_t)1 << 31, "dense reduced-precision path needs n < 2^31");
        OFRR_HIP(hipSetDevice(c->device));
        c->profile = plan->profile != 0;
        if (A->format == OFRR_CSR) check_csr(c, A);
        return eig_general_impl(c, A, k, basis, plan, X0, evals_re, evals_im, evecs_re, evecs_im, resid, info);
    });
}

ofrr_status ofrr_svd_partial(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             const ofrr_plan *plan, const double *V0, double *sigma, double *U,
                             double *V, double *resid, ofrr_info *info) {
    return guarded(ctx, [&](Context *c) {
        validate_matrix(A, false);
        validate_plan(plan);
        OFRR_CHECK_ARG(A->format == OFRR_DENSE_COLMAJOR, "svd_partial: dense A only");
        OFRR_CHECK_ARG(plan->svd_form == 0 || plan->svd_form == 1, "svd_partial: svd_form 0 or 1");
        if (plan->svd_form == 1) {
            const int64_t mn = A->rows < A->cols ? A->rows : A->cols;
            OFRR_CHECK_ARG(k >= 1 && k <= basis && basis <= mn, "need 1 <= k <= basis <= min(m, n)");
            OFRR_CHECK_ARG(sigma && U && V && resid, "output pointers must not be NULL");
            OFRR_CHECK_ARG(plan->basis_dtype == OFRR_F64 || plan->basis_dtype == OFRR_BF16 ||
                               plan->basis_dtype == OFRR_F16,
                           "svd_partial (normal equations): basis F64, BF16 or F16");
            OFRR_HIP(hipSetDevice(c->device));
            c->profile = plan->profile != 0;
            return svd_normal_impl(c, A, k, basis, plan, V0, sigma, U, V, resid, info);
        }
        if (plan->stab != 0 || plan->projection != 0)
            fail(OFRR_ERR_UNSUPPORTED, "svd_partial: Hessenberg stabilisation and the OFRR projection only");
        OFRR_CHECK_ARG(plan->filter == OFRR_POWER && plan->degree == 1,
                       "svd_partial: power filter of degree 1");
        const int64_t mn = A->rows < A->cols ? A->rows : A->cols;
        OFRR_CHECK_ARG(k >= 1 && k <= basis && basis <= mn, "need 1 <= k <= basis <= min(m, n)");
        OFRR_CHECK_ARG(basis <= 256, "svd basis must be <= 256");
        OFRR_CHECK_ARG(sigma && U && V && resid, "output pointers must not be NULL");
        if (plan->gram_accum != OFRR_ACC_F64)
            fail(OFRR_ERR_UNSUPPORTED, "svd_partial: the projections are accumulated in FP64 (gram_accum F64)");
        OFRR_HIP(hipSetDevice(c->device));
        c->profile = plan->profile != 0;
        return svd_partial_impl(c, A, k, basis, plan, V0, sigma, U, V, resid, info);
    });
}

ofrr_status ofrr_eig_partial_batched(ofrr_ctx ctx, int32_t nprob, const ofrr_matrix *As, int32_t k,
                                     int32_t basis, ofrr_which which, const ofrr_plan *plan,
                                     const double *const *X0s, double *const *evals,
                                     double *const *evecs, double *const *resid,
                                     ofrr_info *infos) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(nprob >= 1 && As && evals && evecs && resid, "batched: NULL argument");
        validate_plan(plan);
        for (int32_t p = 0; p < nprob; ++p) {
            validate_matrix(&As[p], true);
            OFRR_CHECK_ARG(As[p].format == OFRR_DENSE_COLMAJOR, "batched: dense problems only");
            OFRR_CHECK_ARG(k >= 1 && k <= basis && basis <= As[p].rows, "batched: 1 <= k <= basis <= n");
            OFRR_CHECK_ARG(evals[p] && evecs[p] && resid[p], "batched: NULL output");
        }
        if (plan->basis_dtype == OFRR_F8E4M3 || plan->basis_dtype == OFRR_F32)
            fail(OFRR_ERR_UNSUPPORTED, "batched: basis_dtype F8E4M3/F32 not supported");
        OFRR_HIP(hipSetDevice(c->device));
        c->profile = plan->profile != 0;
        c->batched_last_grouped = 0;
        if (batched_grouped_supported(plan, nprob, As, k, basis)) {
            c->batched_last_grouped = 1;
            return batched_grouped_impl(c, nprob, As, k, basis, which, plan, X0s, evals, evecs, resid, infos);
        }
        // other plans: one problem after another
        ofrr_status worst = OFRR_OK;
        for (int32_t p = 0; p < nprob; ++p) {
            ofrr_status st = eig_partial_impl(c, &As[p], k, basis, which, plan,
                                              X0s ? X0s[p] : nullptr, evals[p], evecs[p], resid[p],
                                              infos ? &infos[p] : nullptr);
            if (st != OFRR_OK) worst = st;
        }
        return worst;
    });
}

ofrr_status ofrr_krylov_eig(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t nev, int32_t restarts,
                            ofrr_dtype basis_dtype, const double *v0, double tol, double *evals,
                            double *evecs, double *resid, ofrr_info *info) {
    return guarded(ctx, [&](Context *c) {
        validate_matrix(A, true);
        OFRR_CHECK_ARG(k >= 2 && k <= 512 && k <= A->rows, "krylov: 2 <= k <= min(512, n)");
        OFRR_CHECK_ARG(nev >= 1 && nev <= k, "krylov: 1 <= nev <= k");
        OFRR_CHECK_ARG(restarts >= 0, "krylov: restarts >= 0");
        OFRR_CHECK_ARG(tol >= 0, "krylov: tol >= 0");
        OFRR_CHECK_ARG(evals && evecs && resid, "krylov: NULL output");
        OFRR_CHECK_ARG(basis_dtype == OFRR_F64 || basis_dtype == OFRR_F32 || basis_dtype == OFRR_F16,
                       "krylov: basis F64, F32 or F16");
        OFRR_HIP(hipSetDevice(c->device));
        if (A->format == OFRR_CSR) check_csr(c, A);
        return krylov_eig_impl(c, A, k, nev, restarts, basis_dtype, v0, tol, evals, evecs, resid, info);
    });
}

ofrr_status ofrr_set_profile(ofrr_ctx ctx, int32_t on) {
    return guarded(ctx, [&](Context *c) {
        c->profile = on != 0;
        return OFRR_OK;
    });
}

ofrr_status ofrr_batched_last_config(ofrr_ctx ctx, int32_t *grouped, int32_t *rows_red, int32_t *rows_f64,
                                     int32_t *replays, double *first_product_ms) {
    return guarded(ctx, [&](Context *c) {
        if (first_product_ms) *first_product_ms = c->batched_last_first_ms;
        if (grouped) *grouped = c->batched_last_grouped;
        if (rows_red) *rows_red = 32 * c->batched_last_waves[0];
        if (rows_f64) *rows_f64 = 32 * c->batched_last_waves[1];
        if (replays) *replays = c->batched_last_replays;
        return OFRR_OK;
    });
}

ofrr_status ofrr_quantize(ofrr_ctx ctx, ofrr_dtype dst_dtype, int64_t count, const float *src, void *dst) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(count >= 0 && (count == 0 || (src && dst)), "quantize: bad arguments");
        OFRR_CHECK_ARG(dst_dtype == OFRR_BF16 || dst_dtype == OFRR_F16, "quantize: BF16 or F16");
        OFRR_HIP(hipSetDevice(c->device));
        if (count == 0) return OFRR_OK;
        if (dst_dtype == OFRR_BF16)
            cast_f32_to_bf16(c, count, src, (uint16_t *)dst);
        else
            cast_f32_to_f16(c, count, src, (uint16_t *)dst);
        c->sync();
        return OFRR_OK;
    });
}

ofrr_status ofrr_quantize_fp8_blocks(ofrr_ctx ctx, int64_t rows, int64_t cols, const float *A,
                                     int64_t lda, uint8_t *codes, float *scales) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(rows >= 1 && cols >= 1 && lda >= rows && A && codes && scales,
                       "quantize_fp8_blocks: bad arguments");
        OFRR_HIP(hipSetDevice(c->device));
        quantize_fp8_blocks(c, rows, cols, A, lda, codes, scales);
        c->sync();
        return OFRR_OK;
    });
}

ofrr_status ofrr_block_product(ofrr_ctx ctx, const ofrr_matrix *A, int32_t trans, int32_t b,
                               ofrr_dtype v_dtype, const void *V, void *W) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(A && V && W && b >= 1 && b <= 4096, "block_product: bad arguments");
        OFRR_CHECK_ARG(trans == 0 || trans == 1, "trans must be 0 or 1");
        OFRR_HIP(hipSetDevice(c->device));
        if (A->format == OFRR_CSR) {
            validate_matrix(A, false);
            OFRR_CHECK_ARG(trans == 0, "CSR product: trans must be 0");
            OFRR_CHECK_ARG(v_dtype == OFRR_F64 || v_dtype == OFRR_F32 || v_dtype == OFRR_F16 ||
                               v_dtype == OFRR_BF16,
                           "CSR product: V type");
            check_csr(c, A);
            product_csr(c, A, b, v_dtype, V, b, W, b);
        } else if (A->dtype == OFRR_BF16 || A->dtype == OFRR_F16) {
            OFRR_CHECK_ARG(A->rows >= 1 && A->cols >= 1 && A->ld >= A->rows && A->values,
                           "block_product: bad dense descriptor");
            OFRR_CHECK_ARG(v_dtype == A->dtype, "block_product: V must have A's type");
            const int64_t m = trans ? A->cols : A->rows, kd = trans ? A->rows : A->cols;
            product_lowp(c, A->dtype, m, kd, (const uint16_t *)A->values, A->ld, trans, b,
                         (const uint16_t *)V, nullptr, b, (float *)W, b);
        } else {
            validate_matrix(A, false);
            OFRR_CHECK_ARG(v_dtype == OFRR_F64, "block_product: FP64 V for an F64/F32 dense A");
            product_f64(c, A, trans, b, (const double *)V, b, (double *)W, b);
        }
        c->sync();
        return OFRR_OK;
    });
}

ofrr_status ofrr_block_product_sliced(ofrr_ctx ctx, const ofrr_matrix *A, int32_t trans, int32_t b,
                                      int32_t digits, const double *V, double *W) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(A && V && W && b >= 1 && b <= 4096, "block_product_sliced: bad arguments");
        OFRR_CHECK_ARG(digits == 0 || (digits >= 4 && digits <= 6), "block_product_sliced: digits 0, 4, 5 or 6");
        OFRR_CHECK_ARG(trans == 0 || trans == 1, "trans must be 0 or 1");
        validate_matrix(A, false);
        OFRR_CHECK_ARG(A->format == OFRR_DENSE_COLMAJOR && (A->dtype == OFRR_F32 || A->dtype == OFRR_F64),
                       "block_product_sliced: dense F32/F64 A");
        OFRR_HIP(hipSetDevice(c->device));
        const SlicedA sa = slice_matrix_i8(c, A, trans);
        product_i8s(c, sa, b, V, b, W, b, nullptr, digits == 0 ? 6 : digits);
        c->sync();
        return OFRR_OK;
    });
}

ofrr_status ofrr_block_product_fp8(ofrr_ctx ctx, int64_t rows, int64_t cols, const uint8_t *codes,
                                   const float *scales, int32_t trans, int32_t b, const float *V,
                                   float *W) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(rows >= 1 && cols >= 1 && codes && scales && V && W && b >= 1 && b <= 4096,
                       "block_product_fp8: bad arguments");
        OFRR_CHECK_ARG(trans == 0 || trans == 1, "trans must be 0 or 1");
        OFRR_HIP(hipSetDevice(c->device));
        const int64_t kdim = trans ? rows : cols, m = trans ? cols : rows;
        const int64_t ldt = f8_ldt(kdim);
        uint8_t *vc = c->buf<uint8_t>("f8_vcodes", (size_t)b * ldt);
        uint8_t *vs = c->buf<uint8_t>("f8_vscales", (size_t)b * (ldt / 32));
        quant_basis_f8(c, kdim, b, V, b, vc, vs);
        product_f8(c, rows, cols, codes, scales, trans, b, vc, vs, W, b);
        (void)m;
        c->sync();
        return OFRR_OK;
    });
}

ofrr_status ofrr_hessenberg(ofrr_ctx ctx, ofrr_dtype dtype, int64_t n, int32_t b, void *Y,
                            int64_t ldy, double tol, int32_t *piv, int32_t *keep, int32_t *kept) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(Y && piv && keep && n >= 1 && b >= 1 && ldy >= b && tol >= 0,
                       "hessenberg: bad arguments");
        OFRR_CHECK_ARG(dtype == OFRR_F64 || dtype == OFRR_F32, "hessenberg: F64 or F32");
        OFRR_HIP(hipSetDevice(c->device));
        const int32_t kk = hessenberg(c, dtype, n, b, Y, ldy, tol, piv, keep);
        if (kept) *kept = kk;
        return OFRR_OK;
    });
}

ofrr_status ofrr_hessenberg_noalloc(ofrr_ctx ctx, ofrr_dtype dtype, int64_t n, int32_t b, void *Y,
                                    int64_t ldy, double tol, int32_t *piv, int32_t *keep, int32_t *kept) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(Y && piv && keep && n >= 1 && b >= 1 && ldy >= b && tol >= 0,
                       "hessenberg_noalloc: bad arguments");
        OFRR_CHECK_ARG(dtype == OFRR_F64 || dtype == OFRR_F32, "hessenberg_noalloc: F64 or F32");
        OFRR_HIP(hipSetDevice(c->device));
        // no kernel timing here: its events are created on demand
        const bool prof = c->profile;
        c->profile = false;
        try {
            const int32_t kk = hessenberg_noalloc(c, dtype, n, b, Y, ldy, tol, piv, keep);
            c->profile = prof;
            if (kept) *kept = kk;
        } catch (...) {
            c->profile = prof;
            throw;
        }
        return OFRR_OK;
    });
}

ofrr_status ofrr_basis_generate(ofrr_ctx ctx, ofrr_basis_method method, ofrr_dtype storage, int64_t m,
                                int32_t n, void *A, int64_t lda, double tol, double *R, int32_t *piv,
                                int32_t *keep, int32_t *kept, double *kernel_ms) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(A && m >= 1 && n >= 1 && tol >= 0, "basis_generate: bad arguments");
        OFRR_CHECK_ARG((int)method >= 0 && (int)method <= 6, "basis_generate: unknown method");
        OFRR_HIP(hipSetDevice(c->device));
        basis_generate(c, (int)method, storage, m, n, A, lda, tol, R, piv, keep, kept, kernel_ms);
        return OFRR_OK;
    });
}

ofrr_status ofrr_project(ofrr_ctx ctx, int64_t n, int32_t b, ofrr_dtype v_dtype, const void *V,
                         ofrr_dtype w_dtype, const void *W, ofrr_accum accum, double *G,
                         double *H) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(V && W && G && H && n >= 1 && b >= 1 && b <= 4096, "project: bad arguments");
        OFRR_CHECK_ARG(w_dtype == OFRR_F64 || w_dtype == OFRR_F32, "project: W is F64 or F32");
        OFRR_CHECK_ARG(v_dtype != OFRR_F8E4M3, "project: V type");
        OFRR_CHECK_ARG(accum == OFRR_ACC_F32 || accum == OFRR_ACC_F32_COMPENSATED || accum == OFRR_ACC_F64,
                       "project: accumulation mode");
        if (accum != OFRR_ACC_F64 && (v_dtype == OFRR_F64 || w_dtype == OFRR_F64))
            fail(OFRR_ERR_UNSUPPORTED, "project: FP32 accumulation takes FP32, BF16 or F16 blocks");
        OFRR_HIP(hipSetDevice(c->device));
        project(c, n, b, v_dtype, V, b, w_dtype, W, b, accum, G, H);
        c->sync();
        return OFRR_OK;
    });
}

ofrr_status ofrr_pencil_eig(ofrr_ctx ctx, int32_t b, const double *H, const double *G,
                            ofrr_which which, double *theta, double *Y, int32_t *rank) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(H && G && theta && Y && b >= 1 && b <= 1024, "pencil_eig: bad arguments");
        OFRR_HIP(hipSetDevice(c->device));
        const int32_t r = pencil_eig(c, b, H, G, which, theta, Y, true);
        if (rank) *rank = r;
        return OFRR_OK;
    });
}

ofrr_status ofrr_pencil_eig_general(ofrr_ctx ctx, int32_t b, const double *H, const double *G, double *theta_re,
                                    double *theta_im, double *Y) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(H && G && theta_re && theta_im && Y && b >= 1 && b <= 1024,
                       "pencil_eig_general: bad arguments");
        OFRR_HIP(hipSetDevice(c->device));
        pencil_general(c, b, H, G, theta_re, theta_im, Y);
        return OFRR_OK;
    });
}

ofrr_status ofrr_svd_pencil(ofrr_ctx ctx, int32_t k1, int32_t k2, const double *B, const double *MU,
                            const double *MV, double *sigma, double *Y, double *Z) {
    return guarded(ctx, [&](Context *c) {
        OFRR_CHECK_ARG(B && MU && MV && sigma && Y && Z && k1 >= 1 && k2 >= 1 && k1 + k2 <= 1024,
                       "svd_pencil: bad arguments");
        OFRR_HIP(hipSetDevice(c->device));
        svd_pencil(c, k1, k2, B, MU, MV, sigma, Y, Z);
        c->sync();
        return OFRR_OK;
    });
}

}  // extern "C"
