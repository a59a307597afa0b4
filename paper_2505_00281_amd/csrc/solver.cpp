// solver.cpp -- host orchestration of the whole method: multi-step subspace
// iteration (Sec. 2, Alg. "Multiple Step Subspace Iteration") with the
// Hessenberg process in place of QR (Sec. 4.2), the orthogonalization-free
// projection (Sec. 3.1, eq. (geig); Sec. 3.2 for the SVD) and the mixed-
// precision plan (end of Sec. 4): reduced-precision products and basis,
// FP64 projected problem, FP64 final residuals.
//
// Per outer iteration (eigenvalues), with X the current Ritz block and
// AX = A X when known:
//   filter     Y1 = p1(A) X from AX (no product) or by a product, then the
//              remaining degree-1 products of the power/Chebyshev filter; every
//              filtered block is column-scaled by powers of two (Sec. 2);
//   stabilise  Hessenberg process on the last block (drops dependent columns);
//   project    W = A V, G = V^T V, H = V^T W;
//   solve      H y = theta G y in FP64;
//   lift       X = V Y, A X = W Y, residual estimates.
// A refined plan runs this first in the reduced precision and switches to
// an all-FP64 tail when the residual estimates stop improving.
#include <cstdlib>
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace ofrr {

namespace {

size_t esize(ofrr_dtype t) {
    switch (t) {
        case OFRR_F64: return 8;
        case OFRR_F32: return 4;
        case OFRR_BF16:
        case OFRR_F16: return 2;
        case OFRR_F8E4M3: return 1;
    }
    return 8;
}

double unit_roundoff(ofrr_dtype t) {
    switch (t) {
        case OFRR_F64: return std::ldexp(1.0, -52);
        case OFRR_F32: return std::ldexp(1.0, -23);
        case OFRR_F16: return std::ldexp(1.0, -10);
        case OFRR_BF16: return std::ldexp(1.0, -7);
        case OFRR_F8E4M3: return std::ldexp(1.0, -3);
    }
    return 0.0;
}

// One precision phase of the eigen iteration.
struct Phase {
    ofrr_dtype basis;    // F64: everything FP64; BF16/F16: reduced products, FP32 master blocks
    bool split = false;  // BF16 with A and the basis as two-term (hi + lo) splits
    bool sliced = false; // FP64 phase with products from exact INT8 digit planes
    bool f64() const { return basis == OFRR_F64; }
    ofrr_dtype master() const { return f64() ? OFRR_F64 : OFRR_F32; }
};

struct EigRun {
    Context *ctx;
    const ofrr_matrix *A;
    const ofrr_plan *plan;
    int64_t n;
    int32_t b;      // current basis size
    int32_t k;
    ofrr_which which;
    int products = 0;
    // reduced-precision copy of dense A (and the low half of its BF16 split)
    uint16_t *A_lo = nullptr;
    uint16_t *A_lo2 = nullptr;
    ofrr_dtype A_lo_t = OFRR_F64;
    SlicedA A_sl;  // digit planes of A for a sliced FP64 phase
    // power of two the method scales A by (A' = sigma A) when A's FP64
    // entries lie far outside the range in which sums of squares of the
    // products stay finite and normal; 1 otherwise (no extra work)
    double sigma = 1.0;
    // normal-equations operator (the A^T A form of the SVD): the products
    // are A^T (A V) with A m x n, n the operator's dimension
    bool normal = false;
    int64_t m = 0;

    // product of the current phase: W (master type) = A * Vblk (master type)
    // W = A V in the phase's arithmetic.  With defer (dense products only),
    // split-K partials may be left unreduced and described in *defer for a
    // consumer that sums them itself; defer->nsplit stays 0 when W is written.
    void product(const Phase &ph, const void *Vm, void *Wm, int32_t bc, SlabOut *defer = nullptr) {
        const bool rounded = plan->matvec_round >= 0 && !ph.f64();
        product_raw(ph, Vm, Wm, bc, sigma == 1.0 && !rounded ? defer : nullptr);
        if (defer && (sigma != 1.0 || rounded)) defer->nsplit = 0;
        // product outputs rounded to a narrower type (the MatVec precision
        // of the Sec. 2 experiment: computed accurately, the result stored
        // in the narrower type)
        if (rounded) round_block(ctx, (ofrr_dtype)plan->matvec_round, n * b0, (float *)Wm);
        // FP64 phases read A as stored: scale their products (exact: a power
        // of two on normal numbers); the reduced phases' copy of A is scaled
        if (sigma != 1.0 && ph.f64()) scale_array(ctx, n * b0, (double *)Wm, sigma);
    }
    void product_raw(const Phase &ph, const void *Vm, void *Wm, int32_t bc, SlabOut *defer) {
        ++products;
        if (defer) defer->nsplit = 0;
        const int64_t ld = b0;
        if (A->format == OFRR_CSR) {
            // the SpMM reads the phase's master block, rounding on load
            if ((sigma == 1.0 || ph.f64()) &&
                product_csr_master(ctx, A, bc, ph.basis, Vm, ld, Wm, nullptr, nullptr, false, 0.0, 0.0, 0.0))
                return;
            if (ph.f64()) {
                product_csr(ctx, A, bc, OFRR_F64, Vm, ld, Wm, ld);
            } else if (ph.basis == OFRR_F32) {
                product_csr(ctx, A, bc, OFRR_F32, Vm, ld, Wm, ld);
            } else {
                // round the FP32 block to the storage type and run the SpMM on it
                uint16_t *vlo = ctx->buf<uint16_t>("spmm_vlo", (size_t)n * ld);
                if (ph.basis == OFRR_F16)
                    cast_f32_to_f16(ctx, n * ld, (const float *)Vm, vlo);
                else
                    cast_f32_to_bf16(ctx, n * ld, (const float *)Vm, vlo);
                product_csr(ctx, A, bc, ph.basis, vlo, ld, Wm, ld);
                if (sigma != 1.0) fail(OFRR_ERR_UNSUPPORTED, "CSR A with entries outside [2^-300, 2^300] "
                                                             "needs the FP64 form");
            }
            return;
        }
        if (normal) {
            // T = A V (m x bc), then W = A^T T, each in the phase's arithmetic
            void *T = ctx->buf<double>("normal_T", (size_t)m * ld);
            if (ph.f64()) {
                product_f64(ctx, A, 0, bc, (const double *)Vm, ld, (double *)T, ld);
                product_f64(ctx, A, 1, bc, (const double *)T, ld, (double *)Wm, ld);
                return;
            }
            const int64_t ldt = lowp_ldt(std::max(m, n));
            uint16_t *vhi = ctx->buf<uint16_t>("prod_vhi", (size_t)ld * ldt);
            uint16_t *vlo = nullptr;
            if (plan->b_split >= 2) vlo = ctx->buf<uint16_t>("prod_vlo", (size_t)ld * ldt);
            split_block_t(ctx, ph.basis, n, bc, (const float *)Vm, ld, vhi, vlo, ldt);
            product_lowp_t(ctx, ph.basis, m, n, A_lo, m, 0, bc, vhi, vlo, ldt, (float *)T, ld, nullptr);
            split_block_t(ctx, ph.basis, m, bc, (const float *)T, ld, vhi, vlo, ldt);
            product_lowp_t(ctx, ph.basis, n, m, A_lo, m, 1, bc, vhi, vlo, ldt, (float *)Wm, ld, nullptr);
            return;
        }
        if (ph.f64()) {
            if (ph.sliced)
                product_i8s(ctx, A_sl, bc, (const double *)Vm, ld, (double *)Wm, ld, defer, i8_digits);
            else
                product_f64(ctx, A, atrans, bc, (const double *)Vm, ld, (double *)Wm, ld);
            return;
        }
        if (ph.basis == OFRR_F32) {
            // FP32 basis and product output; the sums are formed in FP64 from
            // A as stored and the FP32 block, then rounded to FP32
            double *v64 = ctx->buf<double>("f32_v64", (size_t)n * ld);
            double *w64 = ctx->buf<double>("f32_w64", (size_t)n * ld);
            cast_matrix(ctx, OFRR_F32, OFRR_F64, ld, n, Vm, ld, v64, ld);
            product_f64(ctx, A, atrans, bc, v64, ld, w64, ld);
            cast_matrix(ctx, OFRR_F64, OFRR_F32, ld, n, w64, ld, Wm, ld);
            return;
        }
        // dense reduced precision: split the FP32 block into hi (+ lo), written
        // K-contiguous per column for the MFMA product
        const int64_t ldt = lowp_ldt(n);
        uint16_t *vhi = ctx->buf<uint16_t>("prod_vhi", (size_t)ld * ldt);
        uint16_t *vlo = nullptr;
        if (plan->b_split >= 2 || ph.split) vlo = ctx->buf<uint16_t>("prod_vlo", (size_t)ld * ldt);
        split_block_t(ctx, ph.basis, n, bc, (const float *)Vm, ld, vhi, vlo, ldt);
        product_lowp_t(ctx, ph.basis, n, n, A_lo, n, atrans, bc, vhi, vlo, ldt, (float *)Wm, ld,
                       ph.split ? A_lo2 : nullptr, defer);
    }

    // one Chebyshev step Ynext = alpha (A Ycur - c Ycur) - beta Yprev with the
    // combine fused into a CSR product; false when this A or these blocks
    // take the separate product and combine
    bool cheb_fused(const Phase &ph, const void *Ycur, const void *Yprev, double alpha, double c, double beta,
                    void *Ynext, int32_t bc) {
        if (A->format != OFRR_CSR || sigma != 1.0 || normal) return false;
        if (!product_csr_master(ctx, A, bc, ph.basis, Ycur, b0, Ynext, Ycur, Yprev, true, alpha, c, beta))
            return false;
        ++products;
        return true;
    }

    // dense products read A^T (a symmetric A: A^T = A, the K-contiguous
    // form of the column-major storage) or A itself (a general A)
    int atrans = 1;
    int64_t b0 = 0;  // leading dimension of every block (the initial basis size)
    // digits per side of the INT8 digit-plane products (sliced FP64 phase)
    int i8_digits = 6;
};

// Residual level at which a reduced-precision phase hands over to the
// next: plan.switch_resid when set; otherwise, for an FP32 phase, eight
// units of FP32 rounding (9.5e-7 on the scale of anorm: its blocks cannot
// represent a smaller residual), so that a slowly converging problem does
// not leave it early on a pause of the stall rule.  Other phases leave on
// the stall rule alone.
double switch_level(const ofrr_plan *plan, const Phase &ph) {
    if (plan->switch_resid > 0) return plan->switch_resid;
    if (ph.basis == OFRR_F32) return 8.0 * std::ldexp(1.0, -23);
    return -1.0;
}


}  // namespace

// Digits per side for a sliced FP64 iteration, from the largest wanted
// residual estimate of the iteration before it.  A product with S digits
// per side is exact up to about 2^-7S of the row and column scales (four:
// 3.7e-9, five: 2.9e-11, six: 2.3e-13), which bounds the residual the
// iteration can reach.  Fewer digits are taken only while the residual is
// at least a hundred times above that level, with a factor 16 for |A||V|
// over |A V|: the subspace is not perturbed beyond what the iteration still
// has to shed, and the final iterations, which decide the returned pairs,
// run six.
int i8_digits_for(double emax) {
    if (!(emax < INFINITY)) return 6;
    if (emax > 1600.0 * std::ldexp(1.0, -28)) return 4;
    if (emax > 1600.0 * std::ldexp(1.0, -35)) return 5;
    return 6;
}

ofrr_status eig_partial_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             ofrr_which which, const ofrr_plan *plan, const double *X0,
                             double *evals, double *evecs, double *resid, ofrr_info *info, bool normal) {
    // the operator: A (symmetric, n x n), or A^T A for an m x n A (normal)
    const int64_t n = normal ? A->cols : A->rows;
    const int64_t ld = basis;
    hipEvent_t ev0, ev1;
    OFRR_HIP(hipEventCreate(&ev0));
    OFRR_HIP(hipEventCreate(&ev1));
    OFRR_HIP(hipEventRecord(ev0, ctx->stream));

    EigRun run;
    run.ctx = ctx;
    run.A = A;
    run.plan = plan;
    run.n = n;
    run.b = basis;
    run.k = k;
    run.which = which;
    run.b0 = ld;
    run.normal = normal;
    run.m = A->rows;

    std::vector<Phase> phases;
    phases.push_back(Phase{plan->basis_dtype});
    const bool dense = A->format == OFRR_DENSE_COLMAJOR;
    if (plan->refine >= 2 && dense && !normal && plan->basis_dtype == OFRR_BF16) {
        Phase mid{OFRR_BF16};
        mid.split = true;
        phases.push_back(mid);
    }
    // CSR A: an FP32 middle phase after a 16-bit one (the SpMM reads only the
    // block and the sparse structure, so FP32 vectors cost about half the
    // FP64 tail's traffic per iteration)
    if (plan->refine >= 2 && !dense && (plan->basis_dtype == OFRR_F16 || plan->basis_dtype == OFRR_BF16))
        phases.push_back(Phase{OFRR_F32});
    if (plan->refine && plan->basis_dtype != OFRR_F64) {
        Phase tail{OFRR_F64};
        tail.sliced = dense && !normal && plan->tail_product == OFRR_TAIL_I8_SLICED;
        phases.push_back(tail);
    }
    bool any_split = false, any_sliced = false;
    for (auto &p : phases) {
        any_split = any_split || p.split;
        any_sliced = any_sliced || p.sliced;
    }
    // magnitude guard for FP64 entries: sums of squares of products (the
    // small pencil's reductions, residual norms) stay finite and normal for
    // |a| in [2^-300, 2^300]; outside it the method runs on sigma A with
    // sigma a power of two, and eigenvalues are scaled back at the end
    if (A->dtype == OFRR_F64 && !normal) {
        const double amax = absmax_values(ctx, A);
        if (!std::isfinite(amax)) fail(OFRR_ERR_NUMERIC, "A holds NaN or infinity");
        if (amax > 0) {
            int e = 0;
            (void)std::frexp(amax, &e);
            if (e > 300 || e < -300) run.sigma = std::ldexp(1.0, -e);
        }
    }
    // digit planes of A (rows of A^T, K-contiguous) for a sliced FP64 phase
    if (any_sliced) run.A_sl = slice_matrix_i8(ctx, A, 1);

    // quantise dense A once for the reduced-precision phases (Sec. 4: A
    // stored in reduced precision; a split phase also keeps A - bf16(A))
    if (dense && normal && !phases[0].f64()) {
        // the m x n reduced copy, column-major (ld m): both products read it
        run.A_lo_t = phases[0].basis;
        const int64_t m = A->rows;
        run.A_lo = ctx->buf<uint16_t>("A_lo", (size_t)m * n);
        cast_matrix(ctx, A->dtype, run.A_lo_t, m, n, A->values, A->ld, run.A_lo, m);
    } else if (dense && !phases[0].f64() && phases[0].basis != OFRR_F32) {
        run.A_lo_t = phases[0].basis;
        run.A_lo = ctx->buf<uint16_t>("A_lo", (size_t)n * n);
        const float *Af = nullptr;
        int64_t lda = A->ld;
        if (A->dtype == OFRR_F32) {
            Af = (const float *)A->values;
        } else {
            float *tmp = ctx->buf<float>("A_f32", (size_t)n * n);
            cast_matrix(ctx, OFRR_F64, OFRR_F32, n, n, A->values, A->ld, tmp, n, run.sigma);
            Af = tmp;
            lda = n;
        }
        if (any_split) {
            run.A_lo2 = ctx->buf<uint16_t>("A_lo2", (size_t)n * n);
            cast_f32_to_bf16x2(ctx, n, n, Af, lda, run.A_lo, run.A_lo2);
        } else if (lda == n) {
            if (run.A_lo_t == OFRR_BF16)
                cast_f32_to_bf16(ctx, n * n, Af, run.A_lo);
            else
                cast_f32_to_f16(ctx, n * n, Af, run.A_lo);
        } else {
            cast_matrix(ctx, OFRR_F32, run.A_lo_t, n, n, Af, lda, run.A_lo, n);
        }
    }

    // blocks (row-major n x ld), allocated in FP64 size so every phase fits
    const size_t blk = (size_t)n * ld;
    void *X = ctx->buf<double>("X", blk);
    void *AX = ctx->buf<double>("AX", blk);
    void *Y0 = ctx->buf<double>("Y0", blk);
    void *Y1 = ctx->buf<double>("Y1", blk);
    void *Y2 = ctx->buf<double>("Y2", blk);
    void *V = ctx->buf<double>("V", blk);
    void *W = ctx->buf<double>("W", blk);
    float *swork = ctx->buf<float>("scale_work", (size_t)ld * ((n + 4095) / 4096 + 2) + 256);
    double *G = ctx->buf<double>("G", (size_t)ld * ld);
    double *H = ctx->buf<double>("H", (size_t)ld * ld);
    double *Yr = ctx->buf<double>("Yr", (size_t)ld * ld);
    double *theta = ctx->buf<double>("theta", (size_t)ld + 8);
    int32_t *piv = ctx->buf<int32_t>("piv", (size_t)ld);
    int32_t *keep = ctx->buf<int32_t>("keep", (size_t)ld);
    const int64_t nblk = (n + 63) / 64;
    double *res2 = ctx->buf<double>("res2", (size_t)nblk * ld);
    double *xn2 = ctx->buf<double>("xn2", (size_t)nblk * ld);
    double *rest = ctx->buf<double>("res_est", (size_t)ld + 8);

    // start block X0 (column-major FP64) -> row-major master of phase 0
    {
        const double *src = X0;
        if (!src) {
            double *gen = ctx->buf<double>("X0_gen", blk);
            uniform_start(ctx, n, basis, 0x5EEDull, gen);
            src = gen;
        }
        colmajor_to_rowmajor(ctx, n, basis, src, n, phases[0].master(), X, ld);
    }

    const bool cheb = plan->filter == OFRR_CHEBYSHEV;
    // the damping interval of sigma A
    const double cc = cheb ? 0.5 * (plan->hi + plan->lo) * run.sigma : 0.0;
    const double ee = cheb ? 0.5 * (plan->hi - plan->lo) * run.sigma : 1.0;

    int32_t bc = basis;  // current basis size
    scale_columns_reset(ctx);
    bool have_ax = false;
    int iters = 0, iters_low = 0;
    StallDetector stall_det{plan->stall_iters};
    size_t pi = 0;
    std::vector<double> est((size_t)k);
    double anorm_used = plan->anorm * run.sigma;
    // FP32 accumulation of G and H in the first (reduced-precision) phase,
    // switched to FP64 for an iteration when the previous mass matrix was
    // poorly conditioned: t(G) above the plan's bound, or not numerically
    // positive definite (t = inf)
    const double t_switch = plan->gram_switch_t > 0 ? plan->gram_switch_t : 1000.0;
    double gram_t = 1.0, gram_t_max = 0.0;
    int grams_f64 = 0;

    double emax_prev = INFINITY;
    while (iters < plan->max_iters) {
        const Phase &ph = phases[pi];
        const ofrr_dtype mt = ph.master();
        run.i8_digits = !ph.sliced ? 6 : (plan->tail_digits == 0 ? i8_digits_for(emax_prev) : plan->tail_digits);
        // default drop tolerance: machine epsilon of the arithmetic the
        // Hessenberg sweep runs in (FP32 for reduced-precision phases: it
        // works on the FP32 product output before the basis is rounded to
        // its storage type)
        const double tol = plan->drop_tol > 0 ? plan->drop_tol : unit_roundoff(mt);
        // ---- filter
        // Y0 = X: the blocks trade places (X is dead until the lift writes it)
        std::swap(Y0, X);
        // CSR A with a Chebyshev filter: the column scaling of the recurrence
        // is folded into the fused steps (keys of each output merged in its
        // epilogue, the scales applied as the next step reads its inputs),
        // so no pass over the blocks is spent on it
        // (OFRR_CHEB_FOLD=0 selects the separate scaling passes, for
        // comparisons: both give the same values)
        const char *fold_e = std::getenv("OFRR_CHEB_FOLD");
        const bool fold_env = !(fold_e && std::atoi(fold_e) == 0);
        const bool csr_scaled = fold_env && cheb && A->format == OFRR_CSR && run.sigma == 1.0 && !ph.split &&
                                plan->b_split < 2 && ld % 2 == 0 && bc <= 512;
        if (csr_scaled) {
            unsigned *keys = ctx->buf<unsigned>("cheb_keys", (size_t)3 * CM_KEYS);
            double *svec = ctx->buf<double>("cheb_s", 2 * 512);
            zero_keys(ctx, keys, 3 * CM_KEYS);
            auto K = [&](int i) { return keys + (size_t)(i % 3) * CM_KEYS; };
            bool ok = true;
            if (have_ax) {
                axpby_block(ctx, n, bc, mt, AX, Y0, ld, 1.0 / ee, -cc / ee, mt, Y1, ld);
                column_keys(ctx, mt, n, bc, Y1, ld, K(0));
            } else {
                ok = spmm_cheb_scaled(ctx, A, bc, ph.basis, Y0, nullptr, Y1, ld, 1.0 / ee, cc, 0.0, nullptr, nullptr,
                                      false, nullptr, K(0), nullptr);
                ++run.products;
            }
            int ki = 0;
            for (int d = 2; ok && d <= plan->degree; ++d, ++ki) {
                // p0: the scale step d - 1 applied, still pending on Y0
                const double *p0 = d == 2 ? nullptr : svec + (size_t)((d - 1) & 1) * 512;
                ok = spmm_cheb_scaled(ctx, A, bc, ph.basis, Y1, Y0, Y2, ld, 2.0 / ee, cc, 1.0, K(ki), p0, d > 2,
                                      svec + (size_t)(d & 1) * 512, K(ki + 1), K(ki + 2));
                ++run.products;
                std::swap(Y0, Y1);
                std::swap(Y1, Y2);
            }
            if (!ok) fail(OFRR_ERR_HIP, "scaled Chebyshev step: blocks not pair-aligned");
            scale_apply_keys(ctx, mt, n, bc, Y1, ld, K(ki), K(ki + 1));
        } else {
            if (have_ax) {
                if (cheb)
                    axpby_block(ctx, n, bc, mt, AX, Y0, ld, 1.0 / ee, -cc / ee, mt, Y1, ld);
                else
                    OFRR_HIP(hipMemcpyAsync(Y1, AX, (size_t)n * ld * esize(mt), hipMemcpyDeviceToDevice, ctx->stream));
            } else if (cheb) {
                if (!run.cheb_fused(ph, Y0, nullptr, 1.0 / ee, cc, 0.0, Y1, bc)) {
                    // the combine sums the product's split-K partials itself
                    SlabOut so;
                    run.product(ph, Y0, W, bc, &so);
                    if (so.nsplit > 0)
                        cheb_combine_slabs(ctx, n, bc, so, mt, Y0, nullptr, ld, 1.0 / ee, cc, 0.0, mt, Y1);
                    else
                        cheb_combine(ctx, n, bc, mt, W, mt, Y0, nullptr, ld, 1.0 / ee, cc, 0.0, mt, Y1);
                }
            } else {
                run.product(ph, Y0, W, bc);
                OFRR_HIP(hipMemcpyAsync(Y1, W, (size_t)n * ld * esize(mt), hipMemcpyDeviceToDevice, ctx->stream));
            }
            for (int d = 2; d <= plan->degree; ++d) {
                scale_columns_pow2(ctx, mt, n, bc, Y1, ld, mt, cheb ? Y0 : nullptr, ld, swork);
                if (!ph.f64() && !ph.split && plan->b_split < 2) round_block(ctx, ph.basis, n * ld, (float *)Y1);
                if (cheb) {
                    if (!run.cheb_fused(ph, Y1, Y0, 2.0 / ee, cc, 1.0, Y2, bc)) {
                        SlabOut so;
                        run.product(ph, Y1, W, bc, &so);
                        if (so.nsplit > 0)
                            cheb_combine_slabs(ctx, n, bc, so, mt, Y1, Y0, ld, 2.0 / ee, cc, 1.0, mt, Y2);
                        else
                            cheb_combine(ctx, n, bc, mt, W, mt, Y1, Y0, ld, 2.0 / ee, cc, 1.0, mt, Y2);
                    }
                } else {
                    run.product(ph, Y1, W, bc);
                    OFRR_HIP(hipMemcpyAsync(Y2, W, (size_t)n * ld * esize(mt), hipMemcpyDeviceToDevice, ctx->stream));
                }
                std::swap(Y0, Y1);
                std::swap(Y1, Y2);
            }
            scale_columns_pow2(ctx, mt, n, bc, Y1, ld, mt, nullptr, ld, swork);
        }
        // ---- stabilise (Hessenberg process, FP64 or FP32 arithmetic).  Its
        // kept count comes back with the residual estimates (one host
        // synchronisation per iteration): the rest of the iteration assumes
        // every column was kept and is redone on the compacted basis when
        // one was dropped.
        const int32_t *hstat = nullptr;
        // QR in a wider type than the phase stores: its basis is kept at the
        // phase's master precision, not rounded to the storage type
        const bool qr_wide = plan->stab == 1 && !ph.f64() && plan->qr_dtype >= 0 &&
                             !(plan->qr_dtype == OFRR_F16 && ph.basis == OFRR_F16);
        if (plan->stab == 1) {
            // QR by MGS with re-orthogonalisation (the classical comparison of
            // Sec. 5.2), by default in the phase's storage type: column-major
            // copy, the basis-generation kernel, back
            const ofrr_dtype qt = ph.f64() ? OFRR_F64
                                  : plan->qr_dtype >= 0 ? (ofrr_dtype)plan->qr_dtype
                                  : (ph.basis == OFRR_F16 ? OFRR_F16 : OFRR_F32);
            // with plan.drop_tol > 0, columns whose norm the projections
            // reduce to at most drop_tol of their norm before them are
            // excluded; by default none is (on the Gaussian-kernel studies
            // the FP32 and binary16 QR bases otherwise fell below the wanted
            // pair count in their first iteration)
            const double qtol = plan->drop_tol > 0 ? plan->drop_tol : 0.0;
            void *cm = ctx->buf<double>("qr_colmajor", (size_t)n * ld);
            transpose_cast(ctx, mt, qt, n, bc, Y1, ld, cm, n);
            int32_t kept_q = bc;
            basis_generate(ctx, 6, qt, n, bc, cm, n, qtol, nullptr, piv, keep, &kept_q, nullptr);
            transpose_cast(ctx, qt, mt, bc, n, cm, n, Y1, ld);
            hstat = status_pair(ctx, 0, kept_q);
        } else {
            hessenberg(ctx, mt, n, bc, Y1, ld, tol, piv, keep, &hstat);
        }
        std::swap(V, Y1);
        // storage rounding of the basis for a reduced-precision phase
        // (elementwise, so it commutes with the column compaction)
        if (!ph.f64() && !ph.split && plan->b_split < 2 && !qr_wide) round_block(ctx, ph.basis, n * ld, (float *)V);
        double *stage = nullptr;
        const bool f32_gram = pi == 0 && !ph.f64() && plan->gram_accum != OFRR_ACC_F64;
        ofrr_accum acc = OFRR_ACC_F64;
        if (f32_gram) {
            if (gram_t <= t_switch)
                acc = plan->gram_accum;
            else
                ++grams_f64;
        }
        for (bool first = true;; first = false) {
            // ---- project
            run.product(ph, V, W, bc);
            project(ctx, n, bc, mt, V, ld, mt, W, ld, acc, G, H);
            // the classical Rayleigh-Ritz projection takes the basis as
            // orthonormal: H y = theta y
            if (plan->projection == 1) set_identity(ctx, bc, G);
            // ---- solve; the rank comes back with the residual estimates:
            // every column is lifted, those beyond the rank are zero and the
            // next sweep drops them
            const int32_t *rank_dev = pencil_eig_async(ctx, bc, H, G, which, theta, Yr);
            if (f32_gram) gram_condition(ctx, bc, G, Yr, rank_dev, rest + k + 3);
            // ---- lift (X = V Y, AX = W Y) with residual estimates
            const int64_t prow = lift(ctx, n, bc, bc, mt, V, ld, mt, W, ld, Yr, bc, theta, mt, X, AX, ld, res2, xn2);
            // residual estimates of the k wanted pairs
            if (plan->anorm <= 0) {
                std::vector<double> th((size_t)bc);
                OFRR_HIP(hipMemcpyAsync(th.data(), theta, sizeof(double) * bc, hipMemcpyDeviceToHost,
                                        ctx->stream));
                ctx->sync();
                double m = 0.0;
                for (double v : th) m = std::max(m, std::fabs(v));
                anorm_used = m > 0 ? m : 1.0;
            }
            residual_reduce(ctx, res2, xn2, (int)prow, bc, k, anorm_used, rest, rank_dev,
                            first ? hstat : nullptr);
            stage = ctx->host_stage<double>((size_t)k + 4);
            const int nread = f32_gram ? k + 4 : k + (first ? 3 : 1);
            OFRR_HIP(hipMemcpyAsync(stage, rest, sizeof(double) * nread, hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            if (!first) break;
            if (stage[k + 1] != 0.0) fail(OFRR_ERR_HIP, "hessenberg: wait for the column candidates timed out");
            const int32_t kept = (int32_t)stage[k + 2];
            if (kept <= 0) fail(OFRR_ERR_NUMERIC, "every basis column was dropped");
            if (kept == bc) break;
            compact_columns_rm(ctx, mt, n, bc, V, ld, keep, Y1, ld);
            std::swap(V, Y1);
            bc = kept;
            if (bc < k) fail(OFRR_ERR_NUMERIC, "basis lost rank below k");
        }
        ++iters;
        if (!ph.f64()) ++iters_low;
        if (f32_gram) {
            gram_t = stage[k + 3];
            gram_t_max = std::max(gram_t_max, gram_t);
        }
        have_ax = true;
        std::copy(stage, stage + k, est.begin());
        const int32_t rank = (int32_t)stage[k];
        if (rank < k) fail(OFRR_ERR_NUMERIC, "projected mass matrix lost rank below k");
        bc = rank;
        double emax = 0.0;
        for (double v : est) emax = std::max(emax, std::isfinite(v) ? v : INFINITY);
        if (!std::isfinite(emax)) fail(OFRR_ERR_NUMERIC, "non-finite residual estimate");
        emax_prev = emax;
        const bool last_phase = pi + 1 == phases.size();
        // (an iteration whose products took fewer than six digits is
        // followed by one with six before the loop may stop: its Ritz
        // values carry that product's error)
        if (last_phase && plan->tol > 0 && emax <= plan->tol && run.i8_digits == 6) break;
        if (!last_phase) {
            const bool stalled = stall_det.push(emax);
            const bool by_value = emax <= switch_level(plan, ph);
            if (stalled || by_value) {
                // next phase: promote X for the FP64 tail; AX is recomputed by a
                // product of the new phase in every case
                if (phases[pi + 1].f64() && !ph.f64()) promote_block(ctx, n * ld, X);
                ++pi;
                have_ax = false;
                stall_det.reset();
            }
        }
    }

    // ---- final FP64 residuals from A as stored
    const Phase &ph = phases[pi];
    double *Xf = ctx->buf<double>("X_final", (size_t)n * k + 8);
    double *AXf = ctx->buf<double>("AX_final", (size_t)n * k + 8);
    // X (row-major, ld) -> FP64 row-major n x k (ld k)
    cast_matrix(ctx, ph.master(), OFRR_F64, k, n, X, ld, Xf, k);
    {
        ++run.products;
        if (normal) {
            double *Tf = ctx->buf<double>("normal_Tf", (size_t)A->rows * k + 8);
            product_f64(ctx, A, 0, k, Xf, k, Tf, k);
            product_f64(ctx, A, 1, k, Tf, k, AXf, k);
        } else if (A->format == OFRR_CSR)
            product_csr(ctx, A, k, OFRR_F64, Xf, k, AXf, k);
        else
            product_f64(ctx, A, 1, k, Xf, k, AXf, k);
        if (run.sigma != 1.0) scale_array(ctx, n * k, AXf, run.sigma);
    }
    finalize_eig(ctx, n, k, Xf, k, AXf, k, theta, anorm_used, evals, evecs, resid);
    // eigenvalues of A = those of sigma A over sigma (residuals are relative)
    if (run.sigma != 1.0) scale_array(ctx, k, evals, 1.0 / run.sigma);
    OFRR_HIP(hipEventRecord(ev1, ctx->stream));
    std::vector<double> r((size_t)k);
    OFRR_HIP(hipMemcpyAsync(r.data(), resid, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    float ms = 0.f;
    OFRR_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    OFRR_HIP(hipEventDestroy(ev0));
    OFRR_HIP(hipEventDestroy(ev1));
    int nconv = 0;
    double rmax = 0.0;
    for (double v : r) {
        rmax = std::max(rmax, v);
        if (plan->tol > 0 ? v <= plan->tol : true) ++nconv;
    }
    if (info) {
        info->iters = iters;
        info->iters_low = iters_low;
        info->n_converged = nconv;
        info->basis_eff = bc;
        info->products = run.products;
        info->max_resid = rmax;
        info->seconds = ms * 1e-3;
        info->gram_t_max = gram_t_max;
        info->grams_f64 = grams_f64;
    }
    return (plan->tol > 0 && nconv < k) ? OFRR_NOT_CONVERGED : OFRR_OK;
}

// ---------------------------------------------------------------------------
// Real non-symmetric A (Sec. 3.1: complex Ritz values; eq. (geig) with the
// pencil (V^T A V, V^T V) of a non-orthogonal basis).  The same outer
// iteration with products A V, the power filter, the Hessenberg process,
// FP64 projections and the non-symmetric pencil; the Ritz block is held
// packed real (a conjugate pair as Re and Im of its + member), which is
// also the real restart basis.  The k wanted values are those of largest
// modulus.
// ---------------------------------------------------------------------------
ofrr_status eig_general_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis, const ofrr_plan *plan,
                             const double *X0, double *evals_re, double *evals_im, double *evecs_re,
                             double *evecs_im, double *resid, ofrr_info *info) {
    const int64_t n = A->rows;
    const int64_t ld = basis;
    hipEvent_t ev0, ev1;
    OFRR_HIP(hipEventCreate(&ev0));
    OFRR_HIP(hipEventCreate(&ev1));
    OFRR_HIP(hipEventRecord(ev0, ctx->stream));

    EigRun run;
    run.ctx = ctx;
    run.A = A;
    run.plan = plan;
    run.n = n;
    run.b = basis;
    run.k = k;
    run.which = OFRR_LARGEST;
    run.b0 = ld;
    run.atrans = 0;

    const bool dense = A->format == OFRR_DENSE_COLMAJOR;
    std::vector<Phase> phases;
    phases.push_back(Phase{plan->basis_dtype});
    if (plan->refine >= 2 && dense && plan->basis_dtype == OFRR_BF16) {
        Phase mid{OFRR_BF16};
        mid.split = true;
        phases.push_back(mid);
    }
    if (plan->refine >= 2 && !dense && (plan->basis_dtype == OFRR_F16 || plan->basis_dtype == OFRR_BF16))
        phases.push_back(Phase{OFRR_F32});
    if (plan->refine && plan->basis_dtype != OFRR_F64) {
        Phase tail{OFRR_F64};
        tail.sliced = dense && plan->tail_product == OFRR_TAIL_I8_SLICED;
        phases.push_back(tail);
    }
    bool any_split = false, any_sliced = false;
    for (auto &p : phases) {
        any_split = any_split || p.split;
        any_sliced = any_sliced || p.sliced;
    }
    if (A->dtype == OFRR_F64) {
        const double amax = absmax_values(ctx, A);
        if (!std::isfinite(amax)) fail(OFRR_ERR_NUMERIC, "A holds NaN or infinity");
        if (amax > 0) {
            int e = 0;
            (void)std::frexp(amax, &e);
            if (e > 300 || e < -300) run.sigma = std::ldexp(1.0, -e);
        }
    }
    // digit planes of A's rows (K-contiguous rows of A) for a sliced phase
    if (any_sliced) run.A_sl = slice_matrix_i8(ctx, A, 0);
    if (dense && !phases[0].f64() && phases[0].basis != OFRR_F32) {
        run.A_lo_t = phases[0].basis;
        run.A_lo = ctx->buf<uint16_t>("A_lo", (size_t)n * n);
        const float *Af = nullptr;
        int64_t lda = A->ld;
        if (A->dtype == OFRR_F32) {
            Af = (const float *)A->values;
        } else {
            float *tmp = ctx->buf<float>("A_f32", (size_t)n * n);
            cast_matrix(ctx, OFRR_F64, OFRR_F32, n, n, A->values, A->ld, tmp, n, run.sigma);
            Af = tmp;
            lda = n;
        }
        if (any_split) {
            run.A_lo2 = ctx->buf<uint16_t>("A_lo2", (size_t)n * n);
            cast_f32_to_bf16x2(ctx, n, n, Af, lda, run.A_lo, run.A_lo2);
        } else {
            cast_matrix(ctx, OFRR_F32, run.A_lo_t, n, n, Af, lda, run.A_lo, n);
        }
    }

    const size_t blk = (size_t)n * ld;
    void *X = ctx->buf<double>("X", blk);
    void *AX = ctx->buf<double>("AX", blk);
    void *Y1 = ctx->buf<double>("Y1", blk);
    void *Y2 = ctx->buf<double>("Y2", blk);
    void *V = ctx->buf<double>("V", blk);
    void *W = ctx->buf<double>("W", blk);
    float *swork = ctx->buf<float>("scale_work", (size_t)ld * ((n + 4095) / 4096 + 2) + 256);
    double *G = ctx->buf<double>("G", (size_t)ld * ld);
    double *H = ctx->buf<double>("H", (size_t)ld * ld);
    double *Yr = ctx->buf<double>("Yr", (size_t)ld * ld);
    double *th_re = ctx->buf<double>("theta", (size_t)ld + 8);
    double *th_im = ctx->buf<double>("theta_im", (size_t)ld + 8);
    int32_t *piv = ctx->buf<int32_t>("piv", (size_t)ld);
    int32_t *keep = ctx->buf<int32_t>("keep", (size_t)ld);
    const int64_t nblk = (n + 63) / 64;
    double *res2 = ctx->buf<double>("res2", (size_t)nblk * ld);
    double *xn2 = ctx->buf<double>("xn2", (size_t)nblk * ld);
    double *rest = ctx->buf<double>("res_est", (size_t)ld + 8);
    {
        const double *src = X0;
        if (!src) {
            double *gen = ctx->buf<double>("X0_gen", blk);
            uniform_start(ctx, n, basis, 0x5EEDull, gen);
            src = gen;
        }
        colmajor_to_rowmajor(ctx, n, basis, src, n, phases[0].master(), X, ld);
    }

    int32_t bc = basis;
    scale_columns_reset(ctx);
    bool have_ax = false;
    int iters = 0, iters_low = 0;
    StallDetector stall_det{plan->stall_iters};
    size_t pi = 0;
    double anorm_used = plan->anorm * run.sigma;
    double emax_prev = INFINITY;
    std::vector<double> hre, him;
    while (iters < plan->max_iters) {
        const Phase &ph = phases[pi];
        const ofrr_dtype mt = ph.master();
        run.i8_digits = !ph.sliced ? 6 : (plan->tail_digits == 0 ? i8_digits_for(emax_prev) : plan->tail_digits);
        const double tol = plan->drop_tol > 0 ? plan->drop_tol : unit_roundoff(mt);
        // ---- power filter: Y1 = A^degree X, every block column-scaled
        if (have_ax)
            OFRR_HIP(hipMemcpyAsync(Y1, AX, (size_t)n * ld * esize(mt), hipMemcpyDeviceToDevice, ctx->stream));
        else
            run.product(ph, X, Y1, bc);
        for (int d = 2; d <= plan->degree; ++d) {
            scale_columns_pow2(ctx, mt, n, bc, Y1, ld, mt, nullptr, ld, swork);
            if (!ph.f64() && !ph.split && plan->b_split < 2) round_block(ctx, ph.basis, n * ld, (float *)Y1);
            run.product(ph, Y1, Y2, bc);
            std::swap(Y1, Y2);
        }
        scale_columns_pow2(ctx, mt, n, bc, Y1, ld, mt, nullptr, ld, swork);
        // ---- stabilise
        const int32_t *hstat = nullptr;
        hessenberg(ctx, mt, n, bc, Y1, ld, tol, piv, keep, &hstat);
        std::swap(V, Y1);
        if (!ph.f64() && !ph.split && plan->b_split < 2) round_block(ctx, ph.basis, n * ld, (float *)V);
        double *stage = nullptr;
        for (bool first = true;; first = false) {
            // ---- project, solve, lift
            run.product(ph, V, W, bc);
            project(ctx, n, bc, mt, V, ld, mt, W, ld, OFRR_ACC_F64, G, H);
            const int32_t *pst = pencil_general_async(ctx, bc, H, G, th_re, th_im, Yr);
            lift(ctx, n, bc, bc, mt, V, ld, mt, W, ld, Yr, bc, nullptr, mt, X, AX, ld, nullptr, nullptr);
            residual_partials_general(ctx, mt, n, bc, X, AX, ld, th_re, th_im, res2, xn2);
            if (plan->anorm <= 0) {
                hre.resize((size_t)bc);
                him.resize((size_t)bc);
                OFRR_HIP(hipMemcpyAsync(hre.data(), th_re, sizeof(double) * bc, hipMemcpyDeviceToHost, ctx->stream));
                OFRR_HIP(hipMemcpyAsync(him.data(), th_im, sizeof(double) * bc, hipMemcpyDeviceToHost, ctx->stream));
                ctx->sync();
                double m = 0.0;
                for (int32_t i = 0; i < bc; ++i) m = std::max(m, std::hypot(hre[i], him[i]));
                anorm_used = m > 0 ? m : 1.0;
            }
            // estimates of the k wanted slots, then {pencil status, hessenberg
            // error flag, kept count}
            residual_reduce(ctx, res2, xn2, (int)nblk, bc, k, anorm_used, rest, pst, first ? hstat : nullptr);
            stage = ctx->host_stage<double>((size_t)k + 4);
            const int nread = k + (first ? 3 : 1);
            OFRR_HIP(hipMemcpyAsync(stage, rest, sizeof(double) * nread, hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            if (first) {
                // a dropped column leaves G singular: the pencil is redone
                // on the compacted basis before its status counts
                if (stage[k + 1] != 0.0) fail(OFRR_ERR_HIP, "hessenberg: wait for the column candidates timed out");
                const int32_t kept = (int32_t)stage[k + 2];
                if (kept <= 0) fail(OFRR_ERR_NUMERIC, "every basis column was dropped");
                if (kept != bc) {
                    compact_columns_rm(ctx, mt, n, bc, V, ld, keep, Y1, ld);
                    std::swap(V, Y1);
                    bc = kept;
                    if (bc < k) fail(OFRR_ERR_NUMERIC, "basis lost rank below k");
                    continue;
                }
            }
            if (stage[k] == 1.0) fail(OFRR_ERR_NUMERIC, "projected mass matrix is not positive definite");
            if (stage[k] == 2.0) fail(OFRR_ERR_NUMERIC, "small non-symmetric eigensolver did not converge");
            break;
        }
        ++iters;
        if (!ph.f64()) ++iters_low;
        have_ax = true;
        double emax = 0.0;
        for (int i = 0; i < k; ++i) emax = std::max(emax, std::isfinite(stage[i]) ? stage[i] : INFINITY);
        if (!std::isfinite(emax)) fail(OFRR_ERR_NUMERIC, "non-finite residual estimate");
        emax_prev = emax;
        const bool last_phase = pi + 1 == phases.size();
        if (last_phase && plan->tol > 0 && emax <= plan->tol && run.i8_digits == 6) break;
        if (!last_phase) {
            const bool stalled = stall_det.push(emax);
            const bool by_value = emax <= switch_level(plan, ph);
            if (stalled || by_value) {
                if (phases[pi + 1].f64() && !ph.f64()) promote_block(ctx, n * ld, X);
                ++pi;
                have_ax = false;
                stall_det.reset();
            }
        }
    }

    // ---- final FP64 residuals from A as stored; a pair cut at k keeps its
    // second column
    const Phase &ph = phases[pi];
    double cut_im = 0.0;
    OFRR_HIP(hipMemcpyAsync(&cut_im, th_im + (k - 1), sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    const int32_t kk = (cut_im > 0.0 && k < bc) ? k + 1 : k;
    double *Xf = ctx->buf<double>("X_final", (size_t)n * kk + 8);
    double *AXf = ctx->buf<double>("AX_final", (size_t)n * kk + 8);
    cast_matrix(ctx, ph.master(), OFRR_F64, kk, n, X, ld, Xf, kk);
    ++run.products;
    if (A->format == OFRR_CSR)
        product_csr(ctx, A, kk, OFRR_F64, Xf, kk, AXf, kk);
    else
        product_f64(ctx, A, 0, kk, Xf, kk, AXf, kk);
    if (run.sigma != 1.0) scale_array(ctx, n * kk, AXf, run.sigma);
    finalize_general(ctx, n, k, Xf, AXf, kk, th_re, th_im, anorm_used, evals_re, evals_im, evecs_re, evecs_im,
                     resid);
    if (run.sigma != 1.0) {
        scale_array(ctx, k, evals_re, 1.0 / run.sigma);
        scale_array(ctx, k, evals_im, 1.0 / run.sigma);
    }
    OFRR_HIP(hipEventRecord(ev1, ctx->stream));
    std::vector<double> r((size_t)k);
    OFRR_HIP(hipMemcpyAsync(r.data(), resid, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    float ms = 0.f;
    OFRR_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    OFRR_HIP(hipEventDestroy(ev0));
    OFRR_HIP(hipEventDestroy(ev1));
    int nconv = 0;
    double rmax = 0.0;
    for (double v : r) {
        rmax = std::max(rmax, v);
        if (plan->tol > 0 ? v <= plan->tol : true) ++nconv;
    }
    if (info) {
        info->iters = iters;
        info->iters_low = iters_low;
        info->n_converged = nconv;
        info->basis_eff = bc;
        info->products = run.products;
        info->max_resid = rmax;
        info->seconds = ms * 1e-3;
        info->gram_t_max = 0.0;
        info->grams_f64 = 0;
    }
    return (plan->tol > 0 && nconv < k) ? OFRR_NOT_CONVERGED : OFRR_OK;
}

}  // namespace ofrr
