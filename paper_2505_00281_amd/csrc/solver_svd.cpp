// solver_svd.cpp -- the SVD form (Sec. 3.2, Alg. "Orthogonalization-Free
// Rayleigh-Ritz Projection for SVD"): alternating products U = A V and
// V = A^T U, each stabilised by the Hessenberg process, then the augmented
// pencil [0 B; B^T 0] vs blkdiag(U^T U, V^T V) with B = U^T A V, whose
// positive eigenvalues are the singular values; the lift sqrt(2) U Y and
// sqrt(2) V Z gives orthonormal singular vectors (Theorem of Sec. 3.2).
//
// B needs no third product: with T = A^T U formed for the right block,
// B = U^T A V = T^T V, where T is kept unscaled before the Hessenberg sweep
// turns it into V.  Restart is from all right Ritz vectors.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.hpp"

namespace ofrr {

namespace {

double unit_roundoff_svd(ofrr_dtype t) {
    switch (t) {
        case OFRR_F64: return std::ldexp(1.0, -52);
        case OFRR_F32: return std::ldexp(1.0, -23);
        case OFRR_F16: return std::ldexp(1.0, -10);
        case OFRR_BF16: return std::ldexp(1.0, -7);
        case OFRR_F8E4M3: return std::ldexp(1.0, -3);
    }
    return 0.0;
}

}  // namespace

ofrr_status svd_partial_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             const ofrr_plan *plan, const double *V0, double *sigma, double *U,
                             double *V, double *resid, ofrr_info *info) {
    const int64_t m = A->rows, n = A->cols;
    const int64_t ld = basis;
    hipEvent_t ev0, ev1;
    OFRR_HIP(hipEventCreate(&ev0));
    OFRR_HIP(hipEventCreate(&ev1));
    OFRR_HIP(hipEventRecord(ev0, ctx->stream));

    std::vector<ofrr_dtype> phases{plan->basis_dtype};
    if (plan->refine && plan->basis_dtype != OFRR_F64) phases.push_back(OFRR_F64);
    if (plan->basis_dtype == OFRR_F32)
        fail(OFRR_ERR_UNSUPPORTED, "svd_partial: basis_dtype F32 not supported");

    // quantise A once for the reduced phase: BF16/F16 elementwise, or FP8
    // e4m3fn with one power-of-two scale per 32 x 32 block (square blocks,
    // so the one copy serves both A V and A^T U)
    uint16_t *A_lo = nullptr;
    uint8_t *A_f8 = nullptr;
    float *A_f8s = nullptr;
    if (phases[0] != OFRR_F64) {
        const float *Af = (const float *)A->values;
        int64_t lda = A->ld;
        if (A->dtype == OFRR_F64) {
            float *tmp = ctx->buf<float>("svd_A_f32", (size_t)m * n);
            cast_matrix(ctx, OFRR_F64, OFRR_F32, m, n, A->values, A->ld, tmp, m);
            Af = tmp;
            lda = m;
        }
        if (phases[0] == OFRR_F8E4M3) {
            A_f8 = ctx->buf<uint8_t>("svd_A_f8", (size_t)m * n);
            A_f8s = ctx->buf<float>("svd_A_f8s", (size_t)((m + 31) / 32) * ((n + 31) / 32));
            quantize_fp8_blocks(ctx, m, n, Af, lda, A_f8, A_f8s);
        } else {
            A_lo = ctx->buf<uint16_t>("svd_A_lo", (size_t)m * n);
            cast_matrix(ctx, OFRR_F32, phases[0], m, n, Af, lda, A_lo, m);
        }
    }

    // FP64 tail with products from exact INT8 digit planes (six digits per
    // side, about 2^-42 of the row and column scales): A's rows for A V and
    // its columns for A^T U, sliced once
    const bool sliced = plan->tail_product == OFRR_TAIL_I8_SLICED && phases.back() == OFRR_F64 &&
                        phases.size() > 1 && (A->dtype == OFRR_F32 || A->dtype == OFRR_F64);
    SlicedA A_rows, A_cols;
    if (sliced) {
        A_rows = slice_matrix_i8(ctx, A, 0, "svd_i8_rows");
        A_cols = slice_matrix_i8(ctx, A, 1, "svd_i8_cols");
    }

    const size_t bm = (size_t)m * ld, bn = (size_t)n * ld;
    void *Ub = ctx->buf<double>("svd_U", bm);
    void *T1 = ctx->buf<double>("svd_T1", bm);
    void *Vb = ctx->buf<double>("svd_V", bn);
    void *T2 = ctx->buf<double>("svd_T2", bn);
    void *Ts = ctx->buf<double>("svd_Ts", bn);
    void *Vt = ctx->buf<double>("svd_Vt", bn);
    void *Ut = ctx->buf<double>("svd_Ut", bm);
    // staging of the product's basis operand: 16-bit codes (hi, lo) or, for
    // FP8, codes in vh and per-32-row scales in vl (both fit in bt halves)
    const size_t bt = (size_t)ld * std::max(lowp_ldt(std::max(m, n)), f8_ldt(std::max(m, n)));
    uint16_t *vh = ctx->buf<uint16_t>("svd_vh", bt);
    uint16_t *vl = ctx->buf<uint16_t>("svd_vl", bt);
    float *swork = ctx->buf<float>("svd_swork", (size_t)ld * ((std::max(m, n) + 4095) / 4096 + 2) + 256);
    double *B = ctx->buf<double>("svd_B", (size_t)ld * ld);
    double *MU = ctx->buf<double>("svd_MU", (size_t)ld * ld);
    double *MV = ctx->buf<double>("svd_MV", (size_t)ld * ld);
    double *Ys = ctx->buf<double>("svd_Ys", (size_t)ld * ld);
    double *Zs = ctx->buf<double>("svd_Zs", (size_t)ld * ld);
    double *sig = ctx->buf<double>("svd_sig", (size_t)ld + 8);
    double *est = ctx->buf<double>("svd_est", (size_t)ld + 8);
    int32_t *piv = ctx->buf<int32_t>("svd_piv", (size_t)ld);
    int32_t *keep = ctx->buf<int32_t>("svd_keep", (size_t)ld);
    int products = 0;

    size_t pi = 0;
    auto master = [&]() { return phases[pi] == OFRR_F64 ? OFRR_F64 : OFRR_F32; };
    auto esz = [&]() { return phases[pi] == OFRR_F64 ? (size_t)8 : (size_t)4; };

    {
        const double *src = V0;
        if (!src) {
            double *gen = ctx->buf<double>("svd_V0_gen", bn);
            uniform_start(ctx, n, basis, 0x5EEDull, gen);
            src = gen;
        }
        colmajor_to_rowmajor(ctx, n, basis, src, n, master(), Vb, ld);
    }

    // digits per side of the tail's digit-plane products: chosen at the start
    // of each tail iteration from the previous largest residual estimate (as
    // for the eigenproblem), so the first tail iterations take fewer
    int dig = 6;
    double emax_prev = INFINITY;
    auto tail_digits = [&]() {
        return plan->tail_digits == 0 ? i8_digits_for(emax_prev) : plan->tail_digits;
    };
    // W (rows x bc) = op(A) * X (cols x bc), phase arithmetic
    auto product = [&](int trans, const void *X, void *Wout, int32_t bc) {
        ++products;
        const int64_t rows = trans ? n : m, cols = trans ? m : n;
        if (phases[pi] == OFRR_F64) {
            if (sliced)
                product_i8s(ctx, trans ? A_cols : A_rows, bc, (const double *)X, ld, (double *)Wout, ld, nullptr,
                            dig);
            else
                product_f64(ctx, A, trans, bc, (const double *)X, ld, (double *)Wout, ld);
        } else if (phases[pi] == OFRR_F8E4M3) {
            // basis quantised per product: one scale per 32 rows of each column
            uint8_t *vc = reinterpret_cast<uint8_t *>(vh);
            uint8_t *vs = reinterpret_cast<uint8_t *>(vl);
            quant_basis_f8(ctx, cols, bc, (const float *)X, ld, vc, vs);
            product_f8(ctx, m, n, A_f8, A_f8s, trans, bc, vc, vs, (float *)Wout, ld);
        } else {
            const int64_t ldt = lowp_ldt(cols);
            split_block_t(ctx, phases[pi], cols, bc, (const float *)X, ld, vh,
                          plan->b_split >= 2 ? vl : nullptr, ldt);
            product_lowp_t(ctx, phases[pi], rows, cols, A_lo, m, trans, bc, vh,
                           plan->b_split >= 2 ? vl : nullptr, ldt, (float *)Wout, ld, nullptr);
        }
    };
    // scale, Hessenberg, compact into dst; returns kept columns
    auto stabilise = [&](void *Tin, int64_t rows, int32_t bc, void *dst) {
        // machine epsilon of the sweep's arithmetic (FP32 in reduced phases)
        const double tol = plan->drop_tol > 0 ? plan->drop_tol : unit_roundoff_svd(master());
        scale_columns_pow2(ctx, master(), rows, bc, Tin, ld, master(), nullptr, ld, swork);
        const int32_t kept = hessenberg(ctx, master(), rows, bc, Tin, ld, tol, piv, keep);
        if (kept < k) fail(OFRR_ERR_NUMERIC, "svd: basis lost rank below k");
        if (kept < bc)
            compact_columns_rm(ctx, master(), rows, bc, Tin, ld, keep, dst, ld);
        else
            OFRR_HIP(hipMemcpyAsync(dst, Tin, (size_t)rows * ld * esz(), hipMemcpyDeviceToDevice, ctx->stream));
        if ((phases[pi] == OFRR_BF16 || phases[pi] == OFRR_F16) && plan->b_split < 2)
            round_block(ctx, phases[pi], rows * ld, (float *)dst);
        return kept;
    };

    int32_t bv = basis;
    scale_columns_reset(ctx);
    int iters = 0, iters_low = 0;
    double anorm = plan->anorm;
    StallDetector stall_det{plan->stall_iters};
    int32_t r = 0;
    std::vector<double> eh((size_t)k), sh((size_t)ld);
    // Convergence test of the triplets of the previous iteration: the first
    // product of an iteration is T1 = A V~ with V~ the previous right Ritz
    // vectors, so ||A v~ - s u~|| comes for free.  (The other side,
    // A^T u~ - s v~, lies in span(V) and is orthogonal to it by the Galerkin
    // condition, i.e. it vanishes and tells nothing.)
    bool have_prev = false;
    const bool debug = std::getenv("OFRR_DEBUG") != nullptr;
    while (true) {
        ofrr_dtype mt = master();  // refreshed below if the phase changes
        dig = (sliced && pi + 1 == phases.size()) ? tail_digits() : 6;
        product(0, Vb, T1, bv);
        if (have_prev) {
            col_resid(ctx, mt, m, k, T1, Ut, ld, sig, anorm, est);
            OFRR_HIP(hipMemcpyAsync(eh.data(), est, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            double emax = 0.0;
            for (double v : eh) emax = std::max(emax, std::isfinite(v) ? v : INFINITY);
            if (!std::isfinite(emax)) fail(OFRR_ERR_NUMERIC, "svd: non-finite residual estimate");
            emax_prev = emax;
            const bool last = pi + 1 == phases.size();
            // (an estimate from products with fewer than six digits is
            // followed by an iteration with six before the loop may stop)
            if (last && plan->tol > 0 && emax <= plan->tol && dig == 6) break;
            if (!last) {
                const bool stalled = stall_det.push(emax);
                if (stalled || (plan->switch_resid > 0 && emax <= plan->switch_resid)) {
                    // FP64 tail: promote the right block and redo its product in
                    // FP64; the left Ritz block is promoted too, since the final
                    // residual reads it in the new phase's type when the
                    // iteration cap ends the loop right after the switch
                    promote_block(ctx, n * ld, Vb);
                    promote_block(ctx, m * ld, Ut);
                    ++pi;
                    stall_det.reset();
                    mt = master();
                    dig = sliced && pi + 1 == phases.size() ? tail_digits() : 6;
                    product(0, Vb, T1, bv);
                }
            }
        }
        if (iters >= plan->max_iters) break;
        const int32_t bu = stabilise(T1, m, bv, Ub);
        product(1, Ub, T2, bu);
        OFRR_HIP(hipMemcpyAsync(Ts, T2, bn * esz(), hipMemcpyDeviceToDevice, ctx->stream));
        bv = stabilise(T2, n, bu, Vb);
        gram_rect(ctx, n, bu, bv, mt, Ts, ld, mt, Vb, ld, B);
        gram_rect(ctx, m, bu, bu, mt, Ub, ld, mt, Ub, ld, MU);
        gram_rect(ctx, n, bv, bv, mt, Vb, ld, mt, Vb, ld, MV);
        if (debug) {
            std::vector<double> mu((size_t)bu * bu), mv((size_t)bv * bv);
            OFRR_HIP(hipMemcpyAsync(mu.data(), MU, sizeof(double) * bu * bu, hipMemcpyDeviceToHost, ctx->stream));
            OFRR_HIP(hipMemcpyAsync(mv.data(), MV, sizeof(double) * bv * bv, hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            double dmin_u = INFINITY, dmin_v = INFINITY, dmax_u = 0, dmax_v = 0;
            for (int i = 0; i < bu; ++i) {
                dmin_u = std::min(dmin_u, mu[(size_t)i * bu + i]);
                dmax_u = std::max(dmax_u, mu[(size_t)i * bu + i]);
            }
            for (int i = 0; i < bv; ++i) {
                dmin_v = std::min(dmin_v, mv[(size_t)i * bv + i]);
                dmax_v = std::max(dmax_v, mv[(size_t)i * bv + i]);
            }
            std::fprintf(stderr, "[ofrr svd] iter %d phase %zu bu %d bv %d diag(MU) [%g, %g] diag(MV) [%g, %g]\n",
                         iters, pi, bu, bv, dmin_u, dmax_u, dmin_v, dmax_v);
        }
        svd_pencil(ctx, bu, bv, B, MU, MV, sig, Ys, Zs);
        r = std::min(bu, bv);
        scale_array(ctx, (int64_t)bu * r, Ys, std::sqrt(2.0));
        scale_array(ctx, (int64_t)bv * r, Zs, std::sqrt(2.0));
        // U~ = U Y, V~ = V Z (orthonormal by the Theorem of Sec. 3.2)
        lift(ctx, m, bu, r, mt, Ub, ld, mt, nullptr, 0, Ys, bu, nullptr, mt, Ut, nullptr, ld, nullptr, nullptr);
        lift(ctx, n, bv, r, mt, Vb, ld, mt, nullptr, 0, Zs, bv, nullptr, mt, Vt, nullptr, ld, nullptr, nullptr);
        ++iters;
        if (phases[pi] != OFRR_F64) ++iters_low;
        OFRR_HIP(hipMemcpyAsync(sh.data(), sig, sizeof(double) * r, hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        if (plan->anorm <= 0) anorm = sh[0] > 0 ? sh[0] : 1.0;
        // restart from all right Ritz vectors
        std::swap(Vb, Vt);
        bv = r;
        have_prev = true;
        // a same-step run (tol = 0) ends after max_iters projections
        if (plan->tol <= 0 && iters >= plan->max_iters) break;
    }
    // final FP64 residuals from A as stored: U~ (m x k), V~ (n x k)
    const ofrr_dtype mt = master();
    double *Uf = ctx->buf<double>("svd_Uf", (size_t)m * k + 8);
    double *Vf = ctx->buf<double>("svd_Vf", (size_t)n * k + 8);
    double *AVf = ctx->buf<double>("svd_AVf", (size_t)m * k + 8);
    double *ATUf = ctx->buf<double>("svd_ATUf", (size_t)n * k + 8);
    cast_matrix(ctx, mt, OFRR_F64, k, m, Ut, ld, Uf, k);
    cast_matrix(ctx, mt, OFRR_F64, k, n, Vb, ld, Vf, k);
    products += 2;
    product_f64(ctx, A, 0, k, Vf, k, AVf, k);
    product_f64(ctx, A, 1, k, Uf, k, ATUf, k);
    finalize_svd(ctx, m, n, k, Uf, AVf, Vf, ATUf, k, sig, anorm, sigma, U, V, resid);
    OFRR_HIP(hipEventRecord(ev1, ctx->stream));
    std::vector<double> rr((size_t)k);
    OFRR_HIP(hipMemcpyAsync(rr.data(), resid, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    float ms = 0.f;
    OFRR_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    OFRR_HIP(hipEventDestroy(ev0));
    OFRR_HIP(hipEventDestroy(ev1));
    int nconv = 0;
    double rmax = 0.0;
    for (double v : rr) {
        rmax = std::max(rmax, v);
        if (plan->tol > 0 ? v <= plan->tol : true) ++nconv;
    }
    if (info) {
        info->iters = iters;
        info->iters_low = iters_low;
        info->n_converged = nconv;
        info->basis_eff = bv;
        info->products = products;
        info->max_resid = rmax;
        info->seconds = ms * 1e-3;
        info->gram_t_max = 0.0;
        info->grams_f64 = 0;
    }
    return (plan->tol > 0 && nconv < k) ? OFRR_NOT_CONVERGED : OFRR_OK;
}

ofrr_status eig_partial_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             ofrr_which which, const ofrr_plan *plan, const double *X0,
                             double *evals, double *evecs, double *resid, ofrr_info *info, bool normal);

namespace {

// sigma_i = sqrt(max(theta_i, 0)); U = (A V) / sigma column by column
__global__ void k_sqrt_clamp(const double *theta, double *sigma, int k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) sigma[i] = sqrt(theta[i] > 0.0 ? theta[i] : 0.0);
}
__global__ void k_div_cols(const double *AV, const double *sigma, double *U, int64_t m, int k) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * k; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % k);
        U[e] = sigma[c] > 0.0 ? AV[e] / sigma[c] : 0.0;
    }
}

}  // namespace

// The normal-equations form of the SVD (the A^T A variant): the eigen
// solver runs on the operator A^T A (each product is A V then A^T (A V), in
// the phase's arithmetic) and returns the largest eigenvalues theta = s^2
// with right vectors V; then s = sqrt(theta), U = A V / s, and the same
// FP64 finalisation as the augmented form (residual sqrt(||A v - s u||^2 +
// ||A^T u - s v||^2) / anorm, unit columns, sign fixed on v).  The
// eigenvalues carry the condition of A^T A: a singular value s is found to
// about u (s_1 / s)^2 relative, against u s_1 / s for the augmented pencil.
ofrr_status svd_normal_impl(Context *ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                            const ofrr_plan *plan, const double *V0, double *sigma, double *U,
                            double *V, double *resid, ofrr_info *info) {
    const int64_t m = A->rows, n = A->cols;
    ofrr_plan p = *plan;
    // the operator's normaliser is ||A||^2; its residual target is tighter by
    // the factor the left vector's division brings in (s_1 / s_k, unknown
    // beforehand: a fixed quarter)
    p.anorm = plan->anorm > 0 ? plan->anorm * plan->anorm : 0.0;
    p.tol = plan->tol * 0.25;
    double *th = ctx->buf<double>("svdn_theta", (size_t)k + 8);
    double *Xv = ctx->buf<double>("svdn_evecs", (size_t)n * k + 8);
    double *re = ctx->buf<double>("svdn_resid", (size_t)k + 8);
    ofrr_info ei;
    std::memset(&ei, 0, sizeof ei);
    const ofrr_status st = eig_partial_impl(ctx, A, k, basis, OFRR_LARGEST, &p, V0, th, Xv, re, &ei, true);
    if (st < 0) return st;
    double *sg = ctx->buf<double>("svdn_sigma", (size_t)k + 8);
    hipLaunchKernelGGL(k_sqrt_clamp, dim3(1), dim3(256), 0, ctx->stream, th, sg, k);
    double *Vf = ctx->buf<double>("svdn_Vf", (size_t)n * k + 8);
    double *AVf = ctx->buf<double>("svdn_AVf", (size_t)m * k + 8);
    double *Uf = ctx->buf<double>("svdn_Uf", (size_t)m * k + 8);
    double *ATUf = ctx->buf<double>("svdn_ATUf", (size_t)n * k + 8);
    colmajor_to_rowmajor(ctx, n, k, Xv, n, OFRR_F64, Vf, k);
    product_f64(ctx, A, 0, k, Vf, k, AVf, k);
    hipLaunchKernelGGL(k_div_cols, dim3((unsigned)std::min<int64_t>(4096, (m * k + 255) / 256)), dim3(256), 0,
                       ctx->stream, AVf, sg, Uf, m, k);
    product_f64(ctx, A, 1, k, Uf, k, ATUf, k);
    OFRR_HIP(hipGetLastError());
    // anorm of the SVD residual: the caller's, else the largest singular value
    double anorm = plan->anorm;
    if (!(anorm > 0)) {
        double s0 = 0.0;
        OFRR_HIP(hipMemcpyAsync(&s0, sg, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        OFRR_HIP(hipStreamSynchronize(ctx->stream));
        anorm = s0 > 0 ? s0 : 1.0;
    }
    finalize_svd(ctx, m, n, k, Uf, AVf, Vf, ATUf, k, sg, anorm, sigma, U, V, resid);
    std::vector<double> rr((size_t)k);
    OFRR_HIP(hipMemcpyAsync(rr.data(), resid, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    OFRR_HIP(hipStreamSynchronize(ctx->stream));
    int nconv = 0;
    double rmax = 0.0;
    for (double v : rr) {
        rmax = std::max(rmax, v);
        if (plan->tol > 0 ? v <= plan->tol : true) ++nconv;
    }
    if (info) {
        *info = ei;
        info->n_converged = nconv;
        info->max_resid = rmax;
        info->products = ei.products * 2 + 2;  // every operator product is two products with A
    }
    return (plan->tol > 0 && nconv < k) ? OFRR_NOT_CONVERGED : OFRR_OK;
}

}  // namespace ofrr
