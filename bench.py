"""Benchmark: Ritz pairs/s of the mixed-precision orthogonalization-free
Rayleigh-Ritz method against its FP64 form, on one MI355X.

Workload (the dense eigenvalue configuration of the method's headline
metric): symmetric A = Q diag(i^-1.5) Q^T + 1e-3 * (G + G^T)/sqrt(2),
n = 16384, stored FP32; k = 64 wanted pairs, basis 128, Chebyshev filter of
degree 4 per outer iteration.  Mixed form: BF16 basis and products (FP32
accumulation) with FP32-compensated projections, then a split-BF16 phase
(FP64 projections), then an FP64-accurate tail, each entered when the
previous one stalls; FP64 pencil throughout.  FP64 form: the same method
with every step in FP64.

One step = one complete eig_partial call (quantisation of A, every outer
iteration, the final FP64 residual check) with A and the start block
resident in HBM.  value = converged pairs / step time, where a returned pair
counts when its final FP64 residual ||Ax - lambda x|| / ||A|| is <= 1e-8 AND
its eigenvalue is within 1e-10 (relative) of the CPU oracle's, run to
convergence (residuals <= 1e-12) on the same stored A and start block after
the timed region.  The same oracle run, timed on the host cores, is the CPU
baseline (the whole run, until its 64 pairs met the same two criteria).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K_WANT, BASIS, DEGREE = 16384, 64, 128, 4
NOISE = 1e-3
TOL = 1e-8
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the current product kernels at n=16384, b=128
# (the FP64 product: 1123.4 MiB, used only by the FP64 form at that width),
# from rocprofv3 FETCH_SIZE + WRITE_SIZE passes over `bench.py --traffic-probe`,
# scaled by the same counters on a plain 1 GiB copy (FETCH x2, WRITE x1).
# The digit-plane product by digits per side; its family's entry is the
# average over the call's launches.  Counters were taken for these kernel
# versions; a changed kernel needs new passes before its entry is trusted.
MEASURED_TRAFFIC = {
    "product_bf16": 553.0 * 2**20,
}
MEASURED_TRAFFIC_I8 = {4: 1214.0 * 2**20, 5: 1488.6 * 2**20, 6: 1760.6 * 2**20}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(device):
    import torch
    import workloads as W
    lam = np.arange(1, N + 1, dtype=np.float64) ** -1.5
    t = time.time()
    A = W.dense_symmetric_prescribed(lam, 1002, noise_scale=NOISE, noise_seed=2002,
                                     dtype=torch.float32, device=device)
    X0 = torch.from_numpy(W.uniform_start(N, BASIS, 1102)).to(device)
    torch.cuda.synchronize()
    log(f"[bench] generated A ({N}x{N} FP32) in {time.time() - t:.1f}s")
    # filter interval: the spectrum below the (basis+1)-th eigenvalue is damped
    t = time.time()
    w = torch.linalg.eigvalsh(A).double().cpu().numpy()[::-1]
    log(f"[bench] spectrum bounds in {time.time() - t:.1f}s: "
        f"l1={w[0]:.6f} l{K_WANT}={w[K_WANT - 1]:.6f} l{BASIS + 1}={w[BASIS]:.6f} lmin={w[-1]:.6f}")
    lo, hi = float(w[-1]) - 1e-3 * abs(float(w[-1])), float(w[BASIS])
    anorm = float(max(abs(w[0]), abs(w[-1])))
    return A, X0, lo, hi, anorm


def run_steps(ctx, A, X0, plan, steps, warmup, label):
    import torch
    for _ in range(warmup):
        ctx.eig_partial(A, K_WANT, BASIS, plan=plan, X0=X0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    results = []
    t0 = time.time()
    e0.record(stream)
    for s in range(steps):
        r = ctx.eig_partial(A, K_WANT, BASIS, plan=plan, X0=X0)
        results.append(r)
        log(f"[bench] {label} step {s + 1}/{steps}: iters={r.info['iters']} "
            f"(low {r.info['iters_low']}) products={r.info['products']} "
            f"max_resid={r.info['max_resid']:.2e} device_s={r.info['seconds']:.4f}")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms = e0.elapsed_time(e1)
    return results, ms / steps, wall


def call_ms_summary(results):
    """Median and mean of the per-call device times (HIP events on the
    library's stream, one per eig_partial call)."""
    import statistics
    ms = [1e3 * r.info["seconds"] for r in results]
    return {"median": statistics.median(ms), "mean": statistics.fmean(ms), "per_call": ms}


EVAL_RTOL = 1e-10   # relative eigenvalue error against the converged oracle
ORACLE_TOL = 1e-12  # the oracle's own stopping residual


def oracle_converged(A, X0, lo, hi, anorm):
    """The oracle as it stands (FP64, MGS2 after every product, classical
    Rayleigh-Ritz, cyclic Jacobi) run to convergence on the host copy of the
    same stored A and start block, with the same filter.  Returns the
    reference pairs and the CPU baseline: the time at which all 64 of the
    oracle's own pairs met the metric's two criteria (residual <= 1e-8 and
    eigenvalue within 1e-10 of the converged value)."""
    from oracle import ofrr_oracle as O
    Ah = A.double().cpu().numpy()
    X0h = X0.cpu().numpy()
    t = time.time()
    ref = O.subspace_eig(Ah, X0h, K_WANT, filt="chebyshev", degree=DEGREE, lo=lo, hi=hi,
                         tol=ORACLE_TOL, anorm=anorm, max_outer=400, history=True)
    total = time.time() - t
    t_conv, it_conv = None, None
    for it, th, r, ts in ref.history:
        ok = (r <= TOL) & (np.abs(th - ref.theta) <= EVAL_RTOL * np.abs(ref.theta))
        if ok.all():
            t_conv, it_conv = ts, it
            break
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    log(f"[bench] oracle: {ref.iters} outer iterations in {total:.1f}s, "
        f"64 pairs met the criteria at iteration {it_conv} ({t_conv}s), {cores} threads")
    cpu = None
    if t_conv:
        cpu = {"value": K_WANT / t_conv, "unit": "Ritz pairs/s", "cores": int(cores), "kind": "oracle",
               "sample": (f"the whole workload (n={N}, k={K_WANT}, basis {BASIS}, degree-{DEGREE} "
                          f"Chebyshev) run by the oracle on the host, not projected: its {K_WANT} pairs "
                          f"met residual <= {TOL:g} and eigenvalue within {EVAL_RTOL:g} of its converged "
                          f"values after {it_conv} outer iterations, {t_conv:.1f}s; it stopped at "
                          f"residual <= {ORACLE_TOL:g} after {ref.iters} iterations, {total:.1f}s"),
               "oracle_iters_to_criteria": it_conv, "oracle_seconds_total": total}
    return ref, cpu


def accuracy(r, ref):
    """Per-result errors against the converged oracle and the number of
    pairs meeting both criteria."""
    ev = r.evals.cpu().numpy()
    res = r.resid.cpu().numpy()
    rel = np.abs(ev - ref.theta) / np.abs(ref.theta)
    nconv = int(((res <= TOL) & (rel <= EVAL_RTOL)).sum())
    return nconv, {"max_rel_eval_err_vs_oracle": float(rel.max()), "max_resid": float(res.max()),
                   "n_converged_both_criteria": nconv}



# --------------------------------------------------------------------------
# The other workloads of the method (one JSON line each; the default run is
# the dense workload above).
# --------------------------------------------------------------------------

def _cores():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def _timed_calls(fn, steps, warmup, label):
    """warmup untimed calls, then `steps` timed ones; returns (results,
    per-call device ms from the library's HIP events, ms per step from
    torch events bracketing the timed calls)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = []
    e0.record()
    for s_ in range(steps):
        res.append(fn())
        log(f"[bench] {label} step {s_ + 1}/{steps}")
    e1.record()
    torch.cuda.synchronize()
    return res, e0.elapsed_time(e1) / steps


def _family_roof(ctx, fam, bytes_per_launch, ops_per_launch, peak_mfma, dtype, kernel):
    n_l, t_l = ctx.kernel_stats(fam)
    avg = t_l / max(n_l, 1)
    sec = avg * 1e-3
    hbm_t = bytes_per_launch / (HBM_PEAK_GBS * 1e9)
    mfma_t = ops_per_launch / (peak_mfma * 1e12)
    if hbm_t >= mfma_t:
        ach = bytes_per_launch / sec / 1e9
        r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = ops_per_launch / sec / 1e12
        r = {"bound": "mfma", "achieved": round(ach, 2), "peak": peak_mfma,
             "unit": "TFLOP/s", "frac": round(ach / peak_mfma, 4)}
    r.update({"traffic": None, "kernel": kernel, "family": fam, "avg_launch_ms": avg, "launches": n_l,
              "algorithmic_bytes_per_launch": bytes_per_launch, "algorithmic_flops_per_launch": ops_per_launch,
              "dtype": dtype})
    return r


def bench_svd(args):
    """65536 x 8192 FP32 A = U diag(exp(-i/200)) V^T; top 100 singular
    triplets, basis 200; FP8 e4m3 basis build with 32 x 32 block scales,
    FP64-class tail (INT8 digit-plane products by default); against the
    FP64 form of the same method."""
    import torch
    import workloads as W
    from paper_2505_00281_amd import ofrr
    from oracle import ofrr_oracle as O
    m, n, k, b = 65536, 8192, 100, 200
    sig = np.exp(-np.arange(1, n + 1) / 200.0)
    t = time.time()
    A = W.svd_prescribed(m, n, sig, 1003, dtype=torch.float32, device="cuda")
    V0 = torch.from_numpy(W.uniform_start(n, b, 1103))
    torch.cuda.synchronize()
    log(f"[bench] svd: generated A in {time.time() - t:.1f}s")
    ctx = ofrr.Context(0)
    mixed_kw = dict(basis_dtype="f8e4m3", refine=1, tol=TOL * 0.5, max_iters=300, stall_iters=3, tail=args.tail)
    steps = max(1, min(args.steps, 5))
    res, ms = _timed_calls(lambda: ctx.svd_partial(A, k, b, plan=ofrr.make_plan(**mixed_kw), V0=V0), steps,
                           max(1, min(args.warmup, 2)), "svd mixed")
    fres, fms, ref = None, None, None
    if not args.no_fp64_form:
        fres, fms = _timed_calls(lambda: ctx.svd_partial(A, k, b, plan=ofrr.make_plan(basis_dtype="f64",
                                                                                      tol=TOL * 0.5, max_iters=300),
                                                         V0=V0), 2, 1, "svd fp64")
        ref = fres[-1]
    # reference values: the FP64 form's (or, without it, the closed form,
    # which holds up to the FP32 storage of A)
    sref = ref.sigma.cpu().numpy() if ref is not None else sig[:k]
    tol_ref = 1e-10 if ref is not None else 1e-6
    acc = []
    for r in res:
        s_ = r.sigma.cpu().numpy()
        rel = np.abs(s_ - sref) / sref
        ok = (r.resid.cpu().numpy() <= TOL) & (rel <= tol_ref)
        acc.append((int(ok.sum()), float(rel.max()), float(r.resid.max().item())))
    closed = float(np.max(np.abs(res[-1].sigma.cpu().numpy() - sig[:k]) / sig[:k]))
    fconv = int((ref.resid.cpu().numpy() <= TOL).sum()) if ref is not None else None
    value = sum(a[0] for a in acc) / (ms * 1e-3 * len(res))
    fvalue = fconv / (fms * 1e-3) if ref is not None else None
    # dominant product family on one profiled call
    ctx.kernel_stats_reset()
    ctx.svd_partial(A, k, b, plan=ofrr.make_plan(profile=True, **mixed_kw), V0=V0)
    torch.cuda.synchronize()
    fams = ["product_f8", "product_i8x", "product_reduce", "product_f64", "hessenberg", "small_eig", "gram", "lift",
            "scale", "quantize", "residual"]
    stats = {f: ctx.kernel_stats(f) for f in fams}
    f8_bytes = m * n + (m // 32) * (n // 32) * 4 + (m + n) * b + max(m, n) * b * 4
    roofline = _family_roof(ctx, "product_f8", f8_bytes, 2.0 * m * n * b, 5000.0, "fp8",
                            "k_gemm_f8 (A V or A^T U, e4m3 with E8M0 block scales, MFMA 32x32x64, FP32 accumulate)")
    roofline["per_family_ms_one_call"] = {f: round(t_, 3) for f, (n_, t_) in stats.items()}
    cpu = None
    if not args.no_oracle:
        # CPU baseline: the oracle's alternating iteration on the host copy, two
        # outer iterations timed and scaled to the FP64 form's iteration count
        Ah = A.double().cpu().numpy()
        t = time.time()
        O.subspace_svd(Ah, V0.numpy(), k, outer=2)
        per_it = (time.time() - t) / 2
        iters_needed = (ref or res[-1]).info["iters"]
        cpu = {"value": k / (per_it * iters_needed), "unit": "singular triplets/s", "cores": int(_cores()),
               "kind": "oracle", "sample": (f"two outer iterations of the oracle (A V, A^T U, MGS2 each, two-sided "
                                            f"Rayleigh-Ritz) on the same stored A, {per_it:.1f}s each, scaled to the "
                                            f"{iters_needed} iterations the FP64 form needs (projected)")}
    ctx.close()
    return {"metric": "singular triplets/sec at residual <=1e-8, mixed vs FP64 form, 1 MI355X; % roofline",
            "value": value, "unit": "singular triplets/s", "n_gpus": 1, "steps": len(res), "warmup": 1,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp8",
            "data": "synthetic",
            "config": {"workload": "dense SVD 65536 x 8192, FP32 A = U diag(exp(-i/200)) V^T; top k=100, basis 200, "
                                   "FP8 e4m3 basis build with 32x32 block scales, FP64-class tail "
                                   f"({'INT8 digit-plane products' if args.tail == 'i8' else 'FP64 products'})",
                       "m": m, "n": n, "k": k, "basis": b, "parallelism": "single GPU"},
            "n_converged": [a[0] for a in acc], "iters": res[-1].info["iters"], "iters_low": res[-1].info["iters_low"],
            "accuracy": {"max_rel_sigma_diff_vs_fp64_form": max(a[1] for a in acc),
                         "max_resid": max(a[2] for a in acc), "max_rel_sigma_err_vs_closed_form": closed,
                         "criterion": "residual <= 1e-8 and singular value within 1e-10 (relative) of the FP64 "
                                      "form's (same-step parity of that form with the oracle is tested at 1e-12); "
                                      "the closed form holds up to the FP32 storage of A"},
            "fp64_form": ({"value": fvalue, "ms_per_step": fms, "iters": ref.info["iters"], "n_converged": fconv}
                          if ref is not None else None),
            "speedup_vs_fp64_form": value / fvalue if fvalue else None,
            "roofline": roofline, "cpu_baseline": cpu}


def bench_general(args):
    """Real non-symmetric dense A (n 16384, FP64 storage) = S D S^-1 with
    moduli j^-1.5, half of the units conjugate pairs; the 64 eigenvalues of
    largest modulus, basis 128, power filter of degree 2; BF16 basis with
    the split-BF16 and sliced-INT8 FP64 phases against the FP64 form."""
    import torch
    import workloads as W
    from paper_2505_00281_amd import ofrr
    from oracle import ofrr_oracle as O
    n, k, b, deg = 16384, 64, 128, 2
    t = time.time()
    reals, pairs, lam = W.general_power_law_spectrum(n, 1006)
    A = W.general_prescribed(reals, pairs, 1007, nonnormal=0.3, dtype=torch.float64, device="cuda")
    X0 = torch.from_numpy(W.uniform_start(n, b, 1107))
    torch.cuda.synchronize()
    log(f"[bench] general: generated A in {time.time() - t:.1f}s")
    ctx = ofrr.Context(0)
    common = dict(degree=deg, tol=TOL * 0.5, anorm=1.0, max_iters=300)
    mixed_kw = dict(basis_dtype="bf16", refine=args.refine, stall_iters=args.stall_iters, tail=args.tail, **common)
    steps = max(1, min(args.steps, 5))
    res, ms = _timed_calls(lambda: ctx.eig_general(A, k, b, plan=ofrr.make_plan(**mixed_kw), X0=X0), steps,
                           max(1, min(args.warmup, 2)), "general mixed")
    fres, fms = None, None
    if not args.no_fp64_form:
        fres, fms = _timed_calls(lambda: ctx.eig_general(A, k, b, plan=ofrr.make_plan(basis_dtype="f64", **common),
                                                         X0=X0), 2, 1, "general fp64")

    def count(r):
        # each returned value matched to the nearest unused prescribed one
        th = r.evals.cpu().numpy()
        res_ = r.resid.cpu().numpy()
        pool = list(lam[:k + 8])
        errs = []
        for z in th:
            d = np.abs(np.array(pool) - z)
            j = int(np.argmin(d))
            errs.append(d[j])
            pool.pop(j)
        errs = np.array(errs)  # |lambda_1| = 1: absolute = relative to the largest modulus
        return int(((res_ <= TOL) & (errs <= 1e-10)).sum()), float(errs.max()), float(res_.max())

    acc = [count(r) for r in res]
    value = sum(a[0] for a in acc) / (ms * 1e-3 * len(res))
    facc = count(fres[-1]) if fres else None
    fvalue = facc[0] / (fms * 1e-3) if fres else None
    ctx.kernel_stats_reset()
    ctx.eig_general(A, k, b, plan=ofrr.make_plan(profile=True, **mixed_kw), X0=X0)
    torch.cuda.synchronize()
    fams = ["product_bf16", "product_bf16x2", "product_i8x", "product_reduce", "product_f64", "hessenberg",
            "small_eig", "gram", "lift", "scale", "quantize", "residual"]
    stats = {f: ctx.kernel_stats(f) for f in fams}
    gemm = 2.0 * n * n * b
    # method bytes per product: A read once as the phase stores it (BF16 copy;
    # FP64 as stored for the FP64-class phases) + the basis + the output
    alg = {"product_bf16": (n * n * 2 + n * b * 2 + n * b * 4, gemm, 2500.0, "bf16",
                            "k_gemm_lp<bf16> (A V, A column-major read M-contiguous, BF16 MFMA, FP32 accumulate)"),
           "product_bf16x2": (n * n * 2 + n * b * 2 + n * b * 4, gemm, 2500.0, "bf16",
                              "k_gemm_lp<bf16, split A and V> (A V)"),
           "product_i8x": (n * n * 8 + n * b * 16, gemm, 5000.0, "int8",
                           "k_gemm_i8s (A V from INT8 digit planes of A's rows; FP64-class product)")}
    dom = max(alg, key=lambda f: stats[f][1])
    by, ops, pk, dt, kern = alg[dom]
    roofline = _family_roof(ctx, dom, by, ops, pk, dt, kern)
    roofline["per_family_ms_one_call"] = {f: round(t_, 3) for f, (n_, t_) in stats.items()}
    cpu = None
    if not args.no_oracle:
        # CPU baseline: one outer iteration of the oracle (two products with
        # MGS2 after each, classical Rayleigh-Ritz with the library's
        # non-symmetric solver) on the host copy, scaled to the FP64 form's
        # iteration count
        Ah = A.cpu().numpy()
        t = time.time()
        O.subspace_eig_general(Ah, X0.numpy(), k, degree=deg, outer=1)
        per_it = time.time() - t
        iters_needed = (fres or res)[-1].info["iters"]
        cpu = {"value": k / (per_it * iters_needed), "unit": "Ritz pairs/s", "cores": int(_cores()),
               "kind": "oracle",
               "sample": (f"one outer iteration of the oracle ({deg} products with MGS2 after each, Rayleigh-Ritz "
                          f"with the library's non-symmetric eigensolver) on the same matrix, {per_it:.1f}s, scaled "
                          f"to the {iters_needed} iterations the FP64 form needs (projected)")}
    ctx.close()
    return {"metric": "Ritz pairs/sec at residual <=1e-8, mixed vs FP64 form, 1 MI355X; % roofline",
            "value": value, "unit": "Ritz pairs/s", "n_gpus": 1, "steps": len(res), "warmup": 1, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "dense real non-symmetric A = S D S^-1, n 16384 (FP64 storage), moduli j^-1.5 "
                                   "with half the units conjugate pairs, S = Q (I + 0.3 N); 64 eigenvalues of largest "
                                   "modulus, basis 128, power filter degree 2, BF16 basis with split-BF16 and "
                                   "sliced-INT8 FP64 phases",
                       "n": n, "k": k, "basis": b, "parallelism": "single GPU"},
            "n_converged": [a[0] for a in acc], "iters": res[-1].info["iters"],
            "iters_low": res[-1].info["iters_low"],
            "accuracy": {"max_eval_err_vs_prescribed": max(a[1] for a in acc), "max_resid": max(a[2] for a in acc),
                         "criterion": "residual <= 1e-8 and eigenvalue within 1e-10 of the prescribed one "
                                      "(|lambda_1| = 1; A stored in FP64)"},
            "fp64_form": ({"value": fvalue, "ms_per_step": fms, "iters": fres[-1].info["iters"],
                           "n_converged": facc[0], "max_eval_err": facc[1]} if fres else None),
            "speedup_vs_fp64_form": value / fvalue if fvalue else None,
            "roofline": roofline, "cpu_baseline": cpu}


def bench_laplacian(args):
    """CSR Dirichlet 5-point Laplacian on a 1024 x 1024 grid (n = 1,048,576);
    32 smallest eigenpairs, basis 64, degree-20 Chebyshev on [lambda_65, 8],
    FP32 vectors with an FP64 tail; against the FP64 form."""
    import torch
    import workloads as W
    from paper_2505_00281_amd import ofrr
    from oracle import ofrr_oracle as O
    Ng, k, b = 1024, 32, 64
    n = Ng * Ng
    rp, ci, v = W.laplacian_2d_csr(Ng)
    ev = W.laplacian_2d_eigenvalues(Ng)
    X0 = torch.from_numpy(W.uniform_start(n, b, 1104))
    mat = ofrr.csr_matrix(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(v).cuda())
    ctx = ofrr.Context(0)
    common = dict(filter="chebyshev", degree=20, lo=float(ev[b]), hi=8.0, tol=TOL * 0.5, anorm=8.0,
                  max_iters=3000)
    # FP32 vectors, then the FP64 tail once the residual reaches the FP32
    # level (a binary16 phase before it gains nothing here: the CSR steps
    # read the FP32 master block either way)
    mixed_kw = dict(basis_dtype="f32", refine=1, stall_iters=100, **common)
    steps = max(1, min(args.steps, 2))
    res, ms = _timed_calls(lambda: ctx.eig_partial(mat, k, b, which="smallest", plan=ofrr.make_plan(**mixed_kw),
                                                   X0=X0), steps, max(0, min(args.warmup, 1)), "laplacian mixed")
    fres, fms = None, None
    if not args.no_fp64_form:
        fres, fms = _timed_calls(lambda: ctx.eig_partial(mat, k, b, which="smallest",
                                                         plan=ofrr.make_plan(basis_dtype="f64", **common), X0=X0),
                                 1, 0, "laplacian fp64")

    def count(r):
        th = r.evals.cpu().numpy()
        res_ = r.resid.cpu().numpy() * 8.0 / 8.0
        rel = np.abs(th - ev[:k]) / ev[:k]
        return int(((res_ <= TOL) & (rel <= 1e-10)).sum()), float(rel.max()), float(res_.max())

    acc = [count(r) for r in res]
    value = sum(a[0] for a in acc) / (ms * 1e-3 * len(res))
    facc = count(fres[-1]) if fres else None
    fvalue = facc[0] / (fms * 1e-3) if fres else None
    ctx.kernel_stats_reset()
    ctx.eig_partial(mat, k, b, which="smallest", plan=ofrr.make_plan(profile=True, **mixed_kw), X0=X0)
    torch.cuda.synchronize()
    fams = ["spmm", "hessenberg", "small_eig", "gram", "lift", "scale", "quantize", "residual", "product_reduce"]
    stats = {f: ctx.kernel_stats(f) for f in fams}
    nnz = int(rp[-1])
    # one Chebyshev step per launch: the CSR arrays (FP32 values, int32
    # columns and row pointers) once, Y_j and Y_{j-1} read, Y_{j+1} written,
    # in the storage type of the phase the launch belongs to (2, 4 or 8 bytes)
    sub = {2: "spmm_f16", 4: "spmm_f32", 8: "spmm_f64"}
    per = {es: ctx.kernel_stats(f) for es, f in sub.items()}
    step_bytes = {es: nnz * 4 + nnz * 4 + (n + 1) * 4 + 3 * n * b * es for es in sub}
    launches = sum(nl for nl, _ in per.values())
    tot_ms = sum(t_ for _, t_ in per.values())
    tot_bytes = sum(per[es][0] * step_bytes[es] for es in sub)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_spmm_cheb_scaled (CSR Chebyshev step with the product, the three-term combine and the "
                          "column scaling fused)",
                "family": "spmm", "avg_launch_ms": tot_ms / max(launches, 1), "launches": launches,
                "algorithmic_bytes_per_launch": tot_bytes / max(launches, 1),
                "algorithmic_bytes_per_step_by_storage": {sub[es]: step_bytes[es] for es in sub},
                "per_storage": {sub[es]: {"launches": per[es][0], "avg_launch_ms": per[es][1] / max(per[es][0], 1),
                                          "GB_s": round(step_bytes[es] * per[es][0] / (per[es][1] * 1e-3) / 1e9, 1)
                                          if per[es][1] > 0 else None} for es in sub},
                "dtype": "f32/f64 phases"}
    roofline["per_family_ms_one_call"] = {f: round(t_, 3) for f, (n_, t_) in stats.items()}
    # CPU baseline: a bounded sample, one outer iteration of the oracle with a
    # degree-10 filter (10 CSR products, MGS2 after each, Rayleigh-Ritz),
    # scaled per product to the products the FP64 form needs
    cpu = None
    if not args.no_oracle:
        t = time.time()
        O.subspace_eig((rp, ci, v.astype(np.float64)), X0.numpy(), k, which="smallest", filt="chebyshev",
                       degree=10, lo=float(ev[b]), hi=8.0, outer=1)
        per_prod = (time.time() - t) / 10
        prods_needed = (fres or res)[-1].info["products"]
        cpu = {"value": k / (per_prod * prods_needed), "unit": "Ritz pairs/s", "cores": int(_cores()),
               "kind": "oracle",
               "sample": (f"one outer iteration of the oracle with a degree-10 filter (10 CSR products with MGS2 "
                          f"after each, Rayleigh-Ritz) on the same matrix, {per_prod:.2f}s per product, scaled to "
                          f"the {prods_needed} products the FP64 form needs (projected)")}
    ctx.close()
    return {"metric": "Ritz pairs/sec at residual <=1e-8, mixed vs FP64 form, 1 MI355X; % roofline",
            "value": value, "unit": "Ritz pairs/s", "n_gpus": 1, "steps": len(res), "warmup": 1, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "sparse SPD 5-point 2-D Laplacian, 1024 x 1024 grid (n=1,048,576, CSR, FP32 "
                                   "values); 32 smallest, degree-20 Chebyshev on [lambda_65, 8], basis 64, FP32 vectors "
                                   "with an FP64 tail",
                       "n": n, "nnz": nnz, "k": k, "basis": b, "refine": 1, "parallelism": "single GPU"},
            "n_converged": [a[0] for a in acc], "iters": res[-1].info["iters"], "iters_low": res[-1].info["iters_low"],
            "products": res[-1].info["products"],
            "accuracy": {"max_rel_eval_err_vs_closed_form": max(a[1] for a in acc),
                         "max_resid": max(a[2] for a in acc),
                         "criterion": "residual <= 1e-8 and eigenvalue within 1e-10 (relative) of the closed form "
                                      "4 - 2cos(p pi/1025) - 2cos(q pi/1025) (exact for the stored integer matrix)"},
            "fp64_form": ({"value": fvalue, "ms_per_step": fms, "iters": fres[-1].info["iters"],
                           "n_converged": facc[0]} if fres else None),
            "speedup_vs_fp64_form": value / fvalue if fvalue else None,
            "roofline": roofline, "cpu_baseline": cpu}


def bench_batched(args):
    """512 independent dense symmetric problems, n uniform in [256, 4096]
    (seeded), lambda_i = 0.9^i, FP32 storage; top 8, basis 16, power filter,
    BF16 basis with an FP64 tail, grouped launches replayed from a graph;
    against the FP64 form of the same batched method."""
    import torch
    import workloads as W
    from paper_2505_00281_amd import ofrr
    from oracle import ofrr_oracle as O
    k, b = 8, 16
    sizes = W.batched_sizes(1005)
    t = time.time()
    As, X0s = [], []
    for p, n in enumerate(sizes):
        lam = 0.9 ** np.arange(1, n + 1)
        As.append(W.dense_symmetric_prescribed(lam, 1005000 + p, dtype=torch.float32, device="cuda"))
        X0s.append(torch.from_numpy(W.uniform_start(int(n), b, 1105000 + p)))
    torch.cuda.synchronize()
    log(f"[bench] batched: generated {len(sizes)} problems in {time.time() - t:.1f}s")
    ctx = ofrr.Context(0)
    mixed = ofrr.make_plan(basis_dtype="bf16", refine=1, tol=TOL * 0.5, max_iters=200, stall_iters=3)
    f64 = ofrr.make_plan(basis_dtype="f64", tol=TOL * 0.5, max_iters=200)
    steps = max(1, min(args.steps, 10))
    res, ms = _timed_calls(lambda: ctx.eig_partial_batched(As, k, b, plan=mixed, X0s=X0s), steps,
                           max(1, args.warmup), "batched mixed")
    cfg = ctx.batched_last_config()
    call_ms = [1e3 * r[0].info["seconds"] for r in res]
    fres, fms = _timed_calls(lambda: ctx.eig_partial_batched(As, k, b, plan=f64, X0s=X0s), 3, 1, "batched fp64")
    fcfg = ctx.batched_last_config()
    # accuracy: every problem against the closed form within the FP32
    # storage bound, a sample of problems against the oracle run to
    # convergence (residual <= 1e-13) on the same stored matrices
    lam8 = 0.9 ** np.arange(1, k + 1)
    sample = list(range(0, len(sizes), 64))
    t = time.time()
    refs = {}
    for p in sample:
        refs[p] = O.subspace_eig(As[p].double().cpu().numpy(), X0s[p].numpy(), k, tol=1e-13, max_outer=300)
    cpu_s = time.time() - t
    def count(outs):
        nconv, worst_rel, worst_res, worst_closed = 0, 0.0, 0.0, 0.0
        for p, o in enumerate(outs):
            ev_ = o.evals.cpu().numpy()
            rs = o.resid.cpu().numpy()
            ok = rs <= TOL
            ok &= np.abs(ev_ - lam8) <= 5e-8
            worst_closed = max(worst_closed, float(np.max(np.abs(ev_ - lam8))))
            if p in refs:
                rel = np.abs(ev_ - refs[p].theta) / np.abs(refs[p].theta)
                worst_rel = max(worst_rel, float(rel.max()))
                ok &= rel <= 1e-10
            worst_res = max(worst_res, float(rs.max()))
            nconv += int(ok.sum())
        return nconv, worst_rel, worst_res, worst_closed
    acc = [count(r) for r in res]
    value = sum(a[0] for a in acc) / (ms * 1e-3 * len(res))
    facc = count(fres[-1]) if fres else None
    fvalue = facc[0] / (fms * 1e-3) if fres else None
    # roofline of the grouped BF16 product over all 512 problems (its first
    # launch in the call, timed with HIP events on the library's stream)
    nn = sizes.astype(np.float64)
    red_bytes = float(np.sum(2 * nn * nn + 2 * nn * b + 4 * nn * b))
    red_flops = float(np.sum(2 * nn * nn * b))
    sec = cfg["first_product_ms"] * 1e-3
    ach = red_bytes / sec / 1e9
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": f"kb_product_lp<bf16, {cfg['rows_red'] // 32} waves> (grouped over (problem, "
                          f"{cfg['rows_red']}-row tile), MFMA 32x32x16, FP32 accumulate)",
                "avg_launch_ms": cfg["first_product_ms"], "algorithmic_bytes_per_launch": red_bytes,
                "algorithmic_flops_per_launch": red_flops,
                "fp64_grouped_product": {"rows": fcfg["rows_f64"], "first_launch_ms": fcfg["first_product_ms"],
                                          "TFLOP_s": round(red_flops / (fcfg["first_product_ms"] * 1e-3) / 1e12, 2),
                                          "peak": 78.6}}
    cpu = {"value": len(sample) * k / cpu_s, "unit": "Ritz pairs/s", "cores": int(_cores()), "kind": "oracle",
           "sample": (f"{len(sample)} of the 512 problems (every 64th, n = "
                      f"{[int(sizes[p]) for p in sample]}) run by the oracle to convergence, one at a time, "
                      f"{cpu_s:.1f}s")}
    ctx.close()
    return {"metric": "Ritz pairs/sec at residual <=1e-8, mixed vs FP64 form, 1 MI355X; % roofline",
            "value": value, "unit": "Ritz pairs/s", "n_gpus": 1, "steps": len(res), "warmup": max(1, args.warmup),
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic",
            "config": {"workload": "batched: 512 dense symmetric problems, n uniform in [256, 4096] (seeded), "
                                   "lambda_i = 0.9^i, FP32 storage; top k=8, basis 16, power filter, BF16 basis, "
                                   "one grouped launch per step, graph-replayed iterations, autotuned tiles",
                       "problems": len(sizes), "sum_n2": float(np.sum(nn * nn)), "k": k, "basis": b,
                       "parallelism": "single GPU"},
            "n_converged": [a[0] for a in acc], "batched_config": cfg, "call_ms": call_ms,
            "iters_max": max(o.info["iters"] for o in res[-1]),
            "accuracy": {"max_rel_eval_err_vs_oracle_sample": max(a[1] for a in acc),
                         "max_resid": max(a[2] for a in acc), "max_abs_eval_err_vs_closed_form": max(a[3] for a in acc),
                         "criterion": "residual <= 1e-8, eigenvalue within 5e-8 of 0.9^i (FP32 storage bound) for "
                                      "every problem, and within 1e-10 (relative) of the converged oracle for the "
                                      "sampled problems"},
            "fp64_form": {"value": fvalue, "ms_per_step": fms, "n_converged": facc[0], "batched_config": fcfg},
            "speedup_vs_fp64_form": value / fvalue if fvalue else None,
            "roofline": roofline, "cpu_baseline": cpu}



# The paper's basis-generation timings (ms, mean of 5 runs, RTX 3070 Ti;
# Sec. 5.3, Table 3): context only, other hardware.
PAPER_T3 = {
    "f64": {"mgs_l": (359.805, 369.862, 1402.376), "mgs_r": (42.936, 67.040, 219.855),
            "cgs": (46.322, 65.882, 182.747), "cgs2": (55.346, 82.591, 243.225),
            "hess_l": (119.293, 132.390, 480.391), "hess_r": (24.677, 39.528, 138.033)},
    "f32": {"mgs_l": (334.379, 335.997, 1331.892), "mgs_r": (23.062, 27.906, 99.559),
            "cgs": (14.824, 21.894, 72.658), "cgs2": (18.987, 30.062, 102.819),
            "hess_l": (111.796, 121.182, 446.195), "hess_r": (16.571, 24.286, 77.928)},
    "f16": {"mgs_l": (334.164, 335.369, 1328.612), "mgs_r": (29.499, 17.821, 57.887),
            "cgs": (12.971, 15.894, 47.782), "cgs2": (15.025, 20.742, 64.865),
            "hess_l": (111.314, 120.955, 441.900), "hess_r": (12.754, 17.273, 49.223)},
}
T3_SHAPES = ((25000, 200), (50000, 200), (50000, 400))


def bench_t3(args):
    """The six basis-generation processes (left/right-looking MGS without
    re-orthogonalisation, CGS, CGS-2, left/right-looking Hessenberg) on
    U(0,1) blocks of the paper's three shapes in FP64, FP32 and binary16
    storage with FP32 arithmetic; mean of 5 timed runs after one warm-up
    (each run on a fresh copy of the same block, the copy outside the timed
    launch).  Also the library's production Hessenberg sweep (row-major
    register/LDS kernel) on the same blocks in FP64 and FP32."""
    import statistics
    import torch
    from paper_2505_00281_amd import ofrr
    ctx = ofrr.Context(0)
    dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
    tol = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "f16": 2.0 ** -10}
    table = {}
    for prec in ("f64", "f32", "f16"):
        table[prec] = {}
        for si, (m, n) in enumerate(T3_SHAPES):
            A64 = np.random.default_rng(3000 + si).random((m, n))
            src = torch.from_numpy(np.ascontiguousarray(A64.T)).to(dt[prec]).cuda()  # n x m = column-major m x n
            work = torch.empty_like(src)
            for meth in ("mgs_l", "mgs_r", "cgs", "cgs2", "hess_l", "hess_r"):
                times = []
                for rep in range(6):
                    work.copy_(src)
                    _, _, _, kept, ms = ctx.basis_generate(work.t(), meth, tol=tol[prec])
                    if rep:
                        times.append(ms)
                table[prec].setdefault(meth, []).append(round(statistics.fmean(times), 3))
                log(f"[bench] t3 {prec} {m}x{n} {meth}: {statistics.fmean(times):.3f} ms (kept {kept})")
            if prec in ("f64", "f32"):
                # the production sweep on the row-major copy of the same block
                Yrow = torch.from_numpy(np.ascontiguousarray(A64)).to(dt[prec]).cuda()
                wrow = torch.empty_like(Yrow)
                times = []
                for rep in range(6):
                    wrow.copy_(Yrow)
                    ctx.kernel_stats_reset()
                    ctx.set_profile(True)
                    ctx.hessenberg(wrow, tol[prec])
                    nl, tl = ctx.kernel_stats("hessenberg")
                    if rep:
                        times.append(tl)
                ctx.set_profile(False)
                table[prec].setdefault("hess_r_sweep", []).append(round(statistics.fmean(times), 3))
                log(f"[bench] t3 {prec} {m}x{n} production sweep: {statistics.fmean(times):.3f} ms")
    ctx.close()
    ratios = {p: {meth: [round(PAPER_T3[p][meth][i] / table[p][meth][i], 2) for i in range(3)]
                  for meth in PAPER_T3[p]} for p in table}
    return {"metric": "basis generation time (ms, mean of 5) at the paper's timing-table shapes, 1 MI355X",
            "value": table["f32"]["hess_r"][2], "unit": "ms", "n_gpus": 1, "steps": 5, "warmup": 1,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32/f16-storage",
            "data": "synthetic U(0,1)",
            "config": {"workload": "basis generation: MGS-L, MGS-R, CGS, CGS-2, Hess-L, Hess-R on U(0,1) blocks "
                                   "25000x200, 50000x200, 50000x400 (column-major, one cooperative launch per "
                                   "process); value = Hess-R, FP32, 50000x400",
                       "shapes": T3_SHAPES, "parallelism": "single GPU"},
            "ms": table, "paper_ms_rtx3070ti": PAPER_T3, "paper_over_ours": ratios}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-oracle", "--no-cpu-baseline", dest="no_oracle", action="store_true",
                    help="skip the converged oracle run (the accuracy reference and the CPU baseline)")
    ap.add_argument("--gram-accum", choices=["f32c", "f32", "f64"], default="f32c",
                    help="accumulation of G and H in the BF16 phase")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--b-split", type=int, default=1)
    ap.add_argument("--refine", type=int, default=2,
                    help="1: BF16 then FP64 tail; 2: BF16, split-BF16, FP64 tail")
    ap.add_argument("--stall-iters", type=int, default=3)
    ap.add_argument("--tail", choices=["f64", "i8"], default="i8",
                    help="products of the final FP64 phase: FP64 arithmetic or exact INT8 digit planes")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the three product kernels of the path (BF16 MFMA, INT8 digit planes, "
                         "FP64 MFMA) three times each on a random n=16384 FP32 matrix and a 128-column "
                         "block, for hardware-counter passes (no solver library calls)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write) three times; "
                         "used to scale rocprofv3 FETCH_SIZE/WRITE_SIZE readings")
    ap.add_argument("--workload", choices=["dense", "svd", "laplacian", "batched", "t3", "general"], default="dense",
                    help="dense (default): the n=16384 eigenvalue workload of the headline metric; "
                         "svd: 65536 x 8192 FP8 SVD; laplacian: CSR 2-D Laplacian, 32 smallest; "
                         "batched: 512 problems n in [256, 4096]; t3: basis-generation processes at the "
                         "shapes and precisions of the paper's basis-generation timing table")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU "
              "row partition is a design, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                          "launches": 3}))
        return
    from paper_2505_00281_amd import ofrr
    device = torch.device("cuda", 0)
    if args.workload != "dense":
        out = {"svd": bench_svd, "laplacian": bench_laplacian, "batched": bench_batched,
               "t3": bench_t3, "general": bench_general}[args.workload](args)
        print(json.dumps(out))
        return
    if args.traffic_probe:
        ctx = ofrr.Context(0)
        g = torch.Generator(device=device).manual_seed(7)
        A = torch.randn((N, N), generator=g, device=device, dtype=torch.float32)
        V = torch.randn((N, BASIS), generator=g, device=device, dtype=torch.float64)
        Ab = A.to(torch.bfloat16)
        Vb = V.to(torch.bfloat16)
        for _ in range(3):
            # column-major views (the values are random; only the traffic counts)
            ctx.block_product(Ab.t(), Vb, trans=True)
            for d in (6, 5, 4):
                ctx.block_product_sliced(A.t(), V, trans=True, digits=d)
            ctx.block_product(A.t(), V, trans=True)
        torch.cuda.synchronize()
        ctx.close()
        print(json.dumps({"traffic_probe": {"n": N, "b": BASIS, "launches_per_kernel": 3}}))
        return
    A, X0, lo, hi, anorm = make_problem(device)
    ctx = ofrr.Context(0)

    common = dict(filter="chebyshev", degree=DEGREE, lo=lo, hi=hi, tol=TOL * 0.5, anorm=anorm,
                  max_iters=400)
    mixed_kw = dict(basis_dtype="bf16", refine=args.refine, stall_iters=args.stall_iters,
                    b_split=args.b_split, tail=args.tail, gram_accum=args.gram_accum, **common)
    mixed = ofrr.make_plan(**mixed_kw)
    f64 = ofrr.make_plan(basis_dtype="f64", **common)

    res, ms_step, wall = run_steps(ctx, A, X0, mixed, args.steps, args.warmup, "mixed")

    # FP64 form of the same method on the same GPU
    fres, fms = None, None
    if not args.no_fp64_form:
        fres, fms, _ = run_steps(ctx, A, X0, f64, 3, 1, "fp64")

    # where the time goes: every kernel family timed with HIP events on the
    # library's stream over one more (profiled) call of each form
    fams = ["product_bf16", "product_bf16x2", "product_i8x", "product_reduce", "product_f64", "hessenberg",
            "small_eig", "gram", "lift", "scale", "quantize", "residual"]
    ctx.kernel_stats_reset()
    ctx.eig_partial(A, K_WANT, BASIS, plan=ofrr.make_plan(profile=True, **mixed_kw), X0=X0)
    torch.cuda.synchronize()
    stats = {f: ctx.kernel_stats(f) for f in fams}
    # digit-plane launches by digits per side (4, 5, 6: 10, 15, 21 pairs)
    i8_by_digits = {d: ctx.kernel_stats(f"product_i8x_d{d}") for d in (4, 5, 6)}
    kernel_ms_fp64 = None
    if not args.no_fp64_form:
        ctx.kernel_stats_reset()
        ctx.eig_partial(A, K_WANT, BASIS, plan=ofrr.make_plan(basis_dtype="f64", profile=True, **common), X0=X0)
        torch.cuda.synchronize()
        kernel_ms_fp64 = {}
        for f in fams:
            n_l, t_l = ctx.kernel_stats(f)
            if n_l:
                kernel_ms_fp64[f] = {"launches": n_l, "total_ms": round(t_l, 3)}

    # Roofline of the product families on the METHOD's work per launch:
    # bytes = A read once in the basis build's storage type (BF16, the
    # method's reduced copy) + the basis block + the product; flops = 2 n^2 b.
    # The split-BF16 and INT8 digit-plane kernels do more than that (they are
    # how this build gets FP32- and FP64-class accuracy out of 16-bit and
    # 8-bit units): their own bytes and operations are reported beside it as
    # kernel_rate, not as the roofline.  Peaks are MI355X's data-sheet ones.
    gemm = 2.0 * N * N * BASIS
    bf16_bytes = N * N * 2 + N * BASIS * 2 + N * BASIS * 4
    alg = {
        "product_bf16": dict(bytes=bf16_bytes, ops=gemm, peak_mfma=2500.0, dtype="bf16",
                             kernel="k_gemm_lp<bf16> (A*V, BF16 MFMA 32x32x16, FP32 accumulate)",
                             kernel_bytes=bf16_bytes, kernel_ops=gemm),
        "product_bf16x2": dict(bytes=bf16_bytes, ops=gemm, peak_mfma=2500.0, dtype="bf16",
                               kernel="k_gemm_lp<bf16, split A and V> (hi+lo BF16 operands, 3 MFMAs per step)",
                               kernel_bytes=N * N * 4 + N * BASIS * 4 + N * BASIS * 4, kernel_ops=3 * gemm),
        # FP64-class product: the method's flops on the kernel's own unit
        # (INT8); the kernel's own bytes and operations averaged over its
        # launches by digits per side (d planes of A and V, d(d+1)/2 pairs)
        "product_i8x": dict(bytes=N * N * 4 + N * BASIS * 8 + N * BASIS * 8, ops=gemm, peak_mfma=5000.0,
                            dtype="int8",
                            kernel="k_gemm_i8s (4, 5 or 6 INT8 digit planes per side chosen per iteration; "
                                   "10, 15 or 21 MFMA 32x32x32 pairs, exact int32)",
                            kernel_bytes=sum(n_ * (d * N * N + d * N * BASIS + 8 * N * BASIS)
                                             for d, (n_, _) in i8_by_digits.items())
                            / max(1, sum(n_ for n_, _ in i8_by_digits.values())),
                            kernel_ops=sum(n_ * d * (d + 1) // 2 * gemm for d, (n_, _) in i8_by_digits.items())
                            / max(1, sum(n_ for n_, _ in i8_by_digits.values()))),
        # in the mixed call the only FP64 product is the final residual check
        "product_f64": dict(bytes=N * N * 4 + N * K_WANT * 16, ops=2.0 * N * N * K_WANT, peak_mfma=78.6,
                            dtype="f64", kernel="k_gemm_f64 (final residual product, k columns, FP64 MFMA)",
                            kernel_bytes=N * N * 4 + N * K_WANT * 16, kernel_ops=2.0 * N * N * K_WANT),
    }

    def roof(f):
        a = alg[f]
        n_l, t_l = stats[f]
        avg = t_l / max(n_l, 1)
        sec = avg * 1e-3
        hbm_t = a["bytes"] / (HBM_PEAK_GBS * 1e9)
        mfma_t = a["ops"] / (a["peak_mfma"] * 1e12)
        if hbm_t >= mfma_t:
            ach = a["bytes"] / sec / 1e9
            r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(ach / HBM_PEAK_GBS, 4)}
        else:
            ach = a["ops"] / sec / 1e12
            r = {"bound": "mfma", "achieved": round(ach, 2), "peak": a["peak_mfma"],
                 "unit": "TOP/s" if a["dtype"] == "int8" else "TFLOP/s", "frac": round(ach / a["peak_mfma"], 4)}
        traffic = MEASURED_TRAFFIC.get(f)
        if f == "product_i8x":
            n_i8 = sum(n_ for n_, _ in i8_by_digits.values())
            traffic = (sum(n_ * MEASURED_TRAFFIC_I8[d] for d, (n_, _) in i8_by_digits.items()) / n_i8
                       if n_i8 else None)
        r.update({"traffic": traffic if N == 16384 and BASIS == 128 else None,
                  "kernel": a["kernel"], "family": f, "avg_launch_ms": avg, "launches": n_l,
                  "algorithmic_bytes_per_launch": a["bytes"], "algorithmic_flops_per_launch": a["ops"],
                  "kernel_rate": {"bytes_per_launch": a["kernel_bytes"], "ops_per_launch": a["kernel_ops"],
                                  "GB_s": round(a["kernel_bytes"] / sec / 1e9, 1),
                                  "TOP_s": round(a["kernel_ops"] / sec / 1e12, 2)}})
        if f == "product_i8x":
            # the same product at FP64 accuracy on the FP64 MFMA roof
            r["fp64_equivalent"] = {"achieved_TFLOP_s": round(gemm / sec / 1e12, 2), "peak": 78.6,
                                    "frac": round(gemm / sec / 1e12 / 78.6, 3)}
            r["launches_by_digits"] = {str(d): {"launches": n_, "avg_launch_ms": round(t_ / n_, 4) if n_ else None}
                                       for d, (n_, t_) in i8_by_digits.items()}
        return r

    # the product family with the largest share of the call; the two
    # latency-bound kernels (one-workgroup small eigensolver, grid-exchange
    # Hessenberg sweep) have no bandwidth or MFMA roofline and are reported by time
    dom = max(alg, key=lambda f: stats[f][1])
    roofline = roof(dom)
    roofline["latency_bound_ms_one_call"] = {f: round(stats[f][1], 3) for f in ("small_eig", "hessenberg")}
    roofline["per_family"] = {f: {k: v for k, v in roof(f).items()
                                  if k in ("bound", "achieved", "unit", "frac", "avg_launch_ms", "fp64_equivalent")}
                              for f in alg if stats[f][0]}
    kernel_ms = {f: {"launches": n, "total_ms": round(t, 3)} for f, (n, t) in stats.items()}

    # accuracy against the converged oracle (after the timed region), which
    # is also the CPU baseline
    ref, cpu = None, None
    if not args.no_oracle:
        ref, cpu = oracle_converged(A, X0, lo, hi, anorm)
        acc = [accuracy(r, ref) for r in res]
        nconv = [a[0] for a in acc]
        acc_mixed = acc[-1][1]
    else:
        nconv = [int((r.resid <= TOL).sum().item()) for r in res]
        acc_mixed = None
    value = sum(nconv) / (ms_step * 1e-3 * len(res))

    f64_out = None
    if fres:
        fr = fres[-1]
        if ref is not None:
            fconv, facc = accuracy(fr, ref)
        else:
            fconv, facc = int((fr.resid <= TOL).sum().item()), None
        ev_diff = float(torch.max(torch.abs(fr.evals - res[-1].evals) / torch.abs(fr.evals)).item())
        f64_out = {"value": fconv / (fms * 1e-3), "ms_per_step": fms, "steps": len(fres),
                   "call_ms": call_ms_summary(fres), "iters": fr.info["iters"], "n_converged": fconv,
                   "accuracy_vs_oracle": facc, "max_rel_eval_diff_mixed_vs_fp64": ev_diff}

    out = {
        "metric": "Ritz pairs/sec at residual <=1e-8, mixed vs FP64 form, 1 MI355X; % roofline",
        "value": value, "unit": "Ritz pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "dense symmetric n=16384, lambda_i=i^-1.5 + 1e-3 N(0,1) symmetric "
                               "noise, FP32 storage; top k=64, basis 128, degree-4 Chebyshev",
                   "n": N, "k": K_WANT, "basis": BASIS, "degree": DEGREE, "filter_interval": [lo, hi],
                   "filter_interval_source": "exact spectrum of the stored A (FP32 eigendecomposition "
                                             "on the GPU, outside the timed region)",
                   "plan": (f"bf16 basis + FP32 accumulate{', split-BF16 middle phase' if args.refine >= 2 else ''}, "
                            f"{ {'f32c': 'FP32-compensated', 'f32': 'FP32', 'f64': 'FP64'}[args.gram_accum]} "
                            f"first-phase G/H (FP64 when t(G) > 1000), FP64 pencil, FP64 tail with "
                            f"{'INT8 digit-plane' if args.tail == 'i8' else 'FP64'} products"),
                   "parallelism": "single GPU"},
        "n_converged": nconv, "iters": res[-1].info["iters"], "iters_low": res[-1].info["iters_low"],
        "accuracy_vs_oracle": acc_mixed,
        "gram": {"t_max": res[-1].info["gram_t_max"], "projections_switched_to_f64": res[-1].info["grams_f64"]},
        "call_ms": call_ms_summary(res),
        "fp64_form": f64_out,
        "speedup_vs_fp64_form": (value / f64_out["value"]) if f64_out and f64_out["value"] else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_ms_one_call": kernel_ms,
        "kernel_ms_one_call_fp64_form": kernel_ms_fp64,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
