"""Whole-method parity through the C ABI: the GPU path against the CPU
oracle on the same seeded inputs.

* FP64 form, same-step mode: after the same number of outer iterations the
  GPU's Hessenberg/OFRR subspace equals the oracle's orthonormal/classical-RR
  subspace (span(p(A)^s X0)), so the Ritz values agree to rounding (the
  tolerance 1e-12 relative is the one stated for the FP64 form).
* Mixed forms, converged mode: final residual <= 1e-8 and relative
  eigenvalue error <= 1e-10 against the oracle's converged pairs.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ofrr_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_00281_amd import ofrr
    c = ofrr.Context(0)
    yield c
    c.close()


def _plan(**kw):
    from paper_2505_00281_amd import ofrr
    return ofrr.make_plan(**kw)


def _check_same_step(r, ref, k, vec_tol=1e-8):
    th = r.evals.cpu().numpy()
    np.testing.assert_allclose(th, ref.theta, rtol=1e-12, atol=0)
    res = r.resid.cpu().numpy()
    np.testing.assert_allclose(res, ref.resid, rtol=1e-6, atol=1e-12)
    X = r.evecs.cpu().numpy()
    np.testing.assert_allclose(np.linalg.norm(X, axis=0), 1.0, atol=1e-14)
    np.testing.assert_allclose(X, ref.X, atol=vec_tol)


def test_eig_dense_n512_power_fp64_same_step(ctx):
    """The n=512 configuration: A = Q diag(0.95^i) Q^T (FP64), k=8, basis 16,
    20 power steps, FP64 form."""
    n, b, k, outer = 512, 16, 8, 20
    lam = 0.95 ** np.arange(1, n + 1)
    A = W.dense_symmetric_prescribed(lam, 1001)
    X0 = W.uniform_start(n, b, 1101)
    print("eig n512 fp64 same-step", flush=True)
    r = ctx.eig_partial(A.cuda(), k, b, plan=_plan(max_iters=outer), X0=torch.from_numpy(X0))
    ref = O.subspace_eig(A.numpy(), X0, k, outer=outer)
    assert r.info["iters"] == outer
    _check_same_step(r, ref, k)


@pytest.mark.parametrize("scale", [1e295, 1e-300])
def test_eig_fp64_extreme_magnitudes_same_step(ctx, scale):
    """FP64 form on c * A with c far outside FP32's range: the column scaling
    must bring every product column to infinity-norm (1/2, 1] (an FP32 view
    of the magnitudes saturates at 1e295 and flushes 1e-300 to zero, which
    leaves the columns unscaled and the Hessenberg sweep drops them all).
    Ritz values scale with c, vectors and relative residuals do not."""
    n, b, k, outer = 200, 12, 5, 6
    lam = 0.9 ** np.arange(1, n + 1)
    A0 = W.dense_symmetric_prescribed(lam, 1201)
    X0 = W.uniform_start(n, b, 1202)
    ref = O.subspace_eig(A0.numpy(), X0, k, outer=outer)
    print("eig fp64 extreme magnitude", scale, flush=True)
    r = ctx.eig_partial((A0 * scale).cuda(), k, b, plan=_plan(max_iters=outer), X0=torch.from_numpy(X0))
    assert r.info["basis_eff"] == b
    np.testing.assert_allclose(r.evals.cpu().numpy() / scale, ref.theta, rtol=1e-12, atol=0)
    np.testing.assert_allclose(r.evecs.cpu().numpy(), ref.X, atol=1e-8)
    np.testing.assert_allclose(r.resid.cpu().numpy(), ref.resid, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("n,b,k,deg", [(300, 10, 4, 3), (257, 9, 3, 5)])
def test_eig_dense_chebyshev_fp64_same_step(ctx, n, b, k, deg):
    lam = np.linspace(1.0, -0.5, n) ** 3
    A = W.dense_symmetric_prescribed(lam, 77 + n)
    X0 = W.uniform_start(n, b, 78 + n)
    lo, hi = -0.2, 0.3
    print("eig chebyshev fp64", n, b, k, deg, flush=True)
    r = ctx.eig_partial(A.cuda(), k, b, plan=_plan(filter="chebyshev", degree=deg, lo=lo, hi=hi,
                                                    max_iters=6), X0=torch.from_numpy(X0))
    ref = O.subspace_eig(A.numpy(), X0, k, filt="chebyshev", degree=deg, lo=lo, hi=hi, outer=6)
    _check_same_step(r, ref, k, vec_tol=1e-7)


def test_eig_csr_laplacian_smallest_fp64_same_step(ctx):
    from paper_2505_00281_amd import ofrr
    N, b, k = 24, 16, 6
    rp, ci, v = W.laplacian_2d_csr(N)
    ev = W.laplacian_2d_eigenvalues(N)
    X0 = W.uniform_start(N * N, b, 9)
    mat = ofrr.csr_matrix(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                          torch.from_numpy(v).cuda())
    print("eig csr laplacian fp64", flush=True)
    plan = _plan(filter="chebyshev", degree=8, lo=float(ev[b]), hi=8.0, anorm=8.0, max_iters=10)
    r = ctx.eig_partial(mat, k, b, which="smallest", plan=plan, X0=torch.from_numpy(X0))
    ref = O.subspace_eig((rp, ci, v), X0, k, which="smallest", filt="chebyshev", degree=8,
                         lo=float(ev[b]), hi=8.0, outer=10, anorm=8.0)
    th = r.evals.cpu().numpy()
    np.testing.assert_allclose(th, ref.theta, rtol=1e-12)
    # the Laplacian has exact double eigenvalues: inside such a cluster the
    # individual Ritz vectors (and their residuals) are not unique, but the
    # cluster's residual norm sqrt(sum r_i^2) and its span are
    res, rres = r.resid.cpu().numpy(), ref.resid
    X = r.evecs.cpu().numpy()
    i = 0
    while i < k:
        j = i + 1
        while j < k and abs(ref.theta[j] - ref.theta[i]) <= 1e-9 * abs(ref.theta[i]):
            j += 1
        np.testing.assert_allclose(np.linalg.norm(res[i:j]), np.linalg.norm(rres[i:j]), rtol=1e-3,
                                   atol=1e-11)
        if j == k and j - i > 1:
            break  # the cluster may continue past k: its span within the first k is not unique
        assert O.subspace_sin(X[:, i:j], ref.X[:, i:j]) < 1e-6
        i = j


def test_eig_csr_malformed_is_rejected(ctx):
    """A CSR with an out-of-range column index is refused before any
    product runs."""
    from paper_2505_00281_amd import ofrr
    rp, ci, v = W.laplacian_2d_csr(8)
    ci = ci.copy()
    ci[10] = 10 ** 6
    rpg, cig, vg = (torch.from_numpy(a).cuda() for a in (rp, ci, v))
    mat = ofrr.csr_matrix(rpg, cig, vg)
    with pytest.raises(ofrr.OfrrError) as e:
        ctx.eig_partial(mat, 2, 4, which="smallest", plan=_plan(max_iters=2))
    assert e.value.status == ofrr.ERR_INVALID_ARG


def test_eig_converged_to_tolerance_fp64(ctx):
    n, b, k = 400, 12, 5
    lam = 0.8 ** np.arange(n)
    A = W.dense_symmetric_prescribed(lam, 5)
    print("eig converged fp64", flush=True)
    r = ctx.eig_partial(A.cuda(), k, b, plan=_plan(tol=1e-12, anorm=1.0, max_iters=500))
    assert r.status == 0
    np.testing.assert_allclose(r.evals.cpu().numpy(), lam[:k], rtol=1e-13)
    assert r.resid.cpu().numpy().max() <= 1e-12


@pytest.mark.parametrize("lowp,refine,tail", [("bf16", 1, "f64"), ("f16", 1, "f64"), ("bf16", 2, "f64"),
                                               ("bf16", 2, "i8")])
def test_eig_mixed_refined_converged(ctx, lowp, refine, tail):
    """Mixed form with the FP64 tail (refine=2: with the split-BF16 middle
    phase; tail i8: FP64-phase products from exact INT8 digit planes)
    reaches residual <= 1e-8 and relative eigenvalue error <= 1e-10 against
    the oracle's converged pairs."""
    n, b, k = 2048, 32, 12
    lam = np.arange(1, n + 1) ** -1.5
    A = W.dense_symmetric_prescribed(lam, 1002, noise_scale=1e-4, noise_seed=2002, dtype=torch.float32)
    Ad = A.double().numpy()
    w, Z = np.linalg.eigh(Ad)
    w = w[::-1]
    X0 = W.uniform_start(n, b, 1102)
    lo, hi = float(w[-1]), float(w[b])
    print("eig mixed refined", lowp, flush=True)
    plan = _plan(basis_dtype=lowp, refine=refine, filter="chebyshev", degree=4, lo=lo, hi=hi,
                 tol=1e-9, anorm=float(w[0]), max_iters=400, tail=tail)
    r = ctx.eig_partial(A.cuda(), k, b, plan=plan, X0=torch.from_numpy(X0))
    print("info", r.info, flush=True)
    ref = O.subspace_eig(Ad, X0, k, filt="chebyshev", degree=4, lo=lo, hi=hi, tol=1e-12,
                         anorm=float(w[0]), max_outer=2000)
    th = r.evals.cpu().numpy()
    assert r.info["iters_low"] >= 1
    assert r.resid.cpu().numpy().max() <= 1e-8
    np.testing.assert_allclose(th, ref.theta, rtol=1e-10)
    np.testing.assert_allclose(th, w[:k], rtol=1e-10)


@pytest.mark.parametrize("accum,switch_t", [("f32c", 0.0), ("f32", 0.0), ("f32c", 1.0)])
def test_eig_mixed_fp32_projections_converged(ctx, accum, switch_t):
    """Mixed form whose BF16 phase forms G and H with FP32 accumulation
    (compensated or plain): the same converged pairs as the oracle's
    (residual <= 1e-8, relative eigenvalue error <= 1e-10).  With the
    conditioning bound at 1 (t(G) >= 1, equal only for a diagonal G) every
    first-phase projection after the first is switched to FP64."""
    n, b, k = 2048, 32, 12
    lam = np.arange(1, n + 1) ** -1.5
    A = W.dense_symmetric_prescribed(lam, 1002, noise_scale=1e-4, noise_seed=2002, dtype=torch.float32)
    Ad = A.double().numpy()
    w = np.linalg.eigvalsh(Ad)[::-1]
    X0 = W.uniform_start(n, b, 1102)
    lo, hi = float(w[-1]), float(w[b])
    print("eig mixed fp32 projections", accum, switch_t, flush=True)
    plan = _plan(basis_dtype="bf16", refine=2, filter="chebyshev", degree=4, lo=lo, hi=hi,
                 tol=1e-9, anorm=float(w[0]), max_iters=400, tail="i8", gram_accum=accum,
                 gram_switch_t=switch_t)
    r = ctx.eig_partial(A.cuda(), k, b, plan=plan, X0=torch.from_numpy(X0))
    print("info", r.info, flush=True)
    assert r.info["iters_low"] >= 2
    assert r.info["gram_t_max"] >= 1.0
    # the first phase ends when it stalls; iters_low also counts the split phase
    if switch_t == 1.0:
        assert r.info["grams_f64"] >= 1
    else:
        assert r.info["grams_f64"] == 0 or r.info["gram_t_max"] > 1000.0
    ref = O.subspace_eig(Ad, X0, k, filt="chebyshev", degree=4, lo=lo, hi=hi, tol=1e-12,
                         anorm=float(w[0]), max_outer=2000)
    assert r.resid.cpu().numpy().max() <= 1e-8
    np.testing.assert_allclose(r.evals.cpu().numpy(), ref.theta, rtol=1e-10)


def test_eig_dropped_column_same_step(ctx):
    """A dependent start column is dropped by the first sweep (that
    iteration's projection is redone on the compacted basis); the subspace
    then equals the oracle's from the start block without that column (the
    same span) after the same number of steps."""
    n, b, k, outer = 300, 10, 4, 5
    lam = 0.7 ** np.arange(n)
    A = W.dense_symmetric_prescribed(lam, 15)
    X0 = W.uniform_start(n, b, 16)
    X0[:, 7] = X0[:, 1]
    print("eig dropped column same-step", flush=True)
    r = ctx.eig_partial(A.cuda(), k, b, plan=_plan(max_iters=outer), X0=torch.from_numpy(X0))
    ref = O.subspace_eig(A.numpy(), np.delete(X0, 7, axis=1), k, outer=outer)
    assert r.info["iters"] == outer
    assert r.info["basis_eff"] == b - 1
    _check_same_step(r, ref, k)


def test_eig_rank_deficient_start_block_still_correct(ctx):
    n, b, k = 300, 10, 4
    lam = 0.7 ** np.arange(n)
    A = W.dense_symmetric_prescribed(lam, 15)
    X0 = W.uniform_start(n, b, 16)
    X0[:, 7] = X0[:, 1]  # dependent start column: dropped by the Hessenberg sweep
    print("eig rank-deficient start", flush=True)
    r = ctx.eig_partial(A.cuda(), k, b, plan=_plan(tol=1e-12, anorm=1.0, max_iters=300),
                        X0=torch.from_numpy(X0))
    assert r.info["basis_eff"] <= b - 1
    np.testing.assert_allclose(r.evals.cpu().numpy(), lam[:k], rtol=1e-12)


def test_eig_invalid_arguments(ctx):
    from paper_2505_00281_amd import ofrr
    A = torch.eye(10, dtype=torch.float64).cuda()
    with pytest.raises(ofrr.OfrrError) as e:
        ctx.eig_partial(A, 5, 4)  # k > basis
    assert e.value.status == ofrr.ERR_INVALID_ARG
    with pytest.raises(ofrr.OfrrError) as e:
        ctx.eig_partial(A, 2, 4, plan=_plan(filter="chebyshev", lo=1.0, hi=1.0))
    assert e.value.status == ofrr.ERR_INVALID_ARG
    with pytest.raises(ofrr.OfrrError) as e:
        ctx.eig_partial(A, 2, 11)
    assert e.value.status == ofrr.ERR_INVALID_ARG


def test_eig_nan_input_reports_numeric(ctx):
    from paper_2505_00281_amd import ofrr
    A = torch.eye(64, dtype=torch.float64)
    A[3, 5] = float("nan")
    A[5, 3] = float("nan")
    with pytest.raises(ofrr.OfrrError) as e:
        ctx.eig_partial(A.cuda(), 2, 4, plan=_plan(max_iters=3))
    assert e.value.status == ofrr.ERR_NUMERIC


def test_svd_fp64_same_step(ctx):
    m, n, b, k = 700, 240, 14, 6
    sig = np.exp(-np.arange(1, n + 1) / 30.0)
    A = W.svd_prescribed(m, n, sig, 31, dtype=torch.float64)
    V0 = W.uniform_start(n, b, 32)
    print("svd fp64 same-step", flush=True)
    r = ctx.svd_partial(A.cuda(), k, b, plan=_plan(max_iters=5), V0=torch.from_numpy(V0))
    ref = O.subspace_svd(A.numpy(), V0, k, outer=5)
    np.testing.assert_allclose(r.sigma.cpu().numpy(), ref.sigma, rtol=1e-12)
    np.testing.assert_allclose(r.resid.cpu().numpy(), ref.resid, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(r.V.cpu().numpy(), ref.V, atol=1e-8)
    np.testing.assert_allclose(r.U.cpu().numpy(), ref.U, atol=1e-8)


def test_svd_converged_fp64(ctx):
    m, n, b, k = 600, 200, 16, 8
    sig = np.exp(-np.arange(1, n + 1) / 20.0)
    A = W.svd_prescribed(m, n, sig, 41, dtype=torch.float64)
    print("svd converged fp64", flush=True)
    r = ctx.svd_partial(A.cuda(), k, b, plan=_plan(tol=1e-12, max_iters=300))
    print("info", r.info, flush=True)
    assert r.info["iters"] > 5
    np.testing.assert_allclose(r.sigma.cpu().numpy(), sig[:k], rtol=1e-12)
    assert r.resid.cpu().numpy().max() <= 2e-12


@pytest.mark.parametrize("lowp,tail", [("bf16", "f64"), ("f16", "f64"), ("f8e4m3", "f64"), ("f8e4m3", "i8"),
                                       ("bf16", "i8")])
def test_svd_mixed_refined_converged(ctx, lowp, tail):
    # tail i8: the FP64 phase's A V and A^T U from exact INT8 digit planes
    m, n, b, k = 1500, 400, 24, 10
    sig = np.exp(-np.arange(1, n + 1) / 40.0)
    A = W.svd_prescribed(m, n, sig, 43, dtype=torch.float32)
    Ad = A.double().numpy()
    s_ref = np.linalg.svd(Ad, compute_uv=False)
    print("svd mixed", lowp, tail, flush=True)
    r = ctx.svd_partial(A.cuda(), k, b, plan=_plan(basis_dtype=lowp, refine=True, tol=1e-9,
                                                    max_iters=400, tail=tail))
    print("info", r.info, flush=True)
    assert r.info["iters_low"] >= 1
    assert r.resid.cpu().numpy().max() <= 1e-8
    np.testing.assert_allclose(r.sigma.cpu().numpy(), s_ref[:k], rtol=1e-10)


@pytest.mark.parametrize("lowp,tail", [("bf16", "f64"), ("f8e4m3", "f64"), ("f8e4m3", "i8")])
def test_svd_phase_switch_at_iteration_cap(ctx, lowp, tail):
    """The iteration cap lands on the switch to the FP64 tail: the left and
    right Ritz blocks are promoted exactly, so U, V, sigma and the final
    residuals equal those of the same run that does not switch, bit for
    bit (a left block left in FP32 and read as FP64 would not)."""
    m, n, b, k = 900, 300, 16, 6
    sig = np.exp(-np.arange(1, n + 1) / 30.0)
    A = W.svd_prescribed(m, n, sig, 44, dtype=torch.float32).cuda()
    V0 = torch.from_numpy(W.uniform_start(n, b, 45))
    print("svd switch at cap", lowp, flush=True)
    common = dict(basis_dtype=lowp, refine=True, tol=1e-15, max_iters=1, tail=tail)
    sw = ctx.svd_partial(A, k, b, plan=_plan(stall_iters=1, switch_resid=1e3, **common), V0=V0)
    ns = ctx.svd_partial(A, k, b, plan=_plan(stall_iters=50, switch_resid=0.0, **common), V0=V0)
    assert sw.info["iters"] == ns.info["iters"] == 1
    assert sw.info["products"] == ns.info["products"] + 1  # the redone FP64 product
    for a, c in ((sw.sigma, ns.sigma), (sw.U, ns.U), (sw.V, ns.V), (sw.resid, ns.resid)):
        np.testing.assert_array_equal(a.cpu().numpy(), c.cpu().numpy())
    U = sw.U.cpu().numpy()
    np.testing.assert_allclose(np.linalg.norm(U, axis=0), 1.0, atol=1e-3)


def test_batched_matches_single(ctx):
    sizes = [256, 300, 513]
    As, X0s = [], []
    for i, n in enumerate(sizes):
        lam = 0.9 ** np.arange(1, n + 1)
        As.append(W.dense_symmetric_prescribed(lam, 500 + i))
        X0s.append(torch.from_numpy(W.uniform_start(n, 16, 600 + i)))
    print("batched", flush=True)
    outs = ctx.eig_partial_batched([a.cuda() for a in As], 8, 16, plan=_plan(max_iters=10), X0s=X0s)
    for i, o in enumerate(outs):
        ref = O.subspace_eig(As[i].numpy(), X0s[i].numpy(), 8, outer=10)
        np.testing.assert_allclose(o.evals.cpu().numpy(), ref.theta, rtol=1e-12)


@pytest.mark.parametrize("basis_dtype", ["f64", "f16"])
def test_eig_csr_folded_scaling_equals_separate_passes(ctx, monkeypatch, basis_dtype):
    """CSR + Chebyshev: the column scaling folded into the fused steps gives
    the bits of the separate scaling passes (powers of two scale exactly;
    the reduced phase reads its block rounded to binary16 either way)."""
    from paper_2505_00281_amd import ofrr
    N, b, k = 40, 16, 6
    rp, ci, v = W.laplacian_2d_csr(N)
    ev = W.laplacian_2d_eigenvalues(N)
    X0 = torch.from_numpy(W.uniform_start(N * N, b, 19))
    mat = ofrr.csr_matrix(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(v).cuda())
    plan = _plan(basis_dtype=basis_dtype, filter="chebyshev", degree=7, lo=float(ev[b]), hi=8.0, anorm=8.0,
                 max_iters=6)
    print("eig csr folded scaling", basis_dtype, flush=True)
    r1 = ctx.eig_partial(mat, k, b, which="smallest", plan=plan, X0=X0)
    monkeypatch.setenv("OFRR_CHEB_FOLD", "0")
    r2 = ctx.eig_partial(mat, k, b, which="smallest", plan=plan, X0=X0)
    np.testing.assert_array_equal(r1.evals.cpu().numpy(), r2.evals.cpu().numpy())
    np.testing.assert_array_equal(r1.evecs.cpu().numpy(), r2.evecs.cpu().numpy())
    assert r1.info["products"] == r2.info["products"]
