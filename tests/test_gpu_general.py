"""Real non-symmetric A on the GPU path (Sec. 3.1: complex Ritz values;
eq. (geig) with the pencil (V^T A V, V^T V) of a non-orthogonal basis),
through the C ABI, against the CPU oracle.

* The small pencil: values against the oracle's Cholesky-reduced solve of
  the same pencil (ordering rule of both sides: modulus, real part,
  imaginary part descending), vectors compared up to their phase (the
  complex scalar that fixes a vector is not part of the pencil's answer),
  y^H G y = 1 and B y = theta M y checked directly.
* Whole method, FP64 form, same-step mode: after the same outer iterations
  the Ritz values equal the oracle's (a fixed subspace has fixed Ritz
  pairs) to 1e-10 of the largest modulus; vectors up to phase.
* Converged mode, FP64 and mixed plans: prescribed spectra S D S^-1 (dense)
  and the convection-diffusion operator (CSR), against the closed forms.
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


def _unpack(tre, tim, Y):
    """Complex vectors from the packed real form."""
    b = tre.size
    Z = np.zeros((Y.shape[0], b), complex)
    j = 0
    while j < b:
        if tim[j] > 0:
            Z[:, j] = Y[:, j] + 1j * Y[:, j + 1]
            Z[:, j + 1] = np.conj(Z[:, j])
            j += 2
        else:
            Z[:, j] = Y[:, j]
            j += 1
    return Z


def _same_up_to_phase(x, y, M=None):
    """|<x, y>_M| / (||x||_M ||y||_M): 1 when x and y span the same line."""
    M = np.eye(x.size) if M is None else M
    return abs(np.vdot(x, M @ y)) / np.sqrt(np.vdot(x, M @ x).real * np.vdot(y, M @ y).real)


def _pencil_case(b, seed, spread=1e-3):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((3 * b + 5, b)) @ np.diag(np.logspace(0, np.log10(spread), b))
    A = rng.standard_normal((3 * b + 5, 3 * b + 5))
    return U.T @ A @ U, U.T @ U


@pytest.mark.parametrize("b", [1, 2, 3, 17, 64, 120, 121, 200])
def test_pencil_general_vs_oracle(ctx, b):
    B, M = _pencil_case(b, 100 + b)
    print("pencil general b", b, flush=True)
    tre, tim, Y = ctx.pencil_eig_general(torch.from_numpy(B).cuda(), torch.from_numpy(M).cuda())
    tre, tim, Y = tre.cpu().numpy(), tim.cpu().numpy(), Y.cpu().numpy()
    th = tre + 1j * tim
    ref, Yref = O.general_pencil_eig(B, M)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(th, ref, rtol=0, atol=1e-10 * scale)
    Z = _unpack(tre, tim, Y)
    for j in range(b):
        z = Z[:, j]
        assert abs(np.vdot(z, M @ z).real - 1) < 1e-9
        assert np.linalg.norm(B @ z - th[j] * (M @ z)) <= 1e-9 * np.linalg.norm(B) * np.linalg.norm(z)
        # eigenvalues at least 1e-6 apart here: vectors are determined
        assert _same_up_to_phase(z, Yref[:, j], M) > 1 - 1e-8


def test_pencil_general_rotation_and_identity(ctx):
    # H = [[0, 1], [-1, 0]] (eigenvalues +-i), G = I: y = [1, +-i]/sqrt2 up to phase
    H = torch.tensor([[0.0, 1.0], [-1.0, 0.0]], dtype=torch.float64).cuda()
    G = torch.eye(2, dtype=torch.float64).cuda()
    tre, tim, Y = ctx.pencil_eig_general(H, G)
    np.testing.assert_allclose(tre.cpu().numpy(), [0, 0], atol=1e-15)
    np.testing.assert_allclose(tim.cpu().numpy(), [1, -1], atol=1e-15)
    z = _unpack(tre.cpu().numpy(), tim.cpu().numpy(), Y.cpu().numpy())[:, 0]
    assert _same_up_to_phase(z, np.array([1, 1j]) / np.sqrt(2)) > 1 - 1e-15
    # a diagonal H with G = I: the values in modulus order, unit vectors
    d = np.array([3.0, -5.0, 1.0, 4.0, -2.0])
    tre, tim, Y = ctx.pencil_eig_general(torch.from_numpy(np.diag(d)).cuda(), torch.eye(5, dtype=torch.float64).cuda())
    np.testing.assert_array_equal(tre.cpu().numpy(), [-5.0, 4.0, 3.0, -2.0, 1.0])
    np.testing.assert_array_equal(tim.cpu().numpy(), 0.0)
    np.testing.assert_allclose(np.abs(Y.cpu().numpy()), np.eye(5)[:, [1, 3, 0, 4, 2]], atol=1e-15)


def test_pencil_general_rejects_indefinite_mass(ctx):
    from paper_2505_00281_amd import ofrr
    B, _ = _pencil_case(6, 5)
    M = np.diag([1.0, 1.0, -1.0, 1.0, 1.0, 1.0])
    with pytest.raises(ofrr.OfrrError, match="NUMERIC"):
        ctx.pencil_eig_general(torch.from_numpy(B).cuda(), torch.from_numpy(M).cuda())


def _prescribed(n, seed, nonnormal=0.3):
    reals = [6.0, -5.0, 3.0] + list(np.linspace(1.0, 0.1, n - 9))
    pairs = [(4.0, 2.5), (1.5, -1.2), (0.3, 0.2)]
    A = W.general_prescribed(reals, pairs, seed, nonnormal=nonnormal)
    lam = np.array(reals + [complex(a, b) for a, b in pairs] + [complex(a, -b) for a, b in pairs])
    return A, lam[O.general_order(lam)]


def _check_vectors(A, r, tol):
    """||A x - lambda x|| / |lambda_1| for the returned unit vectors, and the
    phase rule (largest-modulus entry real and positive)."""
    th = r.evals.cpu().numpy()
    X = r.evecs.cpu().numpy()
    An = A if isinstance(A, np.ndarray) else None
    for j in range(th.size):
        x = X[:, j]
        assert abs(np.linalg.norm(x) - 1) < 1e-12
        i = int(np.argmax(np.abs(x)))
        assert x[i].imag == 0.0 and x[i].real > 0
        if An is not None:
            assert np.linalg.norm(An @ x - th[j] * x) <= tol * abs(th[0])


@pytest.mark.parametrize("n,b,k,degree,outer", [(1037, 16, 6, 2, 8), (600, 24, 5, 1, 12)])
def test_eig_general_fp64_same_step(ctx, n, b, k, degree, outer):
    A, _ = _prescribed(n, 31 + n)
    X0 = W.uniform_start(n, b, 41 + n)
    print("eig general fp64 same-step", n, b, k, flush=True)
    r = ctx.eig_general(A.cuda(), k, b, plan=_plan(max_iters=outer, degree=degree), X0=torch.from_numpy(X0))
    ref = O.subspace_eig_general(A.numpy(), X0, k, degree=degree, outer=outer, basis="hessenberg")
    assert r.info["iters"] == outer
    th = r.evals.cpu().numpy()
    np.testing.assert_allclose(th, ref.theta, rtol=0, atol=1e-10 * abs(ref.theta[0]))
    X = r.evecs.cpu().numpy()
    for j in range(k):
        assert _same_up_to_phase(X[:, j], ref.X[:, j]) > 1 - 1e-8, j
    np.testing.assert_allclose(r.resid.cpu().numpy(), ref.resid, rtol=1e-5, atol=1e-13)
    _check_vectors(A.numpy(), r, 1.0)


@pytest.mark.parametrize("cfg", ["f64", "bf16_refine1", "bf16_refine2_i8", "f16_refine1"])
def test_eig_general_converged_prescribed(ctx, cfg):
    n, b, k = 2000, 24, 5
    A, lam = _prescribed(n, 7)
    kw = dict(f64=dict(basis_dtype="f64"),
              bf16_refine1=dict(basis_dtype="bf16", refine=1),
              bf16_refine2_i8=dict(basis_dtype="bf16", refine=2, tail="i8"),
              f16_refine1=dict(basis_dtype="f16", refine=1))[cfg]
    # the six-digit INT8 products of the sliced tail are exact to about
    # 2^-42 of A's row scales times the basis column scales, summed over
    # 2000 terms: residuals near 1e-10 are at their floor, so that plan is
    # asked for 1e-9
    tol = 1e-9 if cfg == "bf16_refine2_i8" else 1e-10
    print("eig general converged", cfg, flush=True)
    r = ctx.eig_general(A.cuda(), k, b, plan=_plan(tol=tol, anorm=6.0, degree=2, max_iters=400, **kw),
                        X0=torch.from_numpy(W.uniform_start(n, b, 9)))
    assert r.status == 0, r.info
    th = r.evals.cpu().numpy()
    np.testing.assert_allclose(th, lam[:k], rtol=0, atol=1e-9)
    assert r.resid.cpu().numpy().max() <= tol
    _check_vectors(A.numpy(), r, 1e-9)
    if cfg != "f64":
        assert r.info["iters_low"] > 0


def test_eig_general_float32_matrix(ctx):
    # A stored in FP32: the FP64 products read it as stored; eigenvalues of
    # the stored matrix from LAPACK
    n, b, k = 700, 20, 4
    A, _ = _prescribed(n, 17)
    A32 = A.float().t().contiguous().t()
    lam = np.linalg.eigvals(A32.double().numpy())
    lam = lam[O.general_order(lam)]
    r = ctx.eig_general(A32.cuda(), k, b, plan=_plan(basis_dtype="bf16", refine=1, tol=1e-10, anorm=6.0,
                                                     max_iters=400),
                        X0=torch.from_numpy(W.uniform_start(n, b, 19)))
    assert r.status == 0
    np.testing.assert_allclose(r.evals.cpu().numpy(), lam[:k], rtol=0, atol=1e-9)


@pytest.mark.parametrize("basis_dtype,refine", [("f64", 0), ("f16", 2)])
def test_eig_general_csr_convection_diffusion(ctx, basis_dtype, refine):
    from paper_2505_00281_amd import ofrr
    # gamma 5: complex pairs with condition numbers about 3 (smaller gamma
    # above 1 makes the operator strongly non-normal: at gamma 1.5 the
    # leading values have condition numbers near 1e4, and residuals of 1e-10
    # fix them only to about 1e-6)
    N, gamma, b, k = 20, 5.0, 48, 6
    rp, ci, v = W.convection_diffusion_2d_csr(N, gamma)
    cf = W.convection_diffusion_2d_eigenvalues(N, gamma)
    cf = cf[O.general_order(cf)]
    mat = ofrr.csr_matrix(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(v).cuda())
    print("eig general csr", basis_dtype, refine, flush=True)
    r = ctx.eig_general(mat, k, b, plan=_plan(basis_dtype=basis_dtype, refine=refine, tol=1e-10, degree=4,
                                              anorm=float(abs(cf[0])), max_iters=3000),
                        X0=torch.from_numpy(W.uniform_start(N * N, b, 23)))
    assert r.status == 0, r.info
    th = r.evals.cpu().numpy()
    # values matched one to one (members of near-equal moduli may swap)
    want = list(cf[:k + 4])
    for z in th:
        d = np.abs(np.array(want) - z)
        j = int(np.argmin(d))
        assert d[j] <= 1e-9 * abs(cf[0]), (z, cf[:k + 2])
        want.pop(j)
    assert r.resid.cpu().numpy().max() <= 1e-10


def test_eig_general_same_step_csr_vs_oracle(ctx):
    from paper_2505_00281_amd import ofrr
    N, gamma, b, k, outer = 20, 0.5, 16, 4, 6
    rp, ci, v = W.convection_diffusion_2d_csr(N, gamma)
    X0 = W.uniform_start(N * N, b, 29)
    mat = ofrr.csr_matrix(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(v).cuda())
    r = ctx.eig_general(mat, k, b, plan=_plan(max_iters=outer, degree=3), X0=torch.from_numpy(X0))
    ref = O.subspace_eig_general((rp, ci, v), X0, k, degree=3, outer=outer, basis="hessenberg")
    np.testing.assert_allclose(r.evals.cpu().numpy(), ref.theta, rtol=0, atol=1e-10 * abs(ref.theta[0]))


def test_eig_general_rejects_unsupported_plans(ctx):
    from paper_2505_00281_amd import ofrr
    A, _ = _prescribed(200, 3)
    Ag = A.cuda()
    for kw in (dict(filter="chebyshev", lo=0.0, hi=1.0), dict(stab="qr"), dict(projection="classical"),
               dict(basis_dtype="f32"), dict(gram_accum="f32")):
        with pytest.raises(ofrr.OfrrError, match="UNSUPPORTED|INVALID"):
            ctx.eig_general(Ag, 4, 8, plan=_plan(**kw))
