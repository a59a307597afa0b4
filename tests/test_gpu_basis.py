"""The basis-generation processes of the comparison (Sec. 4.2 table; Sec.
5.3, Table 3) through the C ABI against the oracle.

* Hessenberg process, both forms, in FP64, FP32 and binary16 storage with
  FP32 arithmetic: bit for bit against the oracle's right-looking process
  in the same precision (left- and right-looking forms apply the same fused
  multiply-adds to every entry in the same order), pivots and drops too.
* Gram-Schmidt forms in FP64: Q and R against the oracle's definition of
  the same form, to the rounding the summation order allows for these
  well-conditioned blocks; FP32 and binary16 storage: within the rounding
  of that precision of the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import ofrr_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_00281_amd import ofrr
    c = ofrr.Context(0)
    yield c
    c.close()


def _block(m, n, seed, special=True):
    A = np.random.default_rng(seed).random((m, n))
    if special and n >= 8:
        A[:, 3] = 0.0            # a zero column: dropped by the Hessenberg process
        A[:, 5] = A[:, 1]        # a repeated column: its pivot falls to rounding level
    return A


def _colmajor(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(A.T)).to(dtype).cuda().t()


_TORCH = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
_ORC = {"f64": "f64", "f32": "f32", "f16": "f16s"}
_TOL = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "f16": 2.0 ** -10}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("method", ["hess_l", "hess_r"])
@pytest.mark.parametrize("shape", [(3001, 40), (25000, 200), (700, 9)])
def test_hessenberg_forms_bitwise(ctx, prec, method, shape):
    m, n = shape
    A = _block(m, n, 900 + n)
    Ag = _colmajor(A, _TORCH[prec])
    print("basis", method, prec, shape, flush=True)
    _, piv, keep, kept, _ = ctx.basis_generate(Ag, method, tol=_TOL[prec])
    Ain = torch.from_numpy(np.ascontiguousarray(A.T)).to(_TORCH[prec]).t().double().numpy()
    Q, p_ref, k_ref = O.hessenberg(Ain, _TOL[prec], _ORC[prec])
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    assert kept == int(k_ref.sum()) and kept < n
    got = Ag.cpu().double().numpy()
    np.testing.assert_array_equal(got, np.asarray(Q, dtype=np.float64))


_GS_ORC = {
    "mgs_l": O.gs_mgs_left,
    "mgs_r": O.gs_mgs_right,
    "cgs": O.gs_cgs,
    "cgs2": lambda A: O.gs_cgs(A, reorth=True),
}


@pytest.mark.parametrize("method", ["mgs_l", "mgs_r", "cgs", "cgs2"])
@pytest.mark.parametrize("shape", [(3001, 40), (25000, 200), (64, 64)])
def test_gram_schmidt_fp64_matches_oracle(ctx, method, shape):
    m, n = shape
    A = _block(m, n, 700 + n, special=False)
    Ag = _colmajor(A, torch.float64)
    print("basis", method, "f64", shape, flush=True)
    R, _, _, kept, _ = ctx.basis_generate(Ag, method, want_r=True)
    Qr, Rr = _GS_ORC[method](A)
    assert kept == n
    Q = Ag.cpu().numpy()
    kappa = np.linalg.cond(A)
    # both sides approximate the same factorisation; their difference is
    # bounded by the forms' rounding (kappa u for MGS, kappa^2 u for CGS)
    tol = 50 * (kappa ** 2 if method == "cgs" else kappa) * 2.0 ** -53 * np.sqrt(m)
    np.testing.assert_allclose(Q, Qr, atol=tol)
    np.testing.assert_allclose(R.cpu().numpy(), Rr, atol=tol * np.abs(Rr).max())


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("method", ["mgs_l", "mgs_r", "cgs", "cgs2"])
def test_gram_schmidt_reduced_precision(ctx, prec, method):
    m, n = 25000, 200
    A = _block(m, n, 777, special=False)
    Ag = _colmajor(A, _TORCH[prec])
    Ain = Ag.double().cpu().numpy()
    print("basis", method, prec, flush=True)
    R, _, _, _, _ = ctx.basis_generate(Ag, method, want_r=True)
    Q = Ag.double().cpu().numpy()
    Qr, Rr = _GS_ORC[method](Ain)
    u = 2.0 ** -24 if prec == "f32" else 2.0 ** -11
    kappa = np.linalg.cond(Ain)
    # every form is backward stable: Ain = Q R to a few units of the storage
    # rounding; orthogonality is lost like kappa u (MGS), kappa^2 u (CGS),
    # or stays at u (CGS2); Q near the FP64 oracle's within that loss
    res = np.linalg.norm(Ain - Q @ R.cpu().numpy()) / np.linalg.norm(Ain)
    assert res <= 50 * u * np.sqrt(n), res
    loss = np.linalg.norm(Q.T @ Q - np.eye(n), 2)
    bound = {"mgs_l": kappa, "mgs_r": kappa, "cgs": kappa ** 2, "cgs2": 1.0}[method] * u * 50 * np.sqrt(m)
    assert loss <= bound, (loss, bound)
    assert np.abs(Q - Qr).max() <= 20 * bound


def test_basis_rejects_bad_arguments(ctx):
    from paper_2505_00281_amd import ofrr
    A = _colmajor(np.zeros((10, 20)), torch.float64)  # n > m
    with pytest.raises(ofrr.OfrrError):
        ctx.basis_generate(A, "cgs")


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_mgs2_excludes_dependent_columns(ctx, prec):
    # with tol > 0, MGS2 excludes a column whose norm its projections reduce
    # to at most tol of its norm before them; the kept columns stay
    # orthonormal to the storage rounding and span the input's columns
    m, n = 5000, 24
    A = np.random.default_rng(990).random((m, n))
    A[:, 7] = A[:, 2] - 0.25 * A[:, 5]
    A[:, 15] = 0.0
    A[:, 20] = A[:, 1] + A[:, 3]
    Ag = _colmajor(A, _TORCH[prec])
    print("basis mgs2 exclusion", prec, flush=True)
    # dependent columns keep a few units of the storage rounding; the others
    # about half their norm (U(0,1) columns share their mean direction)
    tol = {"f64": 2.0 ** -40, "f32": 2.0 ** -16, "f16": 2.0 ** -6}[prec]
    _, piv, keep, kept, _ = ctx.basis_generate(Ag, "mgs2", tol=tol)
    k = keep.cpu().numpy()
    assert k[7] == 0 and k[15] == 0 and k[20] == 0 and kept == n - 3 and k.sum() == kept
    np.testing.assert_array_equal(piv.cpu().numpy(), np.where(k == 1, np.arange(n), -1))
    Q = Ag.double().cpu().numpy()[:, k == 1]
    u = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f16": 2.0 ** -11}[prec]
    assert np.linalg.norm(Q.T @ Q - np.eye(kept), 2) <= 50 * u * np.sqrt(m)
    # every input column lies in the span of the kept columns
    Ain = torch.from_numpy(np.ascontiguousarray(A.T)).to(_TORCH[prec]).double().numpy().T
    res = Ain - Q @ (Q.T @ Ain)
    assert np.linalg.norm(res) <= 50 * u * np.sqrt(m) * np.linalg.norm(Ain)
