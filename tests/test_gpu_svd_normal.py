"""The normal-equations (A^T A) form of the SVD against the oracle's form of
the same method: FP64 same-step parity (the Ritz values of A^T A on the same
subspaces), and a BF16 basis with an FP64 tail converged against the
closed-form singular values."""
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
    return ofrr.make_plan(svd_form="normal", **kw)


@pytest.mark.parametrize("m,n,k,b,outer", [(600, 300, 6, 12, 8), (1000, 257, 5, 9, 5)])
def test_svd_normal_fp64_same_step(ctx, m, n, k, b, outer):
    sig = np.exp(-np.arange(1, n + 1) / 20.0)
    A = W.svd_prescribed(m, n, sig, 3600 + n, dtype=torch.float64)
    V0 = W.uniform_start(n, b, 3700 + n)
    print("svd normal f64", m, n, flush=True)
    r = ctx.svd_partial(A.cuda(), k, b, plan=_plan(max_iters=outer), V0=torch.from_numpy(V0))
    ref = O.subspace_svd_normal(A.numpy(), V0, k, outer=outer)
    np.testing.assert_allclose(r.sigma.cpu().numpy(), ref.sigma, rtol=1e-12)
    np.testing.assert_allclose(r.V.cpu().numpy(), ref.V, atol=1e-8)
    np.testing.assert_allclose(r.U.cpu().numpy(), ref.U, atol=1e-8)


def test_svd_normal_bf16_converged(ctx):
    m, n, k, b = 4000, 1024, 8, 16
    sig = np.exp(-np.arange(1, n + 1) / 40.0)
    A = W.svd_prescribed(m, n, sig, 3800, dtype=torch.float32, device="cuda")
    V0 = torch.from_numpy(W.uniform_start(n, b, 3801))
    print("svd normal bf16", flush=True)
    r = ctx.svd_partial(A, k, b, plan=_plan(basis_dtype="bf16", refine=1, tol=5e-9, max_iters=300,
                                            stall_iters=3), V0=V0)
    s = r.sigma.cpu().numpy()
    assert np.all(r.resid.cpu().numpy() <= 1e-8)
    # FP32 storage of A moves each s by at most ||A_stored - A||_2 (~1e-7 s_1 here)
    np.testing.assert_allclose(s, sig[:k], rtol=2e-7)
    A64 = A.double().cpu().numpy()
    U, V = r.U.cpu().numpy(), r.V.cpu().numpy()
    res = np.sqrt(np.linalg.norm(A64 @ V - U * s, axis=0) ** 2 + np.linalg.norm(A64.T @ U - V * s, axis=0) ** 2)
    np.testing.assert_allclose(r.resid.cpu().numpy(), res / s[0], rtol=1e-3, atol=1e-14)
