"""The allocation-free Hessenberg entry point (ofrr_hessenberg_noalloc)
against ofrr_hessenberg, bit for bit: two calls in a row on the fixed
device array, the second smaller than the first (so stale words of the
first call must not leak into the second), for both element types and
both sweep kernels (register rows and LDS slices)."""
import numpy as np
import pytest
import torch

from paper_2505_00281_amd import ofrr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ofrr.Context(0)
    yield c
    c.close()


def _block(n, b, seed, dt):
    Y = np.random.default_rng(seed).random((n, b))
    # a zero column: its pivot is below any tolerance, so the sweep drops it
    # (keep = 0, piv = -1) in both entry points alike
    Y[:, b // 2] = 0.0
    return torch.from_numpy(Y.astype(dt)).cuda()


def _compare(ctx, Y, tol):
    n, b = Y.shape
    Y1 = Y.clone()
    Y2 = Y.clone()
    piv1, keep1, kept1 = ctx.hessenberg(Y1, tol)
    piv2 = torch.full((b,), -7, dtype=torch.int32, device=Y.device)
    keep2 = torch.full((b,), -7, dtype=torch.int32, device=Y.device)
    kept2 = ctx.hessenberg_noalloc(Y2, tol, piv2, keep2)
    torch.cuda.synchronize()
    assert kept2 == kept1
    assert kept1 == b - 1  # the zero column was dropped
    assert torch.equal(piv2, piv1)
    assert torch.equal(keep2, keep1)
    # bitwise, signed zeros included
    assert torch.equal(Y2.view(torch.int64 if Y.dtype == torch.float64 else torch.int32),
                       Y1.view(torch.int64 if Y.dtype == torch.float64 else torch.int32))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kernel", ["reg", "lds"])
def test_noalloc_matches_allocating_entry_two_calls(ctx, monkeypatch, prec, kernel):
    dt = np.float64 if prec == "f64" else np.float32
    tol = 2.0 ** -52 if prec == "f64" else 2.0 ** -23
    if kernel == "lds":
        monkeypatch.setenv("OFRR_HESS_REG", "0")
        shapes = [(20000, 300), (3001, 40)]
    else:
        shapes = [(16384, 128), (5000, 64)]
    for i, (n, b) in enumerate(shapes):
        print("noalloc hessenberg", prec, kernel, n, b, flush=True)
        _compare(ctx, _block(n, b, 100 + i, dt), tol)


def test_noalloc_rejects_wide_blocks_before_launch(ctx):
    Y = torch.zeros((64, 513), dtype=torch.float64, device="cuda")
    piv = torch.zeros(513, dtype=torch.int32, device="cuda")
    keep = torch.zeros(513, dtype=torch.int32, device="cuda")
    with pytest.raises(ofrr.OfrrError) as e:
        ctx.hessenberg_noalloc(Y, 1e-16, piv, keep)
    assert e.value.status == ofrr.ERR_INVALID_ARG
