"""Step-level parity of the HIP kernels against the CPU oracle, called
through the C ABI.  Integer and byte results are compared bit-exactly; float
results within the rounding-error bound of the arithmetic they perform."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ofrr_oracle as O
from oracle import rounding as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_00281_amd import ofrr
    c = ofrr.Context(0)
    yield c
    c.close()


def _cuda(x):
    return torch.as_tensor(x).cuda()


# ---------------------------------------------------------------- quantize

def test_quantize_bf16_f16_bit_exact(ctx):
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(100000).astype(np.float32) * 10,
        np.array([1.0, 1.00390625, 1.01171875, 1.0078125, -2.0, 0.0, 3.0e38, 1e-40, 65504.0,
                  65520.0, 6e-8, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11], dtype=np.float32)])
    print("quantize bf16/f16 count", x.size, flush=True)
    got = ctx.quantize(_cuda(x), "bf16").cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got, R.f32_to_bf16_bits(x))
    got16 = ctx.quantize(_cuda(x), "f16").cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got16, x.astype(np.float16).view(np.uint16))


def test_fp8_block_quantize_bit_exact(ctx):
    rng = np.random.default_rng(2)
    rows, cols = 100, 70  # ragged blocks
    A = (rng.standard_normal((rows, cols)) * np.exp(rng.uniform(-20, 10, (rows, cols)))).astype(np.float32)
    A[:32, :32] = 0.0  # an all-zero block
    A[40, 40] = 448.0 * 2.0 ** -3  # amax exactly 448 * power of two
    print("fp8 blocks", rows, cols, flush=True)
    At = torch.from_numpy(A.T.copy()).cuda().t()  # column-major
    codes, scales = ctx.quantize_fp8_blocks(At)
    c_ref, s_ref = R.fp8_block_quantize(A)
    np.testing.assert_array_equal(scales.cpu().numpy(), s_ref)
    np.testing.assert_array_equal(codes.cpu().numpy(), c_ref)


def test_fp8_block_quantize_hand_worked(ctx):
    """The kernel on the hand-worked 40 x 33 case of the oracle pins (scale 8,
    16, 1 and the 2^-126 floor; subnormal and tie codes), compared with the
    hand-derived values rather than with the oracle."""
    A = np.zeros((40, 33), dtype=np.float32)
    A[3, 5], A[7, 9], A[0, 0] = 3584.0, 8.0, -1.0
    A[10, 32], A[11, 32] = 3585.0, 0.5
    A[33, 32], A[34, 32] = 2.0 ** -130, -(2.0 ** -133)
    want = np.zeros((40, 33), dtype=np.uint8)
    want[3, 5], want[7, 9], want[0, 0] = 0x7E, 0x38, 0xA0
    want[10, 32], want[11, 32] = 0x76, 0x10
    want[33, 32], want[34, 32] = 0x18, 0x84
    print("fp8 blocks hand-worked 40x33", flush=True)
    codes, scales = ctx.quantize_fp8_blocks(torch.from_numpy(A.T.copy()).cuda().t())
    np.testing.assert_array_equal(scales.cpu().numpy(),
                                  np.array([[8.0, 16.0], [1.0, 2.0 ** -126]], np.float32))
    np.testing.assert_array_equal(codes.cpu().numpy(), want)


# ---------------------------------------------------------------- products

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("trans", [0, 1])
def test_product_f64(ctx, dtype, trans):
    rng = np.random.default_rng(3)
    m, kd, b = 300, 257, 13
    A = rng.standard_normal((m, kd) if not trans else (kd, m))
    A = A.astype(np.float32).astype(np.float64) if dtype == torch.float32 else A
    V = rng.standard_normal((kd, b))
    print("product_f64", dtype, trans, flush=True)
    At = torch.from_numpy(np.asfortranarray(A)).to(dtype)
    At = At.t().contiguous().t().cuda()
    Wg = ctx.block_product(At, _cuda(V), trans=bool(trans)).cpu().numpy()
    opA = A.T if trans else A
    ref = opA @ V
    bound = 2 * kd * 2.0 ** -53 * (np.abs(opA) @ np.abs(V))
    assert np.all(np.abs(Wg - ref) <= bound + 1e-300)


def _pow2_above(x):
    """Smallest power of two strictly above each |x| (1 for zeros)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    _, e = np.frexp(x)
    return np.where(x > 0, np.ldexp(1.0, e), 1.0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("shape,digits", [((300, 257, 13), 6), ((130, 20000, 70), 6), ((1000, 1000, 128), 6),
                                          ((1000, 1000, 128), 5), ((300, 257, 13), 4), ((130, 20000, 70), 5)])
def test_product_sliced(ctx, dtype, trans, shape, digits):
    """INT8 digit-plane product against the FP64 product: within the
    truncation bound 2^-7d (2^e_i sum|V_:j| + 2^f_j sum|A_i:| + 1.02 (d - 1) K
    2^(e_i+f_j)) of the d-digit planes (each side truncated below 2^-7d of
    its row/column scale) and the dropped digit pairs (s + t > d + 1, at most
    127^2 2^-7(s+t) each), plus FP64 rounding of both sides.  The (130,
    20000) case needs two K ranges (int32 cap)."""
    rng = np.random.default_rng(21)
    m, kd, b = shape
    A = rng.standard_normal((m, kd) if not trans else (kd, m)) * np.exp(rng.uniform(-3, 0, (1, 1)))
    A = A.astype(np.float32).astype(np.float64) if dtype == torch.float32 else A
    V = rng.standard_normal((kd, b)) * np.exp(rng.uniform(-4, 1, (1, b)))
    print("product_sliced", dtype, trans, shape, digits, flush=True)
    At = torch.from_numpy(np.asfortranarray(A)).to(dtype)
    At = At.t().contiguous().t().cuda()
    Wg = ctx.block_product_sliced(At, _cuda(V), trans=bool(trans), digits=digits).cpu().numpy()
    opA = A.T if trans else A
    ref = opA @ V
    ea = _pow2_above(np.max(np.abs(opA), axis=1))[:, None]
    fv = _pow2_above(np.max(np.abs(V), axis=0))[None, :]
    bound = 2.0 ** (-7 * digits) * (ea * np.sum(np.abs(V), axis=0)[None, :] +
                                     fv * np.sum(np.abs(opA), axis=1)[:, None] +
                                     1.02 * (digits - 1) * kd * ea * fv)
    bound += 4 * kd * 2.0 ** -53 * (np.abs(opA) @ np.abs(V))
    err = np.abs(Wg - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    # and, with six digits, far tighter than an FP32 product could be
    if digits == 6:
        assert np.max(err / (np.abs(opA) @ np.abs(V))) < 1e-10


def test_product_sliced_width_sequence(ctx):
    """Products of different widths in a row on one context (wide, narrow,
    wide): the column maxima merged for one call never leak into a later
    one, so the last product is bit-identical to the same product on a
    fresh context (its trailing columns are smaller than the first call's,
    so a leaked maximum would change their digit planes)."""
    from paper_2505_00281_amd import ofrr
    rng = np.random.default_rng(22)
    n = 2000
    A = rng.standard_normal((n, n))
    At = torch.from_numpy(np.asfortranarray(A)).cuda()
    V1 = rng.standard_normal((n, 128)) * 1e3
    Vn = rng.standard_normal((n, 16)) * 1e6
    V3 = rng.standard_normal((n, 128))
    V3[:, 64:] *= 1e-3
    print("product_sliced width sequence", flush=True)
    fresh = ofrr.Context(0)
    try:
        Wref = fresh.block_product_sliced(At, _cuda(V3)).cpu().numpy()
    finally:
        fresh.close()
    ctx.block_product_sliced(At, _cuda(V1))
    ctx.block_product_sliced(At, _cuda(Vn))
    W3 = ctx.block_product_sliced(At, _cuda(V3)).cpu().numpy()
    np.testing.assert_array_equal(W3.view(np.uint64), Wref.view(np.uint64))


@pytest.mark.parametrize("lowp", ["bf16", "f16"])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("shape", [(300, 1000, 70), (128, 64, 64), (4100, 4096, 128)])
def test_product_lowp(ctx, lowp, trans, shape):
    from paper_2505_00281_amd import ofrr
    rng = np.random.default_rng(4)
    m, kd, b = shape
    A = rng.standard_normal((m, kd) if not trans else (kd, m)).astype(np.float32)
    V = rng.standard_normal((kd, b)).astype(np.float32)
    rnd = R.round_bf16 if lowp == "bf16" else R.round_f16
    Ar, Vr = rnd(A).astype(np.float64), rnd(V).astype(np.float64)
    print("product_lowp", lowp, trans, shape, flush=True)
    Acm = torch.from_numpy(np.asfortranarray(A).T.copy()).cuda()  # storage of A^T row-major = A col-major
    Aq = ctx.quantize(Acm, lowp)  # same memory order
    Vq = ctx.quantize(_cuda(V), lowp)
    mat = ofrr.Matrix()
    mat.format, mat.dtype = ofrr.DENSE, ofrr.BF16 if lowp == "bf16" else ofrr.F16
    mat.rows, mat.cols = A.shape
    mat.ld = A.shape[0]
    mat.values = Aq.data_ptr()
    Wg = ctx.block_product(mat, Vq, trans=bool(trans), v_dtype=lowp).cpu().numpy().astype(np.float64)
    opA = Ar.T if trans else Ar
    ref = opA @ Vr  # products of the rounded values are exact in FP32 and FP64
    bound = (kd + 2) * 2.0 ** -24 * (np.abs(opA) @ np.abs(Vr))
    err = np.abs(Wg - ref)
    assert np.all(err <= bound), float(np.max(err / np.maximum(bound, 1e-300)))


@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("shape", [(300, 1000, 70), (4100, 2080, 128)])
def test_product_fp8_block_scaled(ctx, trans, shape):
    """FP8 e4m3fn product with 32x32 block scales on A and per-(column, 32
    rows) scales on V: equal to the FP64 product of the dequantised operands
    within the FP32 accumulation bound (scaled FP8 products are exact)."""
    rng = np.random.default_rng(12)
    m, kd, b = shape
    ar, ac = (m, kd) if not trans else (kd, m)
    A = (rng.standard_normal((ar, ac)) * np.exp(rng.uniform(-6, 2, (ar, ac)))).astype(np.float32)
    V = rng.standard_normal((kd, b)).astype(np.float32)
    codes_ref, scales_ref = R.fp8_block_quantize(A)
    Adq = R.e4m3_bits_to_f32(codes_ref).astype(np.float64) * np.kron(
        scales_ref.astype(np.float64), np.ones((32, 32)))[:ar, :ac]
    Vdq = R.fp8_colblock_quantize(V)
    print("product_fp8", trans, shape, flush=True)
    At = torch.from_numpy(A.T.copy()).cuda().t()
    codes, scales = ctx.quantize_fp8_blocks(At)
    Wg = ctx.block_product_fp8(codes, scales, _cuda(V), trans=bool(trans)).cpu().numpy().astype(np.float64)
    opA = Adq.T if trans else Adq
    ref = opA @ Vdq
    bound = (kd + 2) * 2.0 ** -24 * (np.abs(opA) @ np.abs(Vdq))
    err = np.abs(Wg - ref)
    assert np.all(err <= bound + 1e-30), float(np.max(err / np.maximum(bound, 1e-300)))


@pytest.mark.parametrize("b", [24, 23, 130])
@pytest.mark.parametrize("vt", ["f64", "f16", "f32"])
def test_spmm_laplacian(ctx, vt, b):
    # even widths take the paired-column kernel (130: more than 64 column
    # pairs per row), odd widths the one-column kernel
    from paper_2505_00281_amd import ofrr
    N = 37
    rp, ci, v = W.laplacian_2d_csr(N)
    n = N * N
    X = np.random.default_rng(5).standard_normal((n, b))
    if vt == "f16":
        X = R.round_f16(X).astype(np.float64)
        Xg = torch.from_numpy(X.astype(np.float16)).cuda()
    elif vt == "f32":
        X = X.astype(np.float32).astype(np.float64)
        Xg = torch.from_numpy(X.astype(np.float32)).cuda()
    else:
        Xg = _cuda(X)
    print("spmm", vt, flush=True)
    rpg, cig, vg = _cuda(rp), _cuda(ci), _cuda(v)
    mat = ofrr.csr_matrix(rpg, cig, vg)
    Wg = ctx.block_product(mat, Xg, v_dtype=vt).cpu().numpy().astype(np.float64)
    ref = O.csr_matmul(rp, ci, v.astype(np.float64), X)
    tol = 1e-14 if vt == "f64" else 2.0 ** -23
    np.testing.assert_allclose(Wg, ref, rtol=tol, atol=tol * 8 * np.abs(X).max())


# -------------------------------------------------------------- Hessenberg

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(1000, 24), (5000, 64), (70000, 128), (16384, 128), (7, 3)])
def test_hessenberg_matches_oracle_bitwise(ctx, prec, shape):
    n, b = shape
    rng = np.random.default_rng(6)
    Y = rng.random((n, b))
    dt = np.float64 if prec == "f64" else np.float32
    Y = Y.astype(dt)
    tol = 2.0 ** -52 if prec == "f64" else 2.0 ** -23
    print("hessenberg", prec, shape, flush=True)
    Yg = torch.from_numpy(Y.copy()).cuda()
    piv, keep, kept = ctx.hessenberg(Yg, tol)
    Q, p_ref, k_ref = O.hessenberg(Y, tol, prec)
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    assert kept == int(k_ref.sum())
    np.testing.assert_array_equal(Yg.cpu().numpy(), Q)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(16384, 128), (5000, 64)])
def test_hessenberg_lds_kernel_matches_oracle(ctx, monkeypatch, prec, shape):
    # the LDS-resident sweep (the one for blocks the register kernel does not
    # take), forced on shapes the register kernel would otherwise run
    monkeypatch.setenv("OFRR_HESS_REG", "0")
    n, b = shape
    rng = np.random.default_rng(13)
    dt = np.float64 if prec == "f64" else np.float32
    Y = rng.random((n, b)).astype(dt)
    tol = 2.0 ** -52 if prec == "f64" else 2.0 ** -23
    print("hessenberg lds kernel", prec, shape, flush=True)
    Yg = torch.from_numpy(Y.copy()).cuda()
    piv, keep, kept = ctx.hessenberg(Yg, tol)
    Q, p_ref, k_ref = O.hessenberg(Y, tol, prec)
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    np.testing.assert_array_equal(Yg.cpu().numpy(), Q)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(1048576, 64), (300001, 37), (70000, 128)])
def test_hessenberg_panel_kernel_matches_oracle(ctx, prec, shape):
    # blocks too tall for the row slices to stay on chip take the panel
    # form (eight columns per panel, trailing block updated once per panel):
    # the same bits as the per-column process, pivots and drops included.
    # Columns 5 and 20 (inside and across panels) depend on earlier ones and
    # column 11 is zero, so drops occur at several positions in a panel
    n, b = shape
    rng = np.random.default_rng(17 + b)
    Y = rng.standard_normal((n, b))
    Y[:, 5] = Y[:, 1] - 0.5 * Y[:, 3]
    Y[:, 11] = 0.0
    Y[:, 20] = Y[:, 2] + Y[:, 13]
    Y /= np.maximum(np.abs(Y).max(axis=0), 1e-300)
    dt = np.float64 if prec == "f64" else np.float32
    Y = Y.astype(dt)
    tol = (2.0 ** -52 if prec == "f64" else 2.0 ** -23) * 64
    print("hessenberg panel", prec, shape, flush=True)
    Yg = torch.from_numpy(Y.copy()).cuda()
    piv, keep, kept = ctx.hessenberg(Yg, tol)
    Q, p_ref, k_ref = O.hessenberg(Y, tol, prec)
    assert k_ref[5] == 0 and k_ref[11] == 0 and k_ref[20] == 0
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    assert kept == int(k_ref.sum())
    np.testing.assert_array_equal(Yg.cpu().numpy(), Q)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hessenberg_drops_like_oracle(ctx, prec):
    rng = np.random.default_rng(7)
    n, b = 3000, 12
    Y = rng.standard_normal((n, b))
    Y[:, 5] = Y[:, 1] - 0.5 * Y[:, 3]
    Y[:, 9] = 0.0
    Y /= np.maximum(np.abs(Y).max(axis=0), 1e-300)
    dt = np.float64 if prec == "f64" else np.float32
    Y = Y.astype(dt)
    tol = (2.0 ** -52 if prec == "f64" else 2.0 ** -23) * 64
    print("hessenberg drops", prec, flush=True)
    Yg = torch.from_numpy(Y.copy()).cuda()
    piv, keep, kept = ctx.hessenberg(Yg, tol)
    Q, p_ref, k_ref = O.hessenberg(Y, tol, prec)
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    assert k_ref[5] == 0 and k_ref[9] == 0
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    np.testing.assert_array_equal(Yg.cpu().numpy(), Q)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nt", ["64", "128", "256"])
@pytest.mark.parametrize("shape", [(16384, 128), (3000, 77), (130, 5)])
def test_hessenberg_register_widths(ctx, monkeypatch, prec, nt, shape):
    # the register sweep (FP32 and FP64 rows) at each workgroup width gives
    # the oracle's pivots and factor bit for bit (ragged last slice included)
    n, b = shape
    monkeypatch.setenv("OFRR_HESS_REG_NT", nt)
    monkeypatch.setenv("OFRR_HESS_REG64", "1")
    rng = np.random.default_rng(11)
    dt = np.float32 if prec == "f32" else np.float64
    Y = rng.standard_normal((n, b)).astype(dt)
    tol = 2.0 ** -23 if prec == "f32" else 2.0 ** -52
    print("hessenberg register width", prec, nt, shape, flush=True)
    Yg = torch.from_numpy(Y.copy()).cuda()
    piv, keep, kept = ctx.hessenberg(Yg, tol)
    Q, p_ref, k_ref = O.hessenberg(Y, tol, prec)
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    np.testing.assert_array_equal(Yg.cpu().numpy(), Q)


@pytest.mark.parametrize("prec,nt", [("f32", "64"), ("f32", "256"), ("f64", "64"), ("f64", "lds"),
                                     ("f32", "lds")])
def test_hessenberg_signed_zeros_bitwise(ctx, monkeypatch, prec, nt):
    # negative zeros in the input: finished columns keep their sign of zero
    # and updated ones get the fused multiply-add's, as in the oracle
    # (compared as bit patterns, where -0.0 == 0.0 would hide a difference)
    if nt == "lds":
        monkeypatch.setenv("OFRR_HESS_REG", "0")
    else:
        monkeypatch.setenv("OFRR_HESS_REG_NT", nt)
    rng = np.random.default_rng(12)
    n, b = 3000, 40
    Y = rng.standard_normal((n, b))
    Y[rng.random((n, b)) < 0.15] = -0.0
    Y[:, 7] = -0.0
    dt = np.float64 if prec == "f64" else np.float32
    Y = Y.astype(dt)
    tol = 2.0 ** -52 if prec == "f64" else 2.0 ** -23
    print("hessenberg signed zeros", prec, nt, flush=True)
    Yg = torch.from_numpy(Y.copy()).cuda()
    piv, keep, kept = ctx.hessenberg(Yg, tol)
    Q, p_ref, k_ref = O.hessenberg(Y, tol, prec)
    np.testing.assert_array_equal(piv.cpu().numpy(), p_ref)
    np.testing.assert_array_equal(keep.cpu().numpy(), k_ref)
    ui = np.uint64 if prec == "f64" else np.uint32
    np.testing.assert_array_equal(Yg.cpu().numpy().view(ui), np.ascontiguousarray(Q).view(ui))


# ------------------------------------------------------------- projection

@pytest.mark.parametrize("vt", ["f64", "bf16", "f32"])
@pytest.mark.parametrize("shape", [(3001, 70), (16384, 128), (5, 3)])
@pytest.mark.parametrize("accum", ["f64", "f32c", "f32"])
def test_project(ctx, vt, shape, accum):
    """G = V^T V and H = V^T W against the FP64 products of the same stored
    values, within the bound of each accumulation: FP64 sums of exact
    products (2n u64); compensated: FP32 runs of 32 rows of FP32-rounded
    products, the runs summed in FP64 ((32+2) u32 + 2n u64); FP32: a sum of
    n rounded products in FP32 ((n+2) u32).  Bounds are elementwise,
    relative to |V|^T |W|; u32 is taken as 2^-23 (one unit in the last
    place per FP32 operation, whatever rounding the MFMA applies inside)."""
    from paper_2505_00281_amd import ofrr
    rng = np.random.default_rng(8)
    n, b = shape
    V = rng.standard_normal((n, b))
    Wm = rng.standard_normal((n, b))
    if vt == "bf16":
        V = R.round_bf16(V).astype(np.float64)
        Vg = ctx.quantize(_cuda(V.astype(np.float32)), "bf16")
        Wm = Wm.astype(np.float32).astype(np.float64)
        Wg = _cuda(Wm.astype(np.float32))
    elif vt == "f32":
        V = V.astype(np.float32).astype(np.float64)
        Vg = _cuda(V.astype(np.float32))
        Wm = Wm.astype(np.float32).astype(np.float64)
        Wg = _cuda(Wm.astype(np.float32))
    else:
        Vg, Wg = _cuda(V), _cuda(Wm)
    print("project", vt, shape, accum, flush=True)
    if vt == "f64" and accum != "f64":
        with pytest.raises(ofrr.OfrrError) as e:
            ctx.project(Vg, Wg, accum=accum, v_dtype=vt)
        assert e.value.status == ofrr.ERR_UNSUPPORTED
        return
    G, H = ctx.project(Vg, Wg, accum=accum, v_dtype=vt)
    G, H = G.cpu().numpy(), H.cpu().numpy()
    u32, u64 = 2.0 ** -23, 2.0 ** -53
    rel = {"f64": 2 * n * u64, "f32c": 34 * u32 + 2 * n * u64, "f32": (n + 2) * u32}[accum]
    aVV, aVW = np.abs(V).T @ np.abs(V), np.abs(V).T @ np.abs(Wm)
    eG, eH = np.abs(G - V.T @ V), np.abs(H - V.T @ Wm)
    assert np.all(eG <= rel * aVV), float(np.max(eG / (rel * aVV)))
    assert np.all(eH <= rel * aVW), float(np.max(eH / (rel * aVW)))
    if accum == "f64":
        assert np.array_equal(G, G.T)
    else:
        # FP32 rounding shows: the result is not the FP64 one
        assert n < 32 or not np.array_equal(H, V.T @ Wm)


# ---------------------------------------------------------- small problems

@pytest.mark.parametrize("b", [1, 2, 7, 16, 64, 128])
def test_pencil_eig(ctx, b):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((400, 400))
    A = A + A.T
    V = rng.standard_normal((400, b))
    H, G = V.T @ A @ V, V.T @ V
    print("pencil", b, flush=True)
    theta, Y, rank = ctx.pencil_eig(_cuda(H), _cuda(G), "largest")
    theta, Y = theta.cpu().numpy(), Y.cpu().numpy()
    t_ref, Y_ref = O.sym_pencil_eig(H, G)
    t_ref, Y_ref = t_ref[::-1], Y_ref[:, ::-1]
    assert rank == b
    scale = np.abs(t_ref).max()
    np.testing.assert_allclose(theta, t_ref, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Y.T @ G @ Y, np.eye(b), atol=1e-10)
    np.testing.assert_allclose(H @ Y, G @ Y * theta, atol=1e-9 * scale * np.abs(Y).max())


@pytest.mark.parametrize("b,which", [(33, "smallest"), (100, "largest"), (128, "smallest")])
def test_pencil_eig_repeated_eigenvalues(ctx, b, which):
    """H = M^T D M, G = M^T M: the pencil's eigenvalues are D's, here with
    multiplicities up to four, so the cluster branch of the eigenvector step
    runs; Y must still be G-orthonormal with a small residual."""
    rng = np.random.default_rng(11 + b)
    M = rng.standard_normal((b, b)) + 4.0 * np.eye(b)
    lam = np.repeat(np.linspace(-1.0, 2.0, (b + 3) // 4), 4)[:b]
    H, G = M.T @ (lam[:, None] * M), M.T @ M
    print("pencil repeated", b, which, flush=True)
    theta, Y, rank = ctx.pencil_eig(_cuda(H), _cuda(G), which)
    theta, Y = theta.cpu().numpy(), Y.cpu().numpy()
    t_ref, _ = O.sym_pencil_eig(H, G)
    t_ref = t_ref if which == "smallest" else t_ref[::-1]
    assert rank == b
    np.testing.assert_allclose(np.sort(lam)[:: 1 if which == "smallest" else -1], t_ref, atol=1e-9)
    np.testing.assert_allclose(theta, t_ref, rtol=0, atol=1e-11)
    np.testing.assert_allclose(Y.T @ G @ Y, np.eye(b), atol=1e-9)
    np.testing.assert_allclose(H @ Y, G @ Y * theta, atol=1e-8 * np.abs(G @ Y).max())


def test_pencil_eig_indefinite_mass_falls_back(ctx):
    rng = np.random.default_rng(10)
    A = rng.standard_normal((200, 200))
    A = A + A.T
    V = rng.standard_normal((200, 8))
    V[:, 6] = V[:, 0] + V[:, 2]  # rank 7
    H, G = V.T @ A @ V, V.T @ V
    print("pencil fallback", flush=True)
    theta, Y, rank = ctx.pencil_eig(_cuda(H), _cuda(G), "largest")
    assert rank == 7
    theta = theta.cpu().numpy()
    Q, _ = np.linalg.qr(V[:, [0, 1, 2, 3, 4, 5, 7]])
    ref = np.sort(np.linalg.eigvalsh(Q.T @ A @ Q))[::-1]
    np.testing.assert_allclose(theta[:7], ref, rtol=1e-8, atol=1e-8)
    assert theta[7] == 0.0


@pytest.mark.parametrize("k1,k2", [(8, 6), (16, 16), (40, 25), (25, 40), (200, 200), (200, 171)])
def test_svd_pencil(ctx, k1, k2):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((300, 240))
    U = rng.standard_normal((300, k1))
    V = rng.standard_normal((240, k2))
    B, MU, MV = U.T @ A @ V, U.T @ U, V.T @ V
    print("svd pencil", k1, k2, flush=True)
    s, Y, Z = ctx.svd_pencil(_cuda(B), _cuda(MU), _cuda(MV))
    s, Y, Z = s.cpu().numpy(), Y.cpu().numpy(), Z.cpu().numpy()
    s_ref, _, _ = O.svd_pencil(B, MU, MV)
    np.testing.assert_allclose(s, s_ref[:min(k1, k2)], rtol=1e-11)
    Ut, Vt = np.sqrt(2) * U @ Y, np.sqrt(2) * V @ Z
    np.testing.assert_allclose(Ut.T @ Ut, np.eye(min(k1, k2)), atol=1e-9)
    np.testing.assert_allclose(Vt.T @ Vt, np.eye(min(k1, k2)), atol=1e-9)
    # the left and right vectors belong together: 2 Y^T B Z = diag(sigma)
    np.testing.assert_allclose(2.0 * Y.T @ B @ Z, np.diag(s), atol=1e-9 * s[0])


@pytest.mark.parametrize("k", [30, 200])
def test_svd_pencil_not_positive_definite(ctx, k):
    # a mass matrix with a negative pivot is reported (U^T U: status 3,
    # V^T V: status 4) before the Jacobi launch, on both sizes of the
    # pipeline; the context then solves a valid pencil as before
    from paper_2505_00281_amd import ofrr
    rng = np.random.default_rng(12)
    U = rng.standard_normal((3 * k, k))
    V = rng.standard_normal((3 * k, k))
    B, MU, MV = U.T @ rng.standard_normal((3 * k, 3 * k)) @ V, U.T @ U, V.T @ V
    bad = np.eye(k)
    bad[k // 2, k // 2] = -1.0
    print("svd pencil not positive definite", k, flush=True)
    for mu, mv, what in ((bad, MV, "U^T U"), (MU, bad, "V^T V")):
        with pytest.raises(ofrr.OfrrError) as e:
            ctx.svd_pencil(_cuda(B), _cuda(mu), _cuda(mv))
        assert e.value.status == ofrr.ERR_NUMERIC and what in str(e.value)
    s, _, _ = ctx.svd_pencil(_cuda(B), _cuda(MU), _cuda(MV))
    s_ref, _, _ = O.svd_pencil(B, MU, MV)
    np.testing.assert_allclose(s.cpu().numpy(), s_ref[:k], rtol=1e-11)
