"""Pins of the CPU oracle against what the paper and the mathematics fix:
closed forms, textbook/library special cases, invariants, brute force and
hand-worked fixtures.  A plausible slip anywhere in the oracle (a wrong
rotation sign, a dropped re-orthogonalisation, a transposed factor, a wrong
pivot rule) fails at least one of these."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import ofrr_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_sym(n, seed):
    g = np.random.default_rng(seed).standard_normal((n, n))
    return g + g.T


def _prescribed(lam, seed):
    return W.dense_symmetric_prescribed(lam, seed).numpy()


# --------------------------------------------------------------- Jacobi ----

def test_jacobi_2x2_closed_form(oracle):
    a, b, d = 3.0, -1.25, 0.5
    w, Z = oracle.jacobi_eig([[a, b], [b, d]])
    m, r = (a + d) / 2, math.hypot((a - d) / 2, b)
    np.testing.assert_allclose(w, [m - r, m + r], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Z.T @ Z, np.eye(2), atol=1e-15)


def test_jacobi_prescribed_spectrum(oracle):
    lam = 0.95 ** np.arange(1, 65)
    A = _prescribed(lam, 7)
    w, Z = oracle.jacobi_eig(A)
    np.testing.assert_allclose(w, np.sort(lam), rtol=0, atol=2e-15 * 64)
    np.testing.assert_allclose(A @ Z, Z * w, atol=1e-14)
    np.testing.assert_allclose(Z.T @ Z, np.eye(64), atol=1e-14)


def test_jacobi_matches_lapack(oracle):
    S = _rand_sym(80, 3)
    w, Z = oracle.jacobi_eig(S)
    np.testing.assert_allclose(w, np.linalg.eigvalsh(S), rtol=0, atol=1e-13 * np.abs(w).max())


def test_jacobi_laplacian_closed_form(oracle):
    rp, ci, v = W.laplacian_2d_csr(8, dtype=np.float64)
    n = 64
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    w, _ = oracle.jacobi_eig(A)
    np.testing.assert_allclose(w, W.laplacian_2d_eigenvalues(8), rtol=0, atol=1e-13)


def test_jacobi_degenerate(oracle):
    w, Z = oracle.jacobi_eig(np.diag([3.0, -1.0, 2.0]))
    np.testing.assert_array_equal(w, [-1.0, 2.0, 3.0])
    np.testing.assert_array_equal(np.abs(Z), np.eye(3)[:, [1, 2, 0]])
    w, Z = oracle.jacobi_eig(np.zeros((4, 4)))
    np.testing.assert_array_equal(w, 0.0)


# ----------------------------------------------------- Cholesky / MGS2 ----

def test_cholesky_matches_lapack(oracle):
    g = np.random.default_rng(1).standard_normal((30, 30))
    G = g @ g.T + 30 * np.eye(30)
    np.testing.assert_allclose(oracle.cholesky(G), np.linalg.cholesky(G), atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky(-np.eye(3))


def test_mgs2_qr(oracle):
    X = np.random.default_rng(2).standard_normal((300, 12))
    Q, R = oracle.mgs2(X)
    np.testing.assert_allclose(Q @ R, X, atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(12), atol=1e-14)
    # same factor as Householder QR up to column signs
    Qh, Rh = np.linalg.qr(X)
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(Rh)), rtol=1e-12)
    assert np.all(np.diag(R) > 0)


def test_mgs2_reorthogonalises_ill_conditioned(oracle):
    # columns of a Vandermonde-type matrix: kappa ~ 1e12; one MGS pass would
    # lose orthogonality to ~1e-4, the sqrt(2)/2 re-orthogonalisation keeps it
    t = np.linspace(0, 1, 400)
    X = np.stack([t ** j for j in range(10)], axis=1)
    Q, R = oracle.mgs2(X)
    assert np.abs(Q.T @ Q - np.eye(10)).max() < 1e-13
    np.testing.assert_allclose(Q @ R, X, atol=1e-13)


# ----------------------------------------------------------- Hessenberg ----

def _read_golden_hess():
    rows = [l.strip() for l in open(os.path.join(GOLDEN, "hessenberg_4x3.txt"))
            if l.strip() and not l.startswith("#")]
    i = rows.index("Q")
    Q = np.array([[float(x) for x in r.split()] for r in rows[i + 1:i + 5]])
    piv = np.array([int(x) for x in rows[rows.index("piv") + 1].split()])
    j = rows.index("U")
    U = np.array([[float(x) for x in r.split()] for r in rows[j + 1:j + 4]])
    return Q, piv, U


def test_hessenberg_hand_worked_example(oracle):
    Y = np.array([[1, 2, 1], [4, 2, 0], [2, 4, 1], [-2, 0, 3]], dtype=float)
    Qe, pe, Ue = _read_golden_hess()
    for prec in ("f64", "f32"):
        Q, piv, keep, U = oracle.hessenberg(Y, 1e-12, prec, want_u=True)
        np.testing.assert_array_equal(piv, pe)
        np.testing.assert_array_equal(keep, 1)
        tol = 1e-15 if prec == "f64" else 1e-7
        np.testing.assert_allclose(Q, Qe, atol=tol)
        np.testing.assert_allclose(U, Ue, atol=tol * 4)


def test_hessenberg_equals_row_pivoted_lu(oracle):
    # Sec. 4.2: the Hessenberg output is P^T L of PA = LU with row pivoting
    X = np.random.default_rng(5).random((500, 24))
    Q, piv, keep = oracle.hessenberg(X, 2.2e-16)
    P, L, U = sla.lu(X)
    np.testing.assert_allclose(Q, P @ L, atol=1e-13)
    # pivot rows are where the permutation puts rows 0..k-1
    perm = np.argmax(P, axis=0)
    np.testing.assert_array_equal(piv, perm[:24])


def test_hessenberg_structure(oracle):
    X = np.random.default_rng(6).standard_normal((300, 16))
    Q, piv, keep, U = oracle.hessenberg(X, 1e-12, want_u=True)
    assert keep.all()
    for j in range(16):
        assert Q[piv[j], j] == 1.0
        assert np.all(Q[piv[:j], j] == 0.0)
    assert np.abs(Q).max() <= 1.0
    np.testing.assert_allclose(Q @ U, X, atol=1e-13)
    assert np.allclose(np.tril(U, -1), 0)


def test_hessenberg_drops_dependent_columns(oracle):
    X = np.random.default_rng(8).standard_normal((200, 5))
    X[:, 2] = X[:, 0] - 2 * X[:, 1]
    X[:, 4] = 0.0
    Xs = X / np.abs(X).max(axis=0, initial=0, where=np.ones_like(X, bool)).clip(1e-300)
    Q, piv, keep = oracle.hessenberg(Xs, 2.2e-16 * 64)
    np.testing.assert_array_equal(keep, [1, 1, 0, 1, 0])
    np.testing.assert_array_equal(piv[[2, 4]], -1)
    Qk = Q[:, keep == 1]
    assert oracle.subspace_sin(Qk, X[:, [0, 1, 3]]) < 1e-12


def test_hessenberg_tie_takes_first_index(oracle):
    Y = np.array([[1.0, 0.3], [-2.0, 1.0], [2.0, 5.0]])
    _, piv, _ = oracle.hessenberg(Y, 1e-12)
    assert piv[0] == 1


def test_hessenberg_f32_agrees_with_f64(oracle):
    X = np.random.default_rng(9).random((2000, 32)).astype(np.float32)
    Q64, p64, _ = oracle.hessenberg(X.astype(np.float64), 1e-7)
    Q32, p32, _ = oracle.hessenberg(X, 1e-7, "f32")
    np.testing.assert_array_equal(p32, p64)
    np.testing.assert_allclose(Q32, Q64, atol=2e-4)


# --------------------------------------------------------------- pencils ---

def test_sym_pencil_matches_lapack_and_basis_invariance(oracle):
    rng = np.random.default_rng(11)
    A = _rand_sym(120, 12)
    Qo, _ = np.linalg.qr(rng.standard_normal((120, 10)))
    R = np.triu(rng.standard_normal((10, 10))) + 5 * np.eye(10)
    V = Qo @ R  # non-orthogonal basis of the same subspace
    H, G = V.T @ A @ V, V.T @ V
    theta, Y = oracle.sym_pencil_eig(H, G)
    np.testing.assert_allclose(theta, sla.eigh(H, G, eigvals_only=True), rtol=1e-11, atol=1e-12)
    # Galerkin condition depends only on the subspace (eq. (geig))
    np.testing.assert_allclose(theta, np.linalg.eigvalsh(Qo.T @ A @ Qo), atol=1e-11)
    np.testing.assert_allclose(Y.T @ G @ Y, np.eye(10), atol=1e-11)
    np.testing.assert_allclose(H @ Y, G @ Y * theta, atol=1e-10)


def test_svd_pencil_theorem(oracle):
    rng = np.random.default_rng(13)
    A = rng.standard_normal((90, 40))
    Uo, _ = np.linalg.qr(rng.standard_normal((90, 8)))
    Vo, _ = np.linalg.qr(rng.standard_normal((40, 6)))
    U = Uo @ (np.triu(rng.standard_normal((8, 8))) + 3 * np.eye(8))
    V = Vo @ (np.triu(rng.standard_normal((6, 6))) + 3 * np.eye(6))
    B, MU, MV = U.T @ A @ V, U.T @ U, V.T @ V
    s, Y, Z = oracle.svd_pencil(B, MU, MV)
    # k1 + k2 = 14 eigenvalues: 6 positive, 6 negative (pairs), 2 zero
    K = np.block([[np.zeros((8, 8)), B], [B.T, np.zeros((6, 6))]])
    M = sla.block_diag(MU, MV)
    ev = sla.eigh(K, M, eigvals_only=True)
    np.testing.assert_allclose(np.sort(ev[ev > 1e-9])[::-1], s, rtol=1e-11)
    np.testing.assert_allclose(np.sort(-ev[ev < -1e-9])[::-1], s, rtol=1e-11)
    assert np.sum(np.abs(ev) <= 1e-9) == 2
    # Theorem: sqrt(2) U Y and sqrt(2) V Z are orthonormal
    Ut, Vt = np.sqrt(2) * U @ Y, np.sqrt(2) * V @ Z
    np.testing.assert_allclose(Ut.T @ Ut, np.eye(6), atol=1e-11)
    np.testing.assert_allclose(Vt.T @ Vt, np.eye(6), atol=1e-11)
    # equals the classical two-sided projection on orthonormal bases
    np.testing.assert_allclose(s, np.linalg.svd(Uo.T @ A @ Vo, compute_uv=False), rtol=1e-11)


# ------------------------------------------------------------- filters -----

def _cheb_T(d, x):
    x = np.asarray(x, dtype=float)
    return np.where(np.abs(x) <= 1, np.cos(d * np.arccos(np.clip(x, -1, 1))),
                    np.sign(x) ** d * np.cosh(d * np.arccosh(np.abs(x))))


def _cheb_plain(A, X, d, lo, hi):
    c, e = (lo + hi) / 2, (hi - lo) / 2
    Y0 = X
    Y1 = (A @ Y0 - c * Y0) / e
    for _ in range(2, d + 1):
        Y0, Y1 = Y1, 2 * (A @ Y1 - c * Y1) / e - Y0
    return Y1


def test_chebyshev_scales_eigenvectors_by_T_d(oracle):
    lam = np.linspace(-1, 3, 40)
    A = _prescribed(lam, 21)
    w, Z = np.linalg.eigh(A)
    lo, hi = -1.0, 1.5
    for d in (1, 4, 7):
        Y = _cheb_plain(A, Z, d, lo, hi)
        gains = np.linalg.norm(Y, axis=0)
        x = (w - (lo + hi) / 2) / ((hi - lo) / 2)
        np.testing.assert_allclose(gains, np.abs(_cheb_T(d, x)), rtol=1e-10, atol=1e-12)


def test_stabilised_filter_spans_plain_recurrence(oracle):
    lam = 0.8 ** np.arange(60)
    A = _prescribed(lam, 22)
    X = W.uniform_start(60, 6, 3)
    for basis in ("mgs2", "hessenberg"):
        Q = oracle.filter_block(oracle.DenseOp(A), X, "chebyshev", 5, 0.0, 0.3, basis=basis)
        assert oracle.subspace_sin(Q, _cheb_plain(A, X, 5, 0.0, 0.3)) < 1e-10
        Q = oracle.filter_block(oracle.DenseOp(A), X, "power", 3, basis=basis)
        assert oracle.subspace_sin(Q, A @ A @ A @ X) < 1e-10


def test_csr_product_matches_dense(oracle):
    rp, ci, v = W.laplacian_2d_csr(12, dtype=np.float64)
    n = 144
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    assert np.array_equal(A, A.T) and np.all(np.diag(A) == 4)
    X = np.random.default_rng(4).standard_normal((n, 5))
    np.testing.assert_allclose(oracle.csr_matmul(rp, ci, v, X), A @ X, atol=1e-14)


# ---------------------------------------------------- subspace iteration ---

def test_subspace_eig_prescribed_spectrum_converged(oracle):
    n = 512
    lam = 0.95 ** np.arange(1, n + 1)
    A = _prescribed(lam, 1001)
    X0 = W.uniform_start(n, 16, 1101)
    r = oracle.subspace_eig(A, X0, 8, tol=1e-13, anorm=0.95, max_outer=2000)
    np.testing.assert_allclose(r.theta, lam[:8], rtol=1e-12)
    assert np.all(r.resid <= 1e-13)
    # eigenvectors match brute force up to sign
    w, Z = oracle.jacobi_eig(A)
    Zt = oracle.normalize_signs(Z[:, ::-1][:, :8])
    np.testing.assert_allclose(r.X, Zt, atol=1e-10)


def test_subspace_eig_basis_invariance_same_step(oracle):
    # the Hessenberg basis and the orthonormal basis span the same subspace,
    # so the Ritz values after the same number of steps agree
    n = 300
    lam = 0.9 ** np.arange(n)
    A = _prescribed(lam, 31)
    X0 = W.uniform_start(n, 10, 32)
    a = oracle.subspace_eig(A, X0, 5, outer=6)
    b = oracle.subspace_eig(A, X0, 5, outer=6, basis="hessenberg")
    np.testing.assert_allclose(a.theta_all, b.theta_all, rtol=1e-12)
    a = oracle.subspace_eig(A, X0, 5, filt="chebyshev", degree=3, lo=-0.1, hi=0.4, outer=4)
    b = oracle.subspace_eig(A, X0, 5, filt="chebyshev", degree=3, lo=-0.1, hi=0.4, outer=4,
                            basis="hessenberg")
    np.testing.assert_allclose(a.theta_all, b.theta_all, rtol=1e-12)


def test_subspace_eig_laplacian_smallest(oracle):
    N = 20
    rp, ci, v = W.laplacian_2d_csr(N, dtype=np.float64)
    ev = W.laplacian_2d_eigenvalues(N)
    X0 = W.uniform_start(N * N, 16, 5)
    r = oracle.subspace_eig((rp, ci, v), X0, 6, which="smallest", filt="chebyshev",
                            degree=10, lo=ev[16], hi=8.0, tol=1e-11, anorm=8.0, max_outer=5000)
    np.testing.assert_allclose(r.theta, ev[:6], rtol=1e-9)


def test_subspace_svd_prescribed(oracle):
    m, n = 600, 150
    sig = np.exp(-np.arange(1, n + 1) / 20.0)
    A = W.svd_prescribed(m, n, sig, 41, dtype=np.float64 and __import__("torch").float64).numpy()
    V0 = W.uniform_start(n, 12, 42)
    r = oracle.subspace_svd(A, V0, 6, tol=1e-12, max_outer=500)
    np.testing.assert_allclose(r.sigma, sig[:6], rtol=1e-11)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Vr, Ur = oracle.normalize_signs(Vt[:6].T, U[:, :6])
    np.testing.assert_allclose(r.V, Vr, atol=1e-8)
    np.testing.assert_allclose(r.U, Ur, atol=1e-8)


# ------------------------------------------------------------- rounding ----

def test_rounding_bit_patterns():
    from oracle import rounding as R
    for line in open(os.path.join(GOLDEN, "e4m3_bf16_bits.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        fmt, val, hexv = line.split()
        if fmt == "bf16":
            got = int(R.f32_to_bf16_bits(np.float32(val)).ravel()[0])
        else:
            got = int(R.f32_to_e4m3_bits(np.float32(val)).ravel()[0])
        assert got == int(hexv, 16), (fmt, val, hex(got), hexv)


def test_rounding_roundtrip_exhaustive_e4m3():
    from oracle import rounding as R
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = R.e4m3_bits_to_f32(codes)
    back = R.f32_to_e4m3_bits(vals)
    # +0 and -0 are distinct codes with the same value
    np.testing.assert_array_equal(back, codes)
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10
    bf = R.round_bf16(x)
    assert np.all(np.abs(bf - x) <= np.abs(x) * 2.0 ** -8)


def _golden_fp8():
    scales, codes = [], []
    for line in open(os.path.join(GOLDEN, "fp8_block_scale.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        kind, a, b = line.split()
        if kind == "scale":
            scales.append((float.fromhex(a), float.fromhex(b)))
        else:
            codes.append((float.fromhex(a), int(b, 16)))
    return scales, codes


def test_fp8_scale_rule_and_codes_hand_worked():
    from oracle import rounding as R
    scales, codes = _golden_fp8()
    for amax, want in scales:
        assert R.e4m3_block_scale(amax) == want, (amax.hex(), want)
    for v, want in codes:
        got = int(R.f32_to_e4m3_bits(np.float32(v)).ravel()[0])
        assert got == want, (v.hex(), hex(got), hex(want))


def test_fp8_block_quantize_hand_worked():
    """40 x 33 matrix = 2 x 2 blocks (one full, three ragged); expected scales
    and codes worked by hand from the format and the scale rule."""
    from oracle import rounding as R
    A = np.zeros((40, 33), dtype=np.float32)
    A[3, 5], A[7, 9], A[0, 0] = 3584.0, 8.0, -1.0     # block (0,0): amax 448*8 -> scale 8
    A[10, 32], A[11, 32] = 3585.0, 0.5                # block (0,1): 3585 > 3584 -> scale 16
    A[33, 32], A[34, 32] = 2.0 ** -130, -(2.0 ** -133)  # block (1,1): scale clamped at 2^-126
    codes, scales = R.fp8_block_quantize(A)           # block (1,0): all zero -> scale 1
    np.testing.assert_array_equal(scales, np.array([[8.0, 16.0], [1.0, 2.0 ** -126]], np.float32))
    want = np.zeros((40, 33), dtype=np.uint8)
    want[3, 5] = 0x7E    # 3584/8 = 448
    want[7, 9] = 0x38    # 8/8 = 1
    want[0, 0] = 0xA0    # -1/8 = -2^-3: exponent field 4, mantissa 0, sign
    want[10, 32] = 0x76  # 3585/16 = 224.0625 -> 224 = 1.75 * 2^7
    want[11, 32] = 0x10  # 0.5/16 = 2^-5: exponent field 2
    want[33, 32] = 0x18  # 2^-130 / 2^-126 = 2^-4: exponent field 3
    want[34, 32] = 0x84  # -2^-7 = -4 * 2^-9 (subnormal)
    np.testing.assert_array_equal(codes, want)


def test_fp8_colblock_quantize_hand_worked():
    """One scale per 32 rows of a column; dequantised values worked by hand."""
    from oracle import rounding as R
    V = np.zeros((70, 2), dtype=np.float32)
    V[40, 0], V[41, 0], V[42, 0], V[43, 0] = 3584.0, 8.0, 3.0, 100.0  # rows 32..63: scale 8
    V[64, 0], V[65, 0] = 1.0, 0.1                                      # rows 64..69: scale 2^-8
    V[0, 1], V[1, 1], V[2, 1], V[3, 1] = 449.0, 2.0 ** -8, 3 * 2.0 ** -10, 2.0 ** -11  # scale 2
    V[69, 1] = -7.0                                                    # 7 * 2^6 = 448: scale 2^-6
    got = R.fp8_colblock_quantize(V)
    want = np.zeros((70, 2))
    want[40, 0], want[41, 0], want[42, 0] = 3584.0, 8.0, 3.0
    want[43, 0] = 96.0          # 100/8 = 12.5: tie between 12 and 13 -> even mantissa -> 12
    want[64, 0] = 1.0
    want[65, 0] = 26.0 / 256.0  # 0.1 * 256 = 25.6 -> 26 (1.625 * 2^4)
    want[0, 1] = 448.0          # 449/2 = 224.5 -> 224
    want[1, 1] = 2.0 ** -8      # 2^-9 exactly (smallest subnormal)
    want[2, 1] = 2.0 ** -8      # 0.75 * 2^-9 -> 2^-9
    want[3, 1] = 0.0            # 0.125 * 2^-9 -> 0
    want[69, 1] = -7.0
    np.testing.assert_array_equal(got, want)


def test_normalize_signs_hand_worked(oracle):
    """Unit 2-norm, largest-magnitude entry positive, first index on ties;
    the partner block (U of an SVD pair) flips with its column."""
    X = np.array([[0.0, 1.0, 0.0, 0.1],
                  [-3.0, 2.0, 0.0, -0.9],
                  [3.0, -2.0, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0]])
    P = np.array([[2.0, 0.0, 0.0, 0.0],
                  [0.0, 0.0, 3.0, 1.0],
                  [0.0, 5.0, 4.0, 0.0]])
    Xn, Pn = oracle.normalize_signs(X, P)
    r2 = 1.0 / math.sqrt(2.0)
    n4 = math.sqrt(0.82)
    np.testing.assert_allclose(Xn, [[0.0, 1 / 3, 0.0, -0.1 / n4],
                                    [r2, 2 / 3, 0.0, 0.9 / n4],
                                    [-r2, -2 / 3, 0.0, 0.0],
                                    [0.0, 0.0, 0.0, 0.0]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Pn, [[-1.0, 0.0, 0.0, 0.0],
                                    [0.0, 0.0, 0.6, -1.0],
                                    [0.0, 1.0, 0.8, 0.0]], rtol=0, atol=1e-15)


def test_eig_residual_normalisation_hand_worked(oracle):
    """||A x - theta x|| / ||x|| / anorm on a 3 x 3 matrix (||A||_2 = 5) for
    non-eigenvectors, a non-unit vector and an exact eigenvector."""
    A = np.array([[2.0, 1.0, 0.0], [1.0, 2.0, 0.0], [0.0, 0.0, 5.0]])
    X = np.array([[1.0, 2.0, 1.0, 1.0],
                  [0.0, 0.0, 2.0, 1.0],
                  [0.0, 0.0, 2.0, 0.0]])
    theta = np.array([2.0, 2.0, 1.0, 3.0])
    # r = (0,1,0) ; (0,2,0)/2 ; (3,3,8)/3 ; 0
    want = np.array([0.2, 0.2, math.sqrt(82.0) / 15.0, 0.0])
    np.testing.assert_allclose(oracle.eig_residuals(A @ X, X, theta, 5.0), want, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(oracle.true_residuals(A, theta, X, 5.0), want, rtol=1e-15, atol=1e-16)


def test_svd_residual_normalisation_hand_worked(oracle):
    """sqrt(||A v - s u||^2 + ||A^T u - s v||^2) / anorm on a 3 x 2 matrix
    with ||A||_2 = 2, for an exact triplet and two inexact ones."""
    A = np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0]])
    U = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    V = np.array([[0.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    s = np.array([2.0, 1.0, 0.5])
    # (1): exact.  (2): A v - u = (-1,2,0), A^T u - v = (1,-1).
    # (3): A v - u/2 = (1,0,-1/2), A^T u - v/2 = (-1/2,0).
    want = np.array([0.0, math.sqrt(7.0) / 2.0, math.sqrt(1.5) / 2.0])
    np.testing.assert_allclose(oracle.svd_residuals(A, s, U, V, 2.0), want, rtol=1e-15, atol=1e-16)


# ------------------------------------------------- binary16 storage ----

def test_round_binary16_matches_numpy_float16(oracle):
    """The oracle's binary16 rounding against numpy's float16 conversion
    (IEEE round to nearest even): normals, subnormals, ties, overflow."""
    rng = np.random.default_rng(3)
    x = np.concatenate([
        (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 12, 200000))).astype(np.float32),
        np.array([65504.0, 65519.0, 65520.0, 70000.0, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -25,
                  2.0 ** -14, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, -0.0, 0.0], dtype=np.float32)])
    got = oracle.round_binary16(x)
    want = x.astype(np.float16).astype(np.float32)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


def test_hessenberg_f16s_exact_inputs_equal_f64(oracle):
    """Y = L U with dyadic L (|entries| <= 1/2 below the unit diagonal) and
    power-of-two pivots U_jj: every intermediate value is a short dyadic
    number, exact in binary16, so the FP16-storage process rounds nothing,
    recovers L (rows already in pivot order) and equals the FP64 one."""
    L = np.array([[1.0, 0.0, 0.0],
                  [0.5, 1.0, 0.0],
                  [0.25, -0.5, 1.0],
                  [-0.5, 0.25, 0.5]])
    U = np.array([[4.0, 2.0, 1.0],
                  [0.0, 2.0, -1.0],
                  [0.0, 0.0, 8.0]])
    Y = L @ U
    Q64, p64, k64 = oracle.hessenberg(Y, 1e-12, "f64")
    Q16, p16, k16 = oracle.hessenberg(Y, 1e-12, "f16s")
    np.testing.assert_array_equal(p64, [0, 1, 2])
    np.testing.assert_array_equal(Q64, L)
    np.testing.assert_array_equal(p16, p64)
    np.testing.assert_array_equal(k16, k64)
    np.testing.assert_array_equal(Q16.astype(np.float64), L)


def test_hessenberg_f16s_is_rounded_f32_process(oracle):
    """Every stored value of the FP16-storage process is a binary16 value,
    the pivots are the row-pivoted LU pivots of the rounded input, and the
    result stays within binary16 rounding of the FP64 process."""
    rng = np.random.default_rng(5)
    Y = rng.uniform(0.0, 1.0, (300, 12))
    Q16, p16, k16 = oracle.hessenberg(Y, 2.0 ** -10, "f16s")
    assert k16.all()
    np.testing.assert_array_equal(Q16, Q16.astype(np.float16).astype(np.float32))
    Yr = Y.astype(np.float16).astype(np.float64)
    Q64, p64, _ = oracle.hessenberg(Yr, 1e-12, "f64")
    np.testing.assert_array_equal(p16[:4], p64[:4])  # early pivots agree (later ones may swap on ties)
    assert np.max(np.abs(Q16[:, :4] - Q64[:, :4])) < 2e-2


# ---------------------------------------------------------------------------
# Gram-Schmidt comparators (Sec. 4.2 comparison table; Sec. 5.3, Table 3)
# ---------------------------------------------------------------------------

_GS = {
    "mgs_left": lambda A: O.gs_mgs_left(A),
    "mgs_right": lambda A: O.gs_mgs_right(A),
    "cgs": lambda A: O.gs_cgs(A),
    "cgs2": lambda A: O.gs_cgs(A, reorth=True),
}


@pytest.mark.parametrize("name", sorted(_GS))
def test_gs_hand_worked_3x2(name):
    # a1 = (3, 4, 0): r11 = 5, q1 = (0.6, 0.8, 0); a2 = (1, 2, 2):
    # r12 = q1.a2 = 2.2, v = a2 - 2.2 q1 = (-0.32, 0.24, 2), r22 = sqrt(4.16)
    A = np.array([[3.0, 1.0], [4.0, 2.0], [0.0, 2.0]])
    Q, R = _GS[name](A)
    r22 = np.sqrt(4.16)
    np.testing.assert_allclose(R, [[5.0, 2.2], [0.0, r22]], rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(Q[:, 0], [0.6, 0.8, 0.0], atol=1e-16)
    np.testing.assert_allclose(Q[:, 1], np.array([-0.32, 0.24, 2.0]) / r22, atol=1e-15)


@pytest.mark.parametrize("name", sorted(_GS))
def test_gs_matches_householder_qr(name):
    A = np.random.default_rng(11).random((300, 40))
    Qh, Rh = np.linalg.qr(A)
    s = np.sign(np.diag(Rh))
    Qh, Rh = Qh * s, Rh * s[:, None]
    Q, R = _GS[name](A)
    np.testing.assert_allclose(Q, Qh, atol=1e-12)
    np.testing.assert_allclose(R, Rh, atol=1e-11)


def test_gs_loss_of_orthogonality_ordering():
    # kappa = 1e6: CGS loses orthogonality like kappa^2 u, MGS like kappa u,
    # CGS with one re-orthogonalisation stays at u; every variant is
    # backward stable (A = Q R to working precision)
    rng = np.random.default_rng(12)
    U, _ = np.linalg.qr(rng.standard_normal((100, 20)))
    V, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    A = (U * np.logspace(0, -6, 20)) @ V.T
    loss = {}
    for name, f in _GS.items():
        Q, R = f(A)
        loss[name] = np.linalg.norm(Q.T @ Q - np.eye(20), 2)
        assert np.linalg.norm(A - Q @ R) <= 1e-14 * np.linalg.norm(A)
    assert loss["cgs2"] <= 1e-13
    assert 1e-14 <= loss["mgs_left"] <= 1e-8 and loss["mgs_right"] <= 1e-8
    assert loss["cgs"] >= 1e-6


def test_mgs_left_and_right_are_bitwise_equal():
    A = np.random.default_rng(13).random((500, 30))
    Ql, Rl = O.gs_mgs_left(A)
    Qr, Rr = O.gs_mgs_right(A)
    np.testing.assert_array_equal(Ql, Qr)
    np.testing.assert_array_equal(Rl, Rr)


# ---------------------------------------------------------------------------
# Krylov-Hessenberg process and the restarted Krylov reference (Sec. 4.1,
# Alg. "Computing non-orthogonal bases from the Krylov-Hessenberg Process";
# Sec. 5.2 sparse experiments)
# ---------------------------------------------------------------------------

def test_krylov_hessenberg_hand_worked_3x3():
    # v = e1: v1 = e1 (pivot 0); A e1 = (2, 1, 0) loses 2 e1 -> e2 (pivot 1,
    # scale 1); A e2 = (1, 3, 1) loses 1 e1 and 3 e2 -> e3 (pivot 2)
    A = np.array([[2.0, 1.0, 0.0], [1.0, 3.0, 1.0], [0.0, 1.0, 4.0]])
    V, piv, H = O.krylov_hessenberg(A, np.array([1.0, 0.0, 0.0]), 3)
    np.testing.assert_array_equal(V, np.eye(3))
    np.testing.assert_array_equal(piv, [0, 1, 2])
    np.testing.assert_array_equal(H, [[2.0, 1.0], [1.0, 3.0], [0.0, 1.0]])


def test_krylov_hessenberg_relation_and_structure():
    rng = np.random.default_rng(21)
    A = _rand_sym(60, 22)
    v = rng.random(60)
    k = 15
    V, piv, H = O.krylov_hessenberg(A, v, k)
    assert V.shape == (60, k) and len(set(piv.tolist())) == k
    # A V_{k-1} = V H (the Krylov relation of the process), H upper Hessenberg
    np.testing.assert_allclose(A @ V[:, :k - 1], V @ H, atol=1e-12 * np.abs(A).max() * 60)
    assert np.all(np.tril(H, -2) == 0.0)
    # unit pivots, exact zeros at earlier pivot rows, |entries| <= 1
    for i in range(k):
        assert V[piv[i], i] == 1.0
        for l in range(i):
            assert V[piv[l], i] == 0.0
    assert np.abs(V).max() <= 1.0
    # the same subspace as the orthonormal Krylov basis
    Q = np.linalg.qr(np.column_stack([np.linalg.matrix_power(A, p) @ v for p in range(6)]))[0]
    Vq = np.linalg.qr(V[:, :6])[0]
    assert O.subspace_sin(Q, Vq) <= 1e-8


def test_krylov_eig_full_space_is_exact():
    # k = n: the Krylov space of a generic start vector is the whole space,
    # so the Ritz values are the eigenvalues (brute force)
    A = _rand_sym(12, 23)
    v = np.random.default_rng(24).random(12)
    r = O.krylov_eig(A, v, 12, 5)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    np.testing.assert_allclose(r.theta, lam[:5], rtol=1e-12, atol=1e-12)
    assert np.all(r.resid <= 1e-12)


def test_krylov_eig_restarts_converge_on_prescribed_spectrum():
    lam = np.concatenate([[10.0, 9.0, 8.0], np.linspace(1.0, 0.0, 397)])
    A = _prescribed(lam, 25)
    v = np.random.default_rng(26).random(400)
    r0 = O.krylov_eig(A, v, 20, 3, restarts=0)
    r4 = O.krylov_eig(A, v, 20, 3, restarts=4)
    assert r4.resid[0] < r0.resid[0]
    np.testing.assert_allclose(r4.theta[0], 10.0, rtol=1e-12)
    assert r4.resid[0] <= 1e-10


def test_krylov_stops_at_an_invariant_subspace():
    # five distinct eigenvalues: K(A, v) has dimension 5 for a generic v
    lam = np.repeat([5.0, 4.0, 3.0, 2.0, 1.0], 10)
    A = _prescribed(lam, 27)
    v = np.random.default_rng(28).random(50)
    V, piv, H = O.krylov_hessenberg(A, v, 12)
    assert V.shape[1] == 5
    r = O.krylov_eig(A, v, 12, 5)
    np.testing.assert_allclose(r.theta, [5.0, 4.0, 3.0, 2.0, 1.0], rtol=1e-13)


def test_svd_normal_equations_matches_lapack():
    # the A^T A form: s = sqrt(theta) of the Ritz values of A^T A, u = A v / s
    rng = np.random.default_rng(29)
    m, n, k = 120, 40, 5
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = 2.0 ** (-np.arange(n) / 3.0)
    A = (U * sig) @ V.T
    V0 = rng.random((n, 10))
    r = O.subspace_svd_normal(A, V0, k, tol=1e-14, max_outer=500)
    s_ref = np.linalg.svd(A, compute_uv=False)[:k]
    np.testing.assert_allclose(r.sigma, s_ref, rtol=1e-11)
    assert np.all(r.resid <= 1e-10)
    # u_i = A v_i / s_i are unit and orthogonal
    np.testing.assert_allclose(r.U.T @ r.U, np.eye(k), atol=1e-10)
