"""CPU oracle for the orthogonalization-free Rayleigh-Ritz (OFRR) path.

TEST INFRASTRUCTURE ONLY: this package is the independent checker of the
HIP library.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product never does, and it imports
nothing from the product.  It shares no code, header or constant with the
HIP path; the only thing both sides use is the seeded input generators in
`workloads/`, which hold none of the method's arithmetic.

Everything is FP64 (inputs stored in FP32 are promoted exactly), except the
FP32 variant of the Hessenberg process that takes pivot decisions in the
precision the GPU kernel uses.  Paper references are to Xu, Zhang, Chen,
Saad and Xi, arXiv 2505.00281.

What the oracle computes
------------------------
* Ritz pairs of a symmetric A on a subspace are fixed by the Galerkin
  condition alone (Sec. 3.1, eq. (geig)): any basis of the same subspace
  gives a congruent pencil and the same Ritz pairs.  So the oracle for
  "OFRR on a Hessenberg basis" is the plain route: an orthonormal basis
  (MGS with re-orthogonalisation) and classical Rayleigh-Ritz (Alg.
  "Rayleigh-Ritz Projection with Orthogonal Bases").  `subspace_eig` runs
  multi-step subspace iteration (Alg. "Multiple Step Subspace Iteration")
  with restart from all Ritz vectors (Sec. 2), power or Chebyshev filter.
* For the SVD: alternating subspaces U_s = span(A V_{s-1}),
  V_s = span(A^T U_s) and the classical two-sided projection (Alg.
  "Rayleigh-Ritz Projection for SVD"), `subspace_svd`.
* For a real non-symmetric A the Ritz values are complex (Sec. 3.1):
  `subspace_eig_general` runs the same iteration with the library's
  non-symmetric eigensolver on Q^T A Q, or, on a Hessenberg basis, on the
  Cholesky-reduced pencil (V^T A V, V^T V), restarting from a real basis
  of all Ritz vectors.
* The pieces the GPU path computes step by step also have their own
  reference here: the Hessenberg process (Sec. 4.2), the symmetric
  definite pencil (eq. (geig), Alg. "Orthogonalization-Free Rayleigh-Ritz
  Projection") and the augmented SVD pencil with the sqrt(2) lift
  (Sec. 3.2, eq. (gev for svd matrix), Theorem, Alg. "Orthogonalization-Free
  Rayleigh-Ritz Projection for SVD").

Readings of the paper taken here (each also listed in the design notes):
* Hessenberg drop test reads |pivot| >= tol (the printed test names q_k);
  a dropped column keeps pivot -1 and eliminates nothing.
* Ties in the pivot search go to the first (smallest) row index.
* Chebyshev filter (named, not defined, in the paper): three-term
  recurrence on [lo, hi], c = (lo+hi)/2, e = (hi-lo)/2,
  Y1 = (A - cI) Y0 / e, Y_{d+1} = 2 (A - cI) Y_d / e - Y_{d-1}.
* Residual of a Ritz pair: ||A x - theta x||_2 / anorm with unit ||x||_2;
  for the SVD sqrt(||A v - s u||^2 + ||A^T u - s v||^2) / anorm.
* Sign of a returned vector: unit 2-norm and its entry of largest
  magnitude (first index on ties) positive; for the SVD the sign is fixed
  on v and u flips with it.
* Non-symmetric A: wanted values are those of largest modulus, ties
  broken by larger real part, then larger imaginary part; a complex Ritz
  vector is scaled to unit 2-norm with its largest-modulus entry (first on
  ties) real and positive; a conjugate pair restarts as its real and
  imaginary parts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_core.c")
_LIB_PATH = os.path.join(_HERE, "liborc_core.so")
_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile oracle_core.c with gcc (FP contraction off so every rounding
    is the one written in the source; fma() is called explicitly)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_jacobi_eig.restype = ctypes.c_int
    lib.orc_jacobi_eig.argtypes = [_i64, _f64p, _i64, _f64p, _f64p, _i64, ctypes.c_int]
    lib.orc_cholesky.restype = ctypes.c_int
    lib.orc_cholesky.argtypes = [_i64, _f64p, _i64]
    lib.orc_mgs2.restype = _i64
    lib.orc_mgs2.argtypes = [_i64, _i64, _f64p, _i64, _f64p, _i64]
    lib.orc_hessenberg_f64.restype = _i64
    lib.orc_hessenberg_f64.argtypes = [_i64, _i64, _f64p, _i64, ctypes.c_double,
                                       _i32p, _i32p, _f64p, _i64]
    lib.orc_hessenberg_f32.restype = _i64
    lib.orc_hessenberg_f32.argtypes = [_i64, _i64, _f32p, _i64, ctypes.c_float,
                                       _i32p, _i32p, _f32p, _i64]
    lib.orc_hessenberg_f16s.restype = _i64
    lib.orc_hessenberg_f16s.argtypes = [_i64, _i64, _f32p, _i64, ctypes.c_float,
                                        _i32p, _i32p, _f32p, _i64]
    lib.orc_round_binary16.restype = ctypes.c_float
    lib.orc_round_binary16.argtypes = [ctypes.c_float]
    lib.orc_round_binary16_array.restype = None
    lib.orc_round_binary16_array.argtypes = [_i64, _f32p]
    lib.orc_csr_mm.restype = None
    lib.orc_csr_mm.argtypes = [_i64, _i32p, _i32p, _f64p, _i64, _f64p, _i64, _f64p, _i64]
    _lib = lib
    return lib


def _p64(a):
    return a.ctypes.data_as(_f64p)


def _p32(a):
    return a.ctypes.data_as(_f32p)


def _pi32(a):
    return a.ctypes.data_as(_i32p)


# ---------------------------------------------------------------------------
# Small dense building blocks
# ---------------------------------------------------------------------------

def jacobi_eig(S, max_sweeps: int = 60):
    """Eigen-decomposition of a symmetric matrix by cyclic Jacobi rotations.
    Returns (w ascending, Z) with S Z = Z diag(w)."""
    S = np.array(S, dtype=np.float64, order="F", copy=True)
    n = S.shape[0]
    assert S.shape == (n, n)
    w = np.empty(n)
    Z = np.empty((n, n), order="F")
    if n == 0:
        return w, Z
    sweeps = _load().orc_jacobi_eig(n, _p64(S), n, _p64(w), _p64(Z), n, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    order = np.argsort(w, kind="stable")
    return w[order], np.asfortranarray(Z[:, order])


def cholesky(G):
    """Lower Cholesky factor L of a symmetric positive definite G."""
    L = np.array(G, dtype=np.float64, order="F", copy=True)
    n = L.shape[0]
    info = _load().orc_cholesky(n, _p64(L), n)
    if info != 0:
        raise np.linalg.LinAlgError(f"pivot {info} not positive")
    return L


def mgs2(X):
    """Modified Gram-Schmidt QR with sqrt(2)/2 re-orthogonalisation test
    (Sec. 5.1).  Returns (Q, R) with X = Q R."""
    Q = np.array(X, dtype=np.float64, order="F", copy=True)
    n, b = Q.shape
    R = np.zeros((b, b), order="F")
    done = _load().orc_mgs2(n, b, _p64(Q), n, _p64(R), b)
    if done != b:
        raise np.linalg.LinAlgError(f"column {done} is linearly dependent")
    return Q, R


def hessenberg(Y, tol: float, precision: str = "f64", want_u: bool = False):
    """Right-looking Hessenberg process (Sec. 4.2) in FP64, FP32 or with
    binary16 storage and FP32 arithmetic ("f16s").  Returns
    (Q, piv, keep[, U]) where Q holds every column after processing (use
    Q[:, keep == 1] for the basis), piv[j] the pivot row of column j (-1 if
    dropped) and U the multipliers (input = Q[:, keep] U[keep, :])."""
    lib = _load()
    if precision == "f64":
        Q = np.array(Y, dtype=np.float64, order="F", copy=True)
        n, k = Q.shape
        piv = np.empty(k, np.int32)
        keep = np.empty(k, np.int32)
        U = np.zeros((k, k), order="F") if want_u else None
        lib.orc_hessenberg_f64(n, k, _p64(Q), n, float(tol), _pi32(piv), _pi32(keep),
                               _p64(U) if want_u else None, k)
    elif precision in ("f32", "f16s"):
        # f16s: binary16 storage (the input is rounded to binary16 first),
        # FP32 arithmetic
        Q = np.array(Y, dtype=np.float32, order="F", copy=True)
        n, k = Q.shape
        if precision == "f16s":
            Q = np.asfortranarray(round_binary16(Q))
        piv = np.empty(k, np.int32)
        keep = np.empty(k, np.int32)
        U = np.zeros((k, k), dtype=np.float32, order="F") if want_u else None
        fn = lib.orc_hessenberg_f32 if precision == "f32" else lib.orc_hessenberg_f16s
        fn(n, k, _p32(Q), n, float(tol), _pi32(piv), _pi32(keep), _p32(U) if want_u else None, k)
    else:
        raise ValueError(precision)
    return (Q, piv, keep, U) if want_u else (Q, piv, keep)


# ---------------------------------------------------------------------------
# Basis-generation comparators (Sec. 4.2 comparison table; Sec. 5.3,
# Table 3): Gram-Schmidt without re-orthogonalisation in its left- and
# right-looking forms, classical Gram-Schmidt and CGS with one re-
# orthogonalisation.  Plain FP64 definitions, column by column; every
# inner product is the same library dot product, so the two MGS forms do
# identical arithmetic on every column (they differ only in when a
# column's projections are applied).  Each returns (Q, R) with A = Q R.
# ---------------------------------------------------------------------------

def _dot(x, y):
    return float(np.dot(x, y))


def gs_mgs_left(A):
    """Left-looking MGS: column j is projected against q_0 .. q_{j-1} one at
    a time, each coefficient taken from the partly projected column."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = A.shape
    Q = np.zeros_like(A)
    R = np.zeros((n, n))
    for j in range(n):
        v = A[:, j].copy()
        for i in range(j):
            R[i, j] = _dot(Q[:, i], v)
            v = v - R[i, j] * Q[:, i]
        R[j, j] = np.sqrt(_dot(v, v))
        Q[:, j] = v / R[j, j]
    return Q, R


def gs_mgs_right(A):
    """Right-looking MGS: once q_i is final, its projection is removed from
    every later column at once."""
    W = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = W.shape
    Q = np.zeros_like(W)
    R = np.zeros((n, n))
    for i in range(n):
        R[i, i] = np.sqrt(_dot(W[:, i], W[:, i]))
        Q[:, i] = W[:, i] / R[i, i]
        for j in range(i + 1, n):
            R[i, j] = _dot(Q[:, i], W[:, j])
            W[:, j] = W[:, j] - R[i, j] * Q[:, i]
    return Q, R


def gs_cgs(A, reorth: bool = False):
    """Classical Gram-Schmidt: all coefficients of column j from the
    original column (r = Q^T a_j, v = a_j - Q r); with `reorth` the
    projection is repeated once on v and the coefficients are added."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = A.shape
    Q = np.zeros_like(A)
    R = np.zeros((n, n))
    for j in range(n):
        a = A[:, j]
        Qj = Q[:, :j]
        r = Qj.T @ a
        v = a - Qj @ r
        if reorth:
            r2 = Qj.T @ v
            v = v - Qj @ r2
            r = r + r2
        R[:j, j] = r
        R[j, j] = np.sqrt(_dot(v, v))
        Q[:, j] = v / R[j, j]
    return Q, R


# ---------------------------------------------------------------------------
# Krylov methods for sparse A (Sec. 4.1, Alg. "Computing non-orthogonal
# bases from the Krylov-Hessenberg Process"; restart with the Ritz vector
# of the largest Ritz value, Sec. 5.2 sparse-matrix experiments)
# ---------------------------------------------------------------------------

def krylov_hessenberg(A, v, k: int, brk: float = 64 * 2.0 ** -52):
    """The Krylov-Hessenberg process in FP64, step by step as the algorithm
    states it: v is scaled by its entry of largest magnitude (first index
    on ties), then for j = 1..k-1 the product w = A v_j loses, for
    i = 1..j in order, its entry at pivot row pi_i times v_i, and is scaled
    by its new largest entry.  Returns (V (n x k_eff), pi, H) with
    A V[:, :k_eff-1] = V H (H (k_eff x k_eff-1) upper Hessenberg: H[i, j]
    the weight w(pi_i) removed at step j, H[j+1, j] the scaling pivot); the
    process stops early (k_eff < k) when what is left of A v_j after the
    removals is at the rounding level of the quantities it came from
    (max |w| <= brk (max |A v_j| + sum_i |H[i, j]|): an invariant subspace
    was reached; the algorithm as printed has no such test, w being exactly
    zero there in exact arithmetic)."""
    op = as_op(A)
    v = np.array(v, dtype=np.float64).ravel()
    n = v.size
    V = np.zeros((n, k))
    H = np.zeros((k, k - 1))
    piv = []
    r = int(np.argmax(np.abs(v)))
    V[:, 0] = v / v[r]
    piv.append(r)
    for j in range(k - 1):
        w = op.apply(V[:, j:j + 1])[:, 0]
        scale = float(np.abs(w).max())
        for i in range(j + 1):
            H[i, j] = w[piv[i]]
            w = w - H[i, j] * V[:, i]
        r = int(np.argmax(np.abs(w)))
        if not abs(w[r]) > brk * (scale + float(np.abs(H[:j + 1, j]).sum())):
            return V[:, :j + 1], np.array(piv, np.int32), H[:j + 1, :j]
        H[j + 1, j] = w[r]
        V[:, j + 1] = w / w[r]
        piv.append(r)
    return V, np.array(piv, np.int32), H


@dataclass
class KrylovResult:
    theta: np.ndarray
    X: np.ndarray
    resid: np.ndarray   # ||A x - theta x|| / |theta| (unit x)
    cycles: int


def krylov_eig(A, v0, k: int, nev: int, restarts: int = 0):
    """Restarted Krylov Rayleigh-Ritz reference for symmetric A: each cycle
    builds an orthonormal basis of K_k(A, v) by Lanczos with full
    orthogonalisation (MGS against every earlier vector, repeated once:
    Arnoldi with MGS, equivalent to Lanczos with full orthogonalisation
    for symmetric A), projects classically and restarts from the Ritz
    vector of the largest Ritz value; `restarts` further cycles after the
    first.  The Ritz pairs depend only on the Krylov subspace (Galerkin
    condition), so any basis of K_k(A, v) gives the same pairs.  Returns
    the nev largest Ritz pairs of the last cycle with the paper's Krylov
    residual ||A x - theta x|| / |theta|."""
    op = as_op(A)
    v = np.array(v0, dtype=np.float64).ravel()
    for cyc in range(restarts + 1):
        n = v.size
        Q = np.zeros((n, k))
        Q[:, 0] = v / np.linalg.norm(v)
        kk = k
        for j in range(1, k):
            w = op.apply(Q[:, j - 1:j])[:, 0]
            scale = np.linalg.norm(w)
            for _ in range(2):
                for i in range(j):
                    w = w - _dot(Q[:, i], w) * Q[:, i]
            nw = np.linalg.norm(w)
            if not nw > 64 * 2.0 ** -52 * scale:  # an invariant subspace: stop there
                kk = j
                break
            Q[:, j] = w / nw
        Q = Q[:, :kk]
        B = Q.T @ op.apply(Q)
        theta, Z = jacobi_eig(0.5 * (B + B.T))
        order = np.argsort(-theta, kind="stable")
        theta, Z = theta[order], Z[:, order]
        X = Q @ Z
        v = X[:, 0]
    AX = op.apply(X[:, :nev])
    th = theta[:nev]
    res = np.linalg.norm(AX - X[:, :nev] * th, axis=0) / np.abs(th)
    Xs = normalize_signs(X[:, :nev])
    return KrylovResult(th.copy(), Xs, res, restarts + 1)


def round_binary16(x):
    """FP32 values rounded to the nearest IEEE binary16 value (ties to
    even), as FP32 (the C oracle's rounding, applied elementwise)."""
    a = np.array(x, dtype=np.float32, copy=True, order="C")
    _load().orc_round_binary16_array(a.size, _p32(a))
    return a


def csr_matmul(row_ptr, col_idx, values, X):
    """Y = A X for CSR A (0-based, sorted) and a dense block X."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    vals = np.ascontiguousarray(values, dtype=np.float64)
    X = np.asfortranarray(X, dtype=np.float64)
    n_rows = row_ptr.size - 1
    b = X.shape[1]
    Y = np.empty((n_rows, b), order="F")
    _load().orc_csr_mm(n_rows, _pi32(row_ptr), _pi32(col_idx), _p64(vals), b,
                       _p64(X), X.shape[0], _p64(Y), n_rows)
    return Y


def sym_pencil_eig(H, G):
    """Eigenpairs of the symmetric definite pencil H y = theta G y
    (eq. (geig)).  Reduction to standard form with the Cholesky factor
    G = L L^T: C = L^{-1} H L^{-T}, C z = theta z, y = L^{-T} z.
    Returns (theta ascending, Y) with Y^T G Y = I."""
    H = np.asarray(H, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    L = cholesky(0.5 * (G + G.T))
    T = sla.solve_triangular(L, 0.5 * (H + H.T), lower=True)
    C = sla.solve_triangular(L, T.T, lower=True)  # L^{-1} (L^{-1} H)^T = L^{-1} H L^{-T}
    C = 0.5 * (C + C.T)
    theta, Z = jacobi_eig(C)
    Y = sla.solve_triangular(L.T, Z, lower=False)
    return theta, Y


def svd_pencil(B, MU, MV):
    """The augmented pencil of the OFRR SVD (Sec. 3.2): eigenpairs of
    [0 B; B^T 0] [y; z] = s blkdiag(MU, MV) [y; z], keeping the positive
    eigenvalues.  Returns (sigma descending, Y, Z) with the normalisation
    [y; z]^T M [y; z] = 1, so that sqrt(2) U Y and sqrt(2) V Z are
    orthonormal (Theorem in Sec. 3.2)."""
    B = np.asarray(B, dtype=np.float64)
    k1, k2 = B.shape
    K = np.zeros((k1 + k2, k1 + k2))
    K[:k1, k1:] = B
    K[k1:, :k1] = B.T
    M = np.zeros_like(K)
    M[:k1, :k1] = MU
    M[k1:, k1:] = MV
    theta, W = sym_pencil_eig(K, M)
    pos = np.nonzero(theta > 0)[0][::-1]
    return theta[pos], W[:k1, pos], W[k1:, pos]


def normalize_signs(X, Xpartner=None):
    """Unit 2-norm columns, largest-magnitude entry (first on ties) positive.
    Xpartner (if given) is flipped together with X."""
    X = np.array(X, dtype=np.float64, copy=True)
    nrm = np.linalg.norm(X, axis=0)
    nrm[nrm == 0] = 1.0
    X /= nrm
    idx = np.argmax(np.abs(X), axis=0)
    sgn = np.sign(X[idx, np.arange(X.shape[1])])
    sgn[sgn == 0] = 1.0
    X *= sgn
    if Xpartner is not None:
        P = np.array(Xpartner, dtype=np.float64, copy=True)
        pn = np.linalg.norm(P, axis=0)
        pn[pn == 0] = 1.0
        return X, P / pn * sgn
    return X


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

class DenseOp:
    """op(X) = A X for a dense matrix held in FP64 (FP32 input promoted
    exactly).  The product is a library matmul."""

    def __init__(self, A):
        self.A = np.asarray(A, dtype=np.float64)
        self.n = self.A.shape[0]

    def apply(self, X):
        return self.A @ X

    def apply_t(self, X):
        return self.A.T @ X


class CsrOp:
    def __init__(self, row_ptr, col_idx, values, n_cols=None):
        self.row_ptr = np.asarray(row_ptr, dtype=np.int32)
        self.col_idx = np.asarray(col_idx, dtype=np.int32)
        self.values = np.asarray(values, dtype=np.float64)
        self.n = self.row_ptr.size - 1

    def apply(self, X):
        return csr_matmul(self.row_ptr, self.col_idx, self.values, X)


class NormalOp:
    """op(X) = A^T (A X) for a dense m x n A held in FP64: the operator of the
    normal-equations (A^T A) form of the SVD."""

    def __init__(self, A):
        self.A = np.asarray(A, dtype=np.float64)
        self.n = self.A.shape[1]

    def apply(self, X):
        return self.A.T @ (self.A @ X)


def as_op(A):
    if isinstance(A, (DenseOp, CsrOp, NormalOp)):
        return A
    if isinstance(A, tuple) and len(A) == 3:
        return CsrOp(*A)
    return DenseOp(A)


# ---------------------------------------------------------------------------
# Subspace iteration + Rayleigh-Ritz (eigenvalues)
# ---------------------------------------------------------------------------

@dataclass
class EigResult:
    theta: np.ndarray      # k Ritz values, sorted by `which`
    X: np.ndarray          # n x k Ritz vectors (unit norm, sign rule)
    resid: np.ndarray      # k relative residuals ||A x - theta x|| / anorm
    theta_all: np.ndarray  # all b Ritz values of the last projection
    X_all: np.ndarray      # all b Ritz vectors (the restart block)
    iters: int
    history: list


def chebyshev_center_halfwidth(lo: float, hi: float):
    return 0.5 * (hi + lo), 0.5 * (hi - lo)


def filter_block(op, X, filt: str, degree: int, lo=None, hi=None, basis: str = "mgs2",
                 tol=None):
    """Apply the degree-`degree` filter to the block X and return a basis
    of the filtered subspace.  The basis is re-stabilised after every
    product (MGS2, or the Hessenberg process when basis='hessenberg'); the
    previous block of the Chebyshev recurrence is carried through the same
    right transform so the recurrence stays consistent."""
    def stab(Y):
        if basis == "mgs2":
            Q, R = mgs2(Y)
            return Q, R, None
        Q, piv, keep, U = hessenberg(Y, 1e-300 if tol is None else tol, "f64", want_u=True)
        sel = keep == 1
        if not sel.all():
            raise np.linalg.LinAlgError("column dropped inside the filter")
        return Q, U, None

    if filt == "power":
        Y = X
        for _ in range(degree):
            Y, _, _ = stab(op.apply(Y))
        return Y
    if filt != "chebyshev":
        raise ValueError(filt)
    c, e = chebyshev_center_halfwidth(lo, hi)
    Y0 = X
    Y1 = (op.apply(Y0) - c * Y0) / e
    Y1, R, _ = stab(Y1)
    Y0 = sla.solve_triangular(R, Y0.T, trans="T", lower=False).T  # Y0 R^{-1}
    for _ in range(2, degree + 1):
        Y2 = 2.0 * (op.apply(Y1) - c * Y1) / e - Y0
        Y2, R, _ = stab(Y2)
        Y1 = sla.solve_triangular(R, Y1.T, trans="T", lower=False).T
        Y0, Y1 = Y1, Y2
    return Y1


def _order(theta, which):
    if which == "largest":
        return np.argsort(-theta, kind="stable")
    if which == "smallest":
        return np.argsort(theta, kind="stable")
    raise ValueError(which)


def rayleigh_ritz(op, Q, which):
    """Classical Rayleigh-Ritz on an orthonormal Q (Alg. "Rayleigh-Ritz
    Projection with Orthogonal Bases"): B = Q^T A Q, B Z = Z Theta,
    X = Q Z.  Returns (theta, X, AX) ordered by `which`."""
    AQ = op.apply(Q)
    B = Q.T @ AQ
    B = 0.5 * (B + B.T)
    theta, Z = jacobi_eig(B)
    o = _order(theta, which)
    theta, Z = theta[o], Z[:, o]
    return theta, Q @ Z, AQ @ Z


def eig_residuals(AX, X, theta, anorm):
    R = AX - X * theta[None, :]
    return np.linalg.norm(R, axis=0) / np.linalg.norm(X, axis=0) / anorm


def subspace_eig(A, X0, k: int, which: str = "largest", filt: str = "power",
                 degree: int = 1, lo=None, hi=None, outer: int = 20,
                 tol: float | None = None, anorm: float | None = None,
                 basis: str = "mgs2", max_outer: int = 100000, history: bool = False):
    """Multi-step subspace iteration with Rayleigh-Ritz and restart from all
    Ritz vectors (Sec. 2).  Same-step mode: `tol=None` runs exactly `outer`
    outer iterations.  Converged mode: `tol` given, iterate (up to
    max_outer) until the k wanted residuals are <= tol.  anorm (None ->
    max |Ritz value| of the last projection) normalises the residuals."""
    t_start = time.perf_counter()
    op = as_op(A)
    X = np.array(X0, dtype=np.float64, order="F", copy=True)
    hist = []
    it = 0
    limit = outer if tol is None else max_outer
    theta = Xr = AX = None
    while it < limit:
        Q = filter_block(op, X, filt, degree, lo, hi, basis=basis)
        if basis != "mgs2":
            Q, _ = mgs2(Q)  # only for the projection; same span
        theta, Xr, AX = rayleigh_ritz(op, Q, which)
        it += 1
        X = Xr
        an = anorm if anorm else float(np.max(np.abs(theta)))
        r = eig_residuals(AX[:, :k], Xr[:, :k], theta[:k], an)
        if history:
            # (outer iteration, wanted Ritz values, their residuals, seconds
            # since the call started): bookkeeping only
            hist.append((it, theta[:k].copy(), r.copy(), time.perf_counter() - t_start))
        if tol is not None and np.all(r <= tol):
            break
    an = anorm if anorm else float(np.max(np.abs(theta)))
    r = eig_residuals(AX[:, :k], Xr[:, :k], theta[:k], an)
    Xk = normalize_signs(Xr[:, :k])
    return EigResult(theta[:k].copy(), Xk, r, theta.copy(), Xr, it, hist)


def true_residuals(A, theta, X, anorm):
    """||A x_i - theta_i x_i||_2 / anorm in FP64 for unit-norm x_i."""
    op = as_op(A)
    AX = op.apply(np.asarray(X, dtype=np.float64))
    return eig_residuals(AX, np.asarray(X, dtype=np.float64), np.asarray(theta), anorm)


# ---------------------------------------------------------------------------
# Subspace iteration + Rayleigh-Ritz (singular values)
# ---------------------------------------------------------------------------

@dataclass
class SvdResult:
    sigma: np.ndarray
    U: np.ndarray
    V: np.ndarray
    resid: np.ndarray
    sigma_all: np.ndarray
    V_all: np.ndarray
    iters: int


def rayleigh_ritz_svd(A, U, V):
    """Classical two-sided projection (Alg. "Rayleigh-Ritz Projection for
    SVD") on orthonormal U, V: B = U^T A V = Z S W^T, U Z and V W.  The
    SVD of B is taken from the Jacobi eigen-decomposition of the symmetric
    augmented matrix [0 B; B^T 0], whose positive eigenvalues are the
    singular values and whose unit eigenvectors are [z; w] / sqrt(2)."""
    A = np.asarray(A, dtype=np.float64)
    B = U.T @ (A @ V)
    k1, k2 = B.shape
    K = np.zeros((k1 + k2, k1 + k2))
    K[:k1, k1:] = B
    K[k1:, :k1] = B.T
    w, E = jacobi_eig(K)
    pos = np.nonzero(w > 0)[0][::-1]
    s = w[pos]
    Zl = np.sqrt(2.0) * E[:k1, pos]
    Wr = np.sqrt(2.0) * E[k1:, pos]
    return s, U @ Zl, V @ Wr


def svd_residuals(A, s, U, V, anorm):
    A = np.asarray(A, dtype=np.float64)
    r1 = A @ V - U * s[None, :]
    r2 = A.T @ U - V * s[None, :]
    return np.sqrt(np.sum(r1 * r1, axis=0) + np.sum(r2 * r2, axis=0)) / anorm


def subspace_svd(A, V0, k: int, outer: int = 10, tol: float | None = None,
                 anorm: float | None = None, max_outer: int = 100000):
    """Alternating subspace iteration for the largest singular triplets:
    U_s = orth(A V_{s-1}), V_s = orth(A^T U_s), then the two-sided
    Rayleigh-Ritz projection; restart from all right Ritz vectors.
    Same-step mode if tol is None, converged mode otherwise."""
    A = np.asarray(A, dtype=np.float64)
    V = np.array(V0, dtype=np.float64, order="F", copy=True)
    it = 0
    limit = outer if tol is None else max_outer
    while it < limit:
        U, _ = mgs2(A @ V)
        V, _ = mgs2(A.T @ U)
        s, Ur, Vr = rayleigh_ritz_svd(A, U, V)
        it += 1
        V = Vr
        an = anorm if anorm else float(s[0])
        r = svd_residuals(A, s[:k], Ur[:, :k], Vr[:, :k], an)
        if tol is not None and np.all(r <= tol):
            break
    an = anorm if anorm else float(s[0])
    r = svd_residuals(A, s[:k], Ur[:, :k], Vr[:, :k], an)
    Vk, Uk = normalize_signs(Vr[:, :k], Ur[:, :k])
    return SvdResult(s[:k].copy(), Uk, Vk, r, s.copy(), Vr, it)


def subspace_svd_normal(A, V0, k: int, outer: int = 10, tol: float | None = None,
                        anorm: float | None = None, max_outer: int = 100000):
    """The normal-equations form of the SVD: subspace iteration with
    Rayleigh-Ritz on A^T A (power filter, restart from all Ritz vectors),
    singular values s = sqrt(theta), right vectors the Ritz vectors, left
    vectors u = A v / s; residuals as for the SVD.  Same-step mode when tol
    is None; converged mode iterates the eigenproblem to tol * (anorm^2)."""
    A = np.asarray(A, dtype=np.float64)
    op = NormalOp(A)
    an2 = anorm * anorm if anorm else None
    r = subspace_eig(op, V0, k, outer=outer, tol=tol, anorm=an2, max_outer=max_outer)
    s = np.sqrt(np.maximum(r.theta, 0.0))
    V = r.X
    U = (A @ V) / s
    an = anorm if anorm else float(s[0])
    res = svd_residuals(A, s, U, V, an)
    Vn, Un = normalize_signs(V, U)
    return SvdResult(s.copy(), Un, Vn, res, s.copy(), Vn, r.iters)


# ---------------------------------------------------------------------------
# General (non-symmetric) real A (Sec. 3.1: for A in R^{n x n} the Galerkin
# condition admits complex Ritz values; with a basis U that need not be
# orthonormal it becomes the pencil U^* A U y = lambda U^* U y, eq. (geig),
# Alg. "Orthogonalization-Free Rayleigh-Ritz Projection"; for a real U the
# conjugate transpose is the transpose).  The k values of largest modulus
# are wanted.
# ---------------------------------------------------------------------------

def general_order(theta):
    """Order of complex Ritz values: modulus descending, then real part
    descending, then imaginary part descending (of a conjugate pair the
    member with positive imaginary part comes first)."""
    th = np.asarray(theta)
    return np.lexsort((-th.imag, -th.real, -np.abs(th)))


def phase_normalize(x):
    """A complex vector scaled to unit 2-norm with its entry of largest
    modulus (the first on ties) real and positive."""
    x = np.asarray(x, dtype=np.complex128)
    i = int(np.argmax(np.abs(x)))
    nrm = np.linalg.norm(x)
    y = x * (np.conj(x[i]) / (abs(x[i]) * nrm))
    y[i] = abs(x[i]) / nrm  # exactly real
    return y


def general_real_basis(Z, theta):
    """Real columns spanning the space of the complex columns of Z (ordered
    as theta, the two members of a conjugate pair adjacent): a real value
    contributes Re z, a pair contributes Re z and Im z of its first member
    (the second member's column is the conjugate: it adds nothing)."""
    cols = []
    j = 0
    b = Z.shape[1]
    while j < b:
        if theta[j].imag != 0.0 and j + 1 < b and theta[j + 1] == np.conj(theta[j]):
            cols += [Z[:, j].real, Z[:, j].imag]
            j += 2
        else:
            cols.append(Z[:, j].real)
            j += 1
    return np.stack(cols, axis=1)


def general_pencil_eig(B, M):
    """Eigenpairs of the pencil B y = theta M y with B = U^T A U real and
    non-symmetric and M = U^T U symmetric positive definite (eq. (geig)).
    Reduction with the Cholesky factor M = L L^T: C = L^{-1} B L^{-T} (a
    real non-symmetric matrix with the pencil's eigenvalues), C z = theta z
    by the library's non-symmetric eigensolver, y = L^{-T} z.  Returns
    (theta ordered by general_order, Y) with y^H M y = 1, so that U y has
    unit 2-norm."""
    B = np.asarray(B, dtype=np.float64)
    L = cholesky(0.5 * (np.asarray(M, dtype=np.float64) + np.asarray(M, dtype=np.float64).T))
    T = sla.solve_triangular(L, B, lower=True)              # L^{-1} B
    C = sla.solve_triangular(L, T.T, lower=True).T           # (L^{-1} (L^{-1} B)^T)^T = L^{-1} B L^{-T}
    theta, Z = np.linalg.eig(C)
    o = general_order(theta)
    theta, Z = theta[o], Z[:, o]
    Z = Z / np.linalg.norm(Z, axis=0)[None, :]
    Y = sla.solve_triangular(L.T, Z, lower=False)
    return theta, Y


@dataclass
class GeneralResult:
    theta: np.ndarray      # complex, the k wanted Ritz values (general_order)
    X: np.ndarray          # complex n x k Ritz vectors (phase_normalize)
    resid: np.ndarray      # ||A x - theta x|| / (||x|| anorm)
    theta_all: np.ndarray  # all b Ritz values of the last projection
    iters: int


def subspace_eig_general(A, X0, k: int, degree: int = 1, outer: int = 20, tol: float | None = None,
                         anorm: float | None = None, basis: str = "mgs2", hess_tol: float = 1e-300,
                         max_outer: int = 100000):
    """Subspace iteration for a real non-symmetric A with restart from all
    Ritz vectors (Sec. 2), `degree` products per outer iteration.

    basis='mgs2': each product is followed by MGS2 and the projection is
    the classical B = Q^T A Q with the library's eigensolver.
    basis='hessenberg': each product is followed by the Hessenberg process
    (Sec. 4.2, every column kept) and the projection is the pencil
    (V^T A V, V^T V) of the orthogonalization-free form
    (general_pencil_eig).  In exact arithmetic both give the same Ritz
    pairs (Sec. 3.1: they depend on the subspace only).

    The restart block is the real basis (general_real_basis) of all Ritz
    vectors.  Same-step mode when tol is None; otherwise iterate until the
    k wanted residuals are <= tol.  anorm (None -> largest Ritz modulus)
    normalises the residuals."""
    op = as_op(A)
    X = np.array(X0, dtype=np.float64, order="F", copy=True)
    if basis not in ("mgs2", "hessenberg"):
        raise ValueError(basis)

    def stab(Y):
        if basis == "mgs2":
            return mgs2(Y)[0]
        Q, _, keep = hessenberg(Y, hess_tol, "f64")
        if not (keep == 1).all():
            raise np.linalg.LinAlgError("the Hessenberg process dropped a column")
        return Q

    it = 0
    limit = outer if tol is None else max_outer
    while it < limit:
        Q = X
        for _ in range(degree):
            Q = stab(op.apply(Q))
        AQ = op.apply(Q)
        if basis == "mgs2":
            theta, Z = np.linalg.eig(Q.T @ AQ)
            o = general_order(theta)
            theta, Z = theta[o], Z[:, o]
        else:
            theta, Z = general_pencil_eig(Q.T @ AQ, Q.T @ Q)
        Xc = Q @ Z
        AXc = AQ @ Z
        it += 1
        an = anorm if anorm else float(np.max(np.abs(theta)))
        r = np.linalg.norm(AXc[:, :k] - Xc[:, :k] * theta[None, :k], axis=0) / \
            np.linalg.norm(Xc[:, :k], axis=0) / an
        X = np.asfortranarray(general_real_basis(Xc, theta))
        if tol is not None and np.all(r <= tol):
            break
    Xk = np.stack([phase_normalize(Xc[:, j]) for j in range(k)], axis=1)
    return GeneralResult(theta[:k].copy(), Xk, r, theta.copy(), it)


# ---------------------------------------------------------------------------
# Subspace comparison helpers (several correct answers inside a cluster)
# ---------------------------------------------------------------------------

def subspace_sin(X, Y):
    """Sine of the largest principal angle between span(X) and span(Y)
    (dimension of Y <= dimension of X), computed as the 2-norm of the part
    of an orthonormal basis of span(Y) outside span(X)."""
    Qx, _ = np.linalg.qr(np.asarray(X, dtype=np.float64))
    Qy, _ = np.linalg.qr(np.asarray(Y, dtype=np.float64))
    P = Qy - Qx @ (Qx.T @ Qy)
    return float(np.linalg.norm(P, 2)) if P.size else 0.0
