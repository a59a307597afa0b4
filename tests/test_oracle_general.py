"""Pins of the oracle for a real non-symmetric A (Sec. 3.1: complex Ritz
values from the Galerkin condition; eq. (geig) and Alg. "Orthogonalization-
Free Rayleigh-Ritz Projection" on a non-orthogonal basis).

Each pin compares against something the oracle does not compute itself: a
closed form (the 2 x 2 rotation), a prescribed spectrum S D S^-1, the QZ
algorithm on the pencil (a different library route than the Cholesky
reduction the oracle takes), the Ritz values of span(A^p X0) from a
library QR, and the symmetric oracle on a positive definite matrix.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import ofrr_oracle as O


def _sorted_c(z):
    z = np.asarray(z)
    return z[O.general_order(z)]


def _assert_same_values(got, want, atol):
    """The two lists hold the same values within atol, matched one to one
    (the order of the members of a conjugate pair is decided by rounding
    when a routine does not return exact conjugates)."""
    want = list(np.asarray(want))
    for z in np.asarray(got):
        d = np.abs(np.asarray(want) - z)
        j = int(np.argmin(d))
        assert d[j] <= atol, (z, want)
        want.pop(j)


def test_order_rule():
    th = np.array([1.0 + 0j, -3.0 + 0j, 2 - 2j, 2 + 2j, 3.0 + 0j, -2 + 2j, 0.5j])
    got = th[O.general_order(th)]
    # |.|: 3, 3, 2.83 (x3), 1, 0.5; ties by larger real part, then by
    # larger imaginary part
    want = np.array([3.0, -3.0, 2 + 2j, 2 - 2j, -2 + 2j, 1.0, 0.5j])
    np.testing.assert_array_equal(got, want)


def test_phase_normalize():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    y = O.phase_normalize(x)
    assert abs(np.linalg.norm(y) - 1) < 1e-15
    i = int(np.argmax(np.abs(y)))
    assert y[i].imag == 0.0 and y[i].real > 0
    # the result depends on the line through x only
    np.testing.assert_allclose(O.phase_normalize(x * np.exp(0.7j) * 3.5), y, atol=1e-15)
    # ties go to the first index
    z = O.phase_normalize(np.array([1j, -1.0, 0.5]))
    assert z[0].imag == 0.0 and z[0].real > 0


@pytest.mark.parametrize("basis", ["mgs2", "hessenberg"])
def test_rotation_closed_form(basis):
    # A = [[0, 1], [-1, 0]]: eigenvalues +i and -i; A [1, i] = i [1, i]
    A = np.array([[0.0, 1.0], [-1.0, 0.0]])
    X0 = np.array([[0.9, 0.2], [0.3, 0.8]])
    r = O.subspace_eig_general(A, X0, 2, outer=1, basis=basis)
    np.testing.assert_allclose(r.theta, [1j, -1j], atol=1e-15)
    s = 1 / np.sqrt(2)
    # both entries have modulus 1/sqrt2 (a tie that rounding decides): the
    # vectors are [1, +-i] / sqrt2 up to a phase, with one entry real
    for j, want in ((0, [s, 1j * s]), (1, [s, -1j * s])):
        x = r.X[:, j]
        assert abs(abs(np.vdot(want, x)) - 1) < 1e-15
        np.testing.assert_allclose(np.abs(x), [s, s], atol=1e-15)
        i = int(np.argmax(np.abs(x)))
        assert x[i].imag == 0 and x[i].real > 0
    assert np.all(r.resid < 1e-15)


def _prescribed(n_real=44, seed=11, nonnormal=0.3):
    reals = [6.0, -5.0, 3.0] + list(np.linspace(1.0, 0.1, n_real))
    pairs = [(4.0, 2.5), (1.5, -1.2), (0.3, 0.2)]
    A = W.general_prescribed(reals, pairs, seed, nonnormal=nonnormal).numpy()
    lam = np.array(reals + [complex(a, b) for a, b in pairs] + [complex(a, -b) for a, b in pairs])
    return A, _sorted_c(lam)


@pytest.mark.parametrize("basis", ["mgs2", "hessenberg"])
def test_prescribed_spectrum_converges(basis):
    # the five eigenvalues of largest modulus (6, 4 +- 2.5i, -5 and 3 are
    # the leading ones; a conjugate pair straddles no boundary at k = 5)
    A, lam = _prescribed()
    n = A.shape[0]
    X0 = W.uniform_start(n, 10, 5)
    r = O.subspace_eig_general(A, X0, 5, degree=2, tol=1e-11, anorm=6.0, basis=basis)
    np.testing.assert_allclose(r.theta, lam[:5], rtol=0, atol=1e-9)
    # the returned vectors are eigenvectors: checked here in complex FP64
    for j in range(5):
        x = r.X[:, j]
        assert abs(np.linalg.norm(x) - 1) < 1e-13
        assert np.linalg.norm(A @ x - r.theta[j] * x) < 1e-9
    assert np.all(r.resid <= 1e-11)
    # the reported residuals are those of the returned pairs
    for j in range(5):
        x = r.X[:, j]
        np.testing.assert_allclose(r.resid[j], np.linalg.norm(A @ x - r.theta[j] * x) / 6.0,
                                   rtol=1e-3, atol=1e-15)


def test_pencil_matches_qz():
    # general_pencil_eig (Cholesky reduction + the non-symmetric solver)
    # against the QZ algorithm on the same pencil
    rng = np.random.default_rng(4)
    k = 12
    U = rng.standard_normal((40, k)) @ np.diag(np.logspace(0, -3, k))
    A = rng.standard_normal((40, 40))
    B = U.T @ A @ U
    M = U.T @ U
    th, Y = O.general_pencil_eig(B, M)
    qz = sla.eigvals(B, M)
    # (QZ returns no exact conjugates, so its pairs are matched, not sorted)
    _assert_same_values(th, qz, 1e-9 * np.abs(qz).max())
    # the oracle's pairs are exact conjugates, ordered + first
    for j in range(0, k - 1):
        if th[j].imag > 0:
            assert th[j + 1] == np.conj(th[j])
    for j in range(k):
        y = Y[:, j]
        np.testing.assert_allclose(np.vdot(y, M @ y).real, 1.0, rtol=1e-10)
        assert np.linalg.norm(B @ y - th[j] * (M @ y)) <= 1e-9 * np.linalg.norm(B) * np.linalg.norm(y)
        # unit Ritz vector
        assert abs(np.linalg.norm(U @ y) - 1) < 1e-10


@pytest.mark.parametrize("degree,outer", [(1, 3), (3, 1), (2, 2)])
def test_same_step_matches_krylov_power_subspace(degree, outer):
    # after `outer` iterations of `degree` products each the subspace is
    # span(A^(degree*outer) X0) (restart from all Ritz vectors keeps the
    # span); its Ritz values from a library QR of the block
    A, _ = _prescribed(n_real=20, seed=12)
    n = A.shape[0]
    X0 = W.uniform_start(n, 8, 6)
    Y = X0.copy()
    for _ in range(degree * outer):
        Y = A @ Y
    Q, _ = np.linalg.qr(Y)
    want = _sorted_c(np.linalg.eigvals(Q.T @ A @ Q))
    for basis in ("mgs2", "hessenberg"):
        r = O.subspace_eig_general(A, X0, 8, degree=degree, outer=outer, basis=basis)
        np.testing.assert_allclose(r.theta_all, want, rtol=0, atol=1e-10 * abs(want[0]))


def test_symmetric_matrix_reduces_to_symmetric_oracle():
    # a symmetric positive definite A: real Ritz values and the same pairs
    # as the symmetric oracle (largest = largest modulus here)
    lam = np.concatenate([np.linspace(10, 5, 6), np.linspace(1, 0.1, 54)])
    A = W.dense_symmetric_prescribed(lam, 21).numpy()
    X0 = W.uniform_start(60, 10, 7)
    g = O.subspace_eig_general(A, X0, 4, outer=6)
    s = O.subspace_eig(A, X0, 4, outer=6)
    assert np.all(g.theta.imag == 0) or np.abs(g.theta.imag).max() < 1e-14
    np.testing.assert_allclose(g.theta.real, s.theta, rtol=1e-12)
    np.testing.assert_allclose(g.X.real, s.X, atol=1e-9)


@pytest.mark.parametrize("basis", ["mgs2", "hessenberg"])
def test_full_space_is_exact(basis):
    # k = b = n: the subspace is the whole space after one iteration
    A, lam = _prescribed(n_real=5, seed=13)
    n = A.shape[0]
    r = O.subspace_eig_general(A, W.uniform_start(n, n, 8), n, outer=1, basis=basis)
    np.testing.assert_allclose(r.theta, lam, atol=1e-11 * abs(lam[0]))


def test_real_basis_spans_the_ritz_vectors():
    A, _ = _prescribed(n_real=10, seed=14)
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((A.shape[0], 9)))
    th, Z = np.linalg.eig(Q.T @ A @ Q)
    o = O.general_order(th)
    th, Z = th[o], Q @ Z[:, o]
    Xr = O.general_real_basis(Z, th)
    assert Xr.shape == Z.shape and Xr.dtype == np.float64
    # rank 9 together with the complex vectors: the same complex span
    s = np.linalg.svd(np.concatenate([Xr, Z], axis=1), compute_uv=False)
    assert s[8] > 1e-8 * s[0] and s[9] < 1e-12 * s[0]


@pytest.mark.parametrize("gamma", [0.5, 1.5])
def test_convection_diffusion_closed_form(gamma):
    # the sparse non-symmetric workload: its eigenvalues (LAPACK on the
    # dense form) are the closed form's, complex for gamma > 1
    import scipy.sparse as sp
    N = 9
    rp, ci, v = W.convection_diffusion_2d_csr(N, gamma)
    A = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(N * N, N * N)).toarray()
    cf = W.convection_diffusion_2d_eigenvalues(N, gamma)
    _assert_same_values(np.linalg.eigvals(A), cf, 1e-12 * np.abs(cf).max())
    assert (np.abs(cf.imag).max() > 0.5) == (gamma > 1)
    # and the oracle's subspace iteration on the CSR form finds the leading
    # values of the closed form
    r = O.subspace_eig_general((rp, ci, v), W.uniform_start(N * N, 24, 3), 4, degree=2, tol=1e-11,
                               basis="hessenberg")
    _assert_same_values(r.theta, _sorted_c(cf)[:4], 1e-9)
