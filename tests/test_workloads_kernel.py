"""Gaussian kernel workloads of the accuracy studies (Sec. 2 kernel
equation; Sec. 5.3 condition-number study; Sec. 5.4 eigenvalue and SVD
studies), pinned to what the paper states about their spectra and to
properties the definition fixes."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def points():
    return W.kernel_points(1000, 7)


def _eig_desc(A):
    return np.linalg.eigvalsh(A.numpy())[::-1]


def test_points_fill_the_square(points):
    # 1000 points uniform in a square of side sqrt(1000)
    assert points.shape == (1000, 2)
    side = np.sqrt(1000.0)
    assert points.min() >= 0.0 and points.max() <= side
    # each coordinate has the mean and variance of U(0, side)
    np.testing.assert_allclose(points.mean(axis=0), side / 2, rtol=0.05)
    np.testing.assert_allclose(points.var(axis=0), side * side / 12, rtol=0.1)
    np.testing.assert_array_equal(points, W.kernel_points(1000, 7))


def test_kernel_definition_entries(points):
    # A_ij = f (exp(-|x_i - x_j|^2 / (2 l^2)) + s delta_ij), evaluated
    # entry by entry for a few pairs
    f, l, s = 0.2, 10.0, 0.01
    A = W.gaussian_kernel(points, f=f, length=l, s=s).numpy()
    for i, j in [(0, 0), (0, 1), (17, 400), (999, 3), (500, 500)]:
        d2 = float(np.sum((points[i] - points[j]) ** 2))
        want = f * (np.exp(-d2 / (2 * l * l)) + (s if i == j else 0.0))
        np.testing.assert_allclose(A[i, j], want, rtol=1e-14, atol=1e-300)
    np.testing.assert_array_equal(A, A.T)


def test_length_scale_one_decays_slowly(points):
    # Sec. 5.3: with l = 1 the twentieth largest eigenvalue is above 6
    lam = _eig_desc(W.gaussian_kernel(points, f=1.0, length=1.0, s=0.01))
    assert lam[19] > 6.0


def test_length_scale_hundred_is_numerically_low_rank(points):
    # Sec. 5.3: with l = 100 the seventh largest eigenvalue is already
    # close to s = 0.01; the kernel part is PSD, so no eigenvalue is below s
    lam = _eig_desc(W.gaussian_kernel(points, f=1.0, length=100.0, s=0.01))
    assert abs(lam[6] - 0.01) < 1e-3
    assert lam[-1] >= 0.01 * (1 - 1e-10)


def test_eigen_configurations_of_the_study(points):
    # Sec. 5.4, eigenvalues: configuration 1 (f 0.2, l 10, s 0.01) decays
    # only to f s = 0.002; configuration 2 (f 0.2, l 100, s 0) decays to 0
    lam1 = _eig_desc(W.gaussian_kernel(points, f=0.2, length=10.0, s=0.01))
    lam2 = _eig_desc(W.gaussian_kernel(points, f=0.2, length=100.0, s=0.0))
    assert lam1[-1] >= 0.002 * (1 - 1e-10) and lam1[49] < 0.01
    assert lam2[10] < 1e-5 and abs(lam2[-1]) < 1e-10
    # the trace is f (1 + s) n in both
    np.testing.assert_allclose(lam1.sum(), 0.2 * 1.01 * 1000, rtol=1e-12)
    np.testing.assert_allclose(lam2.sum(), 0.2 * 1000, rtol=1e-12)


def test_rectangular_kernel_of_a_subset(points):
    # Sec. 5.4, SVD: the 200 columns are points drawn from the same set
    # without replacement, so A holds a 200 x 200 block of the square kernel
    Y, idx = W.kernel_subset(points, 200, 8)
    assert len(set(idx.tolist())) == 200
    A = W.gaussian_kernel(points, Y, f=0.2, length=10.0).numpy()
    K = W.gaussian_kernel(points, f=0.2, length=10.0).numpy()
    assert A.shape == (1000, 200)
    np.testing.assert_allclose(A, K[:, idx], rtol=1e-13, atol=1e-300)
