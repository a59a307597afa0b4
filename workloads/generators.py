"""Seeded generators for the synthetic test and benchmark matrices.

Random draws always come from numpy's PCG64 with an explicit seed, so the
same seed gives the same bits on every machine; the heavy assembly (QR of a
Gaussian matrix, Q diag(lam) Q^T) runs through torch on the requested
device, which is plain input preparation and no part of the eigensolver.

Dense matrices are returned as torch tensors in column-major layout
(stride (1, rows)); for symmetric matrices that is the same memory as
row-major.  Start blocks are U(0,1) drawn in FP64, as in the paper's
experiments (Sec. 5.2: random initial blocks drawn from U(0,1) in FP64 and
cast to the working precision).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _normal(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(size=shape, dtype=np.float64)


def haar_orthogonal(n: int, seed: int, cols: int | None = None,
                    device: str | torch.device = "cpu") -> torch.Tensor:
    """Q from the QR factorisation of a seeded N(0,1) n x cols matrix, with
    the column signs fixed so that diag(R) > 0 (this makes Q Haar
    distributed).  Returned as an FP64 tensor on `device`."""
    cols = n if cols is None else cols
    g = torch.from_numpy(_normal((n, cols), seed)).to(device)
    q, r = torch.linalg.qr(g, mode="reduced")
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    return q * d.unsqueeze(0)


def goe_noise(n: int, scale: float, seed: int,
              device: str | torch.device = "cpu") -> torch.Tensor:
    """Symmetric Gaussian noise E = scale * (G + G^T) / sqrt(2), G ~ N(0,1)."""
    g = torch.from_numpy(_normal((n, n), seed)).to(device)
    return (g + g.T) * (scale / math.sqrt(2.0))


def dense_symmetric_prescribed(lam, seed: int, noise_scale: float = 0.0,
                               noise_seed: int | None = None,
                               dtype=torch.float64,
                               device: str | torch.device = "cpu") -> torch.Tensor:
    """A = Q diag(lam) Q^T (+ optional symmetric noise), assembled in FP64 and
    stored in `dtype` (the stored array is the matrix of record)."""
    lam = torch.as_tensor(np.asarray(lam, dtype=np.float64), device=device)
    n = lam.numel()
    q = haar_orthogonal(n, seed, device=device)
    a = (q * lam.unsqueeze(0)) @ q.T
    del q
    a = (a + a.T) * 0.5
    if noise_scale:
        a += goe_noise(n, noise_scale, seed if noise_seed is None else noise_seed,
                       device=device)
    return a.to(dtype).contiguous()


def svd_prescribed(m: int, n: int, sigma, seed: int, dtype=torch.float32,
                   device: str | torch.device = "cpu") -> torch.Tensor:
    """A = U diag(sigma) V^T with U (m x n) and V (n x n) Haar orthonormal,
    assembled in FP64 and stored column-major in `dtype`."""
    sigma = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    u = haar_orthogonal(m, seed, cols=n, device=device)
    v = haar_orthogonal(n, seed + 7, device=device)
    # A^T = V diag(sigma) U^T stored row-major is A stored column-major.
    at = (v * sigma.unsqueeze(0)) @ u.T
    del u, v
    return at.to(dtype).contiguous().T


def laplacian_2d_csr(N: int, dtype=np.float32):
    """Dirichlet 5-point Laplacian on an N x N grid, lexicographic ordering
    (row = x + N*y), diagonal 4 and -1 to every existing neighbour, CSR with
    sorted int32 column indices.  Returns (row_ptr, col_idx, values)."""
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = idx // N
    cols = []
    vals = []
    # neighbours in increasing column order: y-1, x-1, self, x+1, y+1
    for dc, ok, v in ((-N, y > 0, -1.0), (-1, x > 0, -1.0), (0, np.ones(n, bool), 4.0),
                      (1, x < N - 1, -1.0), (N, y < N - 1, -1.0)):
        c = np.where(ok, idx + dc, -1)
        cols.append(c)
        vals.append(np.where(ok, v, 0.0))
    cols = np.stack(cols, axis=1)
    vals = np.stack(vals, axis=1)
    mask = cols >= 0
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[mask].astype(np.int32)
    values = vals[mask].astype(dtype)
    return row_ptr.astype(np.int32), col_idx, values


def convection_diffusion_2d_csr(N: int, gamma: float, dtype=np.float32):
    """Non-symmetric 5-point convection-diffusion operator on an N x N grid
    (row = x + N*y): diagonal 4, -1 to the y neighbours, -(1 + gamma) to
    x - 1 and -(1 - gamma) to x + 1 (central differences of a flow along x
    with cell Peclet number gamma), CSR with sorted int32 column indices.
    For gamma > 1 most eigenvalues are complex.  Returns (row_ptr, col_idx,
    values)."""
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = idx // N
    cols, vals = [], []
    for dc, ok, v in ((-N, y > 0, -1.0), (-1, x > 0, -(1.0 + gamma)), (0, np.ones(n, bool), 4.0),
                      (1, x < N - 1, -(1.0 - gamma)), (N, y < N - 1, -1.0)):
        cols.append(np.where(ok, idx + dc, -1))
        vals.append(np.where(ok, v, 0.0))
    cols = np.stack(cols, axis=1)
    vals = np.stack(vals, axis=1)
    mask = cols >= 0
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols[mask].astype(np.int32), vals[mask].astype(dtype)


def convection_diffusion_2d_eigenvalues(N: int, gamma: float) -> np.ndarray:
    """All eigenvalues of convection_diffusion_2d_csr(N, gamma): the sum of
    the x part, a tridiagonal Toeplitz matrix (-(1+gamma), 2, -(1-gamma))
    with eigenvalues 2 + 2 sqrt(1 - gamma^2) cos(p pi/(N+1)) (complex square
    root), and the y part 2 - 2 cos(q pi/(N+1)) (textbook closed forms).
    Complex, unsorted."""
    j = np.arange(1, N + 1)
    c = np.cos(j * np.pi / (N + 1))
    ex = 2.0 + 2.0 * np.sqrt(complex(1.0 - gamma * gamma)) * c
    ey = 2.0 - 2.0 * c
    return (ex[:, None] + ey[None, :]).ravel()


def laplacian_2d_eigenvalues(N: int) -> np.ndarray:
    """All eigenvalues of the N x N-grid Dirichlet 5-point Laplacian
    (textbook closed form 4 - 2 cos(p pi/(N+1)) - 2 cos(q pi/(N+1))),
    sorted ascending."""
    t = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    return np.sort((t[:, None] + t[None, :]).ravel())


def general_prescribed(real_eigs, complex_pairs, seed: int, nonnormal: float = 0.0,
                       dtype=torch.float64, device: str | torch.device = "cpu") -> torch.Tensor:
    """Real non-symmetric A = S D S^-1 with D block diagonal: first, for each
    (a, b) in complex_pairs, a 2 x 2 block [[a, b], [-b, a]] (eigenvalues
    a +- ib), then the given real eigenvalues.  S = Q U with Q Haar
    orthogonal and U = I + nonnormal N, N strictly upper triangular with
    N(0, 1/n) entries (U = I: a normal matrix).  Assembled in FP64 on
    `device` as Q (U D U^-1) Q^T and stored column-major in `dtype`."""
    reals = torch.as_tensor(np.asarray(real_eigs, dtype=np.float64), device=device)
    pairs = np.asarray(complex_pairs, dtype=np.float64).reshape(-1, 2)
    n = reals.numel() + 2 * pairs.shape[0]
    q = haar_orthogonal(n, seed, device=device)
    if nonnormal:
        u = torch.from_numpy(np.triu(_normal((n, n), seed + 1), 1)).to(device) * (nonnormal / math.sqrt(n))
        u.diagonal().add_(1.0)
    else:
        u = torch.eye(n, dtype=torch.float64, device=device)
    # T = U D: column operations
    t = u.clone()
    npair = pairs.shape[0]
    if npair:
        a = torch.as_tensor(pairs[:, 0], device=device)
        b = torch.as_tensor(pairs[:, 1], device=device)
        c0 = u[:, 0:2 * npair:2]
        c1 = u[:, 1:2 * npair:2]
        t[:, 0:2 * npair:2] = c0 * a - c1 * b
        t[:, 1:2 * npair:2] = c0 * b + c1 * a
    t[:, 2 * npair:] = u[:, 2 * npair:] * reals
    # T U^-1 (U upper triangular), then Q T Q^T
    t = torch.linalg.solve_triangular(u, t, upper=True, left=False)
    del u
    a_ = q @ t @ q.T
    del q, t
    return a_.to(dtype).T.contiguous().T


def general_power_law_spectrum(n: int, seed: int, pair_fraction: float = 0.5):
    """Eigenvalues for general_prescribed with moduli j^-1.5: walking j = 1,
    2, ..., with probability pair_fraction a conjugate pair of modulus
    j^-1.5 at an angle drawn from U(0.1 pi, 0.9 pi) (taking j and j + 1),
    else a real value +-j^-1.5 with a random sign.  Returns (reals, pairs,
    all n eigenvalues as complex, in the order drawn: moduli non-increasing,
    a pair's + member first)."""
    g = rng(seed)
    reals, pairs, allv = [], [], []
    j = 1
    while j <= n:
        m = float(j) ** -1.5
        if j < n and g.random() < pair_fraction:
            th = np.pi * (0.1 + 0.8 * g.random())
            a, b = m * np.cos(th), m * np.sin(th)
            pairs.append((a, b))
            allv += [complex(a, b), complex(a, -b)]
            j += 2
        else:
            v = m if g.random() < 0.5 else -m
            reals.append(v)
            allv.append(complex(v, 0.0))
            j += 1
    return reals, pairs, np.array(allv)


def kernel_points(n: int, seed: int, d: int = 2) -> np.ndarray:
    """n points drawn uniformly from the square (cube) of side sqrt(n)."""
    return rng(seed).random((n, d)) * np.sqrt(n)


def kernel_subset(X: np.ndarray, m: int, seed: int):
    """m of the points of X drawn without replacement: (the points, their
    row indices in X)."""
    idx = rng(seed).choice(X.shape[0], size=m, replace=False)
    return X[idx], idx


def gaussian_kernel(X: np.ndarray, Y: np.ndarray | None = None, f: float = 1.0, length: float = 10.0,
                    s: float = 0.0, dtype=torch.float64, device: str | torch.device = "cpu") -> torch.Tensor:
    """Gaussian kernel matrix A_ij = f (exp(-||x_i - y_j||^2 / (2 l^2)) + s [i == j])
    (Y = X for the square case), assembled in FP64, column-major."""
    x = torch.as_tensor(X, dtype=torch.float64, device=device)
    y = x if Y is None else torch.as_tensor(Y, dtype=torch.float64, device=device)
    d2 = torch.cdist(x, y, compute_mode="donot_use_mm_for_euclid_dist") ** 2
    a = torch.exp(-d2 / (2.0 * length * length))
    if Y is None and s:
        a = a + s * torch.eye(x.shape[0], dtype=torch.float64, device=device)
    a = f * a
    if Y is None:
        a = 0.5 * (a + a.T)
    return a.to(dtype).T.contiguous().T


def uniform_start(n: int, b: int, seed: int) -> np.ndarray:
    """U(0,1) start block in FP64, column-major (Fortran order)."""
    return np.asfortranarray(rng(seed).random(size=(n, b), dtype=np.float64))


def batched_sizes(seed: int, count: int = 512, lo: int = 256, hi: int = 4096) -> np.ndarray:
    return rng(seed).integers(lo, hi + 1, size=count)


@dataclass
class Workload:
    name: str
    kind: str
    params: dict = field(default_factory=dict)


# The five benchmark/parity configurations (seed = 1000 + index, start
# block seed = 1100 + index).
WORKLOADS = {
    "dense_sym_n512_power": Workload(
        "dense_sym_n512_power", "eig_dense",
        dict(n=512, lam="0.95**i (i=1..n)", k=8, basis=16, degree=1, filter="power",
             outer=20, seed=1001, x0_seed=1101, dtype="f64")),
    "dense_sym_n16384_cheb4": Workload(
        "dense_sym_n16384_cheb4", "eig_dense",
        dict(n=16384, lam="i**-1.5 (i=1..n)", noise=1e-3, k=64, basis=128, degree=4,
             filter="chebyshev", seed=1002, x0_seed=1102, dtype="f32")),
    "dense_svd_65536x8192": Workload(
        "dense_svd_65536x8192", "svd_dense",
        dict(m=65536, n=8192, sigma="exp(-i/200)", k=100, basis=200, seed=1003,
             x0_seed=1103, dtype="f32")),
    "laplacian2d_1024": Workload(
        "laplacian2d_1024", "eig_csr",
        dict(N=1024, k=32, basis=64, degree=20, filter="chebyshev", which="smallest",
             seed=1004, x0_seed=1104)),
    "batched_512": Workload(
        "batched_512", "eig_batched",
        dict(count=512, nlo=256, nhi=4096, lam="0.9**i", k=8, basis=16, seed=1005,
             x0_seed=1105)),
}
