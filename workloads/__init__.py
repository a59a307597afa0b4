"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles test matrices with a
prescribed spectrum or structure.  It holds none of the eigensolver's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.
"""
from .generators import (  # noqa: F401
    rng,
    haar_orthogonal,
    dense_symmetric_prescribed,
    goe_noise,
    svd_prescribed,
    laplacian_2d_csr,
    convection_diffusion_2d_csr,
    convection_diffusion_2d_eigenvalues,
    laplacian_2d_eigenvalues,
    uniform_start,
    batched_sizes,
    general_prescribed,
    general_power_law_spectrum,
    kernel_points,
    kernel_subset,
    gaussian_kernel,
    WORKLOADS,
)
