"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers and shapes them into the inputs the
solver is given: the element coefficient field kappa and the initial
multi-vector U0.  It holds none of the eigensolver's arithmetic, so both the
CPU oracle and the GPU path can take their inputs from here without sharing
any of the method.

Recipes
-------
* ``initial_vectors(N, k, seed)``: U0 with i.i.d. entries uniform on (-1, 1),
  drawn as ``numpy.random.default_rng(seed).uniform(-1, 1, (N, k))``.  Row i
  is grid node i (lexicographic, x fastest); column j is vector j.
* ``kappa_field(dim, n, seed, ell, var)``: a piecewise-constant coefficient,
  one value per element of the uniform n^dim mesh of the unit square/cube,
  kappa = exp(g) where g is a stationary Gaussian random field with mean 0,
  variance ``var`` and squared-exponential covariance
  C(r) = var * exp(-r^2 / (2 ell^2)), sampled at element centres.  It is
  drawn by circulant embedding on a periodic grid of 2n cells per axis
  (period 2, which is > 1 + several correlation lengths, so the embedding is
  exact for ell = 0.1): white noise w ~ N(0, 1) per cell, g = IFFT(sqrt(L) *
  FFT(w)) with L the (clipped, non-negative) DFT of the periodised
  covariance, then the first n cells per axis are kept.  Element (i, j, l)
  is stored at index i + n*j + n*n*l (x fastest).
* ``general_coefficients(n)``: the coefficients of the second workload of
  the paper's tests (Sec. 5, eq. general) on the uniform n^3 mesh, one value
  per element, evaluated at the element centre c: the tensor
  A(c) = I + (c - 1/2)(c - 1/2)^T, stored as its upper triangle
  (a11, a12, a13, a22, a23, a33), and the reaction
  phi(c) = exp((c1 - 1/2)(c2 - 1/2)(c3 - 1/2)).  No randomness.
"""
from __future__ import annotations

import numpy as np

__all__ = ["initial_vectors", "kappa_field", "interior_count", "general_coefficients"]


def interior_count(dim: int, n: int) -> int:
    """Number of interior grid nodes of a uniform n^dim mesh (Dirichlet DOFs removed)."""
    return (n - 1) ** dim


def initial_vectors(N: int, k: int, seed: int) -> np.ndarray:
    """Seeded U0: N x k float64, uniform on (-1, 1), node-major (row = node)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (N, k))


def kappa_field(dim: int, n: int, seed: int, ell: float = 0.1, var: float = 1.0) -> np.ndarray:
    """Seeded log-normal element coefficient (n^dim float64, x fastest).

    See the module docstring for the recipe.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    h = 1.0 / n
    m = 2 * n                      # periodic embedding grid, period 2
    # periodic distance of every embedding cell to cell 0, per axis
    idx = np.arange(m)
    d1 = np.minimum(idx, m - idx) * h
    grids = np.meshgrid(*([d1] * dim), indexing="ij")
    r2 = sum(g * g for g in grids)
    cov = var * np.exp(-r2 / (2.0 * ell * ell))
    lam = np.fft.fftn(cov).real
    lam = np.clip(lam, 0.0, None)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((m,) * dim)
    g = np.fft.ifftn(np.sqrt(lam) * np.fft.fftn(w)).real
    g = g[(slice(0, n),) * dim]
    # axes are (x, y[, z]) in 'ij' order; store x fastest -> transpose to (z, y, x)
    g = np.ascontiguousarray(np.transpose(g))
    return np.exp(g).reshape(-1)


def general_coefficients(n: int):
    """Element-centre tensor (n^3 x 6: a11, a12, a13, a22, a23, a33) and reaction (n^3) of the
    problem -div(A grad u) + phi u = lambda u with A = I + (x - 1/2)(x - 1/2)^T and
    phi = exp((x1 - 1/2)(x2 - 1/2)(x3 - 1/2)); element (i, j, l) at index i + n j + n^2 l."""
    c = (np.arange(n) + 0.5) / n - 0.5
    d1 = np.tile(c, n * n)
    d2 = np.tile(np.repeat(c, n), n)
    d3 = np.repeat(c, n * n)
    tensor = np.stack([1.0 + d1 * d1, d1 * d2, d1 * d3, 1.0 + d2 * d2, d2 * d3, 1.0 + d3 * d3], axis=1)
    reaction = np.exp(d1 * d2 * d3)
    return np.ascontiguousarray(tensor), reaction
