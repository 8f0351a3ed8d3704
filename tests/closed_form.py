"""Closed-form eigenvalues of the Q1 Laplacian pencil on a uniform mesh.

Independent of the oracle: the 1D Q1 stiffness (1/h) tridiag(-1, 2, -1) and
mass (h/6) tridiag(1, 4, 1) on n-1 interior nodes share the sine
eigenvectors sin(k pi x_i), k = 1..n-1, with generalized eigenvalues
mu_k = (6/h^2) (1 - cos k pi h) / (2 + cos k pi h).  The d-dimensional Q1
pencil is the tensor product, so its eigenvalues are sums of d such mu.
"""
import numpy as np


def mu_1d(n):
    h = 1.0 / n
    k = np.arange(1, n)
    c = np.cos(k * np.pi * h)
    return (6.0 / h ** 2) * (1.0 - c) / (2.0 + c)


def q1_laplace_eigs(dim, n, k=None):
    mu = mu_1d(n)
    g = mu
    for _ in range(dim - 1):
        g = np.add.outer(g, mu).ravel()
    g = np.sort(g)
    return g if k is None else g[:k]
