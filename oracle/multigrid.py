"""Oracle: nested Q1 spaces, interpolation, Galerkin coarse operators, V-cycle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Interpolation I_H^h (Alg. 3 inputs): nodal interpolation of a coarse Q1
  function on the fine nodes.  For nested uniform meshes with ratio
  r = n_fine / n_coarse this is the tensor product of 1D hat-function
  weights max(0, 1 - |x_i - X_I| / H).  The augmented space uses the product
  of the level interpolations (Sec. 3: "a single interpolation matrix or ...
  a sequence of interpolation matrices").
* Coarse operators are Galerkin products P^T A P, P^T M P (Sec. 5.1 states
  B_H = I_h^H B_h I_H^h for the AMG hierarchy; for nested Q1 spaces with
  exact integration this coincides with rediscretisation when kappa is
  constant).
* V-cycle preconditioner for the fine solves.  The paper only says that the
  fine linear problems are solved by (block) CG; the multigrid
  preconditioner and its parameters are a reading: damped Jacobi with weight
  omega, nu pre- and nu post-smoothing sweeps from a zero initial guess,
  restriction by P^T, prolongation by P, exact (dense Cholesky) solve on the
  coarsest level.  It is symmetric positive definite, as CG needs.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem


def interp_1d(n_fine: int, n_coarse: int) -> sp.csr_matrix:
    """1D nodal interpolation from coarse interior nodes to fine interior nodes."""
    if n_fine % n_coarse:
        raise ValueError("meshes must be nested")
    xf = np.arange(1, n_fine) / n_fine
    Xc = np.arange(1, n_coarse) / n_coarse
    W = np.maximum(0.0, 1.0 - np.abs(xf[:, None] - Xc[None, :]) * n_coarse)
    W[np.abs(W) < 1e-15] = 0.0
    return sp.csr_matrix(W)


def interp(dim: int, n_fine: int, n_coarse: int) -> sp.csr_matrix:
    """Tensor-product Q1 interpolation I_H^h (fine interior x coarse interior), x fastest."""
    P1 = interp_1d(n_fine, n_coarse)
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    return P.tocsr()


class Hierarchy:
    """Levels n[0] > n[1] > ... > n[L] (elements per side); level 0 is the fine mesh.

    A[l], M[l]: level operators (A[0], M[0] assembled; coarser ones Galerkin).
    P[l] (l >= 1): interpolation from level l to level l-1.
    Pc: composite interpolation from the coarsest level to level 0.
    """

    def __init__(self, dim, levels, kappa=None, omega=2.0 / 3.0, nu=2, operator=None):
        """``operator``: optional (A0, M0) fine-level pair given in place of the kappa assembly
        (the tensor-coefficient workload, ``fem.assemble_general``)."""
        self.dim = dim
        self.n = list(levels)
        self.omega = omega
        self.nu = nu
        A0, M0 = fem.assemble(dim, self.n[0], kappa) if operator is None else operator
        self.A = [A0]
        self.M = [M0]
        self.P = [None]
        for l in range(1, len(self.n)):
            Pl = interp(dim, self.n[l - 1], self.n[l])
            self.P.append(Pl)
            self.A.append((Pl.T @ self.A[l - 1] @ Pl).tocsr())
            self.M.append((Pl.T @ self.M[l - 1] @ Pl).tocsr())
        self.D = [A.diagonal() for A in self.A]
        Pc = sp.identity(self.A[0].shape[0], format="csr")
        for l in range(1, len(self.n)):
            Pc = (Pc @ self.P[l]).tocsr()
        self.Pc = Pc
        self.L = len(self.n) - 1
        AL = self.A[self.L].toarray()
        self.AL_chol = sla.cho_factor(0.5 * (AL + AL.T), lower=True)

    @classmethod
    def from_matrices(cls, A, M, P, omega=2.0 / 3.0, nu=2):
        """Algebraic hierarchy (Alg. 3's "Require" given as matrices): level operators A[l], M[l]
        (sparse, fine first) and interpolations P[l] from level l to l - 1 (P[0] unused), as an AMG
        setup would give them.  The V-cycle and the composite interpolation are the same as for a
        grid hierarchy."""
        self = cls.__new__(cls)
        self.dim = None
        self.n = None
        self.omega = omega
        self.nu = nu
        self.A = [sp.csr_matrix(a) for a in A]
        self.M = [sp.csr_matrix(m) for m in M]
        self.P = [None] + [sp.csr_matrix(p) for p in P[1:]]
        self.D = [a.diagonal() for a in self.A]
        Pc = sp.identity(self.A[0].shape[0], format="csr")
        for l in range(1, len(self.A)):
            Pc = (Pc @ self.P[l]).tocsr()
        self.Pc = Pc
        self.L = len(self.A) - 1
        AL = self.A[self.L].toarray()
        self.AL_chol = sla.cho_factor(0.5 * (AL + AL.T), lower=True)
        return self

    # --- V-cycle -----------------------------------------------------------
    def jacobi(self, l, x, b):
        """One damped-Jacobi sweep x <- x + omega D^{-1} (b - A x) on level l."""
        return x + self.omega * (b - self.A[l] @ x) / self.D[l][:, None]

    def vcycle(self, b, l=0):
        """Approximate A[l]^{-1} b (b: N_l x k) by one V-cycle from x = 0."""
        b = np.asarray(b, dtype=np.float64)
        squeeze = b.ndim == 1
        if squeeze:
            b = b[:, None]
        if l == self.L:
            x = sla.cho_solve(self.AL_chol, b)
        else:
            x = self.omega * b / self.D[l][:, None]          # first sweep from zero
            for _ in range(self.nu - 1):
                x = self.jacobi(l, x, b)
            r = b - self.A[l] @ x
            e = self.vcycle(self.P[l + 1].T @ r, l + 1)
            x = x + self.P[l + 1] @ e
            for _ in range(self.nu):
                x = self.jacobi(l, x, b)
        return x[:, 0] if squeeze else x
