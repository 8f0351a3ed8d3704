"""Oracle: the fixed point of the method, written out directly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Alg. 3's "Ensure" asks for the first k eigenpairs of the fine pencil,
A_h u = lambda B_h u (Sec. 2.1, the discrete eigenproblem with eigenvalues
counted with multiplicity).  Whatever iteration reaches them, a converged
solve returns those k pairs, so they can be computed here without the
method: the assembled Q1 matrices of ``fem`` and the shift-invert Lanczos of
ARPACK (``scipy.sparse.linalg.eigsh`` with sigma = 0, a library primitive),
which returns the eigenvalues nearest 0 of the positive definite pencil,
i.e. the smallest ones.

Pins (``tests/test_oracle.py``): the closed-form Q1 eigenvalues for kappa = 1
and a dense ``scipy.linalg.eigh`` of the same pencil on a small mesh.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def lowest_eigenpairs(dim: int, n: int, k: int, kappa=None, vectors: bool = False, operator=None):
    """The k smallest eigenvalues (ascending) of the Q1 pencil (A, M) on the n^dim mesh,
    and with ``vectors`` the M-orthonormal eigenvectors (N x k).  ``operator``: an assembled
    (A, M) pair in place of the kappa assembly (the tensor-coefficient workload)."""
    A, M = fem.assemble(dim, n, kappa) if operator is None else operator
    w, V = spla.eigsh(A.tocsc(), k=k, M=M.tocsc(), sigma=0.0, which="LM", tol=1e-14)
    order = np.argsort(w)
    w = w[order]
    if not vectors:
        return w
    V = V[:, order]
    return w, V
