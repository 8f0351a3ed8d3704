"""Pins of the oracle's algebraic hierarchy (``multigrid.Hierarchy.from_matrices``: Alg. 3's
"Require" given as matrices, as an AMG setup gives them).  CPU only.

* ``from_matrices`` with a grid hierarchy's own matrices reproduces that hierarchy's V-cycle exactly
  (the algebraic constructor adds no arithmetic of its own).
* With a non-nested coarse space -- unsmoothed aggregation of 2x2x2 node blocks, coarse operators
  P^T A P, P^T M P -- the V-cycle is symmetric in the A inner product (a transposed or missing
  restriction breaks that), and the outer loop still reaches ARPACK shift-invert's eigenvalues of
  the fine pencil (the fixed point does not depend on the coarse space).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import multigrid, pase


def aggregation(m):
    """Interpolation (m^3 x mc^3, mc = ceil(m / 2)) of unsmoothed aggregation: node (x, y, z) takes the
    value of aggregate (x // 2, y // 2, z // 2)."""
    mc = (m + 1) // 2
    i = np.arange(m ** 3)
    x, y, z = i % m, (i // m) % m, i // (m * m)
    j = (x // 2) + mc * (y // 2) + mc * mc * (z // 2)
    return sp.csr_matrix((np.ones(m ** 3), (i, j)), shape=(m ** 3, mc ** 3)), mc


def aggregation_hierarchy(n, kappa, nlev=3):
    geo = multigrid.Hierarchy(3, [n, n // 2], kappa)
    A, M, P = [geo.A[0]], [geo.M[0]], [None]
    m = n - 1
    for _ in range(nlev - 1):
        Pl, m = aggregation(m)
        P.append(Pl)
        A.append((Pl.T @ A[-1] @ Pl).tocsr())
        M.append((Pl.T @ M[-1] @ Pl).tocsr())
    return multigrid.Hierarchy.from_matrices(A, M, P)


def test_from_matrices_reproduces_the_grid_vcycle():
    kap = synth.kappa_field(3, 16, 2)
    H = multigrid.Hierarchy(3, [16, 8, 4], kap)
    Ha = multigrid.Hierarchy.from_matrices(H.A, H.M, H.P)
    B = np.random.default_rng(0).standard_normal((H.A[0].shape[0], 3))
    assert np.array_equal(Ha.vcycle(B), H.vcycle(B))
    assert abs(Ha.Pc - H.Pc).max() == 0.0


def test_aggregation_vcycle_is_symmetric():
    """x^T V(y) = y^T V(x) (in the Euclidean inner product V approximates A^{-1}, a symmetric
    operator when the post-smoother mirrors the pre-smoother and R = P^T)."""
    H = aggregation_hierarchy(16, synth.kappa_field(3, 16, 4))
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, H.A[0].shape[0]))
    a, b = x @ H.vcycle(y), y @ H.vcycle(x)
    assert abs(a - b) < 1e-12 * abs(a)


def test_pase_with_an_aggregation_hierarchy_reaches_the_library_eigenvalues():
    kap = synth.kappa_field(3, 16, 4)
    H = aggregation_hierarchy(16, kap)
    r = pase.solve(H, 6, 1e-10, synth.initial_vectors(H.A[0].shape[0], 10, 3), guard=4)
    assert r.converged
    w = spla.eigsh(H.A[0].tocsc(), k=6, M=H.M[0].tocsc(), sigma=0.0, which="LM", return_eigenvectors=False,
                   tol=1e-14)
    np.testing.assert_allclose(r.lam, np.sort(w), rtol=1e-10)
