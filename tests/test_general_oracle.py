"""Pins of the oracle's tensor-coefficient + reaction assembly (Sec. 5, eq. general) against facts
that do not come from it.  CPU only.

* ``fem.element_matrices_general`` -- a constant tensor's element stiffness applied to the nodal
  values of a linear function equals the closed form (T g) . int grad phi_i, which fixes every
  directional block K[a][b] (a wrong axis or a transposed pair fails); the blocks sum to the
  unit-coefficient stiffness; the mass equals ``element_matrices``'.
* ``fem.assemble_general`` -- with T = kappa I and no reaction it equals ``fem.assemble`` for the
  same kappa field; with a constant diagonal tensor diag(k1, k2, k3) and a constant reaction c its
  eigenvalues are the closed form k1 mu_i + k2 mu_j + k3 mu_l + c (the pencil is a Kronecker sum of
  1D Q1 pencils); symmetric positive definite for the paper's coefficients.
* ``multigrid.Hierarchy(operator=...)`` / ``pase.solve`` on it -- the outer loop reaches ARPACK
  shift-invert's eigenvalues of the assembled pencil.
"""
import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import fem, multigrid, pase
from tests.closed_form import mu_1d


def _cell_linear_values(g, h):
    """Nodal values of p(x) = g . x at the 8 corners of the cell [0, h]^3 (local vertex a has
    coordinate bit_d(a) h along axis d)."""
    return np.array([sum(g[d] * ((a >> d) & 1) * h for d in range(3)) for a in range(8)])


def test_element_blocks_on_linear_functions():
    """sum_ab T_ab K[a][b] p = (T g) . int grad phi_i for p linear (grad p = g exactly in Q1), and
    int d_a phi_i = +-h^2 / 4 by the vertex's bit along a."""
    h = 0.25
    K, M = fem.element_matrices_general(3, h)
    rng = np.random.default_rng(0)
    B = rng.standard_normal((3, 3))
    T = B @ B.T + np.eye(3)
    g = rng.standard_normal(3)
    p = _cell_linear_values(g, h)
    Ke = sum(T[a, b] * K[a, b] for a in range(3) for b in range(3))
    intgrad = np.array([[(1.0 if (i >> d) & 1 else -1.0) * h * h / 4 for d in range(3)] for i in range(8)])
    np.testing.assert_allclose(Ke @ p, intgrad @ (T @ g), rtol=1e-13, atol=1e-15)
    # the same for each single block: K[a][b] p = g_b int d_a phi
    for a, b in itertools.product(range(3), repeat=2):
        np.testing.assert_allclose(K[a, b] @ p, g[b] * intgrad[:, a], atol=1e-15)
    K1, M1 = fem.element_matrices(3, h)
    np.testing.assert_allclose(K[0, 0] + K[1, 1] + K[2, 2], K1, atol=1e-15)
    np.testing.assert_allclose(M, M1, atol=1e-16)


def test_isotropic_tensor_equals_the_kappa_assembly():
    """T = kappa I per element, no reaction: the same matrices as fem.assemble(kappa)."""
    n = 6
    kap = synth.kappa_field(3, n, 3)
    T = np.zeros((n ** 3, 6))
    T[:, 0] = T[:, 3] = T[:, 5] = kap
    A, M = fem.assemble_general(n, T)
    A0, M0 = fem.assemble(3, n, kap)
    assert abs(A - A0).max() < 1e-13 * abs(A0).max()
    assert abs(M - M0).max() == 0.0


def test_constant_diagonal_tensor_and_reaction_closed_form():
    """T = diag(1, 2, 3), phi = 5: eigenvalues k1 mu_i + k2 mu_j + k3 mu_l + 5 (all 343 of them on
    8^3) by dense eigh."""
    n = 8
    ks = (1.0, 2.0, 3.0)
    T = np.zeros((n ** 3, 6))
    T[:, 0], T[:, 3], T[:, 5] = ks
    A, M = fem.assemble_general(n, T, np.full(n ** 3, 5.0))
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
    mu = mu_1d(n)
    ref = np.sort((ks[0] * mu[:, None, None] + ks[1] * mu[None, :, None] + ks[2] * mu[None, None, :]).ravel() + 5.0)
    np.testing.assert_allclose(w, ref, rtol=1e-12)


def test_paper_coefficients_give_an_spd_pencil():
    """synth.general_coefficients on 8^3: A symmetric and positive definite (its reaction and its
    tensor I + c c^T are positive)."""
    T, phi = synth.general_coefficients(8)
    A, M = fem.assemble_general(8, T, phi)
    assert abs(A - A.T).max() < 1e-15 * abs(A).max()
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_pase_on_the_general_problem_matches_the_library_eigensolver():
    """16^3 mesh, V_H = 4^3, nev 6: the oracle's outer loop reaches ARPACK's eigenvalues to 1e-10."""
    n = 16
    T, phi = synth.general_coefficients(n)
    op = fem.assemble_general(n, T, phi)
    H = multigrid.Hierarchy(3, [16, 8, 4], operator=op)
    r = pase.solve(H, 6, 1e-10, synth.initial_vectors(H.A[0].shape[0], 6, 2))
    assert r.converged
    w = spla.eigsh(op[0].tocsc(), k=6, M=op[1].tocsc(), sigma=0.0, which="LM", return_eigenvectors=False,
                   tol=1e-14)
    np.testing.assert_allclose(r.lam, np.sort(w), rtol=1e-10)
