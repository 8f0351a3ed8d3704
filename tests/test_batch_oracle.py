"""Pins of the oracle's batch scheme (Sec. "Batch scheme for computing plenty of eigenpairs", Alg. 7
and eq. largest_component) against facts that do not come from it.  CPU only.

* ``components`` -- the B-norm of the B-orthogonal projection onto span(u_hat), formed in the fine
                    space from the vectors themselves by a least-squares solve (not by the paper's
                    identity X beta = u_H^T b + gamma^T beta); vectors inside the span keep their
                    whole norm.  Planted slips (a dropped coarse term, a transposed beta) fail.
* ``nearest``     -- a diagonal pencil with known eigenvalues.
* ``solve_batch`` -- the first batch and interior batches (one of them ragged) reach the library
                    eigensolver's eigenpairs of the fine pencil by index, with residuals <= tol and
                    M-orthonormal vectors; planted slips in the shift (the printed difference of
                    step (b)) or in the selection (smallest instead of largest component) fail.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import batch, multigrid
from tests.test_oracle import _planted


@pytest.fixture(scope="module")
def hier64():
    """2D 64^2 kappa field, V_H = 32^2 (N_H = 961), and the 40 smallest pairs of its fine pencil."""
    H = multigrid.Hierarchy(2, [64, 32], synth.kappa_field(2, 64, 3))
    w, V = spla.eigsh(H.A[0].tocsc(), k=40, M=H.M[0].tocsc(), sigma=0.0, which="LM", tol=1e-14)
    o = np.argsort(w)
    return H, w[o], V[:, o]


def _fine_projection_norms(H, uH, gamma, W):
    """||Pi_h v||_M^2 for v = P uH + W gamma, by least squares in the M inner product."""
    M = H.M[0]
    V = H.Pc @ uH + W @ gamma
    G = W.T @ (M @ W)
    X = np.linalg.solve(G, W.T @ (M @ V))
    return np.einsum("ji,jk,ki->i", X, G, X), np.einsum("ij,ij->j", V, M @ V)


@pytest.mark.parametrize("seed", [0, 1])
def test_components_equal_the_fine_space_projection(hier64, seed):
    H, _, _ = hier64
    rng = np.random.default_rng(seed)
    NH = H.A[H.L].shape[0]
    k, n = 7, 12
    W = rng.standard_normal((H.A[0].shape[0], k))
    _, _, _, _, b, beta = batch.composite_parts(H, W)
    uH, gamma = rng.standard_normal((NH, n)), rng.standard_normal((k, n))
    ref, vv = _fine_projection_norms(H, uH, gamma, W)
    got = batch.components(uH, gamma, b, beta)
    np.testing.assert_allclose(got, ref, rtol=1e-10)
    assert np.all(got <= vv * (1 + 1e-12))
    # a vector inside span(u_hat) keeps its whole norm; a coarse one outside it loses some
    inside = batch.components(np.zeros((NH, 1)), gamma[:, :1], b, beta)
    np.testing.assert_allclose(inside, gamma[:, 0] @ beta @ gamma[:, 0], rtol=1e-12)


@pytest.mark.parametrize("old,new", [
    ("rhs = uH.T @ b + gamma.T @ beta", "rhs = gamma.T @ beta"),        # dropped coarse term
    ("rhs = uH.T @ b + gamma.T @ beta", "rhs = uH.T @ b + beta @ gamma"),   # transposed product
])
def test_planted_component_slips_are_caught(hier64, old, new):
    H, _, _ = hier64
    rng = np.random.default_rng(5)
    NH = H.A[H.L].shape[0]
    W = rng.standard_normal((H.A[0].shape[0], 5))
    _, _, _, _, b, beta = batch.composite_parts(H, W)
    uH, gamma = rng.standard_normal((NH, 5)), rng.standard_normal((5, 5))
    ref, _ = _fine_projection_norms(H, uH, gamma, W)
    bad = _planted(batch.components, old, new)(uH, gamma, b, beta)
    assert not np.allclose(bad, ref, rtol=1e-6)


def test_nearest_on_a_diagonal_pencil():
    vals = np.arange(1.0, 11.0)
    B = np.diag(np.full(10, 2.0))
    w, Y = batch.nearest(np.diag(vals * 2.0), B, 4.4, 3)
    np.testing.assert_allclose(w, [3.0, 4.0, 5.0], rtol=1e-14)
    assert np.allclose(np.abs(Y[[2, 3, 4], [0, 1, 2]]), 1 / np.sqrt(2.0))
    w, _ = batch.nearest(np.diag(vals), np.eye(10), 0.0, 2)
    np.testing.assert_allclose(w, [1.0, 2.0])


def _check(H, w, V, r, first, nb, tol):
    assert r.converged
    np.testing.assert_allclose(r.lam, w[first:first + nb], rtol=1e-10)
    A, M = H.A[0], H.M[0]
    R = A @ r.U - (M @ r.U) * r.lam[None, :]
    res = np.linalg.norm(R, axis=0) / (np.abs(r.lam) * np.linalg.norm(M @ r.U, axis=0))
    assert res.max() <= tol
    G = r.U.T @ (M @ r.U)
    assert np.abs(G - np.eye(nb)).max() < 1e-8


@pytest.mark.parametrize("first, nb", [(0, 10), (10, 10), (20, 7)])
def test_batches_reach_the_library_eigenpairs(hier64, first, nb):
    """Interior batches converge to the pairs first .. first + nb - 1 of the fine pencil."""
    H, w, V = hier64
    r = batch.solve_batch(H, first, nb, 1e-10, guard=4, max_outer=60)
    _check(H, w, V, r, first, nb, 1e-10)


@pytest.mark.parametrize("old,new", [
    ("theta = 0.5 * (lamH[b0] + lamH[b0 + k - 1])", "theta = 0.5 * (lamH[b0] - lamH[b0 + k - 1])"),
    ("keep = np.sort(np.argsort(-score, kind=\"stable\")[:k])", "keep = np.sort(np.argsort(score, kind=\"stable\")[:k])"),
])
def test_planted_batch_slips_are_caught(hier64, old, new):
    """Pairs 20 .. 26 with a window of n = 19 composite pairs (the block holds 15): the right shift
    and selection still converge, the slipped ones do not."""
    H, w, V = hier64
    good = batch.solve_batch(H, 20, 7, 1e-10, guard=4, max_outer=60, n=19)
    _check(H, w, V, good, 20, 7, 1e-10)
    bad = _planted(batch.solve_batch, old, new)(H, 20, 7, 1e-10, guard=4, max_outer=15, n=19)
    assert not (bad.converged and np.allclose(bad.lam, w[20:27], rtol=1e-8))
