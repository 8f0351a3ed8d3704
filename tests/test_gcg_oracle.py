"""Pins of the oracle's PRECOND-A and GCG_AUG (Sec. 4: eqs. Transformation_0 and
Eigen_Problem_Hh_2, Alg. 4 and 5) against facts that do not come from it.

CPU only.  Each function of ``oracle.gcg_aug`` and ``oracle.pase.small_solve_precond_a`` is
named in the docstring of the test that pins it:

* ``block_factors``  -- the product of the three factors is the matrix it factorises.
* ``precond_a``      -- its blocks equal the congruence of the composite pencil by the right
                        factor, computed by dense solves (a sign or transposition slip in any of
                        alpha~, b~, beta~ fails; planted slips check that).
* ``AugPencil``      -- its products equal the dense transformed matrices.
* ``gcg_aug``        -- the k smallest eigenpairs of random and PASE-born pencils equal dense
                        ``scipy.linalg.eigh``'s; the eigenvalues of eq. Eigen_Problem_Hh_2 equal
                        those of eq. Eigenvalue_Problem_AHh.
* ``solve_augmented`` / ``small_solve_precond_a`` -- one correction equals the dense generalized
                        eigensolver on the literal composite pencil of eq. Definition_Hh with
                        V_H = an intermediate level.
* ``solve(small="precond_a")`` -- converges to the library eigensolver's eigenpairs of the
                        assembled pencil.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import gcg_aug as gcg
from oracle import multigrid, pase
from tests.test_oracle import _planted


def _spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


def _random_composite(nH=40, k=6, seed=0):
    rng = np.random.default_rng(seed)
    Ahh = _spd(nH + k, rng)
    Bhh = _spd(nH + k, rng, cond=50.0)
    Ahh, Bhh = 0.5 * (Ahh + Ahh.T), 0.5 * (Bhh + Bhh.T)
    return Ahh, Bhh, nH, k


def _blocks(M, nH):
    return M[:nH, :nH], M[:nH, nH:], M[nH:, nH:]


def test_block_factorisation_identity():
    """block_factors: L D R reproduces [[A_H, a], [a^T, alpha]] to round-off, L = R^T, and D is
    block-diagonal with the Schur complement alpha - a^T A_H^{-1} a (eq. Transformation_0)."""
    Ahh, _, nH, k = _random_composite()
    AH, a, alpha = _blocks(Ahh, nH)
    Lf, D, Rf = gcg.block_factors(AH, a, alpha)
    assert np.abs(Lf @ D @ Rf - Ahh).max() < 1e-12 * np.abs(Ahh).max()
    assert np.array_equal(Lf, Rf.T)
    assert np.abs(D[:nH, nH:]).max() == 0.0 and np.abs(D[nH:, :nH]).max() == 0.0
    S = alpha - a.T @ sla.solve(AH, a)
    assert np.abs(D[nH:, nH:] - S).max() < 1e-12 * np.abs(S).max()


def _congruence(Ahh, Bhh, nH):
    """R^{-T} X R^{-1} with R = [[I, A_H^{-1} a], [0, I]], by dense solves only."""
    AH, a, _ = _blocks(Ahh, nH)
    k = Ahh.shape[0] - nH
    R = np.block([[np.eye(nH), sla.solve(AH, a)], [np.zeros((k, nH)), np.eye(k)]])
    Ri = np.linalg.inv(R)
    return Ri.T @ Ahh @ Ri, Ri.T @ Bhh @ Ri


def _precond_blocks(Ahh, Bhh, nH, fn=gcg.precond_a):
    AH, a, alpha = _blocks(Ahh, nH)
    BH, b, beta = _blocks(Bhh, nH)
    return fn(lambda F: sla.solve(AH, F), BH, a, alpha, b, beta)


def test_precond_a_blocks_are_the_congruence():
    """precond_a: alpha~, b~_h and beta~ of eq. Eigen_Problem_Hh_2 are the blocks of the congruence
    of (A_Hh, B_Hh) by the right factor of eq. Transformation_0, and the left matrix becomes
    block-diagonal."""
    Ahh, Bhh, nH, k = _random_composite(seed=1)
    ahat, at, bt, bet = _precond_blocks(Ahh, Bhh, nH)
    At, Bt = _congruence(Ahh, Bhh, nH)
    sA, sB = np.abs(Ahh).max(), np.abs(Bhh).max()
    assert np.abs(At[:nH, nH:]).max() < 1e-11 * sA
    assert np.abs(At[nH:, nH:] - at).max() < 1e-11 * sA
    assert np.abs(Bt[:nH, nH:] - bt).max() < 1e-11 * sB
    assert np.abs(Bt[nH:, nH:] - bet).max() < 1e-11 * sB
    assert np.abs(Bt[:nH, :nH] - Bhh[:nH, :nH]).max() < 1e-11 * sB


@pytest.mark.parametrize("old,new", [
    ("- ahat.T @ b + ahat.T @ (BH @ ahat)", "+ ahat.T @ b + ahat.T @ (BH @ ahat)"),   # sign slip in beta~
    ("b_t = b - BH @ ahat", "b_t = b - BH.T @ ahat + 0 * ahat"),                      # kept (B_H symmetric)
    ("alpha_t = alpha - ahat.T @ a", "alpha_t = alpha - ahat.T @ ahat"),               # wrong operand
    ("b_t = b - BH @ ahat", "b_t = b"),                                                # dropped term
])
def test_planted_precond_a_slips_are_caught(old, new):
    """Slips planted in precond_a break the congruence pin (the transposed B_H is no slip:
    B_H is symmetric, and the pin must pass it)."""
    Ahh, Bhh, nH, k = _random_composite(seed=2)
    bad = _planted(gcg.precond_a, old, new)
    ahat, at, bt, bet = _precond_blocks(Ahh, Bhh, nH, bad)
    At, Bt = _congruence(Ahh, Bhh, nH)
    err = max(np.abs(At[nH:, nH:] - at).max(), np.abs(Bt[:nH, nH:] - bt).max(),
              np.abs(Bt[nH:, nH:] - bet).max())
    if "BH.T" in new:
        assert err < 1e-11 * np.abs(Bhh).max()
    else:
        assert err > 1e-6 * np.abs(Bhh).max()


def test_transformed_pencil_has_the_same_eigenpairs():
    """The pencils of eqs. Eigenvalue_Problem_AHh and Eigen_Problem_Hh_2 have the same eigenvalues
    (dense eigh of each), and Alg. 5 step 3's back-transform u_H = u~_H - a_hat gamma~ of the
    transformed eigenvectors solves the original pencil."""
    Ahh, Bhh, nH, k = _random_composite(seed=3)
    ahat, at, bt, bet = _precond_blocks(Ahh, Bhh, nH)
    AH, BH = Ahh[:nH, :nH], Bhh[:nH, :nH]
    At = np.block([[AH, np.zeros((nH, k))], [np.zeros((k, nH)), at]])
    Bt = np.block([[BH, bt], [bt.T, bet]])
    w0, _ = sla.eigh(Ahh, Bhh)
    w1, Y = sla.eigh(At, Bt)
    np.testing.assert_allclose(w1, w0, rtol=1e-11)
    U = np.vstack([Y[:nH] - ahat @ Y[nH:], Y[nH:]])
    R = Ahh @ U - Bhh @ U * w1[None, :]
    assert np.abs(R).max() < 1e-10 * np.abs(Ahh).max()


def test_aug_pencil_products_match_dense():
    """AugPencil.A / .B equal the dense transformed matrices times a block."""
    Ahh, Bhh, nH, k = _random_composite(seed=4)
    ahat, at, bt, bet = _precond_blocks(Ahh, Bhh, nH)
    AH, BH = Ahh[:nH, :nH], Bhh[:nH, :nH]
    pen = gcg.AugPencil(AH, BH, at, bt, bet, lambda R: sla.solve(AH, R))
    Y = np.random.default_rng(5).standard_normal((nH + k, 3))
    At = np.block([[AH, np.zeros((nH, k))], [np.zeros((k, nH)), at]])
    Bt = np.block([[BH, bt], [bt.T, bet]])
    assert np.abs(pen.A(Y) - At @ Y).max() < 1e-12 * np.abs(At).max()
    assert np.abs(pen.B(Y) - Bt @ Y).max() < 1e-12 * np.abs(Bt).max()


@pytest.mark.parametrize("precond", ["exact", "jacobi"])
def test_gcg_aug_matches_dense_eigh_on_a_random_pencil(precond):
    """gcg_aug from a random start reaches dense eigh's k smallest eigenpairs (eigenvalues to
    1e-10, every residual within tol) with an exact or a Jacobi H-block preconditioner.  The
    tolerance 1e-8 sits above this pencil's residual floor (about 1e-9: eps ||A|| ||B|| / lambda_1
    with cond(A) = 1e3 and ||B|| = 50)."""
    Ahh, Bhh, nH, k = _random_composite(nH=60, k=5, seed=6)
    ahat, at, bt, bet = _precond_blocks(Ahh, Bhh, nH)
    AH, BH = Ahh[:nH, :nH], Bhh[:nH, :nH]
    inv = (lambda R: sla.solve(AH, R)) if precond == "exact" else (lambda R: R / np.diag(AH)[:, None])
    pen = gcg.AugPencil(AH, BH, at, bt, bet, inv)
    kk = 4
    X0 = np.random.default_rng(7).standard_normal((nH + k, kk))
    r = gcg.gcg_aug(pen, X0, 1e-8, s=3, max_iter=500, stall=50)
    At = np.block([[AH, np.zeros((nH, k))], [np.zeros((k, nH)), at]])
    Bt = np.block([[BH, bt], [bt.T, bet]])
    w = sla.eigh(At, Bt, eigvals_only=True)[:kk]
    assert r.converged
    np.testing.assert_allclose(r.lam, w, rtol=1e-10)
    assert np.all(r.res <= 1e-8)
    assert np.abs(r.X.T @ (Bt @ r.X) - np.eye(kk)).max() < 1e-10


def _pase_correction(n=16, levels=(16, 8, 4), nev=8, kseed=5, useed=1):
    kap = synth.kappa_field(3, n, kseed)
    H = multigrid.Hierarchy(3, list(levels), kap)
    U = pase.cholqr_m(synth.initial_vectors(H.A[0].shape[0], nev, useed), H.M[0])
    lam = np.einsum("ij,ij->j", U, H.A[0] @ U)
    for _ in range(3):   # a few dense corrections: a start block like the outer loop's
        W = pase.pcg(H, (H.M[0] @ U) * lam[None, :], U, 2)
        AHh, BHh = pase.composite(H, W)
        lam, Y = pase.small_solve(AHh, BHh, nev)
        NH = AHh.shape[0] - nev
        U = H.Pc @ Y[:NH] + W @ Y[NH:]
    W = pase.pcg(H, (H.M[0] @ U) * lam[None, :], U, 2)
    return H, W


def test_one_correction_equals_the_dense_composite_on_an_intermediate_level():
    """small_solve_precond_a with V_H = level 1 (8^3 of 16^3): eigenvalues equal dense eigh on the
    literal composite pencil of eq. Definition_Hh built on level 1 to 1e-11, and the new vectors
    span the same eigenvectors (|cos| = 1 to 1e-8 in the M inner product)."""
    H, W = _pase_correction()
    k = W.shape[1]
    c = 1
    Pc = pase.interp_from(H, c)
    A, M = H.A[0], H.M[0]
    AHh = np.block([[H.A[c].toarray(), Pc.T @ (A @ W)], [(Pc.T @ (A @ W)).T, W.T @ A @ W]])
    BHh = np.block([[H.M[c].toarray(), Pc.T @ (M @ W)], [(Pc.T @ (M @ W)).T, W.T @ M @ W]])
    w, Y = sla.eigh(0.5 * (AHh + AHh.T), 0.5 * (BHh + BHh.T), subset_by_index=[0, k - 1])
    nH = H.A[c].shape[0]
    Uref = Pc @ Y[:nH] + W @ Y[nH:]
    lam, U, r = pase.small_solve_precond_a(H, W, k, c, 1e-11, max_iter=300, stall=300)
    np.testing.assert_allclose(lam, w, rtol=1e-11)
    cos = np.abs(np.einsum("ij,ij->j", U, M @ Uref)) / np.sqrt(
        np.einsum("ij,ij->j", U, M @ U) * np.einsum("ij,ij->j", Uref, M @ Uref))
    assert np.abs(cos - 1).max() < 1e-8, cos


def test_vector_form_of_precond_a():
    """The complement W~ = W - I_H^h a_hat (the form the GPU path computes) is A-orthogonal to V_H and
    gives the same blocks: alpha~ = W~^T A W~, b~_h = I_h^H M W~, beta~ = W~^T M W~."""
    H, W = _pase_correction()
    c = 1
    Pc = pase.interp_from(H, c)
    A, M = H.A[0], H.M[0]
    a, b = Pc.T @ (A @ W), Pc.T @ (M @ W)
    lu = spla.splu(H.A[c].tocsc())
    ahat, at, bt, bet = gcg.precond_a(lu.solve, H.M[c], a, W.T @ A @ W, b, W.T @ M @ W)
    Wt = W - Pc @ ahat
    s = np.abs(W.T @ A @ W).max()
    assert np.abs(Pc.T @ (A @ Wt)).max() < 1e-12 * np.abs(a).max()
    assert np.abs(Wt.T @ (A @ Wt) - at).max() < 1e-11 * s
    assert np.abs(Pc.T @ (M @ Wt) - bt).max() < 1e-11 * np.abs(b).max()
    assert np.abs(Wt.T @ (M @ Wt) - bet).max() < 1e-11 * np.abs(W.T @ M @ W).max()


def test_pase_with_precond_a_matches_the_library_eigensolver():
    """solve(small="precond_a", coarse_level=1): 16^3 kappa field, nev 8 (4 guard pairs), V_H = 8^3:
    every eigenvalue within 1e-10 of ARPACK shift-invert on the assembled pencil, in fewer
    corrections than V_H = 4^3 takes."""
    kap = synth.kappa_field(3, 16, 5)
    H = multigrid.Hierarchy(3, [16, 8, 4], kap)
    nev, guard = 8, 4
    U0 = synth.initial_vectors(H.A[0].shape[0], nev + guard, 1)
    tl = lambda res: np.maximum(1e-11, 1e-2 * res)   # noqa: E731
    r = pase.solve(H, nev, 1e-10, U0, guard=guard, small="precond_a", coarse_level=1, aug_tol=tl)
    r4 = pase.solve(H, nev, 1e-10, U0, guard=guard, small="precond_a", coarse_level=2, aug_tol=tl)
    assert r.converged and r4.converged
    w = spla.eigsh(H.A[0].tocsc(), k=nev, M=H.M[0].tocsc(), sigma=0.0, which="LM",
                   return_eigenvectors=False, tol=1e-14)
    np.testing.assert_allclose(r.lam, np.sort(w), rtol=1e-10)
    np.testing.assert_allclose(r4.lam, np.sort(w), rtol=1e-10)
    assert r.iters < r4.iters, (r.iters, r4.iters)
