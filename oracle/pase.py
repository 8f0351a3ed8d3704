"""Oracle: the augmented subspace eigensolver outer loop (Alg. 1-3), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

One outer iteration, in the paper's order (Alg. 3):

* step 3 -- fine linear solves A_h u_hat = B_h u Lambda with initial guess
  u, one per eigenvector (eq. presoomthing); the paper uses (block) CG with
  a step limit, and the batch variant uses "s CG steps".  Reading taken here:
  per column (the columns are independent), preconditioned CG, exactly
  ``s`` steps, Fletcher-Reeves beta, V-cycle preconditioner (multigrid).
* step 4 -- composite matrices A_Hh = [[A_H, a_h], [a_h^T, alpha]],
  B_Hh = [[B_H, b_h], [b_h^T, beta]] with a_h = I_h^H A_h u_hat,
  alpha = u_hat^T A_h u_hat, b_h = I_h^H B_h u_hat, beta = u_hat^T B_h u_hat
  (eq. Definition_Hh).
* steps 5-6 -- the k smallest eigenpairs of the pencil (A_Hh, B_Hh) (eq.
  Augmented_GCGE), here by a dense LAPACK generalized eigensolver, and the
  prolongation u_hat <- I_H^h u_H + u_hat gamma (gamma multiplies from the
  right: u_hat is N x k, gamma is k x k).
* step 7 (post-smoothing solve) is optional (``post_smooth``); Alg. 1
  defines one correction step as one solve followed by one Rayleigh-Ritz.

Start (readings): the seeded U0 is B_h-orthonormalised by two passes of
Cholesky-QR and Lambda0 = diag(U0^T A_h U0); Alg. 3 steps 1-2 (coarse
eigenvectors as the start) are available with ``coarse_init=True``.

Stopping rule (Sec. 5): ||A x - lambda B x||_2 / |lambda| <= tol.  The
paper does not fix the scale of x; the primary test here is the
scale-invariant res_i = ||A u_i - lambda_i M u_i||_2 / (|lambda_i| ||M u_i||_2),
and the literal value with u^T M u = 1 is reported beside it.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import gcg_aug as gcg
from .multigrid import Hierarchy


def cholqr_m(U, M, passes=2):
    """M-orthonormalise the columns of U by repeated Cholesky-QR."""
    for _ in range(passes):
        G = U.T @ (M @ U)
        G = 0.5 * (G + G.T)
        L = np.linalg.cholesky(G)
        U = sla.solve_triangular(L, U.T, lower=True).T      # U L^{-T}
    return U


def residuals(A, M, U, lam):
    """Scale-invariant and literal residuals of the pairs (lam_i, U[:, i])."""
    AU = A @ U
    MU = M @ U
    R = AU - MU * lam[None, :]
    rn = np.linalg.norm(R, axis=0)
    res = rn / (np.abs(lam) * np.linalg.norm(MU, axis=0))
    # literal: u scaled to u^T M u = 1
    s = np.sqrt(np.einsum("ij,ij->j", U, MU))
    lit = rn / (s * np.abs(lam))
    return res, lit, R, MU


def pcg(hier: Hierarchy, rhs, x0, s):
    """s steps of V-cycle-preconditioned CG on A x = rhs, per column, from x0.

    Columns are independent: every scalar (alpha_j, beta_j) is per column.
    A step whose denominator is zero (converged column) leaves x unchanged.
    """
    A = hier.A[0]
    x = x0.copy()
    r = rhs - A @ x
    z = hier.vcycle(r)
    p = z.copy()
    rho = np.einsum("ij,ij->j", r, z)
    for j in range(s):
        q = A @ p
        pq = np.einsum("ij,ij->j", p, q)
        alpha = np.where(pq > 0, rho / np.where(pq > 0, pq, 1.0), 0.0)
        x += p * alpha
        r -= q * alpha
        if j + 1 < s:
            z = hier.vcycle(r)
            rho_new = np.einsum("ij,ij->j", r, z)
            beta = np.where(rho != 0, rho_new / np.where(rho != 0, rho, 1.0), 0.0)
            p = z + p * beta
            rho = rho_new
    return x


def composite(hier: Hierarchy, W):
    """Composite matrices A_Hh, B_Hh of eq. Definition_Hh (dense, symmetrised)."""
    A, M, P = hier.A[0], hier.M[0], hier.Pc
    AH = hier.A[hier.L].toarray()
    BH = hier.M[hier.L].toarray()
    AW = A @ W
    MW = M @ W
    a = P.T @ AW
    b = P.T @ MW
    alpha = W.T @ AW
    beta = W.T @ MW
    AHh = np.block([[AH, a], [a.T, alpha]])
    BHh = np.block([[BH, b], [b.T, beta]])
    return 0.5 * (AHh + AHh.T), 0.5 * (BHh + BHh.T)


def small_solve(AHh, BHh, k):
    """k smallest eigenpairs of (A_Hh, B_Hh); vectors are B_Hh-orthonormal."""
    vals, Y = sla.eigh(AHh, BHh, subset_by_index=[0, k - 1])
    return vals, Y


def small_solve_complement(hier: Hierarchy, W, k):
    """Cross-check form of steps 4-5: B-orthogonal complement of u_hat against V_H.

    W_perp = W - I_H^h B_H^{-1} I_h^H B_h W (the vector form of the PRECOND-B
    block factorisation, Sec. 4), then the pencil in the basis
    [I_H^h, W_perp] has b_h = 0.  Same span, so the same Ritz values.
    Returns (vals, U_new).
    """
    A, M, P = hier.A[0], hier.M[0], hier.Pc
    AH = hier.A[hier.L].toarray()
    BH = hier.M[hier.L].toarray()
    c = sla.solve(BH, P.T @ (M @ W), assume_a="pos")
    Wp = W - P @ c
    AW = A @ Wp
    MW = M @ Wp
    AHh = np.block([[AH, P.T @ AW], [(P.T @ AW).T, Wp.T @ AW]])
    BHh = np.block([[BH, P.T @ MW], [(P.T @ MW).T, Wp.T @ MW]])
    vals, Y = small_solve(0.5 * (AHh + AHh.T), 0.5 * (BHh + BHh.T), k)
    NH = AH.shape[0]
    return vals, P @ Y[:NH] + Wp @ Y[NH:]


def interp_from(hier: Hierarchy, c):
    """Composite interpolation I_H^h from level c to the fine level (product of P[1] .. P[c])."""
    Pc = None
    for l in range(1, c + 1):
        Pc = hier.P[l] if Pc is None else (Pc @ hier.P[l]).tocsr()
    return Pc


def small_solve_precond_a(hier: Hierarchy, W, k, c, tol, s=2, max_iter=200, stall=4):
    """Steps 4-6 with V_H = level c and the augmented problem solved by PRECOND-A and GCG_AUG
    (Sec. 4, Alg. 5 with Alg. 4): the composite blocks of eq. (Definition_Hh) on level c, then
    ``gcg_aug.solve_augmented`` (the coarse V-cycle below level c preconditions its linear
    solves), then the prolongation u = I_H^h u_H + u_hat gamma.  Returns (vals, U_new, GcgResult)."""
    A, M = hier.A[0], hier.M[0]
    Pc = interp_from(hier, c)
    AW = A @ W
    MW = M @ W
    a = Pc.T @ AW
    b = Pc.T @ MW
    alpha = 0.5 * (W.T @ AW + (W.T @ AW).T)
    beta = 0.5 * (W.T @ MW + (W.T @ MW).T)
    lam, uH, g, r = gcg.solve_augmented(hier.A[c], hier.M[c], a, alpha, b, beta, k, tol,
                                        lambda R: hier.vcycle(R, l=c), s=s, max_iter=max_iter,
                                        stall=stall)
    return lam, Pc @ uH + W @ g, r


class Result:
    def __init__(self):
        self.lam = None
        self.U = None
        self.iters = 0
        self.converged = False
        self.res = None
        self.res_literal = None
        self.ritz_history = []
        self.res_history = []
        self.aug_iters = []          # GCG_AUG iterations per correction (small="precond_a")


def solve(hier: Hierarchy, nev, tol, U0=None, s=2, max_outer=500, post_smooth=False,
          coarse_init=False, callback=None, guard=0, small="dense", coarse_level=None,
          aug_tol=1e-12, aug_s=2) -> Result:
    """Run the augmented subspace method until every pair meets ``tol``.

    ``U0``: N x (nev + guard) start (seeded, see ``synth``), ignored with coarse_init.
    ``max_outer``: number of corrections allowed; the residual test is made
    before each correction and once more at the end.
    ``guard`` (reading; the algorithms iterate exactly nev vectors): the block
    carries nev + guard pairs, every step treats them alike, and only the nev
    smallest decide convergence and are returned.
    ``small``: "dense" solves the augmented problem of step 5 with V_H = the
    coarsest level by a dense generalized eigensolver; "precond_a" takes
    V_H = level ``coarse_level`` (default the coarsest) and solves it by
    PRECOND-A and GCG_AUG (Sec. 4) to the relative residual ``aug_tol`` (a
    scalar, or a function of the outer residuals giving one value per pair),
    with ``aug_s`` CG steps in GCG_AUG's linear solves.
    """
    want = nev
    nev = nev + guard
    A, M, P = hier.A[0], hier.M[0], hier.Pc
    if coarse_init:
        # Alg. 3 steps 1-2: coarse eigenpairs, interpolated
        AH = hier.A[hier.L].toarray()
        BH = hier.M[hier.L].toarray()
        lam, uH = sla.eigh(AH, BH, subset_by_index=[0, nev - 1])
        U = cholqr_m(P @ uH, M)
        lam = np.einsum("ij,ij->j", U, A @ U)
    else:
        U = cholqr_m(np.array(U0, dtype=np.float64, copy=True), M)
        lam = np.einsum("ij,ij->j", U, A @ U)
    out = Result()
    out.ritz_history.append(lam.copy())
    it = 0
    while True:
        res, lit, _, MU = residuals(A, M, U, lam)
        out.res_history.append(res.copy())
        if np.all(res[:want] <= tol) or it >= max_outer:
            out.converged = bool(np.all(res[:want] <= tol))
            break
        # step 3: fine solves A w = M u lambda, x0 = u
        W = pcg(hier, MU * lam[None, :], U, s)
        # steps 4-6
        if small == "precond_a":
            c = hier.L if coarse_level is None else coarse_level
            tl = aug_tol(res) if callable(aug_tol) else aug_tol
            lam, U, gr = small_solve_precond_a(hier, W, nev, c, tl, s=aug_s)
            out.aug_iters.append(gr.iters)
        else:
            AHh, BHh = composite(hier, W)
            lam, Y = small_solve(AHh, BHh, nev)
            NH = AHh.shape[0] - nev
            U = P @ Y[:NH] + W @ Y[NH:]
        if post_smooth:
            # step 7: A u = M u_hat Lambda from u_hat, then a Rayleigh quotient
            U = pcg(hier, (M @ U) * lam[None, :], U, s)
            U = cholqr_m(U, M)
            lam = np.einsum("ij,ij->j", U, A @ U)
        it += 1
        out.ritz_history.append(lam.copy())
        if callback is not None:
            callback(it, lam, U)
    out.lam = lam[:want]
    out.U = U[:, :want]
    out.iters = it
    out.res = res[:want]
    out.res_literal = lit[:want]
    return out
