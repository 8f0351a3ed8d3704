"""Oracle: PRECOND-A and the GCG_AUG eigensolver of the augmented problem (Sec. 4), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The augmented problem of Alg. 3 step 5, written in the basis [I_H^h, u_hat] of
V_H + span(u_hat) (eq. Eigenvalue_Problem_AHh), couples the coarse block A_H
with the k fine directions through a_h = I_h^H A_h u_hat.  Sec. 4 removes that
coupling from the left matrix with the block factorisation of eq.
(Transformation_0): with a_hat = A_H^{-1} a_h the pencil becomes eq.
(Eigen_Problem_Hh_2), whose left matrix is diag(A_H, alpha~) and whose right
matrix keeps a coupling b~_h.  Alg. 5 transforms, solves the transformed pencil
with GCG_AUG (Alg. 4) and transforms the eigenvectors back.

* ``block_factors`` -- the three factors of eq. (Transformation_0).
* ``precond_a``     -- Alg. 5 step 1: a_hat and the blocks alpha~, b~_h, beta~,
                       from the formulas printed with eq. (Eigen_Problem_Hh_2).
* ``AugPencil``     -- the transformed pencil applied matrix-free.
* ``gcg_aug``       -- Alg. 4 on a pencil given as operators.
* ``solve_augmented`` -- Alg. 5 (steps 1-3) for one correction of the outer loop.

Readings of points the paper leaves open (each also in the function that takes it):

* R-G1 shift: step 2 of Alg. 4 asks for a shift mu that keeps A - mu B SPD; the
  left matrix of eq. (Eigen_Problem_Hh_2) is SPD already, so mu = 0.
* R-G2 linear solver of step 2: ``s`` steps of preconditioned CG per column from
  the initial value X, on the full left operator; the preconditioner is the
  block-diagonal inverse diag(V-cycle on A_H, alpha~^{-1}): one V-cycle of the
  coarse hierarchy below V_H on the H block, the exact inverse of the k x k
  block alpha~ on the other.  Because the left matrix of eq.
  (Eigen_Problem_Hh_2) is block-diagonal this is what PRECOND-A buys: the
  solve splits into a coarse-grid problem and a k x k one.
* R-G3 orthogonalisation of step 3: Gram-Schmidt in the B inner product, two
  passes, columns in the order X, P, W; a column whose B-norm after the passes
  is below 1e-10 of its norm before them is dropped (the paper does not say
  how a numerically dependent column is treated).
* R-G4 active columns: W and P are formed for the pairs that have not yet met
  the tolerance only (converged pairs stay in X, as in GCGE's practice).
* R-G5 step 6 "P = X_new minus X": the part of X_new = V C that the P and W
  blocks contribute, P = [P, W] C_{PW}.
* R-G6 convergence of step 5: res_j = ||A x_j - l_j B x_j|| / (|l_j| ||B x_j||)
  <= tol_j for every column of the block (a per-column tolerance may be given);
  the test is also made on the Rayleigh-Ritz pairs of step 1, so a start block
  that already meets it costs no iteration.  The iteration also stops when the
  largest residual of the unconverged pairs has not reached a new low for
  ``stall`` iterations: the residuals of the transformed pencil stagnate at its
  attainable accuracy (about 1e-11 to 1e-10 relative on the Q1 pencils here,
  set by the condition of A_H and by the cancellation in alpha~ and beta~).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def _sym(a):
    return 0.5 * (a + a.T)


def block_factors(AH, a, alpha):
    """Left, middle and right factors of eq. (Transformation_0) (dense):
    [[A_H, a], [a^T, alpha]] = [[I, 0], [a^T A_H^{-1}, I]] diag(A_H, alpha - a^T A_H^{-1} a) [[I, A_H^{-1} a], [0, I]]."""
    AH = np.asarray(AH, dtype=np.float64)
    nH, k = a.shape
    ahat = np.linalg.solve(AH, a)
    Lf = np.block([[np.eye(nH), np.zeros((nH, k))], [ahat.T, np.eye(k)]])
    D = np.block([[AH, np.zeros((nH, k))], [np.zeros((k, nH)), alpha - a.T @ ahat]])
    Rf = np.block([[np.eye(nH), ahat], [np.zeros((k, nH)), np.eye(k)]])
    return Lf, D, Rf


def precond_a(AH_solve, BH, a, alpha, b, beta):
    """Alg. 5 step 1: a_hat = A_H^{-1} a_h, then (formulas printed with eq. Eigen_Problem_Hh_2)
    alpha~ = alpha - a_hat^T a_h, b~_h = b_h - B_H a_hat,
    beta~ = beta - b_h^T a_hat - a_hat^T b_h + a_hat^T B_H a_hat.
    ``AH_solve`` applies A_H^{-1} to a block; ``BH`` is sparse or dense."""
    ahat = AH_solve(a)
    alpha_t = alpha - ahat.T @ a
    b_t = b - BH @ ahat
    beta_t = beta - b.T @ ahat - ahat.T @ b + ahat.T @ (BH @ ahat)
    return ahat, _sym(alpha_t), b_t, _sym(beta_t)


class AugPencil:
    """The pencil of eq. (Eigen_Problem_Hh_2) on vectors y = [y_H ; y_g] (N_H + k rows):
    A~ y = [A_H y_H ; alpha~ y_g],  B~ y = [B_H y_H + b~ y_g ; b~^T y_H + beta~ y_g].

    ``vcycle_H`` approximates A_H^{-1} on a block (the preconditioner of R-G2)."""

    def __init__(self, AH, BH, alpha_t, b_t, beta_t, vcycle_H):
        self.AH, self.BH = AH, BH
        self.alpha_t, self.b_t, self.beta_t = alpha_t, b_t, beta_t
        self.nH = AH.shape[0]
        self.k = alpha_t.shape[0]
        self.vcycle_H = vcycle_H
        self.alpha_chol = sla.cho_factor(alpha_t, lower=True)

    def split(self, Y):
        return Y[: self.nH], Y[self.nH:]

    def A(self, Y):
        yH, yg = self.split(Y)
        return np.vstack([self.AH @ yH, self.alpha_t @ yg])

    def B(self, Y):
        yH, yg = self.split(Y)
        return np.vstack([self.BH @ yH + self.b_t @ yg, self.b_t.T @ yH + self.beta_t @ yg])

    def precond(self, R):
        """diag(V-cycle on A_H, alpha~^{-1}) (R-G2)."""
        rH, rg = self.split(R)
        return np.vstack([self.vcycle_H(rH), sla.cho_solve(self.alpha_chol, rg)])


def _pcg(pencil, F, X0, s):
    """s steps of preconditioned CG on A~ w = F per column from X0 (R-G2)."""
    x = X0.copy()
    r = F - pencil.A(x)
    z = pencil.precond(r)
    p = z.copy()
    rho = np.einsum("ij,ij->j", r, z)
    for j in range(s):
        q = pencil.A(p)
        pq = np.einsum("ij,ij->j", p, q)
        al = np.where(pq > 0, rho / np.where(pq > 0, pq, 1.0), 0.0)
        x += p * al
        r -= q * al
        if j + 1 < s:
            z = pencil.precond(r)
            rho_new = np.einsum("ij,ij->j", r, z)
            beta = np.where(rho != 0, rho_new / np.where(rho != 0, rho, 1.0), 0.0)
            p = z + p * beta
            rho = rho_new
    return x


def _b_orthonormalise(Bop, X, Y, drop=1e-10):
    """Columns of Y made B-orthonormal against the B-orthonormal X and among themselves by
    Gram-Schmidt, two passes; numerically dependent columns are dropped (R-G3)."""
    kept = []
    for j in range(Y.shape[1]):
        v = Y[:, j].copy()
        n0 = np.sqrt(max(float(v @ Bop(v[:, None])[:, 0]), 0.0))
        if n0 == 0.0:
            continue
        for _ in range(2):
            for Q in (X, np.column_stack(kept) if kept else None):
                if Q is None or Q.shape[1] == 0:
                    continue
                v = v - Q @ (Q.T @ Bop(v[:, None])[:, 0])
        n1 = np.sqrt(max(float(v @ Bop(v[:, None])[:, 0]), 0.0))
        if n1 <= drop * n0:
            continue
        kept.append(v / n1)
    return np.column_stack(kept) if kept else np.zeros((Y.shape[0], 0))


def _rayleigh_ritz(pencil, V, k):
    """Step 4 on a B-orthonormal V: the k smallest eigenpairs of V^T A V."""
    G = _sym(V.T @ pencil.A(V))
    lam, C = np.linalg.eigh(G)
    return lam[:k], C[:, :k]


def _residuals(pencil, X, lam):
    AX = pencil.A(X)
    BX = pencil.B(X)
    R = AX - BX * lam[None, :]
    return np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(BX, axis=0))


class GcgResult:
    def __init__(self, lam, X, iters, res, converged):
        self.lam, self.X, self.iters, self.res, self.converged = lam, X, iters, res, converged


def gcg_aug(pencil: AugPencil, X0, tol, s=2, max_iter=200, stall=4) -> GcgResult:
    """Alg. 4 for the k = X0.shape[1] smallest eigenpairs of (A~, B~).

    ``tol``: scalar or one value per column; ``stall``: the stagnation stop (R-G6)."""
    k = X0.shape[1]
    tolv = np.broadcast_to(np.asarray(tol, dtype=np.float64), (k,))
    best, since = np.inf, 0
    # step 1: Rayleigh-Ritz on the start block
    X = _b_orthonormalise(pencil.B, np.zeros((X0.shape[0], 0)), X0, drop=0.0)
    lam, C = _rayleigh_ritz(pencil, X, k)
    X = X @ C
    P = np.zeros((X.shape[0], 0))
    it = 0
    while True:
        res = _residuals(pencil, X, lam)
        act = np.flatnonzero(res > tolv)
        if act.size:
            worst = float(res[act].max())
            best, since = (worst, 0) if worst < best else (best, since + 1)
        if act.size == 0 or it >= max_iter or since >= stall:
            return GcgResult(lam, X, it, res, act.size == 0)
        # step 2: W = A~^{-1} (B~ X Lambda) approximately, from X, for the active pairs (R-G1, R-G2, R-G4)
        Xa = X[:, act]
        W = _pcg(pencil, pencil.B(Xa) * lam[act][None, :], Xa, s)
        # step 3: V = [X, P, W], B-orthonormal
        Ynew = _b_orthonormalise(pencil.B, X, np.hstack([P, W]))
        V = np.hstack([X, Ynew])
        # step 4: Rayleigh-Ritz
        lam, C = _rayleigh_ritz(pencil, V, k)
        X_new = V @ C
        # step 6: P = the part of X_new that the P and W blocks contribute (R-G5), for the active pairs
        P = (Ynew @ C[k:, :])[:, act] if Ynew.shape[1] else np.zeros((X.shape[0], 0))
        X = X_new
        it += 1


def solve_augmented(AH, BH, a, alpha, b, beta, k, tol, vcycle_H, AH_solve=None, s=2, max_iter=200,
                    start=None, stall=4):
    """Alg. 5 for eq. (Eigenvalue_Problem_AHh): returns (lam, u_H, gamma, GcgResult).

    Step 1 transforms (``AH_solve`` defaults to a sparse LU of A_H), step 2 runs GCG_AUG on
    eq. (Eigen_Problem_Hh_2) from ``start`` (transformed coordinates; default [a_hat ; I]: the
    fine directions themselves, whose coordinates in the original basis are [0 ; I]), and step 3
    maps the eigenvectors back: u_H = u~_H - a_hat gamma~, gamma = gamma~."""
    if AH_solve is None:
        lu = spla.splu(AH.tocsc())
        AH_solve = lu.solve
    ahat, alpha_t, b_t, beta_t = precond_a(AH_solve, BH, a, alpha, b, beta)
    pencil = AugPencil(AH, BH, alpha_t, b_t, beta_t, vcycle_H)
    if start is None:
        start = np.vstack([ahat, np.eye(a.shape[1])])[:, :k]
    r = gcg_aug(pencil, start, tol, s=s, max_iter=max_iter, stall=stall)
    nH = AH.shape[0]
    uH_t, g_t = r.X[:nH], r.X[nH:]
    return r.lam, uH_t - ahat @ g_t, g_t, r
