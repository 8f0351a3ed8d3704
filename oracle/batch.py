"""Oracle: the batch scheme for many eigenpairs (Sec. "Batch scheme for computing plenty of
eigenpairs", Alg. 7 with the selection of eq. largest_component), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The wanted pairs m .. m + k - 1 of a batch are no longer the smallest of the augmented problem, so
each correction computes the n > k eigenpairs of the composite pencil closest to a shift theta and
keeps the k whose eigenfunctions have the largest components, in the B inner product, in the span
of the batch's current fine directions u_hat.  Steps of one batch, in the order of Alg. 7 step 3:

(a) start: the coarse eigenvectors m .. m + k - 1 of (A_H, B_H), interpolated; Lambda = their
    coarse eigenvalues;
(b) theta = the midpoint of the batch's first and last coarse eigenvalue;
(c) s CG steps on A_h u_hat = B_h u Lambda from u;
(d) the composite matrices of eq. Definition_Hh for the k columns of u_hat; the n eigenpairs
    closest to theta;
(e) the k of them with the largest ||Pi_h v||_b^2 (eq. largest_component), prolongated:
    u_hat = I_H^h u_H + u_hat gamma;
(f) s CG steps on A_h u = B_h u_hat Lambda from u_hat;
(g) repeat from (c) until every pair of the batch meets tol (R-B4).

Readings (also in the design doc's table):
* R-B1 step (b) prints theta as half the difference of the two coarse eigenvalues; the text before
  Alg. 7 defines it as their mean, which is what a shift inside the batch's window needs: theta =
  (lambda_{m,H} + lambda_{m+k-1,H}) / 2.
* R-B2 n (how many pairs closest to theta) is not fixed: n = min(2 k, N_H + k).
* R-B3 the eigenproblem of step (d) is solved on the composite pencil as it is (dense generalized
  eigensolver, all pairs, the n nearest theta taken); Alg. 6 (the harmonic Rayleigh-Ritz GCG_AUG)
  is one way to compute the same n pairs.
* R-B4 the convergence test of step (g) is taken on the pairs of step (e) (Ritz pairs of the
  augmented problem, B-orthonormal, the same test as the plain solve's); its residual
  B_h u Lambda - A_h u is also the start residual of the post-smoothing (f).  Lambda stays the
  eigenvalues of step (e) through (f) and the next (c), and the post-smoothed block is used as it
  is (both steps are linear in u and the composite space depends only on the span).
* R-B6 guard pairs, as in the library's plain solve: the block carries up to ``guard`` extra pairs
  below the batch (fewer for the first batches) and ``guard`` above it, started from the adjacent
  coarse eigenvectors; theta is the midpoint of the block's first and last coarse eigenvalue and
  only the batch's own pairs (positions lo .. lo + nb - 1 of the block's ascending Ritz values)
  decide convergence.  Without them a batch whose edge pair has a close neighbour outside it
  converges at the rate of that gap, or not at all.
* R-B5 the selection's ||Pi_h v||_b^2: with X the coordinates of the B-orthogonal projection of v
  onto span(u_hat), X beta = u_H^T b_h + gamma^T beta (the equality printed before eq.
  largest_component), and ||Pi_h v||_b^2 = X beta X^T; the k selected pairs are kept in ascending
  order of their eigenvalues.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .multigrid import Hierarchy
from .pase import pcg, residuals


def composite_parts(hier: Hierarchy, W):
    """Blocks of eq. Definition_Hh for the fine directions W (V_H = the coarsest level)."""
    A, M, P = hier.A[0], hier.M[0], hier.Pc
    AW, MW = A @ W, M @ W
    return (hier.A[hier.L].toarray(), P.T @ AW, W.T @ AW, hier.M[hier.L].toarray(), P.T @ MW, W.T @ MW)


def components(uH, gamma, b, beta):
    """||Pi_h v_i||_b^2 for v_i = I_H^h u_H[:, i] + u_hat gamma[:, i] (eq. largest_component): X beta =
    u_H^T b_h + gamma^T beta, then the diagonal of X beta X^T."""
    rhs = uH.T @ b + gamma.T @ beta
    X = sla.solve(beta, rhs.T, assume_a="pos").T
    return np.einsum("ij,jk,ik->i", X, beta, X)


def nearest(AHh, BHh, theta, n):
    """The n eigenpairs of (A_Hh, B_Hh) closest to theta (dense, all pairs computed), ascending."""
    w, Y = sla.eigh(AHh, BHh)
    idx = np.sort(np.argsort(np.abs(w - theta), kind="stable")[:n])
    return w[idx], Y[:, idx]


class BatchResult:
    def __init__(self, lam, U, iters, converged, res):
        self.lam, self.U, self.iters, self.converged, self.res = lam, U, iters, converged, res


def solve_batch(hier: Hierarchy, first, nb, tol, guard=0, s=2, max_outer=200, n=None) -> BatchResult:
    """Alg. 7 step 3 for the pairs first .. first + nb - 1, with up to ``guard`` guard pairs on each
    side of the batch (R-B6); returns the batch's pairs in ascending order."""
    A, M, P = hier.A[0], hier.M[0], hier.Pc
    AH = hier.A[hier.L].toarray()
    BH = hier.M[hier.L].toarray()
    NH = AH.shape[0]
    lamH, uH_all = sla.eigh(AH, BH)
    lo = min(guard, first)
    b0 = first - lo
    k = lo + nb + guard
    assert b0 + k <= NH
    if n is None:
        n = min(2 * k, NH + k)
    # (a), (b)
    U = P @ uH_all[:, b0:b0 + k]
    lam = lamH[b0:b0 + k].copy()
    theta = 0.5 * (lamH[b0] + lamH[b0 + k - 1])
    it = 0
    while True:
        # (c)
        W = pcg(hier, (M @ U) * lam[None, :], U, s)
        # (d)
        AH_, a, alpha, BH_, b, beta = composite_parts(hier, W)
        AHh = np.block([[AH_, a], [a.T, alpha]])
        BHh = np.block([[BH_, b], [b.T, beta]])
        w, Y = nearest(0.5 * (AHh + AHh.T), 0.5 * (BHh + BHh.T), theta, n)
        # (e)
        score = components(Y[:NH], Y[NH:], b, 0.5 * (beta + beta.T))
        keep = np.sort(np.argsort(-score, kind="stable")[:k])
        lam = w[keep]
        U = P @ Y[:NH, keep] + W @ Y[NH:, keep]
        it += 1
        # (g) on the pairs of step (e)
        res = residuals(A, M, U, lam)[0]
        want = np.arange(lo, lo + nb)
        if np.all(res[want] <= tol) or it >= max_outer:
            return BatchResult(lam[want], U[:, want], it, bool(np.all(res[want] <= tol)), res[want])
        # (f)
        U = pcg(hier, (M @ U) * lam[None, :], U, s)
