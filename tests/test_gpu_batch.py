"""GPU parity of the batch scheme (Alg. 7, eq. largest_component) through the C ABI.

Expected values: the oracle's batch scheme (``oracle.batch.solve_batch``) on the same hierarchy,
the library eigensolver's pairs of the fine pencil by index, and tests/golden/ for the tensor-coefficient
problem.  2D 64^2 kappa field with V_H = 32^2 (N_H = 961, composite pencils of 961 + k) and the 3D
tensor-coefficient problem on 32^3 with V_H = 16^3 (N_H = 3375).
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import batch, multigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Solver(*a, **kw):
    from paper_2502_04589_amd import Solver as S
    return S(*a, **kw)


@pytest.fixture(scope="module")
def problem2d():
    kap = synth.kappa_field(2, 64, 3)
    H = multigrid.Hierarchy(2, [64, 32], kap)
    w = np.sort(spla.eigsh(H.A[0].tocsc(), k=40, M=H.M[0].tocsc(), sigma=0.0, which="LM",
                           return_eigenvectors=False, tol=1e-14))
    return kap, H, w


def _check_pairs(s, lam, U, tol):
    AU, MU = s.apply(0, U)
    G = (U.T.contiguous() @ MU).cpu().numpy()
    assert np.max(np.abs(G - np.eye(U.shape[1]))) < 1e-9
    R = AU - MU * torch.from_numpy(lam).cuda()[None, :]
    res = torch.linalg.norm(R, dim=0) / (torch.from_numpy(np.abs(lam)).cuda() * torch.linalg.norm(MU, dim=0))
    assert float(res.max()) <= tol * 1.01


@pytest.mark.parametrize("first, nb", [(0, 10), (10, 10), (20, 7)])
def test_batch_matches_the_oracle(problem2d, first, nb):
    """Each batch (guard 4, the last one ragged) equals the oracle's batch scheme and the library
    eigensolver's pairs first .. first + nb - 1 to 1e-10, in about as many corrections."""
    kap, H, w = problem2d
    print(f"batch 2D 64^2 first {first} nb {nb}", flush=True)
    r = batch.solve_batch(H, first, nb, 1e-10, guard=4, max_outer=60)
    assert r.converged
    s = Solver(2, [64, 32], kap, nev_max=18, guard=4, max_outer=60)
    lam, U, rep = s.solve_batch(first, nb, 1e-10)
    np.testing.assert_allclose(lam, r.lam, rtol=1e-10)
    np.testing.assert_allclose(lam, w[first:first + nb], rtol=1e-10)
    _check_pairs(s, lam, U, 1e-10)
    assert abs(rep["outer_iters"] - r.iters) <= max(2, r.iters // 5), (rep["outer_iters"], r.iters)
    print(f"  gpu {rep['outer_iters']} corrections, oracle {r.iters}", flush=True)


def test_batches_cover_the_first_m_pairs(problem2d):
    """pase_solve_batches: 30 pairs in batches of 10 equal the library eigensolver's 30 smallest;
    the batches' blocks are M-orthonormal each (pairs of different batches are not
    orthogonalised against each other: Alg. 7 solves them independently)."""
    kap, H, w = problem2d
    s = Solver(2, [64, 32], kap, nev_max=18, guard=4, max_outer=60)
    lam, U, rep = s.solve_batches(30, 10, 1e-10)
    np.testing.assert_allclose(lam, w[:30], rtol=1e-10)
    assert rep["n_converged"] == 30 and np.all(rep["res"] <= 1e-10)
    for b in range(3):
        _check_pairs(s, lam[10 * b:10 * b + 10], U[:, 10 * b:10 * b + 10].contiguous(), 1e-10)
    print(f"batches: {rep['outer_iters']} corrections, {rep['t_solve_ms']:.1f} ms", flush=True)


def test_mixed_batch(problem2d):
    kap, H, w = problem2d
    s = Solver(2, [64, 32], kap, nev_max=18, guard=4, max_outer=60, precision="mixed")
    lam, U, rep = s.solve_batch(10, 10, 1e-9)
    np.testing.assert_allclose(lam, w[10:20], rtol=1e-8)
    _check_pairs(s, lam, U, 1e-9)


def test_3d_batches_match_golden():
    """The batch workload of the paper (Sec. 5, eq. general: tensor coefficient and reaction) on
    32^3 with V_H = 16^3: the 40 smallest pairs in two batches of 20 with 8 guard pairs, every
    eigenvalue (multiplicities included) within 1e-10 of the oracle's lowest eigenpairs of the
    assembled pencil."""
    d = np.load(os.path.join(GOLDEN, "general3d_32_k40.npz"))
    lam_ref, n = d["lam"], int(d["n"])
    T, phi = synth.general_coefficients(n)
    s = Solver(3, [32, 16], None, nev_max=36, guard=8, max_outer=80, tensor=T, reaction=phi)
    print("batch 3D general 32^3 / 16^3, 2 x 20", flush=True)
    lam, U, rep = s.solve_batches(40, 20, 1e-10)
    np.testing.assert_allclose(lam, lam_ref, rtol=1e-10)
    for b in range(2):
        _check_pairs(s, lam[20 * b:20 * b + 20], U[:, 20 * b:20 * b + 20].contiguous(), 1e-10)
    print(f"  {rep['outer_iters']} corrections, {rep['t_solve_ms']:.1f} ms", flush=True)


def test_batch_argument_checks(problem2d):
    from paper_2502_04589_amd.solver import PaseError
    kap, _, _ = problem2d
    s = Solver(2, [64, 32], kap, nev_max=12, guard=4)
    with pytest.raises(PaseError):
        s.solve_batch(10, 10, 1e-10)          # 4 + 10 + 4 columns > nev_max
    with pytest.raises(PaseError):
        s.solve_batch(955, 4, 1e-10)          # past the coarse space
    d = Solver(2, [64, 32], kap, nev_max=12, small_solver="dense")
    with pytest.raises(PaseError):
        d.solve_batch(0, 4, 1e-10)            # no coarse eigenbasis on the dense-only path
