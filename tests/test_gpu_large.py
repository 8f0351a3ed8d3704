"""GPU parity of the large-coarse-space path (N_H = 15^3 = 3375 of a 16^3 coarse mesh).

Covers what a coarse space of thousands of nodes needs beyond one workgroup: the blocked
Cholesky / triangular inverse and the diagonalisation of C0 in setup, the grid-wide dense
eigensolver (setup and the dense path of the augmented eigenproblem), the structured solver
with rows of Gt streamed from L2 (k > 64), the MFMA GEMM of the coarse products, and the
coarse start of Alg. 3 steps 1-2.  Expected eigenvalues come from tests/golden/ (written by
tests/golden/make_golden.py, which calls only oracle.reference) or from numpy/scipy dense
solvers on the host.  All calls go through the C ABI.
"""
import os

import numpy as np
import pytest

import synth
from tests.closed_form import q1_laplace_eigs

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


def golden(name):
    d = np.load(os.path.join(GOLDEN, name + ".npz"))
    return d["lam"], int(d["n"]), int(d["kappa_seed"])


def _check_pairs(s, lam, U, kappa, dim, n, tol):
    """U^T M U = I and every residual within tol (explicit operator, through the C ABI)."""
    AU, MU = s.apply(0, U)
    G = (U.T @ MU).cpu().numpy()
    assert np.max(np.abs(G - np.eye(U.shape[1]))) < 1e-11
    R = AU - MU * torch.from_numpy(lam).cuda()[None, :]
    res = torch.linalg.norm(R, dim=0) / (torch.from_numpy(np.abs(lam)).cuda() * torch.linalg.norm(MU, dim=0))
    assert float(res.max()) <= tol * 1.01


@pytest.mark.parametrize("n, k, spectrum", [(700, 40, "random"), (3475, 112, "random"), (3475, 100, "clustered")])
def test_large_dense_eigensolver(n, k, spectrum):
    """The grid-wide dense eigensolver (pase_small_eig above 512) against numpy.linalg.eigh."""
    print(f"large dense eig n={n} k={k} {spectrum}", flush=True)
    s = Solver(3, [32, 16], nev_max=112)      # N_H + K = 3487 >= n
    assert s.small_eig_max_n() >= n
    rng = np.random.default_rng(n + k)
    if spectrum == "random":
        A = rng.standard_normal((n, n))
        T = (A + A.T) / 2
    else:
        # exact multiplicities (the coarse Laplacian of kappa = 1 has 3- and 6-fold clusters)
        w = np.repeat(np.arange(1, n // 4 + 2, dtype=np.float64), 4)[:n]
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        T = (Q * w) @ Q.T
        T = (T + T.T) / 2
    wref = np.linalg.eigvalsh(T)[:k]
    w, V = s.small_eig(torch.from_numpy(T).cuda(), k)
    scale = np.abs(wref).max()
    assert np.max(np.abs(w - wref)) < 1e-12 * max(scale, 1.0) * 10
    Vh = V.cpu().numpy()
    assert np.max(np.abs(Vh.T @ Vh - np.eye(k))) < 1e-12
    assert np.max(np.abs(T @ Vh - Vh * w[None, :])) < 1e-11 * np.abs(T).max() * np.sqrt(n)


@pytest.mark.parametrize("small_solver, start", [("auto", "given"), ("dense", "given"), ("auto", "coarse")])
def test_coarse_3375_solve_matches_golden(small_solver, start):
    """32^3 fine mesh, V_H = 16^3 (N_H = 3375), kappa field, 40 pairs to 1e-10: every eigenvalue within
    1e-10 (relative) of the oracle's lowest eigenpairs of the assembled pencil."""
    lam_ref, n, seed = golden("kappa3d_32_s5_k40")
    kap = synth.kappa_field(3, n, seed)
    nev = 40
    print(f"coarse-3375 solve {small_solver} {start}", flush=True)
    s = Solver(3, [n, n // 2], kap, nev_max=nev, small_solver=small_solver, guard=8, start=start)
    U0 = None if start == "coarse" else torch.from_numpy(synth.initial_vectors(s.N[0], nev, 3)).cuda()
    lam, U, rep = s.solve(nev, 1e-10, U0)
    np.testing.assert_allclose(lam, lam_ref[:nev], rtol=1e-10)
    _check_pairs(s, lam, U, kap, 3, n, 1e-10)
    if small_solver == "auto":
        assert rep["small_fast_iters"] > 0
    print(f"  iters {rep['outer_iters']} structured {rep['small_fast_iters']} paths {rep['small_path'].tolist()}",
          flush=True)


def test_coarse_3375_constant_kappa_closed_form():
    """kappa = 1: closed-form Q1 eigenvalues (the constant-coefficient stencil on every level)."""
    nev = 20
    s = Solver(3, [32, 16], None, nev_max=nev, guard=8, start="coarse")
    lam, U, rep = s.solve(nev, 1e-10, None)
    np.testing.assert_allclose(lam, q1_laplace_eigs(3, 32, nev), rtol=1e-10)


@pytest.mark.parametrize("precision, nev, rtol", [("fp64", 100, 1e-10), ("mixed", 100, 1e-8)])
def test_coarse_3375_nev100_64cubed(precision, nev, rtol):
    """64^3 fine mesh, V_H = 16^3 (N_H = 3375), kappa field, nev 100 (block of 128): the plain form within
    1e-10 and the mixed form within 1e-8 of the oracle's eigenvalues."""
    lam_ref, n, seed = golden("kappa3d_64_s21_k120")
    kap = synth.kappa_field(3, n, seed)
    print(f"64^3 N_H=3375 nev {nev} {precision}", flush=True)
    s = Solver(3, [n, n // 2, n // 4], kap, nev_max=nev, precision=precision, guard=28, start="coarse")
    lam, U, rep = s.solve(nev, 1e-9, None)
    np.testing.assert_allclose(lam, lam_ref[:nev], rtol=rtol)
    _check_pairs(s, lam, U, kap, 3, n, 1e-9)
    print(f"  iters {rep['outer_iters']} structured {rep['small_fast_iters']} t {rep['t_solve_ms']:.0f} ms "
          f"lowprec {rep['lowprec_projection_iters']}", flush=True)


@pytest.mark.parametrize("precision, rtol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_coarse_3375_nev100_32cubed(precision, rtol):
    """32^3 fine mesh, V_H = 16^3 (N_H = 3375), kappa field, nev 100 with 28 guard pairs (block of 128,
    the structured solver's and the split-BF16 Gram's largest k): every eigenvalue within 1e-10 (plain)
    or 1e-8 (mixed) of the oracle's lowest eigenpairs of the assembled pencil."""
    lam_ref, n, seed = golden("kappa3d_32_s7_k120")
    kap = synth.kappa_field(3, n, seed)
    nev = 100
    print(f"32^3 N_H=3375 nev {nev} {precision}", flush=True)
    s = Solver(3, [n, n // 2], kap, nev_max=nev, precision=precision, guard=28, start="coarse")
    lam, U, rep = s.solve(nev, 1e-9, None)
    np.testing.assert_allclose(lam, lam_ref[:nev], rtol=rtol)
    _check_pairs(s, lam, U, kap, 3, n, 1e-9)
    if precision == "mixed":
        assert rep["lowprec_projection_iters"] > 0
    print(f"  iters {rep['outer_iters']} structured {rep['small_fast_iters']} lowprec "
          f"{rep['lowprec_projection_iters']}", flush=True)
