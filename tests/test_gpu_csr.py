"""GPU parity of the algebraic input (CSR level operators and transfers) through the C ABI.

Alg. 3's "Require" is given as matrices: per level the pencil (A_l, M_l) and the transfers P_l, R_l
as device CSR (``pase_hierarchy_csr``), applied by the CSR multi-vector kernels.  Expected values:
the oracle's grid hierarchy (``oracle.multigrid``), the oracle's algebraic hierarchy of unsmoothed
aggregation (``tests/test_csr_oracle.aggregation_hierarchy``) and its outer loop, and tests/golden/.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import multigrid, pase as opase
from tests.test_csr_oracle import aggregation_hierarchy

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


def to_scipy(c):
    return sp.csr_matrix((c.val.cpu().numpy(), c.colind.cpu().numpy(), c.rowptr.cpu().numpy()),
                         shape=(c.rows, c.cols))


def hierarchy_of(H):
    """The oracle hierarchy as the hierarchy= argument (scipy matrices, copied to the device)."""
    L = len(H.A)
    return {"A": list(H.A), "M": list(H.M), "P": [None] + [H.P[l] for l in range(1, L)],
            "R": [None] + [H.P[l].T.tocsr() for l in range(1, L)]}


def _check_pairs(s, lam, U, tol):
    AU, MU = s.apply(0, U)
    G = (U.T.contiguous() @ MU).cpu().numpy()
    assert np.max(np.abs(G - np.eye(U.shape[1]))) < 1e-11
    R = AU - MU * torch.from_numpy(lam).cuda()[None, :]
    res = torch.linalg.norm(R, dim=0) / (torch.from_numpy(np.abs(lam)).cuda() * torch.linalg.norm(MU, dim=0))
    assert float(res.max()) <= tol * 1.01


@pytest.mark.parametrize("dim, levels", [(3, [16, 8, 4]), (2, [32, 16, 8])])
def test_exported_hierarchy_equals_the_oracle(dim, levels):
    """pase_export_csr: A_l, M_l, P_l, R_l of a grid handle equal the oracle's assembled / Galerkin
    matrices and interpolations (explicit zeros dropped) to 1e-13."""
    kap = synth.kappa_field(dim, levels[0], 3)
    H = multigrid.Hierarchy(dim, levels, kap)
    s = Solver(dim, levels, kap, nev_max=4)
    for l in range(len(levels)):
        for which, ref in (("A", H.A[l]), ("M", H.M[l])) + ((("P", H.P[l]), ("R", H.P[l].T)) if l else ()):
            X = to_scipy(s.export_csr(l, which))
            X.eliminate_zeros()
            assert X.shape == ref.shape, (l, which)
            err = abs(X - ref).max() / abs(ref).max()
            assert err < 1e-13, (l, which, err)


def test_csr_operators_and_transfers_match_the_grid_kernels():
    """Through the algebraic input the library applies the same operators: A, M on every level,
    restriction, prolongation and the V-cycle equal the grid handle's to 1e-13."""
    kap = synth.kappa_field(3, 16, 5)
    g = Solver(3, [16, 8, 4], kap, nev_max=8)
    c = Solver(hierarchy=g.export_hierarchy(), dim=None, levels=None, nev_max=8)
    rng = np.random.default_rng(2)
    for l in range(3):
        X = torch.from_numpy(rng.standard_normal((g.N[l], 7))).cuda()
        for a, b in zip(g.apply(l, X), c.apply(l, X)):
            assert float((a - b).abs().max() / a.abs().max()) < 1e-13
    X = torch.from_numpy(rng.standard_normal((g.N[0], 5))).cuda()
    assert float((g.restrict(X) - c.restrict(X)).abs().max() / g.restrict(X).abs().max()) < 1e-13
    Y = torch.from_numpy(rng.standard_normal((g.N[-1], 5))).cuda()
    assert float((g.prolong(Y) - c.prolong(Y)).abs().max() / g.prolong(Y).abs().max()) < 1e-13
    assert float((g.vcycle(X) - c.vcycle(X)).abs().max() / g.vcycle(X).abs().max()) < 1e-12


@pytest.mark.parametrize("precision, small_solver, rtol", [("fp64", "auto", 1e-10), ("mixed", "auto", 1e-8),
                                                            ("fp64", "gcg", 1e-10)])
def test_csr_solve_of_the_grid_problem_matches_golden(precision, small_solver, rtol):
    """32^3 kappa field given as a CSR hierarchy (exported from the grid handle), V_H = 8^3, nev 40:
    every eigenvalue within rtol of the oracle's lowest eigenpairs of the assembled pencil."""
    d = np.load(os.path.join(GOLDEN, "kappa3d_32_s5_k40.npz"))
    lam_ref, n, seed = d["lam"], int(d["n"]), int(d["kappa_seed"])
    kap = synth.kappa_field(3, n, seed)
    g = Solver(3, [32, 16, 8], kap, nev_max=4)
    hier = g.export_hierarchy()
    del g
    kw = dict(small_solver="gcg", coarse_level=1) if small_solver == "gcg" else {}
    print(f"csr 32^3 {precision} {small_solver}", flush=True)
    s = Solver(hierarchy=hier, dim=None, levels=None, nev_max=40, guard=8, precision=precision, **kw)
    tol = 1e-10 if precision == "fp64" else 1e-9
    lam, U, rep = s.solve(40, tol, None)
    np.testing.assert_allclose(lam, lam_ref, rtol=rtol)
    _check_pairs(s, lam, U, tol)
    print(f"  {rep['outer_iters']} corrections", flush=True)


def test_aggregation_hierarchy_matches_the_oracle():
    """A non-nested algebraic coarse space (unsmoothed aggregation, 3 levels, 16^3 kappa field):
    the GPU solve and the oracle's outer loop on the same matrices reach ARPACK's eigenvalues to
    1e-10, in about the same number of corrections."""
    kap = synth.kappa_field(3, 16, 4)
    H = aggregation_hierarchy(16, kap)
    nev = 6
    U0 = synth.initial_vectors(H.A[0].shape[0], nev, 3)
    r = opase.solve(H, nev, 1e-10, U0)
    w = np.sort(spla.eigsh(H.A[0].tocsc(), k=nev, M=H.M[0].tocsc(), sigma=0.0, which="LM",
                           return_eigenvectors=False, tol=1e-14))
    s = Solver(hierarchy=hierarchy_of(H), dim=None, levels=None, nev_max=nev, locking=False)
    lam, U, rep = s.solve(nev, 1e-10, torch.from_numpy(U0).cuda())
    np.testing.assert_allclose(lam, w, rtol=1e-10)
    np.testing.assert_allclose(r.lam, w, rtol=1e-10)
    _check_pairs(s, lam, U, 1e-10)
    assert abs(rep["outer_iters"] - r.iters) <= max(2, r.iters // 10), (rep["outer_iters"], r.iters)
    print(f"aggregation: gpu {rep['outer_iters']} corrections, oracle {r.iters}", flush=True)


def test_csr_argument_checks():
    from paper_2502_04589_amd.solver import PaseError
    kap = synth.kappa_field(3, 8, 1)
    g = Solver(3, [8, 4], kap, nev_max=2)
    hier = g.export_hierarchy()
    bad = dict(hier)
    bad["R"] = [None, hier["P"][1]]          # R must be N_1 x N_0
    with pytest.raises(PaseError):
        Solver(hierarchy=bad, dim=None, levels=None, nev_max=2)
    with pytest.raises(PaseError):
        Solver(hierarchy=hier, dim=None, levels=None, nev_max=2, precision="learned")
    c = Solver(hierarchy=hier, dim=None, levels=None, nev_max=2)
    with pytest.raises(PaseError):
        c.export_csr(0, "A")
