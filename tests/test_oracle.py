"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every test here runs on the CPU (no GPU marker).  Each pin is chosen so that a
plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand) fails at least one of them; ``test_planted_*`` check
that claim for a few slips by planting them in the oracle.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import fem, multigrid, pase
from tests.closed_form import q1_laplace_eigs


# ---------------------------------------------------------------- elements
def _tensor_element(dim, h):
    """Analytic Q1 element matrices as tensor products of the 1D ones."""
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    nv = 2 ** dim
    K = np.zeros((nv, nv))
    M = np.ones((nv, nv))
    for a, b in itertools.product(range(nv), repeat=2):
        bits_a = [(a >> d) & 1 for d in range(dim)]
        bits_b = [(b >> d) & 1 for d in range(dim)]
        for d in range(dim):
            t = k1[bits_a[d], bits_b[d]]
            for e in range(dim):
                if e != d:
                    t *= m1[bits_a[e], bits_b[e]]
            K[a, b] += t
        for d in range(dim):
            M[a, b] *= m1[bits_a[d], bits_b[d]]
    return K, M


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matrices_match_tensor_closed_form(dim):
    h = 0.37
    K, M = fem.element_matrices(dim, h)
    Kt, Mt = _tensor_element(dim, h)
    np.testing.assert_allclose(K, Kt, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(M, Mt, rtol=1e-13, atol=1e-15)
    # textbook facts: constants are in the stiffness null space; mass integrates to the volume
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-13)
    assert abs(M.sum() - h ** dim) < 1e-14


def test_2d_stiffness_entries_textbook_values():
    """Unit-square Q1 stiffness: diagonal 2/3, edge neighbour -1/6, opposite corner -1/3."""
    rng = np.random.default_rng(3)
    n = 4
    kap = rng.uniform(0.5, 2.0, n * n)
    A, M = fem.assemble(2, n, kap)
    A = A.toarray()
    ke = lambda ex, ey: kap[ex + n * ey]
    node = lambda ix, iy: ix + (n - 1) * iy      # interior node (ix, iy) at ((ix+1)h, (iy+1)h)
    # interior node (1,1) sits at grid point (2,2): elements (1,1),(2,1),(1,2),(2,2)
    diag = 2.0 / 3.0 * (ke(1, 1) + ke(2, 1) + ke(1, 2) + ke(2, 2))
    assert abs(A[node(1, 1), node(1, 1)] - diag) < 1e-13
    # horizontal neighbour (2,1): shared edge between grid points (2,2)-(3,2): elements (2,1),(2,2)
    assert abs(A[node(1, 1), node(2, 1)] - (-1.0 / 6.0) * (ke(2, 1) + ke(2, 2))) < 1e-13
    # diagonal neighbour (2,2): only element (2,2) holds both
    assert abs(A[node(1, 1), node(2, 2)] - (-1.0 / 3.0) * ke(2, 2)) < 1e-13
    # mass: 1D (h/6)(1,4,1) tensor product, independent of kappa
    h = 1.0 / n
    assert abs(M[node(1, 1), node(1, 1)] - (4 * h / 6) ** 2) < 1e-15
    assert abs(M[node(1, 1), node(2, 2)] - (h / 6) ** 2) < 1e-15


@pytest.mark.parametrize("dim,n", [(2, 8), (3, 8), (2, 12)])
def test_discrete_eigenvalues_match_closed_form(dim, n):
    A, M = fem.assemble(dim, n)
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
    np.testing.assert_allclose(w, q1_laplace_eigs(dim, n), rtol=1e-12)


# ---------------------------------------------------------------- hierarchy
@pytest.mark.parametrize("dim,nf,nc", [(2, 16, 8), (3, 8, 4), (2, 16, 4), (3, 8, 2)])
def test_galerkin_equals_rediscretisation(dim, nf, nc):
    """Nested Q1 spaces with exact integration: P^T A_h P = A_H, P^T M_h P = M_H."""
    Ah, Mh = fem.assemble(dim, nf)
    AH, MH = fem.assemble(dim, nc)
    P = multigrid.interp(dim, nf, nc)
    assert abs(P.T @ Ah @ P - AH).max() < 1e-12
    assert abs(P.T @ Mh @ P - MH).max() < 1e-15


def test_interpolation_reproduces_linear_functions():
    """I_H^h applied to the nodal values of a (bi)linear function gives its fine nodal values."""
    nf, nc = 16, 4
    P = multigrid.interp(2, nf, nc)
    X = np.arange(1, nc) / nc
    x = np.arange(1, nf) / nf
    f = lambda a, b: 0.3 + 1.7 * a - 0.9 * b + 2.1 * a * b
    fc = f(X[None, :], X[:, None]).ravel()        # x fastest
    ff = f(x[None, :], x[:, None]).ravel()
    # the Dirichlet trace is not zero, so only compare nodes whose interpolation stencil is interior
    inner = np.zeros((nf - 1, nf - 1), bool)
    inner[nf // nc - 1:nf - nf // nc, nf // nc - 1:nf - nf // nc] = True
    np.testing.assert_allclose((P @ fc)[inner.ravel()], ff[inner.ravel()], atol=1e-14)


@pytest.mark.parametrize("dim,levels", [(2, [16, 8, 4]), (3, [8, 4, 2])])
def test_vcycle_symmetric_positive_and_convergent(dim, levels):
    rng = np.random.default_rng(1)
    kap = synth.kappa_field(dim, levels[0], seed=5)
    H = multigrid.Hierarchy(dim, levels, kap)
    N = H.A[0].shape[0]
    V = H.vcycle(np.eye(N))
    assert np.abs(V - V.T).max() < 1e-13 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    E = np.eye(N) - V @ H.A[0].toarray()
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert rho < 0.35, rho
    x = rng.standard_normal(N)
    # repeated V-cycles as a stationary iteration converge to A^{-1} b
    b = H.A[0] @ x
    y = np.zeros(N)
    for _ in range(30):
        y = y + H.vcycle(b - H.A[0] @ y)
    assert np.linalg.norm(y - x) < 1e-10 * np.linalg.norm(x)


def test_vcycle_on_coarsest_level_is_exact_solve():
    H = multigrid.Hierarchy(2, [8, 4])
    b = np.random.default_rng(0).standard_normal((H.A[1].shape[0], 3))
    np.testing.assert_allclose(H.A[1] @ H.vcycle(b, l=1), b, atol=1e-12)


# ---------------------------------------------------------------- PCG
def test_pcg_equals_krylov_energy_minimiser():
    """s PCG steps = the A-norm best approximation in x0 + K_s(V A, V r0)."""
    H = multigrid.Hierarchy(2, [8, 4, 2], synth.kappa_field(2, 8, seed=2))
    A = H.A[0].toarray()
    N = A.shape[0]
    rng = np.random.default_rng(4)
    b = rng.standard_normal((N, 3))
    x0 = rng.standard_normal((N, 3))
    V = H.vcycle(np.eye(N))
    for s in (1, 2, 3):
        x = pase.pcg(H, b, x0, s)
        for j in range(3):
            r0 = b[:, j] - A @ x0[:, j]
            K = [V @ r0]
            for _ in range(s - 1):
                K.append(V @ (A @ K[-1]))
            K = np.array(K).T
            c = np.linalg.solve(K.T @ A @ K, K.T @ r0)
            ref = x0[:, j] + K @ c
            np.testing.assert_allclose(x[:, j], ref, rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------- outer loop
def _dense_eigs(H, k):
    return sla.eigh(H.A[0].toarray(), H.M[0].toarray(), subset_by_index=[0, k - 1])


@pytest.mark.parametrize("dim,levels,k,kap_seed", [
    (2, [8, 4, 2], 4, None), (3, [8, 4, 2], 5, None), (2, [16, 8, 4], 6, 7), (3, [8, 4], 4, 9)])
def test_pase_matches_dense_generalized_eigensolve(dim, levels, k, kap_seed):
    kap = None if kap_seed is None else synth.kappa_field(dim, levels[0], seed=kap_seed)
    H = multigrid.Hierarchy(dim, levels, kap)
    N = H.A[0].shape[0]
    U0 = synth.initial_vectors(N, k, seed=0)
    r = pase.solve(H, k, 1e-11, U0, max_outer=300)
    assert r.converged
    w, X = _dense_eigs(H, k + 1)
    np.testing.assert_allclose(r.lam, w[:k], rtol=1e-12)
    G = r.U.T @ (H.M[0] @ r.U)
    assert np.abs(G - np.eye(k)).max() < 1e-12
    # eigenvectors are unique only per complete cluster: compare the subspace of
    # the clusters that end before index k (a cluster cut by k is skipped)
    kc = k
    while kc > 0 and abs(w[kc] - w[kc - 1]) < 1e-8 * w[kc]:
        kc -= 1
    cos = np.linalg.svd(X[:, :kc].T @ (H.M[0] @ r.U[:, :kc]), compute_uv=False)
    assert cos.min() > 1 - 1e-9


def test_pase_invariants_every_iteration():
    """U^T M U = I; Ritz values >= exact (Courant-Fischer) and nonincreasing."""
    H = multigrid.Hierarchy(2, [32, 16, 8, 4], synth.kappa_field(2, 32, seed=1))
    k = 6
    w, _ = _dense_eigs(H, k)
    seen = []

    def cb(it, lam, U):
        G = U.T @ (H.M[0] @ U)
        assert np.abs(G - np.eye(k)).max() < 1e-12
        seen.append(lam.copy())

    U0 = synth.initial_vectors(H.A[0].shape[0], k, seed=3)
    r = pase.solve(H, k, 1e-10, U0, callback=cb)
    assert r.converged and len(seen) > 3
    for lam in seen:
        assert np.all(lam >= w * (1 - 1e-11))   # LAPACK and oracle both carry ~1e-13 rounding
    for a, b in zip(seen[:-1], seen[1:]):
        assert np.all(b <= a * (1 + 1e-12))


def test_complement_form_gives_same_ritz_values():
    H = multigrid.Hierarchy(3, [8, 4, 2], synth.kappa_field(3, 8, seed=4))
    k = 5
    N = H.A[0].shape[0]
    U = pase.cholqr_m(synth.initial_vectors(N, k, 2), H.M[0])
    lam = np.einsum("ij,ij->j", U, H.A[0] @ U)
    W = pase.pcg(H, (H.M[0] @ U) * lam, U, 2)
    v1, _ = pase.small_solve(*pase.composite(H, W), k)
    v2, U2 = pase.small_solve_complement(H, W, k)
    np.testing.assert_allclose(v1, v2, rtol=1e-12)


def test_correction_equation_gives_the_same_pcg_iterate():
    """s PCG steps on A w = lam M u from w = u equal u + (s PCG steps on A e = lam M u - A u from e = 0).

    The V-cycle is a fixed linear operator, so every Krylov quantity depends on
    the initial residual alone: the mixed form solves for the correction and
    adds it to the FP64 master vectors.
    """
    H = multigrid.Hierarchy(2, [16, 8, 4], synth.kappa_field(2, 16, seed=8))
    k = 4
    N = H.A[0].shape[0]
    U = pase.cholqr_m(synth.initial_vectors(N, k, 5), H.M[0])
    lam = np.einsum("ij,ij->j", U, H.A[0] @ U)
    rhs = (H.M[0] @ U) * lam
    for s in (1, 2, 3):
        W = pase.pcg(H, rhs, U, s)
        E = pase.pcg(H, rhs - H.A[0] @ U, np.zeros_like(U), s)
        np.testing.assert_allclose(U + E, W, rtol=0, atol=1e-12 * np.abs(W).max())
    # the V-cycle is linear: V(a r1 + r2) = a V(r1) + V(r2)
    r1, r2 = synth.initial_vectors(N, 2, 6).T
    lhs = H.vcycle((2.5 * r1 + r2)[:, None])[:, 0]
    rhs2 = 2.5 * H.vcycle(r1[:, None])[:, 0] + H.vcycle(r2[:, None])[:, 0]
    np.testing.assert_allclose(lhs, rhs2, rtol=0, atol=1e-13 * np.abs(lhs).max())


@pytest.mark.slow
def test_config1_closed_form():
    """2D 128x128, coarse 16x16, nev 10, 2 CG steps, tol 1e-10: closed-form eigenvalues."""
    H = multigrid.Hierarchy(2, [128, 64, 32, 16])
    U0 = synth.initial_vectors(127 ** 2, 10, seed=0)
    r = pase.solve(H, 10, 1e-10, U0)
    assert r.converged
    np.testing.assert_allclose(r.lam, q1_laplace_eigs(2, 128, 10), rtol=1e-11)


def test_coarse_init_path():
    H = multigrid.Hierarchy(2, [16, 8, 4])
    r = pase.solve(H, 4, 1e-11, coarse_init=True)
    assert r.converged
    np.testing.assert_allclose(r.lam, q1_laplace_eigs(2, 16, 4), rtol=1e-12)


@pytest.mark.slow
def test_variable_kappa_against_shift_invert_lanczos():
    """Independent algorithm: ARPACK shift-invert Lanczos on the assembled pencil."""
    H = multigrid.Hierarchy(3, [16, 8, 4], synth.kappa_field(3, 16, seed=11))
    k = 8
    U0 = synth.initial_vectors(H.A[0].shape[0], k, seed=1)
    r = pase.solve(H, k, 1e-11, U0)
    assert r.converged
    w = spla.eigsh(H.A[0].tocsc(), k=k, M=H.M[0].tocsc(), sigma=0.0, which="LM",
                   return_eigenvectors=False, tol=1e-14)
    np.testing.assert_allclose(r.lam, np.sort(w), rtol=1e-10)


# ---------------------------------------------------------------- planted slips
def test_planted_transposed_interpolation_is_caught(monkeypatch):
    """A 1D interpolation with a wrong weight breaks the Galerkin identity pin."""
    orig = multigrid.interp_1d

    def bad(nf, nc):
        P = orig(nf, nc).toarray()
        P[P == 0.5] = 0.25
        import scipy.sparse as sp
        return sp.csr_matrix(P)

    monkeypatch.setattr(multigrid, "interp_1d", bad)
    Ah, _ = fem.assemble(2, 8)
    AH, _ = fem.assemble(2, 4)
    P = multigrid.interp(2, 8, 4)
    assert abs(P.T @ Ah @ P - AH).max() > 1e-3


def _planted(func, old, new):
    """Copy of an oracle function with one slip planted in its source."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(func))
    assert old in src
    ns = dict(func.__globals__)
    exec(src.replace(old, new), ns)
    return ns[func.__name__]


@pytest.mark.parametrize("old,new", [
    ("p = z + p * beta", "p = z"),                     # dropped conjugation term
    ("r -= q * alpha", "r += q * alpha"),              # sign slip in the residual update
    ("x += p * alpha", "x += z * alpha"),              # wrong direction
])
def test_planted_pcg_slips_are_caught(old, new):
    """Slips planted in the oracle's PCG break the Krylov-minimiser pin."""
    H = multigrid.Hierarchy(2, [8, 4, 2], synth.kappa_field(2, 8, seed=2))
    A = H.A[0].toarray()
    N = A.shape[0]
    rng = np.random.default_rng(4)
    b = rng.standard_normal((N, 1))
    x0 = rng.standard_normal((N, 1))
    V = H.vcycle(np.eye(N))
    bad = _planted(pase.pcg, old, new)(H, b, x0, 3)
    r0 = b[:, 0] - A @ x0[:, 0]
    K = [V @ r0]
    for _ in range(2):
        K.append(V @ (A @ K[-1]))
    K = np.array(K).T
    ref = x0[:, 0] + K @ np.linalg.solve(K.T @ A @ K, K.T @ r0)
    assert np.linalg.norm(bad[:, 0] - ref) > 1e-6 * np.linalg.norm(ref)


def test_planted_vcycle_slip_is_caught():
    """A V-cycle whose post-smoother is dropped is no longer symmetric."""
    H = multigrid.Hierarchy(2, [16, 8, 4])
    bad = _planted(multigrid.Hierarchy.vcycle, "for _ in range(self.nu):", "for _ in range(0):")
    N = H.A[0].shape[0]
    V = bad(H, np.eye(N))
    assert np.abs(V - V.T).max() > 1e-6 * np.abs(V).max()


# ---------------------------------------------------------------- synthetic inputs
def test_kappa_field_statistics():
    n = 64
    g = np.log(synth.kappa_field(3, n, seed=0)).reshape(n, n, n)
    assert abs(g.mean()) < 0.2
    assert 0.6 < g.var() < 1.4
    # correlation at lag ell along x: exp(-1/2) for the squared exponential
    lag = int(round(0.1 * n))
    c = np.mean((g[:, :, :-lag] - g.mean()) * (g[:, :, lag:] - g.mean())) / g.var()
    assert abs(c - np.exp(-0.5)) < 0.15
    # seeded: same seed -> same field
    np.testing.assert_array_equal(synth.kappa_field(2, 16, 3), synth.kappa_field(2, 16, 3))


def test_guard_pairs_reach_the_same_fixed_point():
    """Guard pairs change the block, not the answer: the nev wanted pairs still match the closed
    form (kappa = 1) and a dense generalized eigensolve (kappa field) of the assembled pencil."""
    H = multigrid.Hierarchy(2, [16, 8, 4])
    r = pase.solve(H, 4, 1e-11, synth.initial_vectors(15 ** 2, 7, seed=3), guard=3)
    assert r.converged and r.lam.shape == (4,) and r.U.shape == (15 ** 2, 4)
    np.testing.assert_allclose(r.lam, q1_laplace_eigs(2, 16, 4), rtol=1e-11)
    kap = synth.kappa_field(3, 8, seed=4)
    H = multigrid.Hierarchy(3, [8, 4], kap)
    r = pase.solve(H, 5, 1e-11, synth.initial_vectors(7 ** 3, 8, seed=2), guard=3)
    A, M = fem.assemble(3, 8, kap)
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)[:5]
    np.testing.assert_allclose(r.lam, w, rtol=1e-10)


def test_post_smoothing_option_reaches_the_dense_eigenpairs():
    """Alg. 3 step 7 (post-smoothing solve, solve(post_smooth=True)) on an 8 x 8 mesh: the same fixed
    point as the plain iteration, the k smallest eigenpairs of the dense generalized eigenproblem."""
    H = multigrid.Hierarchy(2, [8, 4])
    k = 4
    r = pase.solve(H, k, 1e-12, synth.initial_vectors(49, k, seed=9), post_smooth=True)
    assert r.converged
    A, M = fem.assemble(2, 8)
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)[:k]
    np.testing.assert_allclose(r.lam, w, rtol=1e-11)
    np.testing.assert_allclose(r.lam, q1_laplace_eigs(2, 8, k), rtol=1e-11)
    np.testing.assert_allclose(r.U.T @ (M @ r.U), np.eye(k), atol=1e-12)
