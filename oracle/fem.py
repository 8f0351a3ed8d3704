"""Oracle: Q1 finite elements for -div(kappa grad u) = lambda u, u = 0 on the boundary.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper, Sec. 2.1: the weak form a(u, v) = lambda b(u, v) with
a(u, v) = int A grad u . grad v and b(u, v) = int u v, discretised in a
Lagrange space V_h on a mesh of rectangles / hexahedra.  Here A = kappa * I
with kappa constant on each element, V_h = continuous Q1 functions on the
uniform n^dim mesh of the unit square / cube, and the Dirichlet condition is
imposed by keeping only interior nodes.

Element matrices are computed by tensor Gauss quadrature (2 points per axis,
exact for the Q1 x Q1 products involved); the global matrices by summing
element contributions, which is the plain definition of the FE matrices.

The second workload of the paper's tests (Sec. 5, eq. general) has a tensor
coefficient and a reaction term: a(u, v) = int A grad u . grad v + phi u v
with A symmetric positive definite.  ``assemble_general`` takes A (upper
triangle, 3D) and phi constant on each element, the same element quadrature
and the same Dirichlet elimination; B = M is unchanged.

Node numbering: interior node (i_0, ..., i_{d-1}), 0 <= i_a <= n-2, at
position ((i_a + 1) h), has index sum_a i_a (n-1)^a (x fastest).
Element (e_0, ..., e_{d-1}), 0 <= e_a <= n-1, covers prod [e_a h, (e_a+1) h]
and has index sum_a e_a n^a.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _gauss2():
    """Two-point Gauss rule on [0, 1]."""
    g = 0.5 / np.sqrt(3.0)
    return np.array([0.5 - g, 0.5 + g]), np.array([0.5, 0.5])


def element_matrices(dim: int, h: float):
    """Unit-coefficient Q1 stiffness K_e and mass M_e on a cell of side h.

    Local vertex a = sum_d bit_d(a) 2^d sits at the corner with coordinate
    bit_d(a) * h along axis d.  K_e[a, b] = int grad phi_a . grad phi_b,
    M_e[a, b] = int phi_a phi_b, by tensor Gauss quadrature.
    """
    pts, wts = _gauss2()
    nv = 2 ** dim
    K = np.zeros((nv, nv))
    Mm = np.zeros((nv, nv))
    for q in itertools.product(range(2), repeat=dim):
        xi = pts[list(q)]
        w = float(np.prod(wts[list(q)])) * h ** dim
        phi = np.empty(nv)
        grad = np.empty((nv, dim))
        for a in range(nv):
            bits = [(a >> d) & 1 for d in range(dim)]
            f = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(dim)]
            df = [(1.0 if bits[d] else -1.0) / h for d in range(dim)]
            phi[a] = np.prod(f)
            for d in range(dim):
                grad[a, d] = df[d] * np.prod([f[e] for e in range(dim) if e != d])
        K += w * grad @ grad.T
        Mm += w * np.outer(phi, phi)
    return K, Mm


def n_interior(dim: int, n: int) -> int:
    return (n - 1) ** dim


def assemble(dim: int, n: int, kappa=None):
    """Global stiffness A = sum_e kappa_e K_e and mass M = sum_e M_e (CSR, float64).

    ``kappa``: None (kappa = 1) or an array of n^dim element values.
    Rows / columns of boundary nodes are dropped (Dirichlet elimination).
    """
    h = 1.0 / n
    Ke, Me = element_matrices(dim, h)
    ne = n ** dim
    if kappa is None:
        kap = np.ones(ne)
    else:
        kap = np.asarray(kappa, dtype=np.float64).reshape(-1)
        if kap.size != ne:
            raise ValueError("kappa must have n^dim entries")
    # element multi-indices, x fastest
    e = np.arange(ne)
    ecoord = [(e // n ** d) % n for d in range(dim)]
    m = n - 1
    nv = 2 ** dim
    node = np.empty((nv, ne), dtype=np.int64)
    for a in range(nv):
        idx = np.zeros(ne, dtype=np.int64)
        ok = np.ones(ne, dtype=bool)
        for d in range(dim):
            c = ecoord[d] + ((a >> d) & 1)   # full-grid coordinate 0..n
            ok &= (c >= 1) & (c <= n - 1)
            idx += (c - 1) * m ** d
        node[a] = np.where(ok, idx, -1)
    rows, cols, va, vm = [], [], [], []
    for a in range(nv):
        for b in range(nv):
            mask = (node[a] >= 0) & (node[b] >= 0)
            rows.append(node[a][mask])
            cols.append(node[b][mask])
            va.append(kap[mask] * Ke[a, b])
            vm.append(np.full(int(mask.sum()), Me[a, b]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    N = m ** dim
    A = sp.coo_matrix((np.concatenate(va), (rows, cols)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((np.concatenate(vm), (rows, cols)), shape=(N, N)).tocsr()
    A.sum_duplicates()
    M.sum_duplicates()
    return A, M


def element_matrices_general(dim: int, h: float):
    """Reference matrices of one cell of side h: K[a][b][i, j] = int d_a phi_i d_b phi_j (so that
    the stiffness of a constant tensor T is sum_ab T_ab K[a][b]) and the mass M[i, j], by tensor
    Gauss quadrature (exact for these polynomial integrands)."""
    pts, wts = _gauss2()
    nv = 2 ** dim
    K = np.zeros((dim, dim, nv, nv))
    Mm = np.zeros((nv, nv))
    for q in itertools.product(range(2), repeat=dim):
        xi = pts[list(q)]
        w = float(np.prod(wts[list(q)])) * h ** dim
        phi = np.empty(nv)
        grad = np.empty((nv, dim))
        for a in range(nv):
            bits = [(a >> d) & 1 for d in range(dim)]
            f = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(dim)]
            df = [(1.0 if bits[d] else -1.0) / h for d in range(dim)]
            phi[a] = np.prod(f)
            for d in range(dim):
                grad[a, d] = df[d] * np.prod([f[e] for e in range(dim) if e != d])
        for a in range(dim):
            for b in range(dim):
                K[a, b] += w * np.outer(grad[:, a], grad[:, b])
        Mm += w * np.outer(phi, phi)
    return K, Mm


def assemble_general(n: int, tensor, reaction=None):
    """3D: A = sum_e (sum_ab T_e[a, b] K[a][b] + phi_e M_e), M = sum_e M_e (CSR, float64).

    ``tensor``: n^3 x 6 element values (upper triangle a11, a12, a13, a22, a23, a33);
    ``reaction``: n^3 element values or None (phi = 0)."""
    dim = 3
    h = 1.0 / n
    K, Me = element_matrices_general(dim, h)
    ne = n ** dim
    T = np.asarray(tensor, dtype=np.float64).reshape(ne, 6)
    phi = np.zeros(ne) if reaction is None else np.asarray(reaction, dtype=np.float64).reshape(ne)
    full = np.empty((ne, 3, 3))
    for (a, b), col in zip([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)], range(6)):
        full[:, a, b] = T[:, col]
        full[:, b, a] = T[:, col]
    e = np.arange(ne)
    ecoord = [(e // n ** d) % n for d in range(dim)]
    m = n - 1
    nv = 2 ** dim
    node = np.empty((nv, ne), dtype=np.int64)
    for a in range(nv):
        idx = np.zeros(ne, dtype=np.int64)
        ok = np.ones(ne, dtype=bool)
        for d in range(dim):
            c = ecoord[d] + ((a >> d) & 1)
            ok &= (c >= 1) & (c <= n - 1)
            idx += (c - 1) * m ** d
        node[a] = np.where(ok, idx, -1)
    rows, cols, va, vm = [], [], [], []
    for i in range(nv):
        for j in range(nv):
            mask = (node[i] >= 0) & (node[j] >= 0)
            val = phi[mask] * Me[i, j]
            for a in range(dim):
                for b in range(dim):
                    val = val + full[mask, a, b] * K[a, b, i, j]
            rows.append(node[i][mask])
            cols.append(node[j][mask])
            va.append(val)
            vm.append(np.full(int(mask.sum()), Me[i, j]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    N = m ** dim
    A = sp.coo_matrix((np.concatenate(va), (rows, cols)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((np.concatenate(vm), (rows, cols)), shape=(N, N)).tocsr()
    A.sum_duplicates()
    M.sum_duplicates()
    return A, M
