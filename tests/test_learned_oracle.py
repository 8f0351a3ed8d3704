"""Pins of the learned-preconditioner oracle (oracle/unet.py), CPU only.

Every check compares the oracle with something other than itself: explicit
loops, central finite differences, adjoint identities, a closed-form Adam step,
and the plain PCG of oracle/pase.py.
"""
import numpy as np
import pytest

import synth
from oracle import multigrid, pase, unet


def conv_loops(x, w, m):
    """conv3d written as plain loops over nodes, offsets and channels."""
    B, N, cin = x.shape
    out = np.zeros((B, N, w.shape[2]))
    for b in range(B):
        for z in range(m):
            for y in range(m):
                for xx in range(m):
                    n = xx + m * (y + m * z)
                    for o in range(27):
                        dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
                        X, Y, Z = xx + dx, y + dy, z + dz
                        if 0 <= X < m and 0 <= Y < m and 0 <= Z < m:
                            out[b, n] += x[b, X + m * (Y + m * Z)] @ w[o]
    return out


def test_conv3d_matches_loops():
    rng = np.random.default_rng(0)
    m = 4
    x = rng.standard_normal((2, m ** 3, 3))
    w = rng.standard_normal((27, 3, 5))
    np.testing.assert_allclose(unet.conv3d(x, w, m), conv_loops(x, w, m), rtol=1e-13, atol=1e-12)


def test_conv3d_backward_adjoint_and_fd():
    rng = np.random.default_rng(1)
    m = 5
    x = rng.standard_normal((2, m ** 3, 3))
    w = rng.standard_normal((27, 3, 4))
    d = rng.standard_normal((2, m ** 3, 4))
    dx, dw = unet.conv3d_backward(x, w, d, m)
    # adjoint: <conv(x, w), d> = <x, dX> = <w, dW> (the map is linear in x and in w)
    lhs = np.sum(unet.conv3d(x, w, m) * d)
    assert abs(lhs - np.sum(x * dx)) <= 1e-11 * abs(lhs)
    assert abs(lhs - np.sum(w * dw)) <= 1e-11 * abs(lhs)
    # central differences on a few entries
    eps = 1e-6
    for (o, ci, co) in [(0, 0, 0), (13, 2, 3), (26, 1, 2)]:
        wp, wm = w.copy(), w.copy()
        wp[o, ci, co] += eps
        wm[o, ci, co] -= eps
        fd = (np.sum(unet.conv3d(x, wp, m) * d) - np.sum(unet.conv3d(x, wm, m) * d)) / (2 * eps)
        assert abs(fd - dw[o, ci, co]) <= 1e-6 * max(1.0, abs(fd))


def test_unet_gradient_matches_finite_differences():
    """Loss gradient through every layer (tiny mesh n = 8, channels 2/4/8)."""
    net = unet.UNet(8, channels=(2, 4, 8))
    W = net.init(3)
    N = net.m[0] ** 3
    rng = np.random.default_rng(4)
    R = rng.standard_normal((N, 2))
    C = rng.standard_normal((N, 2))
    logk = rng.standard_normal(N) * 0.3
    L, G = unet.loss_and_grad(net, W, R, C, logk)
    eps = 1e-6
    for layer in range(11):
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += eps
            Wm[layer][idx] -= eps
            fd = (unet.loss_and_grad(net, Wp, R, C, logk)[0] - unet.loss_and_grad(net, Wm, R, C, logk)[0]) / (2 * eps)
            assert abs(fd - G[layer][idx]) <= 1e-6 * max(1e-3, abs(fd)), (layer, idx, fd, G[layer][idx])


def test_network_output_scales_with_the_residual():
    net = unet.UNet(8, channels=(2, 4, 8))
    W = net.init(5)
    rng = np.random.default_rng(6)
    R = rng.standard_normal((net.m[0] ** 3, 3))
    logk = np.zeros(net.m[0] ** 3)
    Z = net.apply(W, R, logk)
    np.testing.assert_allclose(net.apply(W, 7.5 * R, logk), 7.5 * Z, rtol=1e-13, atol=1e-14)


def test_output_scale_is_node_wise_and_in_the_gradient():
    """N with a node-wise output scale s equals s * N without it, and the gradient of the loss
    with the scale matches central differences."""
    net = unet.UNet(8, channels=(2, 4, 8))
    W = net.init(9)
    N = net.m[0] ** 3
    rng = np.random.default_rng(10)
    R = rng.standard_normal((N, 2))
    C = rng.standard_normal((N, 2))
    logk = rng.standard_normal(N) * 0.2
    sc = np.exp(rng.standard_normal(N))
    np.testing.assert_allclose(net.apply(W, R, logk, sc), sc[:, None] * net.apply(W, R, logk), rtol=1e-13)
    L, G = unet.loss_and_grad(net, W, R, C, logk, sc)
    eps = 1e-6
    for layer, idx in [(0, (4, 1, 1)), (5, (13, 3, 7)), (10, (20, 1, 0))]:
        Wp = [w.copy() for w in W]
        Wm = [w.copy() for w in W]
        Wp[layer][idx] += eps
        Wm[layer][idx] -= eps
        fd = (unet.loss_and_grad(net, Wp, R, C, logk, sc)[0] - unet.loss_and_grad(net, Wm, R, C, logk, sc)[0]) / (2 * eps)
        assert abs(fd - G[layer][idx]) <= 1e-6 * max(1e-3, abs(fd)), (layer, fd, G[layer][idx])


def test_node_log_kappa():
    n = 4
    assert np.allclose(unet.node_log_kappa(n, np.full(n ** 3, 2.0)), np.log(2.0))
    kap = np.exp(synth.kappa_field(3, n, 2) * 0 + np.arange(n ** 3) % 5)     # log kappa = element index mod 5
    lk = np.log(kap).reshape(n, n, n)
    node = unet.node_log_kappa(n, kap).reshape(n - 1, n - 1, n - 1)
    # node (x=1, y=0, z=2) sits between elements x in {1,2}, y in {0,1}, z in {2,3}
    assert np.isclose(node[2, 0, 1], lk[2:4, 0:2, 1:3].mean())


def test_adam_first_step_closed_form():
    g = np.array([[0.5, -2.0, 1e-3]])
    opt = unet.Adam([g.shape], lr=1e-2)
    W = opt.step([np.zeros_like(g)], [g])
    # t = 1: bias-corrected m = g, v = g^2, so the step is -lr g / (|g| + eps)
    np.testing.assert_allclose(W[0], -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    W = opt.step(W, [g])
    np.testing.assert_allclose(W[0], -2e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _setup(n=8):
    H = multigrid.Hierarchy(3, [n, n // 2, n // 4])
    N = H.A[0].shape[0]
    U = pase.cholqr_m(synth.initial_vectors(N, 3, 7), H.M[0])
    lam = np.einsum("ij,ij->j", U, H.A[0] @ U)
    return H, U, (H.M[0] @ U) * lam


def test_flexible_pcg_with_the_vcycle_equals_pcg():
    """With a fixed SPD preconditioner the flexible beta equals the standard one."""
    H, U, rhs = _setup()
    x, on = unet.flexible_pcg(H, rhs, U, 3, lambda R, cols: H.vcycle(R))
    np.testing.assert_allclose(x, pase.pcg(H, rhs, U, 3), rtol=0, atol=1e-11 * np.abs(x).max())
    assert on.all()


def test_zero_network_falls_back_to_the_vcycle():
    """A network that returns zero makes no progress, trips the 0.5 test at step 1, and
    the remaining steps are V-cycle PCG from the unchanged iterate."""
    H, U, rhs = _setup()
    x, on = unet.flexible_pcg(H, rhs, U, 3, lambda R, cols: np.zeros_like(R))
    assert not on.any()
    np.testing.assert_allclose(x, pase.pcg(H, rhs, U, 2), rtol=0, atol=1e-11 * np.abs(x).max())


def test_bad_network_step_then_vcycle_pcg_from_the_kept_iterate():
    """A network whose output ignores the residual (a constant field) fails the 0.5 test at
    step 1 in every column; the first step is the exact line search along its output and the
    remaining steps are plain V-cycle PCG from that iterate (restart at the switch)."""
    H, U, rhs = _setup()
    A = H.A[0]
    bad = lambda R, cols: np.ones_like(R)    # noqa: E731
    x, on = unet.flexible_pcg(H, rhs, U, 3, bad)
    assert not on.any()
    r0 = rhs - A @ U
    z0 = bad(r0, None)
    a0 = np.einsum("ij,ij->j", r0, z0) / np.einsum("ij,ij->j", z0, A @ z0)
    x1 = U + z0 * a0
    assert np.all(np.linalg.norm(rhs - A @ x1, axis=0) > 0.5 * np.linalg.norm(r0, axis=0))
    np.testing.assert_allclose(x, pase.pcg(H, rhs, x1, 2), rtol=0, atol=1e-11 * np.abs(x).max())


def test_training_reduces_the_loss():
    """Sixty Adam steps on (r, V(r)) pairs lower the relative loss (tiny network)."""
    H = multigrid.Hierarchy(3, [8, 4, 2])
    net = unet.UNet(8, channels=(2, 4, 8))
    W = net.init(0)
    N = net.m[0] ** 3
    R = np.random.default_rng(8).standard_normal((N, 4))
    C = H.vcycle(R)
    logk = np.zeros(N)
    opt = unet.Adam(net.shapes, lr=3e-3)
    L0 = unet.loss_and_grad(net, W, R, C, logk)[0]
    for _ in range(60):
        L, G = unet.loss_and_grad(net, W, R, C, logk)
        W = opt.step(W, G)
    assert unet.loss_and_grad(net, W, R, C, logk)[0] < 0.6 * L0


# ---------------------------------------------------------------- wiring of the forward pass
def _interp1d(nf, nc):
    """1D linear interpolation from the nc - 1 interior nodes of a mesh of nc elements to the
    nf - 1 interior nodes of the mesh of nf = 2 nc elements (written here, not taken from oracle)."""
    P = np.zeros((nf - 1, nc - 1))
    for j in range(nc - 1):
        i = 2 * j + 1                     # fine index of coarse node j
        P[i, j] = 1.0
        P[i - 1, j] += 0.5
        P[i + 1, j] += 0.5
    return P


def _interp3d(nf, nc):
    p = _interp1d(nf, nc)
    return np.kron(p, np.kron(p, p))      # x fastest: z (outer) x y x x (inner)


def _centre_tap(S):
    w = np.zeros((27,) + S.shape)
    w[13] = S                             # offset (0, 0, 0)
    return w


def test_unet_forward_wiring_is_the_explicit_composition():
    """UNet.forward pinned by weights that make it an explicit linear map: centre-tap convolutions
    that mix channels by fixed non-negative matrices, on non-negative inputs (so every ReLU passes its
    input through).  The expected output is the composition written out here with its own trilinear
    interpolation: down by P^T, up by P, skips concatenated after the up-sampled channels, skips taken
    from the second convolution of each encoder level.  Distinct coefficients on every path make a
    swapped concatenation, a skip from the wrong tensor or an up/down mix-up change the result."""
    n = 8
    net = unet.UNet(n, channels=(2, 2, 2))
    m0, m1, m2 = net.m
    I2 = np.eye(2)
    S = [np.array([[1.0, 0.0], [0.0, 1.0]]),          # 0: h0 = [r, q]
         np.array([[2.0, 0.0], [0.0, 1.0]]),          # 1: e0 = [2 r, q]
         np.array([[1.0, 0.0], [0.0, 0.0]]),          # 2: h1 = [d1_0, 0]
         np.array([[3.0, 0.0], [0.0, 0.0]]),          # 3: e1 = [3 h1_0, 0]
         np.array([[1.0, 0.0], [0.0, 0.0]]),          # 4: h2 = [d2_0, 0]
         np.array([[2.0, 0.0], [0.0, 0.0]]),          # 5: e2 = [2 h2_0, 0]
         np.array([[1.0, 0.0], [0.0, 0.0], [5.0, 0.0], [0.0, 0.0]]),   # 6: g1_0 = u1_0 + 5 e1_0
         np.array([[4.0, 0.0], [0.0, 0.0]]),          # 7: f1 = [4 g1_0, 0]
         np.array([[1.0, 0.0], [0.0, 0.0], [7.0, 0.0], [11.0, 0.0]]),  # 8: g0_0 = u0_0 + 7 e0_0 + 11 e0_1
         I2 * 0.5,                                     # 9: f0 = g0 / 2
         np.array([[1.0], [0.0]])]                     # 10: y = f0_0
    W = [_centre_tap(s) for s in S]
    rng = np.random.default_rng(5)
    r = rng.uniform(0.1, 1.0, m0 ** 3)
    q = rng.uniform(0.1, 1.0, m0 ** 3)
    x = np.stack([r, q], axis=1)[None]
    y, _ = net.forward(W, x)
    P01, P12 = _interp3d(n, n // 2), _interp3d(n // 2, n // 4)
    e0r, e0q = 2.0 * r, q
    e1 = 3.0 * (P01.T @ e0r)
    e2 = 2.0 * (P12.T @ e1)
    f1 = 4.0 * (P12 @ e2 + 5.0 * e1)
    g0 = P01 @ f1 + 7.0 * e0r + 11.0 * e0q
    expect = 0.5 * g0
    np.testing.assert_allclose(y[0, :, 0], expect, rtol=1e-13)


def test_loss_value_is_the_per_column_definition():
    """loss_and_grad's loss equals the mean over the columns of ||N(r_b) - c_b||^2 / ||c_b||^2 computed
    column by column with apply (pins the normalisation by ||c||^2, the mean and the output scale)."""
    n = 8
    net = unet.UNet(n, channels=(2, 4, 4))
    W = net.init(3)
    rng = np.random.default_rng(6)
    N = net.m[0] ** 3
    R = rng.standard_normal((N, 3))
    C = rng.standard_normal((N, 3))
    logk = rng.standard_normal(N) * 0.3
    sc = rng.uniform(0.5, 2.0, N)
    L, _ = unet.loss_and_grad(net, W, R, C, logk, sc)
    ref = 0.0
    for b in range(3):
        z = net.apply(W, R[:, b:b + 1], logk, sc)[:, 0]
        ref += np.sum((z - C[:, b]) ** 2) / np.sum(C[:, b] ** 2)
    assert abs(L - ref / 3) <= 1e-13 * ref
