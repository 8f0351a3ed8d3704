"""GPU parity of the learned preconditioner's kernels against the oracle network.

BF16 weights and activations with FP32 accumulation on the GPU against the FP64
oracle: outputs and gradients agree to a few BF16 units (relative L2 bounds
below), and the Adam step matches its formula in FP32.
"""
import numpy as np
import pytest

from oracle import multigrid, unet as ounet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def node_logk(n, seed):
    """Node average of a seeded log-kappa field over the 8 surrounding elements (input recipe)."""
    import synth
    lk = np.log(synth.kappa_field(3, n, seed)).reshape(n, n, n)
    m = n - 1
    s = sum(lk[cz:cz + m, cy:cy + m, cx:cx + m] for cz in (0, 1) for cy in (0, 1) for cx in (0, 1))
    return (s / 8.0).ravel()


def setup(n=16, batch=3, seed=1):
    from paper_2502_04589_amd import UNet
    net = ounet.UNet(n)
    W = net.init(seed)
    g = UNet(n, batch_max=8)
    g.set_weights(np.concatenate([w.ravel() for w in W]).astype(np.float32))
    rng = np.random.default_rng(seed + 10)
    R = rng.standard_normal((net.m[0] ** 3, batch))
    logk = node_logk(n, seed)
    return net, W, g, R, logk


def test_forward_matches_oracle():
    net, W, g, R, logk = setup()
    Wr = [w.astype(np.float32).astype(np.float64) for w in W]
    ref = net.apply(Wr, R, logk)
    Z = g.apply(dev(R), dev(logk)).cpu().numpy()
    assert relerr(Z, ref) < 2e-2, relerr(Z, ref)
    # the output scales with the residual (positive homogeneity through the input scaling)
    Z2 = g.apply(dev(3.0 * R), dev(logk)).cpu().numpy()
    np.testing.assert_allclose(Z2, 3.0 * Z, rtol=1e-6, atol=1e-6 * np.abs(Z).max())


def test_loss_and_gradients_match_oracle():
    net, W, g, R, logk = setup(seed=2)
    H = multigrid.Hierarchy(3, [16, 8, 4])
    Cm = H.vcycle(R)
    Wr = [w.astype(np.float32).astype(np.float64) for w in W]
    L, G = ounet.loss_and_grad(net, Wr, R, Cm, logk)
    Lg, Gg = g.loss_grad(dev(R), dev(Cm), dev(logk))
    assert abs(Lg - L) <= 2e-2 * L, (Lg, L)
    Gg = Gg.cpu().numpy().astype(np.float64)
    off = 0
    for i, gi in enumerate(G):
        gg = Gg[off:off + gi.size].reshape(gi.shape)
        off += gi.size
        cos = float(np.sum(gg * gi) / (np.linalg.norm(gg) * np.linalg.norm(gi)))
        assert cos > 0.999 and relerr(gg, gi) < 5e-2, (i, cos, relerr(gg, gi))


def test_adam_step_matches_formula():
    net, W, g, R, logk = setup(seed=3)
    H = multigrid.Hierarchy(3, [16, 8, 4])
    Cm = H.vcycle(R)
    W0 = g.get_weights().cpu().numpy()
    _, G = g.loss_grad(dev(R), dev(Cm), dev(logk))
    G = G.cpu().numpy()
    g.adam_step(1e-3)
    W1 = g.get_weights().cpu().numpy()
    # first step: bias-corrected moments are g and g^2, so the update is -lr g / (|g| + eps)
    expect = W0 - np.float32(1e-3) * G / (np.abs(G) + np.float32(1e-8))
    np.testing.assert_allclose(W1, expect, rtol=1e-5, atol=1e-7)


def test_training_steps_reduce_the_loss():
    """A handful of GPU Adam steps on fixed (r, V(r)) pairs lower the relative loss."""
    net, W, g, R, logk = setup(seed=4, batch=4)
    H = multigrid.Hierarchy(3, [16, 8, 4])
    Cm = dev(H.vcycle(R))
    Rd, lk = dev(R), dev(logk)
    L0, _ = g.loss_grad(Rd, Cm, lk)
    for _ in range(40):
        g.loss_grad(Rd, Cm, lk)
        g.adam_step(3e-3)
    L1, _ = g.loss_grad(Rd, Cm, lk)
    assert L1 < 0.7 * L0, (L0, L1)
