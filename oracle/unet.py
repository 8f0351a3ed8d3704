"""Oracle: the learned preconditioner of the learned form and the flexible PCG that uses it.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy, FP64.

The learned form replaces the V-cycle inside the fine-grid PCG of the outer
step (Alg. 3 step 3) by a small convolutional network N that maps a residual
to a correction, trained on pairs (r, V(r)) produced by the solver itself, and
keeps the V-cycle as the fallback.  The paper does not define this extension;
the readings taken here are:

* Network: a 3-level U-Net on the grid of interior nodes (vertex-centred
  hierarchy m -> (m-1)/2 -> ...).  Per level two 3x3x3 convolutions (zero
  padding, no bias) each followed by ReLU; down-sampling by full-weighting
  restriction P^T, up-sampling by trilinear prolongation P (the multigrid
  transfer operators), skip connections by channel concatenation, a final
  3x3x3 convolution to one channel.  Channels 16/32/64 by default.
* Inputs: the residual divided by its root mean square rho(r) = ||r||_2 / sqrt(N)
  (per-node values of order one, like the other channel) and the node average of
  log kappa (mean over the 2^3 elements around a node; zero when kappa = 1).
  The output is rescaled by rho(r), so N is positively homogeneous in r, and,
  node-wise, by the inverse diagonal of A (D^-1 r is the Jacobi part of V(r) and
  carries its 1/kappa scaling, which the log kappa channel alone learns slowly):
  N(r) = rho(r) D^-1 net(r / rho(r), log kappa).  The scale is an argument
  (None = 1), so the network is also usable without it.
* Loss: mean over the batch of ||N(r) - c||^2 / ||c||^2 with c = V(r) (one
  V-cycle from zero).
* Optimiser: Adam (Kingma and Ba, 2015) with beta1 = 0.9, beta2 = 0.999,
  eps = 1e-8.
* Flexible PCG (Notay, 2000): beta_j = r_{j+1}^T (z_{j+1} - z_j) / (r_j^T z_j);
  a column whose residual norm does not drop below half its previous value
  while it uses the network switches to the V-cycle for the remaining steps
  of that outer iteration (the step itself is kept).  At the switch the CG
  recurrence restarts (beta = 0), so the remaining steps are V-cycle PCG from
  the kept iterate: a direction from a poor network, with r^T z near zero,
  would otherwise dominate the next search direction through beta.

Layout: fields are node-major (B, N, C) with x fastest, as the GPU kernels use.
Convolution offsets o = 0..26 enumerate (dx, dy, dz) in {-1,0,1}^3 with dx
fastest: dx = o % 3 - 1, dy = (o // 3) % 3 - 1, dz = o // 9 - 1.  A weight
tensor has shape (27, Cin, Cout).
"""
from __future__ import annotations

import numpy as np

from . import multigrid

DEFAULT_CHANNELS = (16, 32, 64)


# ---------------------------------------------------------------- primitives

def _offsets():
    return [(o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1) for o in range(27)]


def conv3d(x, w, m):
    """out[b, n, co] = sum_{o, ci} w[o, ci, co] x[b, n + o, ci] (zero outside the m^3 grid)."""
    B, N, cin = x.shape
    X = np.pad(x.reshape(B, m, m, m, cin), ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((B, m, m, m, w.shape[2]))
    for o, (dx, dy, dz) in enumerate(_offsets()):
        out += X[:, 1 + dz:1 + dz + m, 1 + dy:1 + dy + m, 1 + dx:1 + dx + m, :] @ w[o]
    return out.reshape(B, N, w.shape[2])


def conv3d_backward(x, w, dout, m):
    """Gradients of conv3d with respect to its input and its weights."""
    B, N, cin = x.shape
    cout = w.shape[2]
    X = np.pad(x.reshape(B, m, m, m, cin), ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    D = dout.reshape(B, m, m, m, cout)
    dX = np.zeros_like(X)
    dw = np.zeros_like(w)
    for o, (dx, dy, dz) in enumerate(_offsets()):
        sl = (slice(None), slice(1 + dz, 1 + dz + m), slice(1 + dy, 1 + dy + m), slice(1 + dx, 1 + dx + m))
        dX[sl] += D @ w[o].T
        dw[o] = X[sl].reshape(-1, cin).T @ D.reshape(-1, cout)
    return dX[:, 1:-1, 1:-1, 1:-1, :].reshape(B, N, cin), dw


def relu(x):
    return np.maximum(x, 0.0)


def node_log_kappa(n, kappa):
    """Node average of log kappa over the 8 elements around each interior node (x fastest)."""
    m = n - 1
    if kappa is None:
        return np.zeros(m ** 3)
    lk = np.log(np.asarray(kappa, dtype=np.float64).reshape(n, n, n))   # [z, y, x]
    s = np.zeros((m, m, m))
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                s += lk[cz:cz + m, cy:cy + m, cx:cx + m]
    return (s / 8.0).ravel()


# ---------------------------------------------------------------- network

class UNet:
    """3-level U-Net on the interior nodes of an n^3 Q1 mesh (n divisible by 4)."""

    def __init__(self, n, channels=DEFAULT_CHANNELS, cin=2):
        if n % 4:
            raise ValueError("n must be divisible by 4")
        self.n = (n, n // 2, n // 4)
        self.m = tuple(v - 1 for v in self.n)
        self.P01 = multigrid.interp(3, self.n[0], self.n[1])   # level 1 -> level 0
        self.P12 = multigrid.interp(3, self.n[1], self.n[2])   # level 2 -> level 1
        c0, c1, c2 = channels
        self.channels = channels
        self.shapes = [(27, cin, c0), (27, c0, c0),            # encoder level 0
                       (27, c0, c1), (27, c1, c1),             # encoder level 1
                       (27, c1, c2), (27, c2, c2),             # bottom
                       (27, c2 + c1, c1), (27, c1, c1),        # decoder level 1
                       (27, c1 + c0, c0), (27, c0, c0),        # decoder level 0
                       (27, c0, 1)]                            # output

    def init(self, seed):
        """He-normal weights: std = sqrt(2 / (27 cin))."""
        rng = np.random.default_rng(seed)
        return [rng.standard_normal(s) * np.sqrt(2.0 / (27 * s[1])) for s in self.shapes]

    # transfers between levels, applied per batch item and channel
    @staticmethod
    def _apply(P, x):
        return np.stack([P @ x[b] for b in range(x.shape[0])])

    def forward(self, W, x):
        """x: (B, N0, cin) -> (y (B, N0, 1), cache)."""
        m0, m1, m2 = self.m
        cache = {"x": x}
        a0 = conv3d(x, W[0], m0); h0 = relu(a0)
        a1 = conv3d(h0, W[1], m0); e0 = relu(a1)
        d1 = self._apply(self.P01.T, e0)
        a2 = conv3d(d1, W[2], m1); h1 = relu(a2)
        a3 = conv3d(h1, W[3], m1); e1 = relu(a3)
        d2 = self._apply(self.P12.T, e1)
        a4 = conv3d(d2, W[4], m2); h2 = relu(a4)
        a5 = conv3d(h2, W[5], m2); e2 = relu(a5)
        u1 = self._apply(self.P12, e2)
        c1 = np.concatenate([u1, e1], axis=2)
        a6 = conv3d(c1, W[6], m1); g1 = relu(a6)
        a7 = conv3d(g1, W[7], m1); f1 = relu(a7)
        u0 = self._apply(self.P01, f1)
        c0 = np.concatenate([u0, e0], axis=2)
        a8 = conv3d(c0, W[8], m0); g0 = relu(a8)
        a9 = conv3d(g0, W[9], m0); f0 = relu(a9)
        y = conv3d(f0, W[10], m0)
        cache.update(h0=h0, e0=e0, d1=d1, h1=h1, e1=e1, d2=d2, h2=h2, e2=e2, c1=c1, g1=g1, f1=f1, c0=c0,
                     g0=g0, f0=f0, a=(a0, a1, a2, a3, a4, a5, a6, a7, a8, a9))
        return y, cache

    def backward(self, W, cache, dy):
        """Gradients of a scalar loss with respect to the weights, given dL/dy."""
        m0, m1, m2 = self.m
        a = cache["a"]
        g = [None] * 11
        d_f0, g[10] = conv3d_backward(cache["f0"], W[10], dy, m0)
        d_g0, g[9] = conv3d_backward(cache["g0"], W[9], d_f0 * (a[9] > 0), m0)
        d_c0, g[8] = conv3d_backward(cache["c0"], W[8], d_g0 * (a[8] > 0), m0)
        cu = cache["f1"].shape[2]
        d_u0, d_e0 = d_c0[:, :, :cu], d_c0[:, :, cu:]
        d_f1 = self._apply(self.P01.T, d_u0)
        d_g1, g[7] = conv3d_backward(cache["g1"], W[7], d_f1 * (a[7] > 0), m1)
        d_c1, g[6] = conv3d_backward(cache["c1"], W[6], d_g1 * (a[6] > 0), m1)
        cu = cache["e2"].shape[2]
        d_u1, d_e1 = d_c1[:, :, :cu], d_c1[:, :, cu:]
        d_e2 = self._apply(self.P12.T, d_u1)
        d_h2, g[5] = conv3d_backward(cache["h2"], W[5], d_e2 * (a[5] > 0), m2)
        d_d2, g[4] = conv3d_backward(cache["d2"], W[4], d_h2 * (a[4] > 0), m2)
        d_e1 = d_e1 + self._apply(self.P12, d_d2)
        d_h1, g[3] = conv3d_backward(cache["h1"], W[3], d_e1 * (a[3] > 0), m1)
        d_d1, g[2] = conv3d_backward(cache["d1"], W[2], d_h1 * (a[2] > 0), m1)
        d_e0 = d_e0 + self._apply(self.P01, d_d1)
        d_h0, g[1] = conv3d_backward(cache["h0"], W[1], d_e0 * (a[1] > 0), m0)
        _, g[0] = conv3d_backward(cache["x"], W[0], d_h0 * (a[0] > 0), m0)
        return g

    # ------------------------------------------------------------ preconditioner use

    def inputs(self, R, logk):
        """(N0, B) residual columns -> network input (B, N0, 2) and the columns' root mean squares."""
        nr = np.linalg.norm(R, axis=0) / np.sqrt(R.shape[0])
        x = np.empty((R.shape[1], R.shape[0], 2))
        x[:, :, 0] = (R / np.where(nr > 0, nr, 1.0)).T
        x[:, :, 1] = logk[None, :]
        return x, nr

    def apply(self, W, R, logk, oscale=None):
        """N(R) column by column: rho(r) s * net(r / rho(r), log kappa), rho(r) = ||r|| / sqrt(N0);
        R is (N0, B), s the node-wise output scale (oscale, e.g. the inverse diagonal of A; None = 1)."""
        x, nr = self.inputs(R, logk)
        y, _ = self.forward(W, x)
        Z = y[:, :, 0].T * nr[None, :]
        return Z if oscale is None else Z * np.asarray(oscale)[:, None]


def loss_and_grad(net, W, R, C, logk, oscale=None):
    """L = mean_b ||N(r_b) - c_b||^2 / ||c_b||^2 and its gradient (R, C: (N0, B))."""
    x, nr = net.inputs(R, logk)
    y, cache = net.forward(W, x)
    sc = np.ones(R.shape[0]) if oscale is None else np.asarray(oscale, dtype=np.float64)
    Z = y[:, :, 0].T * nr[None, :] * sc[:, None]
    E = Z - C
    cn = np.einsum("ij,ij->j", C, C)
    B = R.shape[1]
    L = float(np.mean(np.einsum("ij,ij->j", E, E) / cn))
    dZ = 2.0 * E / cn[None, :] / B
    dy = (dZ * nr[None, :] * sc[:, None]).T[:, :, None]
    return L, net.backward(W, cache, dy)


class Adam:
    """Adam (Kingma and Ba, 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, shapes, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros(s) for s in shapes]
        self.v = [np.zeros(s) for s in shapes]
        self.t = 0

    def step(self, W, G):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for i, g in enumerate(G):
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            W[i] = W[i] - self.lr * (self.m[i] / c1) / (np.sqrt(self.v[i] / c2) + self.eps)
        return W


# ---------------------------------------------------------------- flexible PCG with fallback

def flexible_pcg(hier, rhs, x0, s, precond, ratio=0.5):
    """s steps of flexible PCG per column from x0 on A x = rhs.

    precond(R, cols) returns the network correction for the residual columns
    listed in cols.  A column falls back to the V-cycle for the remaining steps
    once its residual norm fails to drop below ratio times its previous value
    while it used the network, and its recurrence restarts there (beta = 0).
    Returns (x, used_net_mask).
    """
    A = hier.A[0]
    x = x0.copy()
    r = rhs - A @ x
    k = r.shape[1]
    net_on = np.ones(k, dtype=bool)

    def apply(rr):
        z = hier.vcycle(rr)
        cols = np.flatnonzero(net_on)
        if cols.size:
            z[:, cols] = precond(rr[:, cols], cols)
        return z

    z = apply(r)
    p = z.copy()
    rz = np.einsum("ij,ij->j", r, z)
    for j in range(s):
        q = A @ p
        pq = np.einsum("ij,ij->j", p, q)
        alpha = np.where(pq > 0, rz / np.where(pq > 0, pq, 1.0), 0.0)
        x += p * alpha
        rn = r - q * alpha
        worse = np.linalg.norm(rn, axis=0) > ratio * np.linalg.norm(r, axis=0)
        switched = net_on & worse
        net_on &= ~worse
        if j + 1 < s:
            zn = apply(rn)
            beta = np.where(rz != 0, np.einsum("ij,ij->j", rn, zn - z) / np.where(rz != 0, rz, 1.0), 0.0)
            beta[switched] = 0.0          # restart: plain V-cycle PCG from the kept iterate
            p = zn + p * beta
            z = zn
            rz = np.einsum("ij,ij->j", rn, zn)
        r = rn
    return x, net_on
