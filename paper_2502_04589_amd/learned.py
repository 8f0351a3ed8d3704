"""UNet: a handle on the learned preconditioner of libpase (torch-owned device memory).

Argument marshalling only: the network's forward and backward passes, the loss,
the output-scale fit and Adam run in libpase's HIP kernels on the stream that was
current when the network was created.  Host-side training plumbing uses torch: the
He-normal initial weights come from a seeded CPU generator, and each step's batch
of pair columns is gathered with torch indexing (data movement only).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import _native as nat
from .solver import PaseError, _ptr

CHANNELS = (16, 32, 64)


class UNet:
    """3-level U-Net preconditioner on the interior nodes of an n^3 Q1 mesh (n divisible by 4)."""

    def __init__(self, n, batch_max, device="cuda:0"):
        self.lib = nat.load()
        if not torch.cuda.is_available():
            raise RuntimeError("UNet needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self.n = int(n)
        self.batch_max = int(batch_max)
        self.N = (self.n - 1) ** 3
        ch = (C.c_int * 3)(*CHANNELS)
        cnt = C.c_size_t(0)
        self._check(self.lib.pase_unet_param_count(ch, C.byref(cnt)))
        self.num_params = int(cnt.value)
        nbytes = C.c_size_t(0)
        self._check(self.lib.pase_unet_workspace_bytes(self.n, self.batch_max, ch, C.byref(nbytes)))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._check(self.lib.pase_unet_create(self.n, self.batch_max, ch, _ptr(self.workspace), nbytes,
                                              C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def _check(self, st):
        if st != 0:
            msg = self.lib.pase_unet_last_error(getattr(self, "h", None)) if getattr(self, "h", None) else b""
            raise PaseError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pase_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _mv(self, t, k, name):
        if not (isinstance(t, torch.Tensor) and t.device == self.device and t.dtype == torch.float64):
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if t.shape != (self.N, k) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.N} x {k} tensor")
        return t

    def _logk(self, logk):
        if logk is None:
            return None
        if not (isinstance(logk, torch.Tensor) and logk.dtype == torch.float64 and logk.numel() == self.N):
            raise TypeError("logk must be a float64 device tensor with one value per node")
        return logk.contiguous()

    def set_weights(self, W):
        W = torch.as_tensor(W, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
        if W.numel() != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters")
        self._w = W
        self._check(self.lib.pase_unet_set_weights(self.h, _ptr(W)))

    def get_weights(self):
        W = torch.empty(self.num_params, dtype=torch.float32, device=self.device)
        self._check(self.lib.pase_unet_get_weights(self.h, _ptr(W)))
        return W

    def save(self, path):
        """Write the training state (weights, Adam moments, Adam step count) to the file `path`."""
        self._check(self.lib.pase_unet_save(self.h, os.fsencode(path)))

    def load(self, path):
        """Restore a training state written by save() for a network of the same channel widths."""
        self._check(self.lib.pase_unet_load(self.h, os.fsencode(path)))

    def apply(self, R, logk=None):
        k = R.shape[1]
        R = self._mv(R, k, "R")
        lk = self._logk(logk)
        Z = torch.empty_like(R)
        self._check(self.lib.pase_unet_apply(self.h, k, _ptr(R), _ptr(lk), _ptr(Z)))
        return Z

    def loss_grad(self, R, Cm, logk=None, want_grad=True):
        k = R.shape[1]
        R = self._mv(R, k, "R")
        Cm = self._mv(Cm, k, "C")
        lk = self._logk(logk)
        G = torch.empty(self.num_params, dtype=torch.float32, device=self.device) if want_grad else None
        loss = C.c_double(0.0)
        self._check(self.lib.pase_unet_loss_grad(self.h, k, _ptr(R), _ptr(Cm), _ptr(lk), C.byref(loss), _ptr(G)))
        return float(loss.value), G

    def set_output_scale(self, scale):
        """Node-wise output scale (float64 device tensor with one value per node, or None = 1);
        the learned form uses the inverse diagonal of A (Solver.fine_diag_inverse())."""
        if scale is not None:
            if not (isinstance(scale, torch.Tensor) and scale.dtype == torch.float64 and scale.numel() == self.N
                    and scale.device == self.device):
                raise TypeError("scale must be a float64 device tensor with one value per node")
            scale = scale.contiguous()
        self._oscale = scale              # the library keeps the pointer: hold the memory
        self._check(self.lib.pase_unet_set_output_scale(self.h, _ptr(scale)))

    def fit_scale(self, R, Cm, logk=None):
        """Rescale the output to the targets' norm (s = ||Cm|| / ||N(R)||, spread over the last three
        layers); returns s."""
        k = R.shape[1]
        R = self._mv(R, k, "R")
        Cm = self._mv(Cm, k, "C")
        lk = self._logk(logk)
        sc = C.c_double(0.0)
        self._check(self.lib.pase_unet_fit_scale(self.h, k, _ptr(R), _ptr(Cm), _ptr(lk), C.byref(sc)))
        return float(sc.value)

    def adam_step(self, lr):
        self._check(self.lib.pase_unet_adam_step(self.h, C.c_float(lr)))

    # ------------------------------------------------------------------ training
    @staticmethod
    def layer_shapes(channels=CHANNELS):
        """(27, Cin, Cout) of the 11 convolutions in parameter order (the order libpase uses)."""
        c0, c1, c2 = channels
        io = [(2, c0), (c0, c0), (c0, c1), (c1, c1), (c1, c2), (c2, c2), (c2 + c1, c1), (c1, c1),
              (c1 + c0, c0), (c0, c0), (c0, 1)]
        return [(27, a, b) for a, b in io]

    def init_weights(self, seed=0):
        """He-normal initialisation (std sqrt(2 / (27 Cin))) from a seeded CPU generator."""
        g = torch.Generator().manual_seed(int(seed))
        parts = [torch.randn(sh, generator=g, dtype=torch.float32) * (2.0 / (sh[0] * sh[1])) ** 0.5
                 for sh in self.layer_shapes()]
        self.set_weights(torch.cat([p.reshape(-1) for p in parts]))

    def train(self, R, V, logk=None, steps=100, lr=1e-3, seed=0, fit_scale=True):
        """Adam on the pairs (R[:, j], V[:, j]) (device N x P each): every step draws batch_max
        distinct columns (seeded), runs the loss, its gradient and one Adam step.  With fit_scale
        the output scale is first fitted on one such batch.  Returns the loss of every step."""
        P = R.shape[1]
        R = self._mv(R, P, "R")
        V = self._mv(V, P, "V")
        rng = np.random.default_rng(seed)
        b = min(self.batch_max, P)
        losses = []
        if fit_scale:
            cols = torch.from_numpy(rng.choice(P, size=b, replace=False)).to(self.device)
            self.fit_scale(R.index_select(1, cols).contiguous(), V.index_select(1, cols).contiguous(), logk)
        for _ in range(int(steps)):
            cols = torch.from_numpy(rng.choice(P, size=b, replace=False)).to(self.device)
            Rb = R.index_select(1, cols).contiguous()
            Vb = V.index_select(1, cols).contiguous()
            loss, _ = self.loss_grad(Rb, Vb, logk, want_grad=False)
            self.adam_step(lr)
            losses.append(loss)
        return losses
