"""Solver: a handle on libpase with torch-owned device memory.

Argument marshalling only: shapes are checked, torch tensors are passed by
device pointer, and every computation happens in libpase's HIP kernels on
the stream that was current when the Solver was created.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as nat


class PaseError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = nat.STATUS.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class CsrMatrix:
    """A device CSR matrix for the algebraic input: int32 rowptr / colind and float64 values."""

    def __init__(self, rows, cols, rowptr, colind, val):
        self.rows, self.cols = int(rows), int(cols)
        self.rowptr = rowptr.to(torch.int32).contiguous()
        self.colind = colind.to(torch.int32).contiguous()
        self.val = val.to(torch.float64).contiguous()
        if self.rowptr.numel() != self.rows + 1 or self.colind.numel() != self.val.numel():
            raise ValueError("inconsistent CSR arrays")

    @classmethod
    def from_scipy(cls, M, device="cuda:0"):
        M = M.tocsr()
        dev = torch.device(device)
        return cls(M.shape[0], M.shape[1], torch.from_numpy(M.indptr.astype(np.int32)).to(dev),
                   torch.from_numpy(M.indices.astype(np.int32)).to(dev), torch.from_numpy(M.data.astype(np.float64)).to(dev))

    def _struct(self):
        c = nat.Csr()
        c.rows, c.cols = self.rows, self.cols
        c.rowptr, c.colind, c.val = _ptr(self.rowptr), _ptr(self.colind), _ptr(self.val)
        return c


class Solver:
    """Augmented subspace eigensolver for the Q1 pencil of -div(kappa grad u) = lambda u.

    dim:     2 or 3.
    levels:  elements per side of each grid, fine first, halving each time;
             the last one is the coarse space V_H unless coarse_level says otherwise.
    kappa:   None (kappa = 1) or n^dim element values, x fastest (array or tensor).
    tensor, reaction: the tensor-coefficient workload (3D, kappa None): n^3 x 6 element values of the
             symmetric coefficient (a11, a12, a13, a22, a23, a33) and n^3 values of the reaction
             (None = 0); see synth.general_coefficients.
    nev_max: largest nev a solve may ask for.
    locking: True (default): a correction's fine solves skip the pairs whose residual is already
             below tol / 10 (they keep w = u; the Rayleigh-Ritz still uses every pair); False:
             every pair every correction, as the algorithm is stated.
    guard:   extra pairs carried in the block (default 0); solve(nev) iterates nev + guard pairs
             and returns the nev smallest once they meet tol.
    start:   "given" (default): solve() starts from its U0 (None: a fixed counter-based
             uniform(-1, 1) block); "coarse": from the smallest eigenvectors of the coarse pencil,
             interpolated to the fine mesh (Alg. 3 steps 1-2).
    fallback_ratio: learned form's switch to the V-cycle (default 0.5).
    small_solver: the augmented eigenproblem's solver: "auto" (structured shift-invert path with a
             dense fallback), "dense", or "gcg" (PRECOND-A and GCG_AUG, Sec. 4: matrix-free, so
             V_H may be a level whose N_H no dense eigensolver reaches).
    coarse_level: index in levels of V_H (None = the last; levels above the last need "gcg").
    hierarchy: algebraic input instead of a grid (dim and levels are then ignored): a dict with lists
             "A", "M" (one CSR matrix per level, fine first) and "P", "R" (index 0 None, P[l] the
             interpolation from level l to l-1, R[l] = P[l]^T), each a CsrMatrix or a scipy sparse
             matrix (copied to the device).  The solver keeps them alive.
    aug_rtol: "gcg" only: GCG_AUG's stop, relative to each pair's outer residual (default 1e-2;
             0: to 1e-11).
    """

    def __init__(self, dim, levels, kappa=None, nev_max=16, precision="fp64", cg_steps=2, max_outer=500,
                 nu=2, omega=2.0 / 3.0, small_solver="auto", device="cuda:0", locking=True, guard=0,
                 start="given", fallback_ratio=0.5, coarse_level=None, aug_rtol=1e-2, tensor=None, reaction=None,
                 hierarchy=None):
        self.lib = nat.load()
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        prob = nat.Problem()
        self._csr_keep = None
        if hierarchy is not None:
            if kappa is not None or tensor is not None:
                raise ValueError("hierarchy excludes kappa and tensor")
            mats = {}
            for key in ("A", "M", "P", "R"):
                mats[key] = [None if m is None else (m if isinstance(m, CsrMatrix) else CsrMatrix.from_scipy(m, device))
                             for m in hierarchy[key]]
            nl = len(mats["A"])
            if not 2 <= nl <= nat.MAX_LEVELS or any(len(mats[key]) != nl for key in mats):
                raise ValueError("hierarchy: 2..8 levels, the same count for A, M, P, R")
            hs = nat.HierarchyCsr()
            hs.nlevels = nl
            for key in ("A", "M", "P", "R"):
                arr = getattr(hs, key)
                for l, m in enumerate(mats[key]):
                    if m is not None:
                        arr[l] = m._struct()
            self._csr_keep = (mats, hs)
            prob.csr = C.cast(C.pointer(hs), C.c_void_p)
            self.dim = 0
            self.levels = [m.rows for m in mats["A"]]
            dim, levels = 0, []
        else:
            self.dim = int(dim)
            self.levels = [int(n) for n in levels]
            prob.dim = self.dim
            prob.nlevels = len(self.levels)
            if not 2 <= prob.nlevels <= nat.MAX_LEVELS:
                raise ValueError("need 2..8 levels")
            for i, n in enumerate(self.levels):
                prob.n[i] = n
        self._kappa = None
        if kappa is not None:
            ne = self.levels[0] ** self.dim
            kt = torch.as_tensor(kappa, dtype=torch.float64).reshape(-1)
            if kt.numel() != ne:
                raise ValueError(f"kappa must have {ne} entries")
            self._kappa = kt.to(self.device).contiguous()
        prob.kappa = _ptr(self._kappa)
        self._tensor = self._reaction = None
        if tensor is not None:
            ne = self.levels[0] ** self.dim
            self._tensor = torch.as_tensor(tensor, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
            if self._tensor.numel() != 6 * ne:
                raise ValueError(f"tensor must have {6 * ne} entries")
            if reaction is not None:
                self._reaction = torch.as_tensor(reaction, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
                if self._reaction.numel() != ne:
                    raise ValueError(f"reaction must have {ne} entries")
        elif reaction is not None:
            raise ValueError("reaction needs tensor")
        prob.tensor = _ptr(self._tensor)
        prob.reaction = _ptr(self._reaction)
        opt = nat.Options()
        self.lib.pase_options_default(C.byref(opt))
        opt.precision = nat.PREC[precision]
        opt.nev_max = int(nev_max)
        opt.cg_steps = int(cg_steps)
        opt.max_outer = int(max_outer)
        opt.nu = int(nu)
        opt.omega = float(omega)
        opt.small_solver = {"auto": 0, "dense": 1, "gcg": 2}[small_solver]
        opt.locking = 1 if locking else 0
        opt.guard = int(guard)
        opt.start = {"given": 0, "coarse": 1}[start]
        opt.fallback_ratio = float(fallback_ratio)
        opt.coarse_level = 0 if coarse_level is None else int(coarse_level)
        opt.aug_rtol = float(aug_rtol)
        self.opt = opt
        nbytes = C.c_size_t(0)
        self._check(self.lib.pase_workspace_bytes(C.byref(prob), C.byref(opt), C.byref(nbytes)), None)
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = self.lib.pase_setup(C.byref(prob), C.byref(opt), _ptr(self.workspace), nbytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._check(st, None)
        self.h = h
        self._kappa = None
        self.N = [self.level_size(l) for l in range(len(self.levels))]

    # ------------------------------------------------------------------ helpers
    def _check(self, st, h):
        if st != 0:
            msg = self.lib.pase_last_error(h if h is not None else None)
            raise PaseError(st, msg.decode() if msg else "")

    def _mv(self, t, rows, k, name, dtype=torch.float64):
        if not (isinstance(t, torch.Tensor) and t.device == self.device and t.dtype == dtype):
            raise TypeError(f"{name} must be a {dtype} tensor on {self.device}")
        if t.shape != (rows, k) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {rows} x {k} tensor")
        return t

    def _new(self, rows, k):
        return torch.empty((rows, k), dtype=torch.float64, device=self.device)

    def export_csr(self, level, which):
        """The grid hierarchy's operator as a CsrMatrix on the device: which = "A", "M" (level l),
        "P" (interpolation from level l to l - 1) or "R" (P^T)."""
        w = {"A": 0, "M": 1, "P": 2, "R": 3}[which]
        rows, cols, slots = C.c_int(0), C.c_int(0), C.c_int(0)
        self._check(self.lib.pase_export_csr(self.h, int(level), w, C.byref(rows), C.byref(cols), C.byref(slots),
                                             None, None, None), self.h)
        r, c, sl = rows.value, cols.value, slots.value
        rowptr = torch.empty(r + 1, dtype=torch.int32, device=self.device)
        colind = torch.empty(r * sl, dtype=torch.int32, device=self.device)
        val = torch.empty(r * sl, dtype=torch.float64, device=self.device)
        self._check(self.lib.pase_export_csr(self.h, int(level), w, C.byref(rows), C.byref(cols), C.byref(slots),
                                             _ptr(rowptr), _ptr(colind), _ptr(val)), self.h)
        return CsrMatrix(r, c, rowptr, colind, val)

    def export_hierarchy(self):
        """The whole hierarchy, in the form the hierarchy= argument takes."""
        L = len(self.levels)
        return {"A": [self.export_csr(l, "A") for l in range(L)], "M": [self.export_csr(l, "M") for l in range(L)],
                "P": [None] + [self.export_csr(l, "P") for l in range(1, L)],
                "R": [None] + [self.export_csr(l, "R") for l in range(1, L)]}

    def level_size(self, level):
        n = C.c_longlong(0)
        self._check(self.lib.pase_level_size(self.h, int(level), C.byref(n)), self.h)
        return int(n.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pase_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ solve
    def solve(self, nev, tol, U0, history=False, raise_notconv=True):
        """nev smallest eigenpairs.  Returns (lam [np], U [torch N x nev], report dict)."""
        N = self.N[0]
        if U0 is not None:
            U0 = self._mv(U0, N, nev, "U0")
        U = self._new(N, nev)
        lam = np.zeros(nev)
        res = np.zeros(nev)
        lit = np.zeros(nev)
        hist = np.zeros((self.opt.max_outer + 1, nev)) if history else None
        paths = np.zeros(max(self.opt.max_outer, 1), dtype=np.int32)
        rep = nat.Report()
        rep.res_host = res.ctypes.data
        rep.res_literal_host = lit.ctypes.data
        rep.ritz_history_host = hist.ctypes.data if history else None
        rep.small_path_host = paths.ctypes.data
        st = self.lib.pase_solve(self.h, int(nev), float(tol), _ptr(U0), lam.ctypes.data, _ptr(U), C.byref(rep))
        report = {"outer_iters": rep.outer_iters, "n_converged": rep.n_converged, "res": res,
                  "res_literal": lit, "t_solve_ms": rep.t_solve_ms, "small_fast_iters": rep.small_fast_iters,
                  "small_path": paths[:rep.outer_iters].copy(), "learned_fallbacks": rep.learned_fallbacks,
                  "lowprec_projection_iters": rep.lowprec_projection_iters,
                  "fine_solve_columns": rep.fine_solve_columns,
                  "t_phase_ms": {name: float(rep.t_phase_ms[i]) for i, name in enumerate(nat.PHASES)},
                  "aug_iters": rep.aug_iters, "aug_restarts": rep.aug_restarts,
                  "status": nat.STATUS.get(st, st)}
        if history:
            report["ritz_history"] = hist[:rep.ritz_history_rows].copy()
        if st != 0 and not (st == 4 and not raise_notconv):
            self._check(st, self.h)
        return lam, U, report

    def _batch_report(self, rep, st, res):
        return {"outer_iters": rep.outer_iters, "n_converged": rep.n_converged, "res": res,
                "t_solve_ms": rep.t_solve_ms, "fine_solve_columns": rep.fine_solve_columns,
                "t_phase_ms": {name: float(rep.t_phase_ms[i]) for i, name in enumerate(nat.PHASES)},
                "status": nat.STATUS.get(st, st)}

    def solve_batch(self, first, nb, tol, raise_notconv=True):
        """Alg. 7 step 3: the pairs first .. first + nb - 1 (guard pairs from the options).
        Returns (lam [np], U [torch N x nb], report dict)."""
        U = self._new(self.N[0], nb)
        lam, res = np.zeros(nb), np.zeros(nb)
        rep = nat.Report()
        rep.res_host = res.ctypes.data
        st = self.lib.pase_solve_batch(self.h, int(first), int(nb), float(tol), lam.ctypes.data, _ptr(U), int(nb),
                                       C.byref(rep))
        report = self._batch_report(rep, st, res)
        if st != 0 and not (st == 4 and not raise_notconv):
            self._check(st, self.h)
        return lam, U, report

    def solve_batches(self, m, nb, tol, raise_notconv=True):
        """Alg. 7: the m smallest pairs in batches of nb.  Returns (lam, U [N x m], report)."""
        U = self._new(self.N[0], m)
        lam, res = np.zeros(m), np.zeros(m)
        rep = nat.Report()
        rep.res_host = res.ctypes.data
        st = self.lib.pase_solve_batches(self.h, int(m), int(nb), float(tol), lam.ctypes.data, _ptr(U), C.byref(rep))
        report = self._batch_report(rep, st, res)
        if st != 0 and not (st == 4 and not raise_notconv):
            self._check(st, self.h)
        return lam, U, report

    # ------------------------------------------------------------------ components
    def apply(self, level, X):
        k = X.shape[1]
        X = self._mv(X, self.N[level], k, "X")
        AX, MX = self._new(self.N[level], k), self._new(self.N[level], k)
        self._check(self.lib.pase_apply(self.h, int(level), k, _ptr(X), _ptr(AX), _ptr(MX)), self.h)
        return AX, MX

    def vcycle(self, B):
        k = B.shape[1]
        B = self._mv(B, self.N[0], k, "B")
        Z = self._new(self.N[0], k)
        self._check(self.lib.pase_vcycle(self.h, k, _ptr(B), _ptr(Z)), self.h)
        return Z

    def pcg(self, lam, U):
        k = U.shape[1]
        U = self._mv(U, self.N[0], k, "U")
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        W = self._new(self.N[0], k)
        self._check(self.lib.pase_pcg(self.h, k, lam.ctypes.data, _ptr(U), _ptr(W)), self.h)
        return W

    def restrict(self, Xf):
        k = Xf.shape[1]
        Xf = self._mv(Xf, self.N[0], k, "Xf")
        Xc = self._new(self.N[-1], k)
        self._check(self.lib.pase_restrict(self.h, k, _ptr(Xf), _ptr(Xc)), self.h)
        return Xc

    def prolong(self, Xc):
        k = Xc.shape[1]
        Xc = self._mv(Xc, self.N[-1], k, "Xc")
        Xf = self._new(self.N[0], k)
        self._check(self.lib.pase_prolong(self.h, k, _ptr(Xc), _ptr(Xf)), self.h)
        return Xf

    def gram(self, X, Y):
        N, k = X.shape
        X = self._mv(X, N, k, "X")
        Y = self._mv(Y, N, k, "Y")
        G = self._new(k, k)
        self._check(self.lib.pase_gram(self.h, int(N), k, _ptr(X), _ptr(Y), _ptr(G)), self.h)
        return G

    def gram_bf16x3(self, X, Y):
        """X^T Y of float32 N x k blocks (k <= 128) by split-BF16 products, FP64 result."""
        N, k = X.shape
        X = self._mv(X, N, k, "X", torch.float32)
        Y = self._mv(Y, N, k, "Y", torch.float32)
        G = self._new(k, k)
        self._check(self.lib.pase_gram_bf16x3(self.h, int(N), k, _ptr(X), _ptr(Y), _ptr(G)), self.h)
        return G

    def small_eig(self, T, k):
        n = T.shape[0]
        T = self._mv(T, n, n, "T")
        w = np.zeros(k)
        V = self._new(n, k)
        self._check(self.lib.pase_small_eig(self.h, n, int(k), _ptr(T), w.ctypes.data, _ptr(V)), self.h)
        return w, V

    def small_eig_max_n(self):
        return int(self.lib.pase_small_eig_max_n(self.h))

    KERNELS = {"sweep": 0, "apply": 1, "gram": 2, "vcycle": 3, "cg_update": 5, "apply_A": 6, "apply_M": 7}

    def time_kernel(self, name, k, reps=20):
        """Average device ms per launch of a hot-path kernel (HIP events on the solver's stream)."""
        ms = C.c_double(0.0)
        self._check(self.lib.pase_time_kernel(self.h, self.KERNELS[name], int(k), int(reps), C.byref(ms)), self.h)
        return float(ms.value)

    # ------------------------------------------------------------------ learned form
    def attach(self, net):
        """Use the UNet `net` as the PCG preconditioner (precision="learned" only)."""
        self._check(self.lib.pase_attach_unet(self.h, net.h), self.h)
        self._net = net          # keeps the network's memory alive while attached

    def harvest(self, lam, U):
        """Training pair for the network: R = Lambda M U - A U and V = V-cycle(R)."""
        k = U.shape[1]
        U = self._mv(U, self.N[0], k, "U")
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        R, V = self._new(self.N[0], k), self._new(self.N[0], k)
        self._check(self.lib.pase_harvest(self.h, k, lam.ctypes.data, _ptr(U), _ptr(R), _ptr(V)), self.h)
        return R, V

    def fine_diag_inverse(self):
        """1 / A_ii at the fine nodes (the learned form's network output scale)."""
        out = torch.empty(self.N[0], dtype=torch.float64, device=self.device)
        self._check(self.lib.pase_fine_diag_inverse(self.h, _ptr(out)), self.h)
        return out

    def node_logk(self):
        """Node average of log kappa on the fine mesh (the network's second input)."""
        out = torch.empty(self.N[0], dtype=torch.float64, device=self.device)
        self._check(self.lib.pase_node_logk(self.h, _ptr(out)), self.h)
        return out

    def correction(self, lam, U):
        k = U.shape[1]
        U = self._mv(U, self.N[0], k, "U").clone()
        lam = np.array(lam, dtype=np.float64)
        self._check(self.lib.pase_correction(self.h, k, lam.ctypes.data, _ptr(U)), self.h)
        return lam, U
