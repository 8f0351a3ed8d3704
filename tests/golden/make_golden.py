"""Writes the stored expected values under tests/golden/ by calling only ``oracle``.

    python tests/golden/make_golden.py [name ...]

Each entry is the k smallest eigenvalues of the Q1 pencil of -div(kappa grad u) = lambda u
(Alg. 3 "Ensure"), computed by ``oracle.reference.lowest_eigenpairs`` from the seeded kappa field
of ``synth.kappa_field``, or of -div(A grad u) + phi u = lambda u (the tensor-coefficient workload,
Sec. 5 eq. general) assembled by ``oracle.fem.assemble_general`` from ``synth.general_coefficients``;
the file records the recipe beside the values.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fem, reference  # noqa: E402

# name: (dim, n, k, kappa seed or None)
CASES = {
    # the large coarse space path: 64^3 fine mesh, V_H = 16^3 (N_H = 3375), 120 pairs of a kappa field
    "kappa3d_64_s21_k120": (3, 64, 120, 21),
    # 32^3 fine mesh with the same 16^3 coarse space: 40 and 120 pairs of a kappa field
    "kappa3d_32_s5_k40": (3, 32, 40, 5),
    "kappa3d_32_s7_k120": (3, 32, 120, 7),
    # the tensor-coefficient + reaction workload on 32^3 and 64^3 meshes (kappa seed "general")
    "general3d_32_k40": (3, 32, 40, "general"),
    "general3d_64_k40": (3, 64, 40, "general"),
}


def write(name):
    dim, n, k, seed = CASES[name]
    t = time.time()
    path = os.path.join(HERE, name + ".npz")
    if seed == "general":
        tensor, reaction = synth.general_coefficients(n)
        w = reference.lowest_eigenpairs(dim, n, k, operator=fem.assemble_general(n, tensor, reaction))
        np.savez(path, lam=w, dim=dim, n=n, k=k, kappa_seed=-2,
                 recipe="oracle.reference.lowest_eigenpairs(dim, n, k, operator=oracle.fem.assemble_general("
                        "n, *synth.general_coefficients(n)))")
    else:
        kappa = None if seed is None else synth.kappa_field(dim, n, seed)
        w = reference.lowest_eigenpairs(dim, n, k, kappa)
        np.savez(path, lam=w, dim=dim, n=n, k=k, kappa_seed=-1 if seed is None else seed,
                 recipe="oracle.reference.lowest_eigenpairs(dim, n, k, synth.kappa_field(dim, n, kappa_seed))")
    print(f"{name}: {time.time() - t:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        write(name)
