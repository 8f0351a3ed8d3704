"""Plain FP64 CPU oracle of the augmented subspace eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls or links anything here; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.
It shares no code with the GPU path: the only common module is ``synth``,
which draws the seeded inputs and holds none of the method's arithmetic.

Written from the paper (Xie et al., "A parallel augmented subspace
eigensolver", arXiv 2502.04589) with NumPy/SciPy in float64:

* ``fem``        -- the model problem and its Q1 discretisation (Sec. 2.1).
* ``multigrid``  -- nested spaces, interpolation I_H^h, Galerkin coarse
                    operators (Alg. 3 inputs, Sec. 5.1) and the geometric
                    multigrid V-cycle used to precondition the fine solves.
* ``pase``       -- the outer loop: fine linear solves by CG (Alg. 3 step 3),
                    composite matrices (eq. Definition_Hh), the augmented
                    eigenproblem (Alg. 3 steps 5-6) and the stopping rule
                    (Sec. 5, opening paragraph).
* ``gcg_aug``    -- PRECOND-A (the block factorisation of eq.
                    Transformation_0 and the pencil of eq. Eigen_Problem_Hh_2)
                    and the GCG_AUG eigensolver of the augmented problem
                    (Sec. 4, Alg. 4 and 5), used by ``pase.solve(small=
                    "precond_a")`` with V_H on any level of the hierarchy.
* ``batch``      -- the batch scheme for many eigenpairs (Alg. 7): per batch a
                    shift, the composite pairs nearest it and the selection of
                    eq. largest_component, with guard pairs on both sides.
* ``reference``  -- the fixed point written out: the k smallest eigenpairs of
                    the assembled pencil by a library eigensolver (Alg. 3
                    "Ensure").
* ``unet``       -- the learned form's preconditioner (a small 3D U-Net with
                    hand-written backward pass), its loss and Adam optimiser,
                    and the flexible PCG with fallback to the V-cycle.  The
                    paper does not define this extension; the readings are in
                    the module docstring.

Readings of points the paper leaves open are listed in the docstrings where
they are taken.
"""
from . import batch, fem, gcg_aug, multigrid, pase, reference, unet  # noqa: F401
