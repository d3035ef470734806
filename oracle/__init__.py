"""FP64 CPU oracle for the high-order linear-elasticity operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It is a plain, slow, obviously-correct implementation written from the paper's
definitions, sharing no code with the GPU path:

* ``rules``       -- 1D Gauss-Legendre points/weights and Gauss-Lobatto-Legendre
                     nodes on [0,1]; Lagrange basis values and derivatives
                     (Sec. 4.4: (p+1) GLL nodes, (p+2) GL points; eq. 6).
* ``mesh``        -- structured-box geometry, node numbering, element Jacobians,
                     essential (clamped) dofs.
* ``elasticity``  -- element stiffness matrices by direct quadrature of the weak
                     form (eqs. 3-4) over full 3D basis functions (no sum
                     factorization), the global apply y = sum_e G_e^T K_e G_e x,
                     load vectors, the constrained operator, and the sum of
                     element magnitudes sum_e G_e^T |K_e| G_e x that scales the
                     rounding of an evaluation of A x.
* ``solvers``     -- direct solves (dense, and block Cholesky over x-slabs for
                     cantilevers of ~1e5 dofs), power iteration, Chebyshev
                     smoothing, p/h prolongation matrices, a dense V-cycle and
                     PCG (Sec. 3), used as references on small problems.

Parity status of each function is stated in its docstring; every function here
is pinned by a ``-m "not gpu"`` test (closed forms, invariants, exact symbolic
integration, textbook algorithms) except where it says "parity unpinned".
"""
