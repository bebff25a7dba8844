"""CPU FP64 oracle for the range-space Schur solve of Choi, Farhat, Murray and
Saunders, "A practical factorization of a Schur complement for PDE-constrained
distributed optimal control" (arXiv 1312.5653).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library (the HIP/C-ABI path
under ``paper_1312_5653_amd``) may import, call, link or execute anything in
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  The oracle shares no code with
the GPU path: it assembles its own sparse matrices from the Q1 element
integrals and solves with SciPy's sparse direct solver (SuperLU), in FP64.

Modules
-------
fem      Q1 finite elements on the unit square / cube (Sec. 2, discrete QP).
kkt      KKT saddle-point system, its right-hand side and the accuracy metrics
         (Sec. 2 KKT system; Sec. 6.2 relative constraint violation).
solve    Direct solvers: the paper's two-factor range-space solve (Sec. 3.1
         Schur system + Sec. 4 complex factorization), the reduced real
         saddle system, dense brute force, and the closed form for sine
         targets.
feti     FETI-DP written out from its definitions (Sec. 5: signed Boolean
         matrices, interface operator F and right-hand side d, corner coarse
         problem, Dirichlet preconditioner) with dense local inverses, for
         small meshes.  Used to pin the GPU path's intermediate quantities.
elastic  Trilinear linear-elasticity elements on a box (Sec. 6.2 solid
         cantilever control): stiffness, vector mass, pressure and body
         loads, support reactions.  The KKT and range-space solvers above
         take its K and V unchanged.

Every function cites the passage of the paper it follows.  Where the paper is
silent, the reading taken is stated in the docstring.
"""
