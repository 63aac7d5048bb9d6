"""FP64 CPU oracle for the DG p-multigrid Poisson solver (test infrastructure only).

This package is a plain, slow, obviously-correct restatement of the paper's
method (Stiller, "Robust multigrid for high-order discontinuous Galerkin
methods: a fast Poisson solver suitable for high-aspect ratio Cartesian
grids", arXiv:1603.02524) in numpy/scipy, double precision throughout.

It exists to check the HIP library, and only ``tests/``, the smoke entry
point and the CPU-baseline leg of the benchmark may import it.  It shares no
code, tables or constants with the HIP path; the only common import is the
``synth`` package of seeded inputs, which holds no arithmetic of the method.

Modules
-------
gll        1D spectral toolkit: GLL nodes/weights, differentiation, stiffness,
           embedded interpolation (Sec. 2.4, Sec. 3.2).
operator   the system matrix A, assembled three independent ways
           (textbook SIPG form; mixed LDG form; Kronecker sum of the 1D
           operators of the primal form, eq. (discrete problem)).
schwarz    element- and face-centred subdomains, weights, dense and
           fast-diagonalisation patch solves, additive Schwarz sweeps (Sec. 3.1).
multigrid  level series, transfers, exact coarse solve, V-cycle (Alg. 1) and
           inexact MG-preconditioned CG (Alg. 2).
se         the continuous spectral-element counterpart of Sec. 4.3: direct
           stiffness summation, transfers, element-centred weighted additive
           Schwarz on continuous subdomains (the V-cycle and MGCG are shared).
metrics    convergence and cost measures of Sec. 4.1.
mlp        FP64 reference of the small overlap-weight network (not in the paper).

Parity status per function is stated in each module header; every function
listed there is pinned by a ``-m "not gpu"`` test unless marked
"parity unpinned".
"""
