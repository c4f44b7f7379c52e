"""CPU FP64 oracle for the CISOR hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct numpy/scipy implementation of
what the GPU library computes, written directly from the paper (arXiv
1708.01663: "Problem Formulation", "Proposed Method", and the appendix proofs).
Only the test suite, the package's smoke check and the benchmark's CPU-baseline
leg may import it.  The product path never calls into it, and it shares no
code with the HIP library (only the seeded input generators in ``synth``).

Modules
-------
geometry   cell-centred grids, plane-wave incident fields, receiver rings.
green      discretised Green's function: equal-area cell integrals of the
           scalar Green's function (2D Hankel, 3D spherical wave), the padded
           FFT kernel, dense matrices for brute force.
operators  matrix-free ``A = I - G diag(f)`` and its adjoint via FFT.
krylov     BiCGSTAB in FP64 and a dense direct solve.
cisor      forward model, misfit, Prop. 1 gradient, dense-Jacobian gradient.
tv         isotropic TV value and the FGP proximal map with box constraint.
fista      relaxed FISTA (eqs. algo1-algo3).
stepsize   Born Gauss-Newton Lipschitz estimate used to pick a step size.

Pins: every function is checked by the ``-m "not gpu"`` tests against
something other than itself (closed forms, brute force, invariants).  See the
module docstrings for which pin covers which function.
"""
