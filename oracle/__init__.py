"""Plain FP64 CPU oracle for AMG block-preconditioned GMRES on the multi-group
radiation-diffusion block system (Yue, Zhang, Xu, Shu, Shi, "Algebraic
multigrid block preconditioning for multi-group radiation diffusion
equations", arXiv 2002.04958).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; it exists so that tests, the smoke check and the CPU
baseline leg of the benchmark can compare the GPU library against an
independent, slow, obviously correct implementation.  It shares no code with
the GPU path; both consume the arrays drawn by ``synth_inputs``.

Modules
  assemble  block system of eq. 2.2 from per-cell coefficients
  amg       classical AMG: strength, PMIS and HMIS, modified classical
            interpolation, aggressive coarsening with multipass
            interpolation, Galerkin coarse operators, CF-l1-Jacobi and
            multicolour Gauss-Seidel V(1,1) cycles
  interp.c  the modified classical interpolation as a plain loop over rows
            (built by ``cext`` with gcc, loaded with ctypes)
  cext      builds and loads interp.c
  precond   monolithic AMG, block-diagonal, PCTL (Sec. 3.2), Schur1/Schur2
            (Sec. 3.3) with the diagonal approximations of Sec. 3.4, inner
            solves to a tolerance and option #4 (Sec. 3.4)
  adaptive  Definitions 1 and 2 and the preconditioners they select (Sec. 3.5)
  krylov    restarted right-preconditioned (flexible) GMRES(m)
  adjoint   transposed-system solve and coefficient gradients

Parity status: every function is pinned by a test in tests/test_oracle_*.py
except where its docstring says "parity unpinned".
"""
from . import assemble, amg, precond, krylov, adjoint  # noqa: F401
