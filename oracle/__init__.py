"""Reference oracle for the multi-rhs Wilson-Dirac operator and batched GMRES.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128 NumPy
implementation of what the hot path computes, written from the paper's
definitions (Sec. III-A.1 Wilson-Dirac operator and Algorithm 1, Sec. III-A.2
Algorithm 2 and odd-even preconditioning).  It uses the full 4x4 gamma
matrices and no spin projection, so it shares no arithmetic with the HIP
kernels.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library never does.

Modules:
  geometry      site numbering, neighbours, parity, odd-even compact maps
  gamma         Euclidean chiral gamma matrices
  dirac         D_W applied to a block of spinors, its adjoint, dense assembly
  evenodd       Schur complement, source preparation, odd reconstruction
  gmres         batched restarted GMRES (Algorithm 2) and GMRES with
                iterative refinement in a lower working precision
  gradients     backward of the apply and of the solve, su(3) force
  closed_forms  free-field symbols used to pin the apply (derived)
"""
