"""CPU oracle for the Krylov phi-combination (test infrastructure only).

This package is a plain, slow, float64 reference for what the HIP library
computes.  It is test infrastructure: only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  The product path never calls
it, and it shares no code with the HIP kernels (the only common module is the
seeded input generator in `workloads`, which holds no arithmetic of the
method).

Contents, each following the passage of arXiv:2410.14917 it implements:

  phi.py          phi_k scalar functions (eq. phi_int_def), dense matrix
                  exponential by Taylor series with scaling and squaring, and
                  the dense augmented-matrix definition of the phi combination
                  (Section 2.1, eq. philincomb).
  operators.py    the matrix-free 2D periodic operators (second-order finite
                  differences as in Section 4.3) and their transposes.
  arnoldi.py      Arnoldi with modified Gram-Schmidt (Algorithm 1), the
                  hybrid low-synchronization Arnoldi (Algorithm 4 with the
                  correction matrices of Algorithms 5, 6 and 7) and the
                  incomplete classical Gram-Schmidt process (Section 2.3.1).
  krylov.py       Krylov projection of the exponential (eq. kryexp), substepping
                  (Section 2.2, eq. substep) with a fixed schedule or an adaptive
                  controller, applied to the augmented matrix.
  closed_form.py  closed forms that pin the above: DFT diagonalisation of
                  constant-coefficient periodic stencils and elementwise phi_k
                  for diagonal operators.
  adjoint.py      derivatives of the phi combination (block-triangular
                  exponential of the Frechet derivative, transposed solves).
  integrators.py  the exponential integrators of Section 4.1 (EPI4, EPI5,
                  SRERK3) that drive the phi combination.

Parity status of each function is stated in its docstring; every function here
is pinned by a `-m "not gpu"` test against something other than itself.
"""
