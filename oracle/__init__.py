"""FP64 CPU oracle for the PCG-in-Split-Bregman hot path (test infrastructure).

This package is a plain, slow, obviously correct NumPy implementation of what
the paper's method computes, in float64 / complex128.  It exists only to check
the native HIP path: only the tests, the package smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the native library and
imports nothing from the product package.

Modules
  operators  the data model, the system operator A and its parts (Theory, Eqs.
             ill0, original, system; the difference operators with periodic
             boundaries)
  wavelet    periodised orthonormal wavelet transforms (Haar, Daubechies-4)
  precond    the circulant spectrum k (Eqs. K, Kdiag, precon, diagonalelements),
             its brute-force definition, Jacobi
  pcg        preconditioned conjugate gradients (Complexity section)
  sb         Split Bregman, Algorithm 1
  learned    the learned spectrum correction: CNN, loss, probe statistics
  coils      coil compression to virtual coils (Methods, Coil compression)
  volume     the 3D operator and its circulant spectrum (Discussion)

Parity status: every function here is pinned by the CPU tests against a dense
matrix built from the definition, a closed form, an invariant or a library
routine.  Split Bregman is pinned by closed-form scalar recurrences with inactive
shrinks and with active wavelet shrinks, and with active TV shrinks by its
limit: the inner loop reaches the minimiser of the convex objective that an
independent dual projected-gradient solve computes.  The learned correction's
training trajectory (minibatch order, Adam state over many steps) is pinned only
step by step.
"""
