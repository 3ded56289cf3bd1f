"""CPU FP64 oracle for the batched DNLS inner step (test infrastructure).

This package is a plain, slow, deliberately unoptimised restatement of what
the paper's method computes: Gauss-Newton / Levenberg-Marquardt steps on
Lie-group variables and the implicit-differentiation backward pass through
the final iterate.  It exists to check the HIP path; only the test-suite,
the smoke check and the benchmark's CPU-baseline leg may import it.  It
shares no code with the HIP library: its Lie-group maps, Jacobians and
linear algebra are written here from their mathematical definitions, with
PyTorch (CPU, float64) and SciPy used only as matrix primitives.

Modules
  lie      SE(2)/SE(3) exponential, logarithm, adjoint and right Jacobian
  costs    relative-pose, prior and pinhole reprojection costs with Jacobians
  solve    the inner loop, the final linearisation and the implicit backward
  toy      Euclidean problems with closed-form answers (curve fit, linear-Gaussian)

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` (library routines, finite differences, closed forms,
invariants); none is "parity unpinned".
"""
