"""CPU FP64 oracle for Gaussian-kernel ridge regression with HSS solvers.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the GPU path computes; it exists so that tests, the smoke
check and the CPU baseline leg of the benchmark can compare against it.  The
product library never imports, links or calls anything here, and nothing here
imports the product package: the two share only the seeded input generators
in `synthdata`.

Contents (each function cites the passage of the paper it follows):
  kernel    dense Gaussian kernel, dense Cholesky KRR, prediction, accuracy
  cluster   recursive two-means ordering and cluster tree (C, exact spec)
  hss       HSS reference built by nested interpolative decompositions of
            dense block rows, dense assembly of any HSS given its generators
  grad      validation-loss gradients in (log h, log lambda) and the fused
            kernel-product backward, dense FP64
  cmath     FP64 matrix-free kernel products in C (large-n residuals, samples)

Parity status: every function is pinned by the `-m "not gpu"` tests in
tests/test_oracle_*.py against closed forms, limits, brute force or library
special cases.  The two-means ordering is pinned to its own written spec plus
invariants (valid permutation, leaf sizes, Lloyd fixed point, separated-group
brute force); against the paper itself its exact permutation is "parity
unpinned", because the paper prints no permutation and any Lloyd local optimum
is a valid two-means split.
"""
from . import kernel, cluster, hss, grad, cmath  # noqa: F401
