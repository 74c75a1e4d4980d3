"""CPU FP64 oracle for inverse factorization -- TEST INFRASTRUCTURE ONLY.

Plain, slow, dense numpy implementations of what the GPU path computes:

* ``refinement``: block truncation, the refinement coefficients, iterative
  refinement from a scaled identity (IRSI), localized inverse factorization
  (LIF, Alg. 2) and the recursive inverse Cholesky algorithm (RINCH, Alg. 1);
* ``closed_forms``: the exact results these methods reach without truncation
  (Loewdin S^{-1/2}, inverse Cholesky, the recursive LIF limit), the spectral
  map of one refinement step and the iteration bound of Sec. 3.3;
* ``adjoint``: the reverse sweep of refinement and LIF for L = tr(G^T Z) and
  dense references for it;
* ``blocks``: single output blocks of a block-sparse product, for sampled
  checks at sizes the dense oracle cannot hold;
* ``blocked``: the same IRSI, LIF and RINCH steps on block lists, for sizes
  the dense oracle cannot hold; its products run in ``bsmm.c`` (plain C
  with OpenMP over output rows, built by ``build.py`` into ``libbsmm.so``)
  when that is built, else in a Python loop, the two pinned to each other.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library and never calls it.
"""
