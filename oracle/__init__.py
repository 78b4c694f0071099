"""CPU oracle for randomized QLP (Rand-QLP) -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, fp64 restatement of what the GPU path computes,
written from the paper (Kaloorazi, Liu, Chen, de Lamare, "An Efficient
Randomized QLP Algorithm for Approximating the Singular Value Decomposition",
arXiv 2110.01011).  It exists only so that tests, the smoke check and the
benchmark's CPU-baseline leg can check and time the HIP implementation.
The product path (``paper_2110_01011_amd``) never imports it, and it never
imports the product path: the two share no code.

Modules
  philox  -- Philox4x64-10 counter generator and the Gaussian test matrix
             (Algorithm 1, the ``randn`` step), from the published definition.
  randqlp -- Algorithm 1 generalised to d = k + p sketch columns and q power
             iterations; reduced unpivoted QR with a non-negative R diagonal.
  jacobi  -- one-sided (Hestenes) Jacobi SVD for tiny brute-force checks.
  bounds  -- the per-sample quantities of Theorems 1-3 (Section 4.1).
  flops   -- the flop model of Section 4.2, generalised to (d, q).
"""
from .philox import philox4x64_10, gaussian_matrix, uniforms_from_words  # noqa: F401
from .randqlp import (qr_pos, randqlp, sketch_width, rel_error,  # noqa: F401
                      subspace_sine, orth_error)
from .flops import randqlp_flops, paper_flops_full  # noqa: F401
from .jacobi import jacobi_singular_values  # noqa: F401
