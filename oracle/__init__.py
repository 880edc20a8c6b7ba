"""Plain FP64 CPU oracle of Scalable Laplacian K-modes (Ziko, Granger, Ben Ayed, NeurIPS 2018).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU library
and never imports it; the product path must not route through it.

Modules:
  slk    -- the method step by step: kNN affinity, bandwidth, unary affinities,
            the bound-optimizer z-update, relaxed bound, labels, byproduct modes,
            discrete energy and the outer/inner driver (SLK-BO).
  brute  -- brute-force minimisation of the discrete objective over all labelings
            with modes taken by their definition (small N only).
"""
from . import slk, brute  # noqa: F401
