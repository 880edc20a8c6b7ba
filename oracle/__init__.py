"""Plain FP64 CPU oracle of Scalable Laplacian K-modes (Ziko, Granger, Ben Ayed, NeurIPS 2018).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU library
and never imports it; the product path must not route through it.

Modules:
  slk    -- the method step by step: kNN affinity, bandwidth, unary affinities,
            the bound-optimizer z-update, relaxed bound, labels, byproduct modes,
            discrete energy and the outer/inner loops (SLK-BO).
  brute  -- brute-force minimisation of the discrete objective over all labelings
            with modes taken by their definition (small N only).
  extend -- out-of-sample assignment and the SLK-MS mean-shift mode update.
  seeding -- K-means++ seeding, the nearest-seed assignment and the exact modes of
            Eqs. (1) and (10).
"""
from . import slk, brute, extend, seeding  # noqa: F401
