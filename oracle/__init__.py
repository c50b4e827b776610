"""Plain FP64 CPU oracle for sketched block orthogonalization and s-step GMRES.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or load
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the HIP implementation; the
two meet only in the seeded input generators (``paper_2503_16717_amd.workloads``)
and in the published definition of the SplitMix64 counter generator that both
sides implement independently for the sparse-sign sketch.

Every routine is a slow, direct transcription of the mathematics (numpy float64;
loops where the order of operations matters) and cites the passage of the paper
it follows (arXiv:2503.16717, "Random sketching to enhance the numerical
stability of block orthogonalization algorithms for s-step GMRES").

Modules
  sketch   -- Gaussian and sparse-sign sketches (Section 3; Section 5.2)
  dense    -- Householder QR, Cholesky, right triangular solve (Figs. 2b, 4a)
  orth     -- CholQR/CholQR2, RandHH/RandCholQR, BCGS2, two-stage (Sections 4-7)
  krylov   -- CSR SpMV, matrix-powers kernel, s-step GMRES (Section 4, Fig. 1; Fig. 5)
  metrics  -- orthogonality / backward error with compensated accumulation
"""
from . import sketch, dense, orth, krylov, metrics  # noqa: F401
