"""FP64 CPU oracle for the QFT->FFT transform (test infrastructure).

This package is test infrastructure, not part of the product. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import or
run it. It shares no code, tables or constants with the GPU library.

Contents
  qft_oracle.py  gate-by-gate state-vector simulation of the (approximate) QFT
                 circuit, the naive DFT, the closed-form AQFT matrix, the
                 per-target fused (DIF) form, metrics and AQFT error formulas.
  dft_bins.c     plain C per-output-bin sums (exact DFT and closed-form AQFT)
                 used to check sampled outputs of large transforms.
  qft_state.c    plain C (OpenMP) whole-vector per-target form, the same
                 steps as qft_fused_targets, for full outputs at n = 28-31.
"""

from .qft_oracle import *  # noqa: F401,F403
