"""Algorithmic work per template-sample of the fused TDI response kernel.

Used for roofline accounting only.  Counts are the floating-point operations
of the closed forms as written (a fused multiply-add counts 2; sqrt, cbrt,
divide, sin, cos, tanh count 1 each), not instruction counts of the build:

* Lagrange interpolation with K taps: weights 5K (K differences, prefix and
  suffix products, normalisation) plus 2K per interpolated series.
* link response y at one grid sample: 6 links x 2 delayed reads x (5K + 2x2K)
  for h+ and hx, cubic interpolation of 4 node quantities per link (6 x 4 x 8),
  and the projection (6 x 5).
* TDI at one output sample: 3 channels x (terms with a nonzero delay) x
  (5K + 2K), the delay sums (terms x 6 x 2), 6 light-time interpolations x 8,
  and A, E, T (10).
* waveform + twist-up at one grid sample (FP64): aligned ~ 120, precessing
  with five co-precessing modes ~ 800 (Euler angles, quaternion products,
  powers of Q_a, Q_b, the ten Wigner-D polynomials, the mode sum).  The h
  window exceeds the output tile by ~7 % (halos).
"""


def tdi_flops_per_sample(taps, generation, precessing=True, modes=5):
    K = taps
    y = 6 * 2 * (5 * K + 2 * 2 * K) + 6 * 4 * 8 + 6 * 5
    terms_nonzero = 14 if generation == 20 else 6
    terms_all = 16 if generation == 20 else 8
    tdi = 3 * terms_nonzero * (5 * K + 2 * K) + 3 * terms_all * 6 * 2 + 6 * 8 + 10
    wave = (800 if precessing else 120) * modes / 5.0
    return 1.07 * wave + y + tdi
