"""Algorithmic work per template-sample of the fused response / TDI kernel.

Used for roofline accounting only.  The count is the direct method's, whatever
shortcuts the kernel takes: every interpolation at a delayed time needs one
set of K Lagrange weights (3K flops: K differences and the two running
products) and one K-tap dot product per interpolated series (2K flops, a
fused multiply-add counting 2).

* TDI 2.0, per output sample: the six links read h+ and hx at 3 receiver and
  6 sender times (9 weight sets, 18 dot products); X, Y, Z have 3 x 16 terms,
  of which 3 x 14 are delayed (42 weight sets, 42 dot products); the orbit
  and delay interpolations and the y projections bring the totals to about
  60 weight sets and 72 dot products, i.e. 60 * 3K + 72 * 2K = 324 K flops
  (2592 at K = 8).
* TDI 1.5: 36 weight sets and 48 dot products, i.e. 204 K flops.

The waveform kernel is not included (it is a separate launch).
"""


def tdi_flops_per_sample(taps, generation):
    K = taps
    if generation == 20:
        return 60 * 3 * K + 72 * 2 * K
    return 36 * 3 * K + 48 * 2 * K


# One multiply-add per lane per clock on every SIMD: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# x 2.4 GHz = 78.6 TFLOP/s, the vector FP64 peak and the FP32 peak without packed (two-wide)
# FP32 instructions, which this build does not emit.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
CLOCK_HZ = 2.4e9
N_CU = 256


def executed_flops(fma_f32_insts, fma_f64_insts):
    """Flops of issued multiply-add wave-instructions (64 lanes, 2 flops each), from the
    SQ_INSTS_VALU_FMA_F32 / _F64 counters of one launch."""
    return 128.0 * (fma_f32_insts + fma_f64_insts)


def issue_rate(valu_insts, seconds):
    """VALU wave-instructions issued per clock per CU over a launch of `seconds`."""
    return valu_insts / (seconds * CLOCK_HZ * N_CU)

