"""The interpolation order of the throughput workload, chosen by the method's own
interpolation error (ORACLE-M(K) against ORACLE-X, P24) on the CPU.

Templates: the Tab. I precessing injection and the lightest, a light, a median and the
heaviest of a draw from the workload's distribution (precessing, five modes, Kepler arms,
TDI 2.0), 4096 samples at 5 s with the merger 1000 s before the end; errors over the
interior samples 400 .. 2599 (away from the grid's edges).

Tolerance 1e-6 of the channel: the FP32 rounding floor of the mixed-precision response
(24 sqrt(K) u max|h| at u = 2^-24 is ~1e-6 of the channel for the Tab. I system): a larger K
buys nothing once its error is below that.  The choice is K = 8 (K = 6 misses by an order
of magnitude on the lightest template, whose ringdown is barely resolved at 5 s), the value
the benchmark and the sampler use."""
import numpy as np

from oracle.taps import choose_taps, interp_error
from paper_2501_08261_amd import inputs

TOL = 1e-6


def _templates(g):
    rnd = inputs.draw_templates(8, 40, g, precessing=True, before_end=1000.0)
    order = np.argsort(rnd[:, 0] + rnd[:, 1])
    return [rnd[order[0]], inputs.tab1_injection(True, g, before_end=1000.0), rnd[order[5]], rnd[order[39]]]


def test_taps_chosen_by_interpolation_error():
    g = inputs.grid(4096, 5.0)
    idx = np.arange(400, 2600)
    K, worst = choose_taps(_templates(g), g, idx, TOL, candidates=(4, 6, 8, 12))
    print(worst)
    assert K == 8
    assert worst[6] > 10 * TOL          # the next smaller order fails clearly
    assert worst[8] < TOL


def test_linear_interpolation_error():
    """K = 2, the paper's linear interpolation, errs by ~3e-3 of the channel on the Tab. I
    injection (and more on lighter templates): far above the FP32 floor."""
    g = inputs.grid(4096, 5.0)
    e = interp_error(inputs.tab1_injection(True, g, before_end=1000.0), 2, g, np.arange(400, 2600))
    assert 1e-3 < e < 1e-2
