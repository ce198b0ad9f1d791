"""Plain FP64 CPU oracle for the time-domain LISA likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code, tables or constants with the HIP path.

Every function follows the paper (arXiv:2501.08261, "GPU-accelerated LISA
parameter estimation with full time domain response") section by section and
is written for readability, not speed:

  waveform.py   Sec. II.A  -- the PhenomT-form co-precessing modes
  twist.py      Sec. II.A  -- Euler angles, quaternions (Eq. 2.5), Wigner-D
                             (Eq. 2.6), explicit (Eqs. 2.1-2.3) and
                             single-sum (Eq. 2.4) twist-up
  orbits.py     Sec. II.B  -- spacecraft positions and light travel times
  response.py   Sec. II.B  -- link responses (Eq. 2.8), TDI 1.5 / 2.0
                             (Eqs. 2.9-2.10), A, E, T (Eq. 2.11)
  likelihood.py Sec. II.B  -- PSD (Eqs. 2.14-2.15), inner product (Eq. 2.13),
                             log-likelihood (Eq. 2.12 and its footnote)
  fisher.py     Sec. II.C  -- Fisher matrix and Fisher initialisation
  sampler.py    Sec. II.C  -- ensemble / parallel-tempering MCMC
  flow.py       (learned proposal; not in the paper) -- RealNVP flow

Parity status of each function is stated in its docstring; functions whose
agreement with the paper's (unpublished) code cannot be checked say
"parity unpinned".
"""
