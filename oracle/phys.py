"""Physical constants used by the oracle (SI units).  Test infrastructure only."""

C_SI = 299792458.0                 # speed of light [m/s]
MTSUN_SI = 4.925490947641267e-06   # G Msun / c^3 [s]
MPC_SI = 3.085677581491367e22      # megaparsec [m]
AU_SI = 1.495978707e11             # astronomical unit [m]
YEAR_SI = 31558149.763545603       # sidereal year [s]
ARM_SI = 2.5e9                     # LISA nominal arm length [m]
