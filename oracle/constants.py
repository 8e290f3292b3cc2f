"""Physical constants (cgs) and the fit coefficients printed in the paper.

The paper prints no values for the physical constants (Sections II.A-II.C);
CODATA-2018 cgs values are used.  The fit coefficients are the ones printed in
Section II: bremsstrahlung (II.A), the Pacholczyk emissivity prefactor and the
Mahadevan fit for I'(x) (II.B).  Part of the oracle: test infrastructure only.
"""
import math

# --- CODATA 2018, cgs -------------------------------------------------------
C_LIGHT = 2.99792458e10          # cm s^-1
K_B = 1.380649e-16               # erg K^-1
H_PLANCK = 6.62607015e-27        # erg s
M_E = 9.1093837015e-28           # g
M_P = 1.67262192369e-24          # g
E_CHARGE = 4.803204712570263e-10  # esu (1.602176634e-19 C * c / 10)
SIGMA_T = 6.6524587321e-25       # cm^2
SIGMA_SB = 5.670374419e-5        # erg cm^-2 s^-1 K^-4
G_NEWTON = 6.67430e-8            # cm^3 g^-1 s^-2
M_SUN = 1.98847e33               # g

ME_C2 = M_E * C_LIGHT ** 2       # erg
MP_C2 = M_P * C_LIGHT ** 2       # erg

# --- Section II.A: bremsstrahlung fits ---------------------------------------
BREM_EE_NORM = 2.56e-22
BREM_EE_LOW = (1.1, 1.0, 1.25)   # theta^1.5 (1 + 1.1 th + th^2 - 1.25 th^2.5)
BREM_EE_HIGH = (1.34, 1.123, 1.28)  # 1.34 th [ln(1.123 th) + 1.28]
BREM_EI_NORM = 1.48e-22
BREM_EI_LOW = (1.781, 1.34)      # 4 (2 th / pi^3)^0.5 [1 + 1.781 th^1.34]
BREM_EI_HIGH = (1.123, 0.48, 1.5)  # 9 th / (2 pi) [ln(1.123 th + 0.48) + 1.5]

# --- Section II.B: synchrotron ------------------------------------------------
SYN_EPS_NORM = 4.43e-30          # eq. optically_thin_synch prefactor
IPRIME_NORM = 4.0505             # eq. fitting_I(xm)
IPRIME_C1 = 0.4                  # coefficient of x^-1/4
IPRIME_C2 = 0.5316               # coefficient of x^-1/2
IPRIME_A = 1.8899                # exp(-1.8899 x^1/3)
SYN_LOWT_SWITCH = 1.0e8          # K; K2(1/theta) -> 2 theta^2 at or below this

# --- Section II.G: Coulomb exchange ------------------------------------------
LN_LAMBDA = 20.0                 # Coulomb logarithm (reading: ln Lambda = 20)

# --- Section III.B: internal energy, gamma = 5/3 (Section III.C) --------------
GAMMA_AD = 5.0 / 3.0
U_PER_NKT = 1.0 / (GAMMA_AD - 1.0)  # u = n k T / (gamma - 1) = 1.5 n k T

# --- Section III.B.1: explicit limiter ---------------------------------------
EXPLICIT_CAP = 0.30
EXPLICIT_SUBSTEPS = 16

SQRT3 = math.sqrt(3.0)
