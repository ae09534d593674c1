"""Physical constants used by the oracle (CODATA 2018, cgs).

The paper fixes R* = 1e6 cm (Sec. 2.2, the drag-length estimate) and
B_QED = m_e^2 c^3 / (hbar e) = 4.4e13 G (Sec. 1, Eq. elandau).  Field strengths
enter only as b = B/B_QED, so B_QED itself is never needed numerically.
"""

R_E_CM = 2.8179403262e-13          # classical electron radius r_e [cm]
LAMBDABAR_CM = 3.8615926796e-11    # reduced Compton wavelength hbar/(m_e c) [cm]
ME_C2_KEV = 510.99895000           # electron rest energy [keV]
R_STAR_CM = 1.0e6                  # stellar radius used by the paper [cm]
