"""Resonant inverse Compton scattering (RICS): rate, drag force, photon energy.

Follows Sec. 2.1 (resonance, Eqs. elandau, resomega), Sec. 2.2 (Planck
intensity, Eq. scatteringNdot for the scattering rate, Eq. contdrag for the
drag force) and Appendix A.3 (Eq. perpemit for the up-scattered photon
energy).  Normalisation as in Sec. 3: momenta p = gamma*beta (units m_e c),
force F_hat = F R*/(m_e c^2), i.e. dp/dt_hat = F_hat with t_hat = c t / R*;
the rate is likewise per unit t_hat (Ndot_hat = Ndot R*/c).

The event's kinematics (Appendix A.2-A.3) for a photon leaving the excited
lepton's rest frame at cosine mu_r from its motion: `emission`; mu_r = 0 is the
perpendicular emission of Eq. perpemit.

Closed forms (the radial beam from a blackbody of radius R* subtends
pi/x^2 steradian, which is the solid-angle factor behind the 1/(4 x^2) of
Eq. contdrag):

    y        = b / (Theta gamma (1 - beta mu))            Theta = kT/(m_e c^2)
    F_hat    = A_F / x^2 * gamma (mu - beta) * y^3/(e^y - 1)
    Ndot_hat = A_N / (x^2 gamma) * y^2/(e^y - 1)
    A_F = r_e R* Theta^3 / (4 lambdabar^2),  A_N = r_e R* Theta^2 / (4 lambdabar^2)
    eps      = gamma (1 - (1 + 2b)^(-1/2))                (perpendicular emission)

Pins (tests/test_oracle_rics.py): Wien maximum of g (Sec. 2.2 "g ~ 1.4"),
the drag length ~200 cm and eta ~3.8e4 at x = 10, kT = 1 keV (Sec. 2.2),
F = Ndot * DeltaP (Sec. 2.2) and the attractor beta = mu, the photon-energy
limits and bounds (Sec. 2.1, Appendix A.3), the excitation kinematics
(Appendix A.1, Eq. excitedgamma), eps and excited_gamma rebuilt from
Lorentz boosts of four-momenta (Appendix A.1-A.3), and a numerical quadrature of the rate
integral with a finite-width resonance that converges to the closed form.
"""
import numpy as np

from .constants import LAMBDABAR_CM, ME_C2_KEV, R_E_CM, R_STAR_CM

# Beyond y = 80 the Planck factors are set to zero (g(80) ~ 1e-29, far below any
# momentum change a float64 or float32 state can resolve).  The cutoff is part
# of the method's definition here so that every implementation agrees on which
# particles feel exactly zero force (the drag limiter compares |F| with |p|).
Y_CUTOFF = 80.0


def theta_of_kT(kT_keV):
    return kT_keV / ME_C2_KEV


def prefactors(kT_keV):
    """(A_F, A_N) of the normalised drag force and scattering rate."""
    th = theta_of_kT(kT_keV)
    base = R_E_CM * R_STAR_CM / (4.0 * LAMBDABAR_CM ** 2)
    return base * th ** 3, base * th ** 2


def lorentz(u):
    u = np.asarray(u, dtype=np.float64)
    g = np.sqrt(1.0 + u * u)
    return g, u / g


def resonance_y(u, b, mu, kT_keV):
    """y = hbar omega_X / kT at resonance, omega_X = omega_B/(gamma(1-beta mu)) (Eq. resomega)."""
    gam, beta = lorentz(u)
    return b / (theta_of_kT(kT_keV) * gam * (1.0 - beta * mu))


def _planck_factors(y):
    """(y^2/(e^y-1), y^3/(e^y-1)) with the cutoff beyond Y_CUTOFF."""
    y = np.asarray(y, dtype=np.float64)
    big = y > Y_CUTOFF
    ys = np.where(big, 1.0, y)
    em1 = np.expm1(ys)
    f2 = np.where(big, 0.0, ys * ys / em1)
    f3 = np.where(big, 0.0, ys ** 3 / em1)
    return f2, f3


def g_planck(y):
    """g(y) = y^3 / (e^y - 1) (Sec. 2.2, after Eq. contdrag)."""
    return _planck_factors(y)[1]


def drag_force(u, b, mu, x, kT_keV):
    """F_hat(u) of Eq. contdrag, normalised by m_e c^2 / R*."""
    A_F, _ = prefactors(kT_keV)
    gam, beta = lorentz(u)
    _, g = _planck_factors(resonance_y(u, b, mu, kT_keV))
    return A_F / (x * x) * gam * (mu - beta) * g


def drag_force_du(u, b, mu, x, kT_keV):
    """dF_hat/du, differentiated analytically.

    Write F = (A_F/x^2) (gamma mu - u) g(y) and y = b / (Theta (gamma - u mu)):
    d(gamma mu - u)/du = -(1 - beta mu), dy/du = y (mu - beta)/(gamma - u mu),
    g'(y) = g(y) (3/y - 1 - 1/(e^y - 1)).
    """
    A_F, _ = prefactors(kT_keV)
    u = np.asarray(u, dtype=np.float64)
    gam, beta = lorentz(u)
    y = resonance_y(u, b, mu, kT_keV)
    _, g = _planck_factors(y)
    ys = np.where(y > Y_CUTOFF, 1.0, y)
    gp = np.where(y > Y_CUTOFF, 0.0, g * (3.0 / ys - 1.0 - 1.0 / np.expm1(ys)))
    dy = y * (mu - beta) / (gam - u * mu)
    return A_F / (x * x) * (-(1.0 - beta * mu) * g + (gam * mu - u) * gp * dy)


def scatter_rate(u, b, mu, x, kT_keV):
    """Ndot_hat of Eq. scatteringNdot with the radial beam (solid angle pi/x^2)."""
    _, A_N = prefactors(kT_keV)
    gam, _ = lorentz(u)
    f2, _ = _planck_factors(resonance_y(u, b, mu, kT_keV))
    return A_N / (x * x * gam) * f2


def photon_energy(u, b):
    """Up-scattered photon energy in m_e c^2 for perpendicular emission (Eq. perpemit).

    E_gamma = gamma_i (1 - m_e c^2 / E_B) with E_B / m_e c^2 = (1 + 2b)^(1/2) (Eq. elandau).
    """
    gam, _ = lorentz(u)
    return gam * (1.0 - 1.0 / np.sqrt(1.0 + 2.0 * b))


def deexcitation_energy(b, c):
    """Photon energy E_gamma(theta)/m_e c^2 in the rest frame of the excited lepton
    (Appendix A.2): E_B/sin^2(theta) [1 - (cos^2 theta + sin^2 theta m^2/E_B^2)^(1/2)]
    with c = cos(theta) measured from the field, written without the 0/0 at
    theta = 0 as (q - 1/q) / (1 + (c^2 + (1 - c^2)/q^2)^(1/2)), q = E_B/m_e c^2."""
    q = np.sqrt(1.0 + 2.0 * np.asarray(b, dtype=np.float64))
    c = np.asarray(c, dtype=np.float64)
    return (q - 1.0 / q) / (1.0 + np.sqrt(c * c + (1.0 - c * c) / (q * q)))


EMISSION_PATTERNS = ("perpendicular", "isotropic", "dipole")


def emission_cosine(w1, w2, w3, pattern):
    """Rest-frame emission cosine mu_r (from the excited lepton's motion) drawn from the
    second, third and fourth words of the event's Philox block.  The paper takes the
    pattern from the two polarisation states of an external reference it does not
    reproduce; the patterns offered are readings:
      perpendicular  mu_r = 0 (Eq. perpemit, the estimate the paper works with);
      isotropic      mu_r uniform on [-1, 1]: 2 U1 - 1, U1 from the top 24 bits of w1;
      dipole         density (3/8)(1 + mu_r^2), the classical cyclotron pattern summed
                     over both polarisations, as the mixture 3/4 uniform on [-1, 1]
                     (density 3/8) + 1/4 of density (3/8) mu^2 * 4 = (3/2) mu^2, whose
                     |mu| is the largest of three uniforms (density 3 |mu|^2 on [0, 1])
                     with a random sign.  The low bits of w1 pick the component (both
                     of bits 0 and 1 clear: the second, probability 1/4) and bit 2 the
                     sign; U1, U2, U3 come from the top 24 bits of w1, w2, w3.  Every
                     draw is exact in binary floating point.
    """
    w1 = np.asarray(w1, dtype=np.uint32)
    u1 = (w1 >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
    if pattern == "perpendicular":
        return np.zeros_like(u1)
    if pattern == "isotropic":
        return 2.0 * u1 - 1.0
    if pattern == "dipole":
        u2 = (np.asarray(w2, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
        u3 = (np.asarray(w3, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
        top = np.maximum(u1, np.maximum(u2, u3))
        squared = (w1 & np.uint32(3)) == 0
        sign = np.where((w1 & np.uint32(4)) != 0, -1.0, 1.0)
        return np.where(squared, sign * top, 2.0 * u1 - 1.0)
    raise ValueError(pattern)


def emission(u, b, mu_r):
    """One scattering event with the photon leaving the excited lepton's rest frame at
    cosine mu_r from the lepton's direction of motion (Appendix A.2-A.3).

    The excited lepton moves along the field with gamma_e = gamma / q (Eq. scatlim1,
    q = E_B/m_e c^2); in its rest frame the photon takes E_gamma(theta), the lepton
    E_B - E_gamma and momentum -E_gamma mu_r along the motion; both are boosted back.
    Returns (photon energy eps, lepton momentum u after the event, the photon's
    direction along s), all in the lab.  mu_r = 0 is perpendicular emission (Eq.
    perpemit): eps = gamma (1 - 1/q), the lepton keeps its direction at gamma/q.
    Where gamma < q (gamma_e < 1, outside the resonance kinematics) the boost is
    taken as zero and the lepton's gamma is clamped at 1, as for perpendicular
    emission.
    """
    u = np.asarray(u, dtype=np.float64)
    mu_r = np.asarray(mu_r, dtype=np.float64)
    gam = np.sqrt(1.0 + u * u)
    d = np.where(u >= 0.0, 1.0, -1.0)
    q = np.sqrt(1.0 + 2.0 * np.asarray(b, dtype=np.float64))
    ge = gam / q
    be = np.sqrt(np.maximum(1.0 - 1.0 / (ge * ge), 0.0))
    eg = deexcitation_energy(b, mu_r)
    ee = q - eg
    # 1 - beta_e = 1 / (gamma_e^2 (1 + beta_e)) keeps the Doppler factors exact where
    # they cancel: 1 + beta_e mu_r for backward emission, and for forward emission
    # E_e - beta_e E_gamma mu_r = 1 / (E_e + E_gamma mu_r) + E_gamma mu_r (1 - beta_e),
    # the first term from the rest-frame mass shell E_e^2 - (E_gamma mu_r)^2 = 1
    omb = np.where(ge > 1.0, 1.0 / (ge * ge * (1.0 + be)), 1.0)
    dopp = np.where(mu_r >= 0.0, 1.0 + be * mu_r, be * (1.0 + mu_r) + omb)
    eps = ge * eg * dopp
    g_new = ge * np.where(mu_r >= 0.0, 1.0 / (ee + eg * mu_r) + eg * mu_r * omb, ee - be * eg * mu_r)
    p_new = ge * (be * ee - eg * mu_r)            # along the motion
    u_new = d * np.where(p_new >= 0.0, 1.0, -1.0) * np.sqrt(np.maximum((g_new - 1.0) * (g_new + 1.0), 0.0))
    dir_ph = d * np.where(mu_r + be >= 0.0, 1.0, -1.0)
    return eps, u_new, dir_ph


def excited_gamma(b):
    """Lorentz factor of the excited lepton in the frame of the absorbed photon's
    collision, gamma = (E_B/m + m/E_B)/2 (Appendix A.1, Eq. excitedgamma)."""
    eb = np.sqrt(1.0 + 2.0 * b)
    return 0.5 * (eb + 1.0 / eb)


def scatter_rate_quadrature(u, b, mu, x, kT_keV, width, n_sigma=12.0, n_pts=40001):
    """Ndot_hat from the rate integral with a finite-width resonance (test of the closed form).

    c * Omega * int d(omega) n_omega sigma(omega), with
      n_omega   = omega^2 / (8 pi^3 c^3) / (exp(hbar omega / kT) - 1)   (Sec. 2.2, I_omega / (hbar omega c)),
      Omega     = pi / x^2 (radial beam from the stellar disk),
      int sigma d(omega) = 2 pi^2 r_e c / gamma  (oscillator-strength sum rule of a
                 single classical resonance, transformed to the lab frame),
    and sigma(omega) given a normalised Gaussian profile of relative width
    `width` around omega_X.  In photon energy eps = hbar omega/(m_e c^2) the
    integrand is  c r_e / (4 lambdabar^2 x^2 gamma) * G(eps) eps^2 / (exp(eps/Theta) - 1).
    Scalar inputs only.
    """
    th = theta_of_kT(kT_keV)
    gam = np.sqrt(1.0 + u * u)
    beta = u / gam
    eps_x = b / (gam * (1.0 - beta * mu))
    sig = width * eps_x
    e = np.linspace(max(eps_x - n_sigma * sig, 1e-300), eps_x + n_sigma * sig, n_pts)
    prof = np.exp(-0.5 * ((e - eps_x) / sig) ** 2) / (np.sqrt(2.0 * np.pi) * sig)
    integrand = prof * e * e / np.expm1(e / th)
    integral = np.trapezoid(integrand, e)
    # c * r_e/(4 lambdabar^2 x^2 gamma) * integral, normalised by R*/c:
    return R_E_CM * R_STAR_CM / (4.0 * LAMBDABAR_CM ** 2 * x * x * gam) * integral


# ---------------------------------------------------------------------------
# (log10 gamma, s) table of the u >= 0 half, with the mirror for u < 0.
# ---------------------------------------------------------------------------

def table_axes(n_lg, n_s, L_cells):
    """Table nodes: log10 gamma_i = 8 i/(n_lg-1); s_j = (j + 1/2) L / n_s (cells)."""
    lg = 8.0 * np.arange(n_lg, dtype=np.float64) / (n_lg - 1)
    s = (np.arange(n_s, dtype=np.float64) + 0.5) * (L_cells / n_s)
    return lg, s


def build_table(geom_at, n_lg, n_s, L_cells, kT_keV):
    """Tabulate F_hat and Ndot_hat for u >= 0 on the (log10 gamma, s) grid.

    geom_at(s_cells) must return (b, mu, x) at arc length s (in cells) from the
    exact line geometry.  Returns arrays of shape (n_lg, n_s).
    """
    lg, s = table_axes(n_lg, n_s, L_cells)
    b, mu, x = geom_at(s)
    gam = 10.0 ** lg
    u = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    U = u[:, None]
    F = drag_force(U, b[None, :], mu[None, :], x[None, :], kT_keV)
    N = scatter_rate(U, b[None, :], mu[None, :], x[None, :], kT_keV)
    return F, N


def table_lookup(F_tab, N_tab, u, xcell, L_cells):
    """Bilinear lookup with clamping; u < 0 uses F(-u,s) = -F(u,L-s), N(-u,s) = N(u,L-s).

    Returns (F_hat, Ndot_hat, dF_hat/du of the interpolant).
    """
    n_lg, n_s = F_tab.shape
    u = np.asarray(u, dtype=np.float64)
    xcell = np.asarray(xcell, dtype=np.float64)
    neg = u < 0.0
    ua = np.abs(u)
    sx = np.where(neg, L_cells - xcell, xcell)
    gam = np.sqrt(1.0 + ua * ua)
    fi = np.log10(gam) * ((n_lg - 1) / 8.0)
    inside_i = (fi > 0.0) & (fi < n_lg - 1)
    fi = np.clip(fi, 0.0, n_lg - 1)
    fj = np.clip(sx * (n_s / L_cells) - 0.5, 0.0, n_s - 1)
    i0 = np.minimum(np.floor(fi).astype(np.int64), n_lg - 2)
    j0 = np.minimum(np.floor(fj).astype(np.int64), n_s - 2)
    wi = fi - i0
    wj = fj - j0

    def bil(T):
        a = T[i0, j0] * (1 - wj) + T[i0, j0 + 1] * wj
        c = T[i0 + 1, j0] * (1 - wj) + T[i0 + 1, j0 + 1] * wj
        return a * (1 - wi) + c * wi, c - a

    F, dF_di = bil(F_tab)
    N, _ = bil(N_tab)
    # d fi / d|u| = (n_lg-1)/8 * |u| / (gamma^2 ln 10); zero where clamped.
    dfi = np.where(inside_i, (n_lg - 1) / 8.0 * ua / (gam * gam * np.log(10.0)), 0.0)
    dF = dF_di * dfi          # dF_tab/d|u|; for u<0: d(-F_tab(|u|))/du = +dF_tab/d|u|
    F = np.where(neg, -F, F)
    return F, N, dF
