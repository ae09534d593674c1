"""Pins of oracle/rics.py: printed numbers of Sec. 2.2, identities of Sec. 2.1-2.2 and
Appendix A, and a quadrature of the rate integral."""
import json
import os
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import constants, geometry, rics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_wien_maximum_of_g():
    res = minimize_scalar(lambda y: -rics.g_planck(y), bounds=(0.5, 10.0), method="bounded",
                          options=dict(xatol=1e-10))
    g = GOLD["g_max"]
    assert -res.fun == pytest.approx(g["value"], rel=g["rel"])
    # the Wien-law maximum of y^3/(e^y - 1) sits where y = 3 (1 - e^-y)
    assert res.x == pytest.approx(3.0 * (1.0 - np.exp(-res.x)), abs=1e-6)


def _drag_length_cm(x, kT_keV, g):
    # tau_RICS = p/|dp/dt| for the linearised force at the equatorial attractor
    # (mu = 0, gamma_bar = 1): dp/dt = -(A_F/x^2) beta g(y) m c^2/R*, p = beta m c
    # -> l_RICS = c tau = R* x^2 / (A_F g).
    A_F, _ = rics.prefactors(kT_keV)
    return constants.R_STAR_CM * x * x / (A_F * g)


def test_drag_length_matches_paper():
    d = GOLD["l_rics_cm"]
    assert _drag_length_cm(d["x"], d["kT_keV"], d["g"]) == pytest.approx(d["value"], rel=d["rel"])


def test_drag_length_from_force_itself():
    # the same length measured from drag_force: l = c p / |dp/dt| near u = 0 at mu = 0,
    # with b chosen so that y = b/(Theta gamma) hits the Wien maximum.
    kT, x = 1.0, 10.0
    ymax = minimize_scalar(lambda y: -rics.g_planck(y), bounds=(0.5, 10), method="bounded").x
    b = ymax * rics.theta_of_kT(kT)
    u = 1e-6
    F = rics.drag_force(u, b, 0.0, x, kT)
    gmax = rics.g_planck(ymax)
    assert constants.R_STAR_CM * u / abs(F) == pytest.approx(_drag_length_cm(x, kT, gmax), rel=1e-6)


def test_eta_and_skin_depth_match_paper():
    d = GOLD["d_p_cm"]
    r = d["x"] * constants.R_STAR_CM
    n = d["n_coeff"] / r ** 3
    # d_p = c/omega_p with omega_p^2 = 4 pi n e^2/m_e = 4 pi n r_e c^2
    dp = 1.0 / np.sqrt(4.0 * np.pi * n * constants.R_E_CM)
    assert dp == pytest.approx(d["value"], rel=d["rel"])
    e = GOLD["eta"]
    l = _drag_length_cm(e["x"], e["kT_keV"], GOLD["l_rics_cm"]["g"])
    assert l / dp == pytest.approx(e["value"], rel=e["rel"])


@pytest.mark.parametrize("u", [-50.0, -0.3, 0.0, 0.7, 3.0, 200.0])
@pytest.mark.parametrize("mu", [-0.8, 0.0, 0.5, 0.95])
def test_force_is_rate_times_momentum_kick(u, mu):
    # Sec. 2.2: F = Ndot_sc * DeltaP, DeltaP = gamma mu~ hbar omega_B / c, mu~ = (mu-beta)/(1-beta mu)
    b, x, kT = 0.05, 6.0, 0.5
    gam = np.sqrt(1 + u * u)
    beta = u / gam
    F = rics.drag_force(u, b, mu, x, kT)
    N = rics.scatter_rate(u, b, mu, x, kT)
    dP = gam * (mu - beta) / (1 - beta * mu) * b
    assert F == pytest.approx(N * dP, rel=1e-12, abs=1e-300)


def test_attractor_zero_force_and_sign():
    b, x, kT = 0.02, 8.0, 0.5
    for mu in (-0.7, 0.2, 0.9):
        pt = mu / np.sqrt(1 - mu * mu)
        assert abs(rics.drag_force(pt, b, mu, x, kT)) < 1e-12 * abs(rics.drag_force(pt + 1.0, b, mu, x, kT))
        assert rics.drag_force(pt + 0.5, b, mu, x, kT) < 0
        assert rics.drag_force(pt - 0.5, b, mu, x, kT) > 0


def test_force_derivative_against_finite_difference():
    b, x, kT = 0.03, 5.0, 0.5
    for u in (-20.0, -1.0, 0.1, 2.0, 40.0):
        for mu in (-0.6, 0.3, 0.9):
            h = 1e-6 * max(1.0, abs(u))
            fd = (rics.drag_force(u + h, b, mu, x, kT) - rics.drag_force(u - h, b, mu, x, kT)) / (2 * h)
            an = rics.drag_force_du(u, b, mu, x, kT)
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(rics.drag_force(u, b, mu, x, kT)) + 1e-300)


def test_photon_energy_limits_and_bounds():
    # Sec. 2.1 bounds: gamma(1 - m/E_B) < E/m < gamma(1 - m^2/E_B^2); the perpendicular
    # value is the lower bound (Appendix A.3, Eq. perpemit).
    for b in (1e-3, 0.05, 1.0, 30.0):
        eb = np.sqrt(1 + 2 * b)
        gam = 1e3
        u = np.sqrt(gam * gam - 1)
        e = rics.photon_energy(u, b)
        assert e == pytest.approx(gam * (1 - 1 / eb), rel=1e-14)
        assert e < gam * (1 - 1 / eb ** 2)
    # limits: eps/gamma -> b for b << 1 and -> 1 for b >> 1 (Appendix A.3)
    assert rics.photon_energy(1e4, 1e-6) / 1e4 == pytest.approx(1e-6, rel=1e-5)
    assert rics.photon_energy(1e4, 1e8) / 1e4 == pytest.approx(1.0, rel=1e-3)
    # the printed scaling E ~ 5e4 b^2 keV at gamma_res ~ 1e2 b (b << 1)
    s = GOLD["e_gamma_scaling_keV"]
    b = 0.01
    gam_i = 1e3   # relativistic lepton with b << 1: E ~ gamma_i b m c^2
    e_keV = rics.photon_energy(np.sqrt(gam_i ** 2 - 1), b) * constants.ME_C2_KEV
    assert e_keV / (gam_i * b) == pytest.approx(constants.ME_C2_KEV, rel=s["rel"])
    assert 1e2 * constants.ME_C2_KEV == pytest.approx(s["coeff"], rel=s["rel"])


def test_excitation_kinematics_give_recoil_factor():
    # Appendix A.1-A.3: gamma = (E_B + 1/E_B)/2 in the excitation frame implies
    # gamma (1 - beta) = m/E_B, the lab-frame recoil gamma_e = gamma_i m/E_B; the
    # oracle's post-event gamma - eps equals that.
    for b in (0.01, 0.3, 4.0, 12.0):
        eb = np.sqrt(1 + 2 * b)
        g = rics.excited_gamma(b)
        beta = np.sqrt(1 - 1 / g ** 2)
        assert g * (1 - beta) == pytest.approx(1 / eb, rel=1e-12)
        gi = 5e3
        assert gi - rics.photon_energy(np.sqrt(gi * gi - 1), b) == pytest.approx(gi / eb, rel=1e-12)


@pytest.mark.parametrize("u,mu,b", [(3.0, 0.5, 0.02), (-2.0, 0.9, 0.01), (30.0, -0.4, 0.2), (0.2, 0.0, 0.002)])
def test_rate_quadrature_converges_to_closed_form(u, mu, b):
    # A23: with a finite-width resonance the rate integral tends to the closed
    # form as the width w -> 0, with an O(w^2) error.
    x, kT = 7.0, 0.5
    exact = rics.scatter_rate(u, b, mu, x, kT)
    errs = []
    for w in (0.008, 0.004, 0.002):
        q = rics.scatter_rate_quadrature(u, b, mu, x, kT, w)
        errs.append(abs(q / exact - 1.0))
    assert errs[-1] < 1e-3
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.15)


def test_planck_cutoff_is_negligible():
    assert rics.g_planck(80.0) < 1e-28
    assert rics.g_planck(80.5) == 0.0


def test_table_reproduces_nodes_and_mirror():
    R, n = 4.0, 512
    L = float(n)
    ds = geometry.line_length(R) / n

    def geom_at(sc):
        uu = geometry.cos_of_s(R, sc * ds)
        return geometry.field_b(10.0, R, uu), geometry.photon_mu(uu), geometry.radius(R, uu)

    F, N = rics.build_table(geom_at, 256, 512, L, 0.5)
    lg, s = rics.table_axes(256, 512, L)
    # at a node the lookup returns the node value exactly
    i, jn = 100, 37
    gam = 10 ** lg[i]
    u = np.sqrt(gam * gam - 1)
    Fl, Nl, _ = rics.table_lookup(F, N, u, s[jn], L)
    assert Fl == pytest.approx(F[i, jn], rel=1e-10)
    assert Nl == pytest.approx(N[i, jn], rel=1e-10)
    # mirror: F(-u, s) = -F(u, L - s) is exact on the table too
    Fm, Nm, _ = rics.table_lookup(F, N, -u, L - s[jn], L)
    assert Fm == pytest.approx(-F[i, jn], rel=1e-10)
    assert Nm == pytest.approx(N[i, jn], rel=1e-10)
    # the table's own mirror symmetry: node j and node 511-j are mirror points
    b1, mu1, x1 = geom_at(s)
    np.testing.assert_allclose(b1, b1[::-1], rtol=1e-10)
    np.testing.assert_allclose(mu1, -mu1[::-1], atol=1e-10)


def test_table_interpolation_error_shrinks_with_resolution():
    # bilinear interpolation of a smooth region: the error falls ~4x per doubling
    R, n = 4.0, 512
    L = float(n)
    ds = geometry.line_length(R) / n

    def geom_at(sc):
        uu = geometry.cos_of_s(R, sc * ds)
        return geometry.field_b(10.0, R, uu), geometry.photon_mu(uu), geometry.radius(R, uu)

    rng = np.random.default_rng(1)
    xs = rng.uniform(200, 300, 400)
    gam = 10 ** rng.uniform(1.2, 1.6, 400)
    u = np.sqrt(gam ** 2 - 1)
    b, mu, x = geom_at(xs)
    ex = rics.scatter_rate(u, b, mu, x, 0.5)
    errs = []
    for nl, ns in ((64, 128), (128, 256), (256, 512)):
        F, N = rics.build_table(geom_at, nl, ns, L, 0.5)
        errs.append(np.max(np.abs(rics.table_lookup(F, N, u, xs, L)[1] / ex - 1)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 8.0


def _boost_photon_energy(gam, b):
    """Photon energy and recoil gamma of one resonant scattering from four-momenta
    (m_e = c = 1, momenta along B): a soft photon met head-on is absorbed when the
    pair's invariant mass reaches E_B = (1 + 2b)^(1/2) (Eq. elandau); in the rest frame
    of the excited state the photon leaves perpendicular to B, so the lepton keeps no
    parallel momentum there and drops to the ground level at rest (energy 1), the
    photon taking E_B - 1; both are boosted back along B with the excited state's
    rapidity.  Returns (photon energy, lepton gamma, absorbed photon energy), all lab."""
    p = math.sqrt(gam * gam - 1.0)
    eb = math.sqrt(1.0 + 2.0 * b)
    # invariant mass^2 of (gam, p) + (k, -k) is 1 + 2 k (gam + p): solve for k by bisection
    lo, hi = 0.0, 1.0
    while 1.0 + 2.0 * hi * (gam + p) < eb * eb:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 1.0 + 2.0 * mid * (gam + p) < eb * eb:
            lo = mid
        else:
            hi = mid
    k = 0.5 * (lo + hi)
    # E - p_par and E + p_par of the sum, the first without cancellation (gam - p = 1/(gam + p))
    minus, plus = 1.0 / (gam + p) + 2.0 * k, gam + p
    assert math.sqrt(minus * plus) == pytest.approx(eb, rel=1e-12)
    y = 0.5 * math.log(plus / minus)
    # rest-frame four-momenta (E, p_par): photon (eb - 1, 0), lepton (1, 0)
    return math.cosh(y) * (eb - 1.0), math.cosh(y) * 1.0, k


@pytest.mark.parametrize("b", [1e-3, 0.05, 1.0, 30.0])
def test_photon_energy_from_lorentz_boosts(b):
    # Appendix A.1-A.3 through explicit four-momenta rather than the closed form:
    # the boosted photon energy equals photon_energy up to the neglected energy of
    # the absorbed soft photon (relative k/gamma < b/gamma^2), and the boosted
    # lepton's gamma equals gamma - eps to the same order
    for gam in (50.0, 1e3, 1e5):
        e_boost, g_boost, k = _boost_photon_energy(gam, b)
        e = float(rics.photon_energy(math.sqrt(gam * gam - 1.0), b))
        assert k / gam < b / gam ** 2
        assert abs(e_boost / e - 1.0) <= 1.001 * k / gam + 1e-13
        assert abs(g_boost - (gam - e)) <= 1.001 * k + 1e-13 * gam
    # in the rest frame of the incoming lepton the absorbed photon has energy b and
    # the excited state moves with the Lorentz factor of excited_gamma
    e0, g0, k0 = _boost_photon_energy(1.0, b)
    assert k0 == pytest.approx(b, rel=1e-12)
    assert float(rics.excited_gamma(b)) == pytest.approx(g0, rel=1e-12)
