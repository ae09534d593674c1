"""Angle-resolved de-excitation (Appendix A.2-A.3): the photon leaves the excited
lepton's rest frame at cosine mu_r from its motion, the lepton recoils along B, and
both are boosted back to the lab.  Pinned by the printed E_gamma(theta), the
rest-frame mass shell, explicit Lorentz boosts of four-momenta, energy
conservation, the perpendicular case (Eq. perpemit), the parallel limit (Eq.
paremit) and the bounds the paper states for E_gamma, and for the rest-frame
patterns by their distribution functions."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import philox, pic, rics

B_VALUES = (1e-3, 0.09, 0.5, 3.0, 40.0)


def _printed_e_gamma(b, c):
    """E_gamma(theta) as printed, E_B / sin^2 [1 - (cos^2 + sin^2 m^2/E_B^2)^(1/2)],
    with m_e c^2 = 1 and E_B = (1 + 2b)^(1/2) (Eq. elandau)."""
    eb = math.sqrt(1.0 + 2.0 * b)
    s2 = 1.0 - c * c
    return eb / s2 * (1.0 - math.sqrt(c * c + s2 / (eb * eb)))


@pytest.mark.parametrize("b", B_VALUES)
def test_deexcitation_energy_printed_form_and_limits(b):
    q = math.sqrt(1.0 + 2.0 * b)
    for c in (-0.9, -0.5, 0.0, 0.1, 0.5, 0.8, 0.9):
        assert float(rics.deexcitation_energy(b, c)) == pytest.approx(_printed_e_gamma(b, c), rel=1e-9)
    # sideways the lepton drops to rest: the photon takes E_B - m; along B the
    # two-body decay to a photon and a lepton of mass m gives (E_B^2 - m^2)/(2 E_B)
    assert float(rics.deexcitation_energy(b, 0.0)) == pytest.approx(q - 1.0, rel=1e-14)
    for c in (1.0, -1.0):
        assert float(rics.deexcitation_energy(b, c)) == pytest.approx((q * q - 1.0) / (2.0 * q), rel=1e-14)


@pytest.mark.parametrize("b", B_VALUES)
def test_rest_frame_lepton_on_mass_shell(b):
    # after the decay the lepton (energy E_B - E_gamma, momentum -E_gamma mu_r along B)
    # is a free ground-level lepton of mass m_e
    q = math.sqrt(1.0 + 2.0 * b)
    c = np.linspace(-1.0, 1.0, 41)
    eg = rics.deexcitation_energy(b, c)
    np.testing.assert_allclose((q - eg) ** 2 - (eg * c) ** 2, 1.0, rtol=1e-12)


def _boosted(u, b, c):
    """Lab photon energy, lepton momentum and photon direction from rest-frame
    four-momenta boosted along B, in 60-digit arithmetic: in the excited lepton's rest frame (mass E_B, moving
    with gamma_e = gamma / E_B) the photon has (E', p_par, p_perp) = E_gamma (1, c,
    (1 - c^2)^(1/2)), the lepton (E_B - E_gamma, -E_gamma c, 0); the boost has rapidity
    acosh(gamma_e) in the lepton's direction."""
    with mpmath.workdps(60):
        u, b, c = mpmath.mpf(u), mpmath.mpf(b), mpmath.mpf(c)
        gam = mpmath.sqrt(1 + u * u)
        d = 1 if u >= 0 else -1
        q = mpmath.sqrt(1 + 2 * b)
        y = mpmath.acosh(max(gam / q, 1))
        s2 = 1 - c * c
        eg = q / s2 * (1 - mpmath.sqrt(c * c + s2 / (q * q))) if s2 > 0 else (q * q - 1) / (2 * q)
        boost = mpmath.matrix([[mpmath.cosh(y), mpmath.sinh(y)], [mpmath.sinh(y), mpmath.cosh(y)]])
        ph = boost * mpmath.matrix([eg, eg * c])
        le = boost * mpmath.matrix([q - eg, -eg * c])
        return float(ph[0]), float(d * le[1]), float(d * mpmath.sign(ph[1])), float(le[0])


@pytest.mark.parametrize("b", (0.09, 0.5, 3.0, 40.0))
def test_emission_equals_explicit_lorentz_boosts(b):
    q = math.sqrt(1.0 + 2.0 * b)
    for gam in (1.5 * q, 10.0 * q, 1e3, 1e6):
        for sgn in (1.0, -1.0):
            u = sgn * math.sqrt(gam * gam - 1.0)
            for c in (-1.0, -0.7, -0.2, 0.0, 0.3, 0.95, 1.0):
                eps, un, dph = (float(v[0]) for v in rics.emission(np.array([u]), b, np.array([c])))
                e_b, u_b, d_b, g_b = _boosted(u, b, c)
                assert eps == pytest.approx(e_b, rel=1e-12)
                # the lepton's momentum near zero is ill-conditioned in the boost itself
                assert un == pytest.approx(u_b, rel=1e-9, abs=1e-12 * gam)
                assert dph == d_b
                # energy is conserved and the lepton stays on its mass shell
                assert math.sqrt(1.0 + un * un) + eps == pytest.approx(gam, rel=1e-12)
                assert math.sqrt(1.0 + un * un) == pytest.approx(g_b, rel=1e-12)


@pytest.mark.parametrize("b", B_VALUES)
def test_perpendicular_emission_is_the_printed_estimate(b):
    # mu_r = 0: eps = gamma (1 - m/E_B) (Eq. perpemit) and the lepton keeps its
    # direction at gamma / E_B (Eq. scatlim1)
    u = np.array([-3e5, -40.0, 7.0, 250.0, 2e6])
    eps, un, dph = rics.emission(u, b, np.zeros_like(u))
    np.testing.assert_allclose(eps, rics.photon_energy(u, b), rtol=1e-13)
    gq = np.sqrt(1.0 + u * u) / math.sqrt(1.0 + 2.0 * b)
    np.testing.assert_allclose(np.abs(un), np.sqrt(np.maximum(gq * gq - 1.0, 0.0)), rtol=1e-12)
    np.testing.assert_array_equal(dph, np.sign(u))
    np.testing.assert_array_equal(np.sign(un[np.abs(un) > 0]), np.sign(u[np.abs(un) > 0]))


@pytest.mark.parametrize("b", B_VALUES)
def test_emission_continuous_in_the_cosine_and_unboosted_below_e_b(b):
    # the backward and forward forms of the Doppler factors meet at mu_r = 0 for every
    # gamma; below gamma = E_B (gamma_e < 1, outside the resonance kinematics) the
    # boost is dropped: eps = gamma_e E_gamma(theta), the lepton recoils against the
    # photon, and energy is conserved wherever its energy gamma_e E_e reaches m_e
    q = math.sqrt(1.0 + 2.0 * b)
    for gam in (0.5 * q, 0.999 * q, q, 1.001 * q, 3.0 * q, 1e5 * q):
        if gam < 1.0:
            continue
        u = np.full(3, math.sqrt(gam * gam - 1.0))
        eps, un, _ = rics.emission(u, b, np.array([-1e-300, 0.0, 1e-300]))
        np.testing.assert_allclose(eps, eps[1], rtol=1e-14)
        # (the lepton's gamma: its momentum near rest is sqrt-sensitive to rounding)
        np.testing.assert_allclose(np.sqrt(1.0 + un * un), math.sqrt(1.0 + un[1] ** 2), rtol=1e-14)
        if gam < q:
            c = np.linspace(-1.0, 1.0, 11)
            eps, un, dph = rics.emission(np.full(c.shape, u[0]), b, c)
            np.testing.assert_allclose(eps, gam / q * rics.deexcitation_energy(b, c), rtol=1e-14)
            np.testing.assert_array_equal(dph, np.where(c >= 0.0, 1.0, -1.0))
            moving = un != 0.0
            assert np.all(np.sign(un[moving]) == -np.sign(c[moving]))
            np.testing.assert_allclose(np.sqrt(1.0 + un[moving] ** 2) + eps[moving], gam, rtol=1e-13)
            np.testing.assert_array_equal(moving, gam / q * (q - rics.deexcitation_energy(b, c)) > 1.0)


@pytest.mark.parametrize("b", B_VALUES)
def test_emission_between_the_printed_bounds(b):
    # forward emission in the rest frame (mu_r in [0, 1]) gives the lab energies the
    # paper bounds by gamma (1 - m/E_B) and gamma (1 - m^2/E_B^2); along B it reaches
    # the upper one (Eq. paremit) as gamma_e grows, backward emission gives less than
    # the perpendicular estimate; eps rises with mu_r over backward emission, and over
    # all mu_r once the Doppler factor outweighs the fall of E_gamma(theta) towards B
    q = math.sqrt(1.0 + 2.0 * b)
    c = np.linspace(-1.0, 1.0, 201)
    for gam in (2.0 * q, 30.0 * q, 1e4 * q):
        u = np.full(c.shape, math.sqrt(gam * gam - 1.0))
        eps, _, _ = rics.emission(u, b, c)
        lo, hi = gam * (1.0 - 1.0 / q), gam * (1.0 - 1.0 / (q * q))
        fwd = c >= 0
        assert np.all(eps[fwd] >= lo * (1 - 1e-12)) and np.all(eps[fwd] <= hi * (1 + 1e-12))
        assert np.all(eps[~fwd] < lo)
        assert np.all(np.diff(eps[c <= 0]) > 0)
        if gam >= 30.0 * q:
            assert np.all(np.diff(eps) > 0)
        ge = gam / q
        assert eps[-1] / hi == pytest.approx(1.0, abs=1.0 / ge ** 2)


def _cosines(pattern, n=1 << 20):
    w = philox.philox4x32_10(np.arange(n, dtype=np.uint64), 3, 0, philox.STREAM_RICS, 17, 0)
    return rics.emission_cosine(w[1], w[2], w[3], pattern), w


def _ks(sample, cdf):
    x = np.sort(sample)
    n = x.size
    F = cdf(x)
    return max(np.max(np.arange(1, n + 1) / n - F), np.max(F - np.arange(n) / n))


def test_emission_cosine_patterns():
    mu, w = _cosines("perpendicular", 1024)
    assert np.all(mu == 0.0)
    iso, w = _cosines("isotropic")
    dip, _ = _cosines("dipole")
    np.testing.assert_array_equal(iso, 2.0 * philox.uniform24(w[1]) - 1.0)
    # every draw is exact in float32, inside [-1, 1]
    for m in (iso, dip):
        assert np.all(m.astype(np.float32).astype(np.float64) == m)
        assert np.all(np.abs(m) <= 1.0)
    # Kolmogorov-Smirnov against the distribution functions (mu + 1)/2 and
    # (mu^3 + 3 mu + 4)/8 of the densities 1/2 and (3/8)(1 + mu^2); the 1% critical
    # value is 1.63 / n^(1/2)
    crit = 1.63 / math.sqrt(iso.size)
    assert _ks(iso, lambda m: (m + 1.0) / 2.0) < crit
    assert _ks(dip, lambda m: (m ** 3 + 3.0 * m + 4.0) / 8.0) < crit
    assert _ks(dip, lambda m: (m + 1.0) / 2.0) > 10 * crit
    # moments: <mu^2> = 1/3 and 2/5, <mu^4> = 1/5 and 9/35, each within 4 sigma
    n = iso.size
    for m, m2, m4, m8 in ((iso, 1 / 3, 1 / 5, 1 / 9), (dip, 2 / 5, 9 / 35, 3 / 8 * (2 / 9 + 2 / 11))):
        assert abs(np.mean(m ** 2) - m2) < 4 * math.sqrt((m4 - m2 * m2) / n)
        assert abs(np.mean(m ** 4) - m4) < 4 * math.sqrt((m8 - m4 * m4) / n)
        assert abs(np.mean(m)) < 4 * math.sqrt(m2 / n)
    with pytest.raises(ValueError):
        rics.emission_cosine(w[1], w[2], w[3], "beamed")


def _forced_case(pattern, n, sign):
    """n positrons at one point of the stochastic regime with a certain event whose
    photon converts if emitted perpendicular; field-free, immediate conversion."""
    cfg = pic.make_config(lines=[dict(r_eq=4.0, n_cells=64, ppc_init=0, init="empty")], rics="exact",
                          j_twist=0.0, pairs=True, conversion="immediate", b_pole=10.0, seed=5,
                          emission=pattern)
    st = pic.init_state(cfg)
    ln = st.lines[0]
    x0 = 3.3
    b, mu, xr, rc = ln.geometry_at(np.array([x0]))
    _, _, rate = ln.rics_funcs(np.array([x0]), b, mu, xr)
    for g in np.geomspace(3.0, 1e7, 400):
        u = math.sqrt(g * g - 1.0)
        if rate(np.array([u]))[0] * ln.h >= 1.0 and rics.photon_energy(np.array([u]), b)[0] >= 2.0:
            break
    else:
        pytest.skip("no momentum with a certain event at this position")
    ids = np.arange(n, dtype=np.uint64) * 13 + 5
    pic.load_particles(st, 0, 1, np.full(n, 3, dtype=np.int32), np.full(n, x0 - 3.0), np.full(n, sign * u), ids)
    return st, float(b[0]), sign * u, ids


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("pattern", ["isotropic", "dipole"])
def test_step_draws_the_emission_cosine_from_the_event_block(pattern, sign):
    # every positron scatters; the photons with eps >= 2 convert on the spot into a
    # pair moving along the photon, the others escape.  The recoils match the cosines
    # drawn from the other words of each event's Philox block, energy is conserved
    # through recoil, pairs and escaped photons, and over the ensemble the mean photon
    # energy matches the pattern's average of eps(mu_r)
    n = 4000
    st, b, u0, ids = _forced_case(pattern, n, sign)
    g0 = math.sqrt(1.0 + u0 * u0)
    pic.step(st)
    k0, k1 = philox.seed_key(5)
    lo, hi = philox.split_id(ids)
    w = philox.philox4x32_10(0, lo, hi, philox.STREAM_RICS, k0, k1)
    mu_r = rics.emission_cosine(w[1], w[2], w[3], pattern)
    eps, un, dph = rics.emission(np.full(n, u0), b, mu_r)
    conv = eps >= 2.0
    c = st.counters[0]
    assert c["events"] == n and c["pairs_created"] == int(conv.sum()) and c["photons_escaped"] == n - conv.sum()
    assert conv.sum() > n // 2
    P = st.parts[0]
    parents = np.isin(P[1]["id"], ids)
    order = np.argsort(P[1]["id"][parents])
    up = P[1]["u"][parents][order]
    np.testing.assert_allclose(up, un, rtol=1e-12)
    # the pairs: one member of each sign per converting event, moving along the photon
    ue, upos = P[0]["u"], P[1]["u"][~parents]
    gsum = np.sqrt(1.0 + ue ** 2).sum() + np.sqrt(1.0 + upos ** 2).sum() + np.sqrt(1.0 + up ** 2).sum()
    assert gsum + eps[~conv].sum() == pytest.approx(n * g0, rel=1e-11)
    assert np.sort(np.sign(ue)).tolist() == np.sort(dph[conv]).tolist()
    dens = (lambda m: 0.5) if pattern == "isotropic" else (lambda m: 0.375 * (1.0 + m * m))
    e_of = lambda m: float(rics.emission(np.array([u0]), b, np.array([m]))[0][0])
    mean_eps = integrate.quad(lambda m: e_of(m) * dens(m), -1.0, 1.0, epsabs=0, epsrel=1e-10)[0]
    sd = math.sqrt(integrate.quad(lambda m: (e_of(m) - mean_eps) ** 2 * dens(m), -1.0, 1.0)[0])
    assert abs(eps.mean() - mean_eps) < 4.0 * sd / math.sqrt(n)
    assert 0.0 < mean_eps < g0


def test_unknown_pattern_is_rejected():
    with pytest.raises(ValueError):
        pic.init_state(pic.make_config(lines=[dict(r_eq=4.0, n_cells=8, ppc_init=0, init="empty")],
                                       emission="beamed"))
