"""Pins of the oracle's atmosphere refill and of its event and pair kinematics
(oracle/pic.py) against what the distributions and conservation laws fix."""
import math

import numpy as np
import pytest

from oracle import pic, rics


def _atm_cfg(**kw):
    d = dict(lines=[dict(r_eq=4.0, n_cells=200, ppc_init=0, init="empty")], rics="off", atmosphere=True,
             j_twist=0.5, ppc0=50.0, atm_T=0.01, mass_ratio=100.0)
    d.update(kw)
    return pic.make_config(**d)


def test_atmosphere_refill_is_maxwellian_and_uniform_in_the_cell():
    # from an empty line, one step's refill injects the whole layer at rest in the
    # field-free first step: the momenta are Maxwellian with sigma_u = (T/m)^(1/2)
    # per species (non-relativistic at T = 0.01), the offsets uniform in the cell,
    # and every ion sits on its electron
    st = pic.init_state(_atm_cfg())
    pic.step(st)
    e, i = st.parts[0][2], st.parts[0][3]
    n = e["x"].size
    assert n > 20000 and i["x"].size == n
    np.testing.assert_array_equal(np.sort(e["x"]), np.sort(i["x"]))
    T, mr = 0.01, 100.0
    for u, sig in ((e["u"], math.sqrt(T)), (i["u"], math.sqrt(T / mr))):
        assert abs(u.mean()) < 4.0 * sig / math.sqrt(n)
        assert abs(u.std() / sig - 1.0) < 4.0 / math.sqrt(2.0 * n)
        # fourth moment of a Gaussian: 3 sigma^4
        assert abs(np.mean(u ** 4) / (3.0 * sig ** 4) - 1.0) < 0.05
    off = e["x"] - np.floor(e["x"])
    assert abs(off.mean() - 0.5) < 4.0 * math.sqrt(1.0 / 12.0 / n)
    assert abs(off.var() - 1.0 / 12.0) < 0.02 / 12.0
    # Kolmogorov-Smirnov distance to the uniform distribution
    srt = np.sort(off)
    ks = np.max(np.abs(srt - (np.arange(n) + 0.5) / n))
    assert ks < 1.63 / math.sqrt(n)          # the 1% critical value


def test_atmosphere_layer_is_topped_up_to_the_hydrostatic_profile():
    # Appendix B.1: each layer cell ends every step with at least
    # floor(a0 exp(-d/h) ppc0) electrons and ions (a0 = 18 |j|, h = 3 d0 / a0^(1/2),
    # d the distance of the cell centre from the nearer wall), and from an empty
    # line exactly that many
    st = pic.init_state(_atm_cfg())
    ln = st.lines[0]
    k = np.arange(ln.n)
    d = np.minimum(k + 0.5, ln.n - k - 0.5)
    a0, h = 18.0 * 0.5, 3.0 * 48.0 / math.sqrt(9.0)
    prof = a0 * np.exp(-d / h)
    target = np.where(prof >= 0.01, np.floor(prof * 50.0), 0).astype(np.int64)
    for step in range(3):
        pic.step(st)
        ne = pic.cell_counts(ln, st.parts[0], species=(2,))
        ni = pic.cell_counts(ln, st.parts[0], species=(3,))
        if step == 0:
            np.testing.assert_array_equal(ne, target)
            np.testing.assert_array_equal(ni, target)
        assert np.all(np.minimum(ne, ni) >= target)


def _event_case(u0, x0=3.3, b_pole=10.0):
    """One positron (id 12345) at x0 in the stochastic regime, field-free, with
    immediate pair conversion; returns (state, config)."""
    cfg = pic.make_config(lines=[dict(r_eq=4.0, n_cells=64, ppc_init=0, init="empty")], rics="exact",
                          j_twist=0.0, pairs=True, conversion="immediate", b_pole=b_pole, seed=5)
    st = pic.init_state(cfg)
    c = int(x0)
    pic.load_particles(st, 0, 1, np.array([c], dtype=np.int32), np.array([x0 - c]), np.array([u0]),
                       np.array([12345], dtype=np.uint64))
    return st, cfg


def _forced_event_momentum(ln, x0):
    """A momentum at x0 whose event probability Ndot h is clipped at 1 (so the event
    happens whatever the draw) and whose photon converts (eps >= 2)."""
    b, mu, xr, rc = ln.geometry_at(np.array([x0]))
    _, _, rate = ln.rics_funcs(np.array([x0]), b, mu, xr)
    for g in np.geomspace(3.0, 1e7, 400):
        u = math.sqrt(g * g - 1.0)
        if rate(np.array([u]))[0] * ln.h >= 1.0 and rics.photon_energy(np.array([u]), b)[0] >= 2.0:
            return u, float(b[0])
    pytest.skip("no momentum with a certain event at this position")


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_event_and_pair_conserve_energy(sign):
    # An event takes the photon's energy from the lepton (Sec. 3 and Appendix A.3),
    # and the pair made from the photon shares it equally: gamma before = gamma of
    # the recoiled lepton + gamma(e-) + gamma(e+), both members moving along the
    # parent, at the emission point (immediate conversion), and the recoil keeps the
    # lepton's direction.
    st, cfg = _event_case(1.0)
    ln = st.lines[0]
    x0 = 3.3
    u0, b = _forced_event_momentum(ln, x0)
    u0 *= sign
    st, cfg = _event_case(u0, x0)
    g0 = math.sqrt(1.0 + u0 * u0)
    pic.step(st)
    assert st.counters[0]["events"] == 1 and st.counters[0]["pairs_created"] == 1
    P = st.parts[0]
    parent = P[1]["id"] == np.uint64(12345)
    up = float(P[1]["u"][parent][0])
    ue = float(P[0]["u"][0])
    upos = float(P[1]["u"][~parent][0])
    gp, ge, gpos = (math.sqrt(1.0 + v * v) for v in (up, ue, upos))
    assert gp + ge + gpos == pytest.approx(g0, rel=1e-12)
    assert ge == pytest.approx(gpos, rel=1e-15)
    assert gp < g0 and math.copysign(1.0, up) == sign
    assert math.copysign(1.0, ue) == sign and math.copysign(1.0, upos) == sign
    assert float(P[0]["x"][0]) == pytest.approx(x0, abs=1e-15)
    assert float(P[1]["x"][~parent][0]) == pytest.approx(x0, abs=1e-15)


def test_event_and_pair_yield_follow_the_probability():
    # Sec. 3: each lepton-step scatters with probability p = Ndot h (clipped at 1),
    # decided by an independent uniform draw per particle and step.  N identical
    # positrons with p ~ 0.3 give Binomial(N, p) events; with immediate conversion,
    # eps >= 2 and n_max far away, every event makes one pair.
    st0, cfg = _event_case(1.0)
    ln = st0.lines[0]
    x0 = 3.3
    b, mu, xr, rc = ln.geometry_at(np.array([x0]))
    _, _, rate = ln.rics_funcs(np.array([x0]), b, mu, xr)
    us = np.sqrt(np.geomspace(3.0, 1e7, 2000) ** 2 - 1.0)
    p_all = rate(us) * ln.h
    ok = (p_all > 0.2) & (p_all < 0.4) & (rics.photon_energy(us, np.full(us.shape, b[0])) >= 2.0)
    if not ok.any():
        pytest.skip("no momentum with p in (0.2, 0.4) at this position")
    u0 = float(us[np.nonzero(ok)[0][0]])
    p = float(rate(np.array([u0]))[0] * ln.h)
    n = 40000
    st = pic.init_state(cfg)
    pic.load_particles(st, 0, 1, np.full(n, 3, dtype=np.int32), np.full(n, x0 - 3.0), np.full(n, u0),
                       np.arange(n, dtype=np.uint64) * 7 + 11)
    pic.step(st)
    ev = st.counters[0]["events"]
    assert abs(ev - n * p) < 4.0 * math.sqrt(n * p * (1.0 - p))
    assert st.counters[0]["pairs_created"] == ev
    assert st.parts[0][0]["x"].size == ev
