"""Pins of oracle/pic.py: textbook dynamics the PIC step must reproduce."""
import math

import numpy as np
import pytest

from oracle import philox, pic


def _line(**kw):
    d = dict(r_eq=4.0, n_cells=512, ppc_init=0, init="cold")
    d.update(kw)
    return d


def _single(cfg, s, x, u, pid=7):
    st = pic.init_state(cfg)
    pic.load_particles(st, 0, s, np.array([int(x)], dtype=np.int32), np.array([x - int(x)]),
                       np.array([u]), np.array([pid], dtype=np.uint64))
    return st


def _hyperbolic_error(a, n_steps):
    """Positron in a uniform frozen E with acceleration a = (q/m) E per step^2."""
    cfg = pic.make_config(lines=[_line(n_cells=2000)], rics="off", frozen_field=True, j_twist=0.0)
    st = _single(cfg, 1, 10.0, 0.0)
    C = st.lines[0].C
    st.E[0][:] = a       # q/m = +1 for a positron
    x0 = 10.0
    for _ in range(n_steps):
        pic.step(st)
    x = st.parts[0][1]["x"][0]
    u = st.parts[0][1]["u"][0]
    # leapfrog stores u^{n-1/2}; u(t) = (a/C)(t + 1/2) with u^{-1/2} = 0, and the exact
    # hyperbolic motion gives x(t) = x0 + (C^2/a)(gamma(t) - gamma(0)).
    assert u == pytest.approx(n_steps * a / C, rel=1e-12)
    gam = lambda t: math.sqrt(1.0 + (a * (t + 0.5) / C) ** 2)
    x_exact = x0 + C * C / a * (gam(n_steps) - gam(0))
    span = C * C / a * (gam(n_steps) - gam(0))
    return abs(x - x_exact) / span


def test_hyperbolic_motion_second_order():
    # halving the acceleration and doubling the steps covers the same dimensionless
    # trajectory with half the step relative to C/a: the error must fall ~4x
    e1 = _hyperbolic_error(2e-3, 500)
    e2 = _hyperbolic_error(1e-3, 1000)
    e3 = _hyperbolic_error(5e-4, 2000)
    assert e1 < 1e-3
    assert e1 / e2 == pytest.approx(4.0, rel=0.15)
    assert e2 / e3 == pytest.approx(4.0, rel=0.15)


def test_initial_state_is_neutral_and_stratified():
    cfg = pic.make_config(lines=[_line(n_cells=64, ppc_init=8, init="hot")], rics="off")
    st = pic.init_state(cfg)
    e, p = st.parts[0][0], st.parts[0][1]
    np.testing.assert_array_equal(e["x"], p["x"])
    assert np.all(np.bincount(np.floor(e["x"]).astype(int), minlength=64) == 8)
    ids = np.concatenate([e["id"], p["id"]])
    assert np.unique(ids).size == ids.size
    assert pic.gauss_residual(st, 0) < 1e-15
    g = np.sqrt(1 + e["u"] ** 2)
    assert g.min() >= 1.0 and g.max() <= 1e4 * (1 + 1e-12)


@pytest.mark.parametrize("conversion", ["immediate", "curvature"])
def test_gauss_law_to_roundoff_through_cascade_and_atmosphere(conversion):
    cfg = pic.make_config(lines=[_line(n_cells=256, ppc_init=8, init="hot", init_gamma_max=3e3)],
                          rics="exact", pairs=True, conversion=conversion, atmosphere=True, ppc0=8.0)
    st = pic.init_state(cfg)
    for _ in range(12):
        pic.step(st)
    c = st.counters[0]
    assert c["pairs_created"] > 0 and c["atm_injected"] > 0 and c["absorbed"] > 0 and c["events"] > 0
    assert pic.gauss_residual(st, 0) < 1e-12


def test_charge_continuity_of_deposit_single_particles():
    # for random single moves the deposit equals minus the change of the CIC charge,
    # integrated from the wall (the 1D continuity equation)
    rng = np.random.default_rng(3)
    n = 16
    for _ in range(200):
        x0 = rng.uniform(0, n)
        x1 = x0 + rng.uniform(-0.5, 0.5)
        j = np.zeros(n)
        pic.deposit(j, 1.0, np.array([x0]), np.array([x1]), n)
        def rho(x):
            r = np.zeros(n + 1)
            if 0 <= x < n:
                i = int(math.floor(x)); f = x - i
                r[i] += 1 - f; r[i + 1] += f
            return r
        drho = rho(x1) - rho(x0)
        # interior nodes: drho_i = -(j_i - j_{i-1})
        np.testing.assert_allclose(drho[1:n], -(j[1:] - j[:-1]), atol=1e-14)


def _energy_series(cfg, n_steps):
    st = pic.init_state(cfg)
    K, U, Wt, Ww = [], [], [], []
    for _ in range(n_steps):
        k, u = pic.energies(st, 0)
        K.append(k); U.append(u); Wt.append(st.energy_twist[0]); Ww.append(st.energy_walls[0])
        pic.step(st)
    return [np.array(a) for a in (K, U, Wt, Ww)]


def test_energy_ledger_plasma_oscillation():
    # drag off, no twist: kinetic and field energy exchange completely; the leapfrog
    # ledger (kinetic energy time-centred between half steps) drifts only at O((w_p dt)^2)
    cfg = pic.make_config(lines=[_line(ppc_init=16, init="stream", init_beta=0.1)], rics="off",
                          j_twist=0.0, ppc0=16.0)
    K, U, Wt, Ww = _energy_series(cfg, 1500)
    Kc = 0.5 * (K[:-1] + K[1:])
    led = Kc + U[:-1] + Ww[:-1]
    assert U.max() > 0.9 * K[0]
    assert np.max(np.abs(led - led[0])) / K[0] < 1e-3


def test_energy_ledger_with_twist_current_and_walls():
    cfg = pic.make_config(lines=[_line(n_cells=256, ppc_init=32, init="stream", init_beta=0.3)],
                          rics="off", j_twist=0.5, ppc0=32.0)
    K, U, Wt, Ww = _energy_series(cfg, 1200)
    Kc = 0.5 * (K[:-1] + K[1:])
    led = Kc + U[:-1] - Wt[:-1] + Ww[:-1]
    scale = max(np.abs(Wt).max(), K[0])
    assert Wt.max() > 5 * K[0] * 1e-2 and Ww.max() > 0
    assert np.max(np.abs(led - led[0])) / scale < 5e-3


def test_cold_two_stream_growth_rate():
    # e+ at +v0, e- at -v0 carrying the twist current exactly: the symmetric cold
    # two-stream instability grows at w_b/(2 gamma0^(3/2)) at k v0 = (sqrt3/2) w_b/gamma0^(3/2)
    beta, ppc, n = 0.2, 16, 1024
    cfg = pic.make_config(lines=[_line(n_cells=n, ppc_init=ppc, init="stream", init_beta=beta)],
                          rics="off", ppc0=float(ppc), j_twist=2 * beta)
    st = pic.init_state(cfg)
    g0 = 1 / math.sqrt(1 - beta ** 2)
    wb = st.lines[0].wp0
    v0 = beta * st.lines[0].C
    gth = wb / (2 * g0 ** 1.5)
    kth = math.sqrt(3) / 2 * wb / g0 ** 1.5 / v0
    win = np.hanning(n - 400)
    A, T = [], []
    for i in range(1001):
        if i % 20 == 0 and i >= 400:
            A.append(np.abs(np.fft.rfft(st.E[0][200:n - 200] * win)))
            T.append(i)
        pic.step(st)
    A, T = np.array(A), np.array(T)
    k = 2 * np.pi * np.fft.rfftfreq(n - 400)
    rates = np.polyfit(T, np.log(A + 1e-300), 1)[0]
    band = (k > 0.5 * kth) & (k < 1.5 * kth)
    assert rates[band].max() == pytest.approx(gth, rel=0.10)


def test_pair_cap_blocks_conversion():
    # n_max below the start-of-step count of every cell: no photon converts
    cfg = pic.make_config(lines=[_line(n_cells=128, ppc_init=8, init="hot", init_gamma_max=3e3)],
                          rics="exact", pairs=True, ppc0=8.0, nmax_over_n0=1.0)
    st = pic.init_state(cfg)
    pic.step(st)
    c = st.counters[0]
    assert c["events"] > 0 and c["pairs_created"] == 0
    assert c["photons_escaped"] == c["events"]


def test_rics_draws_keyed_by_id_not_layout():
    # permuting the particle arrays changes nothing in the result (compared by id)
    cfg = pic.make_config(lines=[_line(n_cells=64, ppc_init=8, init="hot", init_gamma_max=3e3)],
                          rics="exact", pairs=True, ppc0=8.0)
    a = pic.init_state(cfg)
    b = pic.init_state(cfg)
    rng = np.random.default_rng(0)
    for s in (0, 1):
        perm = rng.permutation(b.parts[0][s]["x"].size)
        b.parts[0][s] = {k: v[perm] for k, v in b.parts[0][s].items()}
    for _ in range(3):
        pic.step(a)
        pic.step(b)
    for s in range(4):
        oa = np.argsort(a.parts[0][s]["id"])
        ob = np.argsort(b.parts[0][s]["id"])
        np.testing.assert_array_equal(a.parts[0][s]["id"][oa], b.parts[0][s]["id"][ob])
        np.testing.assert_array_equal(a.parts[0][s]["x"][oa], b.parts[0][s]["x"][ob])
        np.testing.assert_array_equal(a.parts[0][s]["u"][oa], b.parts[0][s]["u"][ob])
    np.testing.assert_allclose(a.E[0], b.E[0], rtol=0, atol=1e-15 * np.abs(a.E[0]).max())
