"""Pins of the oracle's circuit potential, layer gravity and node interpolation.

* The circuit potential V_c (Sec. 2: the voltage along the line that the twist
  current needs) is the line integral of E.  Its sign and its 1/c^2 are pinned
  by what it means physically: a test electron that crosses a frozen-field line
  gains e V_c in energy, measured from the oracle's own push.
* The atmosphere's gravity (Appendix B.1: g = -T/h, the force that holds an
  isothermal layer at scale height h) is pinned by relativistic free fall under
  a constant force towards the nearer wall: the fall time from rest and the
  apex of a particle thrown upwards have closed forms.
* interp_nodes is the piecewise-linear interpolant of the node values, pinned
  against numpy's interp and at nodes and midpoints.
"""
import math

import numpy as np
import pytest

from oracle import geometry, pic


def _load(st, s, x, u, pid):
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    cell = np.floor(x).astype(np.int32)
    pic.load_particles(st, 0, s, cell, x - cell, np.atleast_1d(np.asarray(u, dtype=np.float64)),
                       np.atleast_1d(np.asarray(pid, dtype=np.uint64)))


# ---------------------------------------------------------------------------
# circuit potential
# ---------------------------------------------------------------------------

def test_circuit_potential_of_uniform_field():
    cfg = pic.make_config(lines=[dict(r_eq=4.0, n_cells=300, ppc_init=0, init="cold")], rics="off")
    st = pic.init_state(cfg)
    C = st.lines[0].C
    st.E[0][:] = 2.5e-4
    # e V_c / m c^2 = -(1/c^2) integral of E ds over 300 cells, in code units (c = C cells/step)
    assert pic.circuit_potential(st, 0) == pytest.approx(-2.5e-4 * 300 / C ** 2, rel=1e-13)


@pytest.mark.parametrize("species,gamma0", [(0, 30.0), (0, 300.0), (1, 300.0)])
def test_lepton_crossing_the_line_gains_e_times_circuit_potential(species, gamma0):
    # A fast lepton crosses a line whose frozen E is a smooth bump that vanishes at
    # both ends; no drag.  Its energy gain is the work of E along its path,
    # q * integral E ds = q (-V_c), so for an electron (q = -e) exactly e V_c, for a
    # positron -e V_c.  Leapfrog errs at O(kick^2) per step; the bump is weak and
    # the particle relativistic, so 1e-4 relative is ample.
    n = 400
    cfg = pic.make_config(lines=[dict(r_eq=4.0, n_cells=n, ppc_init=0, init="cold")], rics="off",
                          frozen_field=True, j_twist=0.0)
    st = pic.init_state(cfg)
    k = np.arange(n) + 0.5
    bump = np.sin(math.pi * np.clip((k - 20.0) / (n - 40.0), 0.0, 1.0)) ** 2
    amp = 3e-3 * (gamma0 / 30.0) * (1.0 if species == 0 else -1.0)   # decelerate nobody to rest
    st.E[0][:] = -amp * bump                                        # accelerates the electron
    vc = pic.circuit_potential(st, 0)
    u0 = math.sqrt(gamma0 ** 2 - 1.0)
    _load(st, species, 5.0, u0, 11)
    g_start = gamma0
    while st.parts[0][species]["x"][0] < n - 10.0:
        pic.step(st)
    g_end = math.sqrt(1.0 + st.parts[0][species]["u"][0] ** 2)
    gain = g_end - g_start
    expect = vc if species == 0 else -vc
    assert abs(expect) > 0.5                     # a real potential drop, not a rounding test
    assert gain == pytest.approx(expect, rel=1e-4)


# ---------------------------------------------------------------------------
# gravity in the atmosphere layer
# ---------------------------------------------------------------------------

def _gravity_line(n=1024, **kw):
    cfg = pic.make_config(lines=[dict(r_eq=4.0, n_cells=n, ppc_init=0, init="cold")], rics="off",
                          frozen_field=True, atmosphere=True, gravity=True, j_twist=0.5, ppc0=1.0,
                          mass_ratio=100.0, **kw)
    st = pic.init_state(cfg)
    # keep the layer empty of refill particles: a target of zero everywhere, the
    # layer (where gravity acts) unchanged
    st.lines[0].atm_target[:] = 0
    return st


def _accel_per_step(st, mass):
    """du per step of a constant force T/h on mass m (units m_e c^2 / cell for T/h)."""
    ln = st.lines[0]
    return st.cfg["atm_T"] / mass * ln.C / ln.atm_h


@pytest.mark.parametrize("wall,species,mass", [("low", 0, 1.0), ("high", 0, 1.0), ("low", 3, 100.0)])
def test_free_fall_time_to_the_nearer_wall(wall, species, mass):
    st = _gravity_line()
    ln = st.lines[0]
    d = 0.4 * ln.atm_depth
    x0 = d if wall == "low" else ln.n - d
    _load(st, species, x0, 0.0, 5)
    # constant force F towards the wall from rest: gamma(t) - 1 = F z(t) / (m c^2), so the
    # wall at depth d is reached when u(t) = g t satisfies (1 + u^2)^1/2 - 1 = g d / C
    # (g the kick per step, C the light speed in cells per step): t = ((1 + g d/C)^2 - 1)^1/2 / g
    g = _accel_per_step(st, mass)
    t_exact = math.sqrt((1.0 + g * d / ln.C) ** 2 - 1.0) / g
    steps = 0
    while st.parts[0][species]["x"].size:
        u = st.parts[0][species]["u"][0]
        assert (u <= 0.0) if wall == "low" else (u >= 0.0)      # always towards the nearer wall
        pic.step(st)
        steps += 1
        assert steps < 3 * t_exact
    # leapfrog: the kick leads the position by half a step; within a step of the exact time
    assert abs(steps - t_exact) <= 1.5
    assert t_exact > 100.0


def test_apex_of_a_particle_thrown_from_the_wall():
    st = _gravity_line()
    ln = st.lines[0]
    g = _accel_per_step(st, 1.0)
    z_target = 0.5 * ln.atm_depth
    # gamma0 - 1 = g z_max / C for a particle launched upwards with u0 against the force
    gamma0 = 1.0 + g * z_target / ln.C
    u0 = math.sqrt(gamma0 ** 2 - 1.0)
    _load(st, 0, 0.5, u0, 9)
    zmax = 0.0
    for _ in range(100000):
        pic.step(st)
        x = st.parts[0][0]["x"]
        if x.size == 0:
            break
        zmax = max(zmax, x[0])
    assert st.parts[0][0]["x"].size == 0           # it fell back into the wall
    assert zmax - 0.5 == pytest.approx(z_target, rel=2e-3)


def test_no_gravity_outside_the_layer_or_when_switched_off():
    st = _gravity_line()
    ln = st.lines[0]
    assert ln.atm_depth < 0.5 * ln.n - 50
    _load(st, 0, 0.5 * ln.n, 0.0, 3)
    for _ in range(20):
        pic.step(st)
    assert st.parts[0][0]["u"][0] == 0.0
    st = _gravity_line(n=1024)
    st.cfg["gravity"] = False
    _load(st, 0, 20.0, 0.0, 3)
    for _ in range(20):
        pic.step(st)
    assert st.parts[0][0]["u"][0] == 0.0


# ---------------------------------------------------------------------------
# node interpolation
# ---------------------------------------------------------------------------

def test_interp_nodes_is_the_piecewise_linear_interpolant():
    rng = np.random.default_rng(3)
    tab = rng.normal(size=33)
    n = tab.size - 1
    nodes = np.arange(n + 1, dtype=np.float64)
    np.testing.assert_array_equal(geometry.interp_nodes(tab, nodes), tab)
    mid = nodes[:-1] + 0.5
    np.testing.assert_allclose(geometry.interp_nodes(tab, mid), 0.5 * (tab[:-1] + tab[1:]), rtol=0, atol=1e-15)
    x = rng.uniform(0.0, n, 5000)
    np.testing.assert_allclose(geometry.interp_nodes(tab, x), np.interp(x, nodes, tab), rtol=0, atol=1e-14)
    # a linear node table is reproduced everywhere
    lin = 2.0 - 0.75 * nodes
    np.testing.assert_allclose(geometry.interp_nodes(lin, x), 2.0 - 0.75 * x, rtol=0, atol=1e-13)
