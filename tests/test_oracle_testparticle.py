"""Pins of oracle/testparticle.py (Appendix A.4, Fig. 6): test leptons under RICS drag."""
import math

import pytest

from oracle import geometry
from oracle import testparticle as tp


def test_without_drag_the_particle_coasts_and_never_scatters():
    # at kT = 1e-3 keV every resonance on this line sits beyond the Planck cutoff
    # (y >= 0.185 * 511 / (1e-3 * 1000) = 94 at the equator, larger elsewhere)
    r = tp.sweep_line(3.0, kT_keV=1e-3)
    assert r["crossed"] and r["gamma_min"] == pytest.approx(1000.0, rel=1e-12)
    assert r["s_first"] is None and r["l_pp"] == 0.0


@pytest.mark.parametrize("R", [2.0, 3.0])
def test_radau_agrees_with_an_independent_fixed_step_runge_kutta(R):
    r = tp.sweep_line(R)
    g_end, g_min, crossed = tp.rk4_line(R, n_steps=60000)
    assert r["crossed"] and crossed
    assert r["gamma_min"] == pytest.approx(g_min, rel=1e-6)


def test_threshold_point_has_b_equal_to_the_threshold():
    for R in (4.0, 10.0, 50.0):
        v = tp.b_threshold_cos(R, 10.0, 0.1)
        assert geometry.field_b(10.0, R, v) == pytest.approx(0.1, rel=1e-12)
    assert tp.b_threshold_cos(2.0, 10.0, 0.1) is None      # b(equator) = 10/(2 R^3) > 0.1


def test_the_papers_regions_appear():
    # Appendix A.4: the shortest lines keep gamma_min > 1 and their pair zone spans the
    # equator (Region I); the zone grows over the shortest lines and then falls to
    # l_pp ~ 2 R* (Fig. 6 top); beyond a critical radius the drag stops the particle
    # at the equator (gamma_min ~ 1, Region III)
    res = {R: tp.sweep_line(R) for R in (1.5, 2.0, 3.0, 6.0, 10.0)}
    assert all(res[R]["crossed"] and res[R]["gamma_min"] > 2.0 for R in (1.5, 2.0, 3.0))
    assert all(res[R]["s_b"] is None for R in (1.5, 2.0))
    assert res[1.5]["l_pp"] < res[2.0]["l_pp"] < res[3.0]["l_pp"]
    for R in (6.0, 10.0):
        assert not res[R]["crossed"] and res[R]["gamma_min"] - 1.0 < 1e-3
        assert 1.0 < res[R]["l_pp"] < 3.0
