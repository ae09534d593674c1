"""Pins of oracle/geometry.py against the paper's numbers and closed-form facts."""
import json
import os

import numpy as np
import pytest

from oracle import geometry

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_cell_count_of_r_eq10_line_matches_paper():
    g = GOLD["cells_r_eq10"]
    L = geometry.line_length(g["r_eq"])
    assert L / g["dl_over_rstar"] == pytest.approx(g["value"], rel=g["rel"])


@pytest.mark.parametrize("R", [2.0, 4.0, 10.0, 30.0, 100.0])
def test_line_length_against_polyline(R):
    # brute force: sum of chords of r = R sin^2(theta) in the (r, theta) plane
    u0 = geometry.footpoint_cos(R)
    th = np.linspace(np.arccos(u0), np.pi - np.arccos(u0), 400001)
    r = R * np.sin(th) ** 2
    X, Z = r * np.sin(th), r * np.cos(th)
    chords = np.hypot(np.diff(X), np.diff(Z)).sum()
    assert geometry.line_length(R) == pytest.approx(chords, rel=1e-9)


def test_footpoints_on_star_and_equator_radius():
    for R in (2.0, 4.0, 30.0):
        t = geometry.node_tables(R, 64, 10.0)
        assert t["x"][0] == pytest.approx(1.0, abs=1e-12)
        assert t["x"][-1] == pytest.approx(1.0, abs=1e-12)
        assert t["x"][32] == pytest.approx(R, rel=1e-12)     # equator at s = L/2


def test_pole_surface_field_is_b_star():
    # B_d(r = R*, theta = 0) = B*: the footpoint of a very long line approaches the pole
    # (the footpoint field is B* sqrt(4 - 3/R)/2, within 3/(8R) of B*)
    R = 1.0e6
    u = geometry.footpoint_cos(R)
    assert geometry.field_b(10.0, R, u) == pytest.approx(10.0, rel=1e-6)


def test_mirror_symmetry_about_equator():
    t = geometry.node_tables(6.0, 128, 10.0)
    np.testing.assert_allclose(t["b"], t["b"][::-1], rtol=1e-12)
    np.testing.assert_allclose(t["x"], t["x"][::-1], rtol=1e-12)
    np.testing.assert_allclose(t["mu"], -t["mu"][::-1], atol=1e-12)
    np.testing.assert_allclose(t["rc"], t["rc"][::-1], rtol=1e-10)
    assert abs(t["mu"][64]) < 1e-12
    assert t["mu"][0] > 0   # photons and +s point away from the star in the north


def test_mu_and_attractor_at_footpoint_R4():
    u0 = geometry.footpoint_cos(4.0)
    mu = geometry.photon_mu(u0)
    assert mu == pytest.approx(0.9608, abs=1e-4)
    assert mu / np.sqrt(1 - mu * mu) == pytest.approx(3.464, abs=1e-3)


def test_curvature_radius_against_three_point_circle():
    # curvature from the circle through three nearby points of the curve
    R = 7.0
    for th in (0.4, 0.9, np.pi / 2, 2.2):
        d = 1e-4
        pts = []
        for t in (th - d, th, th + d):
            r = R * np.sin(t) ** 2
            pts.append((r * np.sin(t), r * np.cos(t)))
        (x1, y1), (x2, y2), (x3, y3) = pts
        a = np.hypot(x2 - x1, y2 - y1)
        b = np.hypot(x3 - x2, y3 - y2)
        c = np.hypot(x3 - x1, y3 - y1)
        area2 = abs((x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1))
        rc_num = a * b * c / (2.0 * area2)
        assert geometry.curvature_radius(R, np.cos(th)) == pytest.approx(rc_num, rel=1e-6)
    assert geometry.curvature_radius(R, 0.0) == pytest.approx(R / 3.0)


def test_cos_of_s_inverts_s_of_cos():
    R = 30.0
    u = np.linspace(-0.98, 0.98, 101)
    s = geometry.s_of_cos(R, u)
    np.testing.assert_allclose(geometry.cos_of_s(R, s), u, atol=1e-13)
