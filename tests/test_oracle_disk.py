"""Pins of oracle/disk.py: RICS from the finite stellar disk (Sec. 5) against what
the radial beam of Sec. 2.2 and plain integration fix."""
import math

import numpy as np
import pytest

from oracle import disk, geometry, rics


def test_particle_at_rest_has_closed_form_cone_integrals():
    # beta = 0: y = b / Theta for every direction, so the force integral is
    # A_F/pi g(y) integral(mu') dOmega = A_F g(y) mu sin^2(theta_d) -- the radial beam's
    # force exactly -- and the rate A_N/pi f2(y) Omega_cone, with
    # Omega_cone = 2 pi (1 - cos theta_d) = (pi / x^2) 2 / (1 + cos theta_d)
    for x, mu, b in ((1.0, 0.9, 2.0), (1.3, -0.4, 0.3), (3.0, 0.2, 0.05), (12.0, 0.7, 0.01)):
        F, N = disk.disk_rics(0.0, b, mu, x, 0.5)
        Fr = rics.drag_force(0.0, b, mu, x, 0.5)
        Nr = rics.scatter_rate(0.0, b, mu, x, 0.5)
        cd = math.sqrt(1.0 - 1.0 / (x * x))
        assert F == pytest.approx(Fr, rel=1e-12)
        assert N == pytest.approx(Nr * 2.0 / (1.0 + cd), rel=1e-12)


def test_far_from_the_star_the_disk_becomes_the_radial_beam():
    # the cone shrinks as 1/x: the relative difference falls as x^-2
    u, b, mu = 40.0, 0.02, -0.3
    d = []
    for x in (8.0, 16.0, 32.0, 64.0):
        F, N = disk.disk_rics(u, b, mu, x, 1.0)
        Fr = rics.drag_force(u, b, mu, x, 1.0)
        Nr = rics.scatter_rate(u, b, mu, x, 1.0)
        d.append((abs(F / Fr - 1.0), abs(N / Nr - 1.0)))
    d = np.array(d)
    assert d[-1].max() < 1e-3
    ratios = d[:-1] / d[1:]
    assert np.all((ratios > 3.5) & (ratios < 4.5)), ratios


def test_product_rule_matches_an_adaptive_quadrature():
    from scipy import integrate
    A_F, A_N = rics.prefactors(1.0)
    th = rics.theta_of_kT(1.0)
    for u, b, mu, x in ((30.0, 0.5, 0.6, 2.0), (300.0, 0.1, -0.2, 5.0), (5.0, 3.0, 0.95, 1.2)):
        gam = math.sqrt(1.0 + u * u)
        beta = u / gam
        cd = math.sqrt(1.0 - 1.0 / (x * x))

        def f(phi, c, k):
            mup = mu * c + math.sqrt(1.0 - mu * mu) * math.sqrt(max(1.0 - c * c, 0.0)) * math.cos(phi)
            y = b / (th * gam * (1.0 - beta * mup))
            if y > rics.Y_CUTOFF:
                return 0.0
            p = y ** (k + 2) / math.expm1(y)
            return gam * (mup - beta) * p if k == 1 else p

        Fq = A_F / math.pi * integrate.dblquad(lambda p, c: f(p, c, 1), cd, 1.0, 0.0, 2.0 * math.pi,
                                               epsabs=0.0, epsrel=1e-11)[0]
        Nq = A_N / (math.pi * gam) * integrate.dblquad(lambda p, c: f(p, c, 0), cd, 1.0, 0.0, 2.0 * math.pi,
                                                       epsabs=0.0, epsrel=1e-11)[0]
        F, N = disk.disk_rics(u, b, mu, x, 1.0, n_c=64, n_phi=64)
        assert F == pytest.approx(Fq, rel=1e-8)
        assert N == pytest.approx(Nq, rel=1e-8)
        # the model's own rule (24 x 24) on these smooth integrands
        F24, N24 = disk.disk_rics(u, b, mu, x, 1.0)
        assert F24 == pytest.approx(Fq, rel=1e-4)
        assert N24 == pytest.approx(Nq, rel=1e-4)


def test_disk_force_points_to_the_attractor_of_the_cone():
    # one attractor: the force pushes slow particles forward and fast ones back, and
    # vanishes at a beta below the radial beam's (the cone's photons arrive at
    # cosines mu' smaller than mu on average, weighted towards the resonance)
    x, b, mu = 1.5, 0.05, 0.5
    us = np.linspace(0.05, 3.0, 300)
    F, _ = disk.disk_rics(us, b, mu, x, 1.0)
    sign_change = np.nonzero(np.diff(np.sign(F)) != 0)[0]
    assert sign_change.size == 1
    assert F[0] > 0.0 and F[-1] < 0.0
    u_att = us[sign_change[0]]
    assert 0.05 < u_att < mu / math.sqrt(1.0 - mu * mu)


def test_disk_table_looks_up_like_the_radial_table():
    # the same grid and lookup as the radial table; far lines (x >= 3 everywhere except
    # near the footpoints) differ from it by the finite-disk correction only
    R, n = 4.0, 64

    def geom_at(sc):
        ds = geometry.line_length(R) / n
        c = geometry.cos_of_s(R, sc * ds)
        return geometry.field_b(10.0, R, c), geometry.photon_mu(c), geometry.radius(R, c)

    F, N = disk.build_table(geom_at, 12, 16, float(n), 0.5, n_c=8, n_phi=8)
    Fr, Nr = rics.build_table(geom_at, 12, 16, float(n), 0.5)
    assert F.shape == Fr.shape == (12, 16)
    # at gamma = 1 (first row) the force is the radial beam's (particle at rest)
    np.testing.assert_allclose(F[0], Fr[0], rtol=1e-12, atol=0)
    b, mu, x = geom_at(rics.table_axes(12, 16, float(n))[1])
    cd = np.sqrt(1.0 - 1.0 / (x * x))
    np.testing.assert_allclose(N[0], Nr[0] * 2.0 / (1.0 + cd), rtol=1e-12, atol=0)
