"""Test particles under RICS drag along dipole field lines (Appendix A.4, Fig. 6).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Appendix A.4 maps the magnetosphere with test particles: a lepton injected at a
footpoint with gamma_0 = 1000 moves along the field line under the drag force
of Eq. contdrag alone (no electric field), here for B*/B_QED = 10 and 1 keV
photons.  Along its path the appendix reads off

  * gamma_min, the lowest Lorentz factor the drag imposes: on lines beyond a
    critical radius the particle is brought to rest at the equator (gamma_min
    ~ 1), on shorter lines it crosses it with gamma_min > 1;
  * the extent l_pp of the pair-production zone: from the first scattering of
    the lepton to the point where b drops below the pair threshold 0.1; on
    lines with b > 0.1 everywhere the zone spans the equator and is taken
    symmetric about it.

Readings (the appendix gives no formulas for them):
  * the particle starts at the northern footpoint (s = 0) moving along +s, away
    from the star;
  * the first scattering is where the expected number of scatterings,
    integral Ndot_hat dt_hat along the path, reaches 1 (Eq. scatteringNdot);
  * gamma_min is the minimum of gamma between the footpoint and the equator:
    at the equator crossing if the particle crosses, else over the integration
    time t_max (the particle approaching its attractor beta = mu -> 0 at the
    equator);
  * l_pp = s_b - s_first where the zone closes at b = b_pp, L - 2 s_first on
    lines that never reach b < b_pp, 0 when the first scattering comes after
    s_b or never.

The equations, in t_hat = c t / R* with the position as v = cos(theta) on
r = R sin^2(theta) (ds = -R (1 + 3 v^2)^(1/2) dv, Appendix B.2):
    dv/dt_hat = -beta / (R (1 + 3 v^2)^(1/2)),  du/dt_hat = F_hat(u, v),
    dN/dt_hat = Ndot_hat(u, v),
integrated by scipy's Radau (an implicit Runge-Kutta method: the drag is stiff
near the attractor) with events at N = 1 and v = 0.

Pins (tests/test_oracle_testparticle.py): with the drag switched off the
particle keeps gamma_0 and never scatters; the Radau solution agrees with an
independent fixed-step fourth-order Runge-Kutta integration; the paper's
qualitative findings (gamma_min > 1 on the shortest lines and ~1 beyond a
critical radius, and a pair zone that grows over the shortest lines before it
falls to a couple of R* on long ones).
"""
import math

import numpy as np
from scipy.integrate import solve_ivp

from . import geometry, rics


def line_point(R, v, b_pole):
    """(b, mu, x) at cos(theta) = v on the line r = R sin^2(theta)."""
    return geometry.field_b(b_pole, R, v), geometry.photon_mu(v), geometry.radius(R, v)


def b_threshold_cos(R, b_pole, b_pp):
    """v in (0, v0] where b first drops to b_pp going from the northern footpoint,
    or None if b >= b_pp everywhere (b decreases monotonically towards the equator)."""
    v0 = geometry.footpoint_cos(R)
    if geometry.field_b(b_pole, R, 0.0) >= b_pp:
        return None
    lo, hi = 0.0, v0                  # b(lo) < b_pp <= b(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if geometry.field_b(b_pole, R, mid) < b_pp:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def rhs(R, b_pole, kT_keV):
    def f(t, y):
        v, u = y[0], y[1]
        b, mu, x = line_point(R, v, b_pole)
        gam = math.sqrt(1.0 + u * u)
        beta = u / gam
        F = float(rics.drag_force(u, b, mu, x, kT_keV))
        N = float(rics.scatter_rate(u, b, mu, x, kT_keV))
        return [-beta / (R * math.sqrt(1.0 + 3.0 * v * v)), F, N]
    return f


def sweep_line(R, gamma0=1000.0, kT_keV=1.0, b_pole=10.0, b_pp=0.1, t_max=None, rtol=1e-10):
    """gamma_min, s_first, s_b, l_pp (R*), whether the particle crossed the equator,
    and the line length L, for one line of equatorial radius R (R*)."""
    v0 = geometry.footpoint_cos(R)
    L = geometry.line_length(R)
    if t_max is None:
        t_max = 4.0 * L
    u0 = math.sqrt(gamma0 * gamma0 - 1.0)

    def ev_first(t, y):
        return y[2] - 1.0
    ev_first.terminal = False
    ev_first.direction = 1.0

    def ev_equator(t, y):
        return y[0]
    ev_equator.terminal = True
    ev_equator.direction = -1.0

    sol = solve_ivp(rhs(R, b_pole, kT_keV), (0.0, t_max), [v0, u0, 0.0], method="Radau", rtol=rtol,
                    atol=[1e-14, 1e-12, 1e-12], events=[ev_first, ev_equator], dense_output=True)
    crossed = sol.t_events[1].size > 0
    u_path = sol.y[1]
    gam_path = np.sqrt(1.0 + u_path * u_path)
    if crossed:
        ue = sol.y_events[1][0][1]
        gamma_min = min(float(gam_path.min()), math.sqrt(1.0 + ue * ue))
    else:
        gamma_min = float(gam_path.min())
    s_first = None
    if sol.t_events[0].size:
        v_first = sol.y_events[0][0][0]
        s_first = float(geometry.s_of_cos(R, v_first))
    vb = b_threshold_cos(R, b_pole, b_pp)
    s_b = float(geometry.s_of_cos(R, vb)) if vb is not None else None
    if s_first is None:
        l_pp = 0.0
    elif s_b is None:
        l_pp = max(L - 2.0 * s_first, 0.0)
    else:
        l_pp = max(s_b - s_first, 0.0)
    return dict(gamma_min=gamma_min, s_first=s_first, s_b=s_b, l_pp=l_pp, crossed=crossed, L=L)


def rk4_line(R, gamma0=1000.0, kT_keV=1.0, b_pole=10.0, n_steps=200000, t_end=None):
    """Fixed-step classical Runge-Kutta of the same equations up to the equator or t_end
    (an independent check of the Radau solution); returns (gamma at the end, min gamma, crossed)."""
    v0 = geometry.footpoint_cos(R)
    L = geometry.line_length(R)
    t_end = 4.0 * L if t_end is None else t_end
    f = rhs(R, b_pole, kT_keV)
    y = np.array([v0, math.sqrt(gamma0 * gamma0 - 1.0), 0.0])
    h = t_end / n_steps
    gmin = gamma0
    for _ in range(n_steps):
        k1 = np.array(f(0.0, y))
        k2 = np.array(f(0.0, y + 0.5 * h * k1))
        k3 = np.array(f(0.0, y + 0.5 * h * k2))
        k4 = np.array(f(0.0, y + h * k3))
        yn = y + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if yn[0] < 0.0:
            # linear interpolation to the equator crossing
            w = y[0] / (y[0] - yn[0])
            ue = y[1] + w * (yn[1] - y[1])
            return math.sqrt(1.0 + ue * ue), min(gmin, math.sqrt(1.0 + ue * ue)), True
        y = yn
        gmin = min(gmin, math.sqrt(1.0 + y[1] * y[1]))
    return math.sqrt(1.0 + y[1] * y[1]), gmin, False
