"""Pins of oracle/drag.py (the drag half step of Sec. 3): the damping branch is the
exact relaxation, the implicit branch converges at second order to independent
ODE solutions of dp/dt = F(p)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import drag, rics

KT = 0.5
B, MU, X = 0.02, 0.5, 5.0


def _force(u):
    return rics.drag_force(u, B, MU, X, KT)


def _dforce(u):
    return rics.drag_force_du(u, B, MU, X, KT)


def _run(u0, h, n_half, tau_hat, stats=None):
    u = np.array([u0], dtype=np.float64)
    for _ in range(n_half):
        u = drag.half_step(u, _force, _dforce, h, tau_hat, np.array([MU]), stats=stats)
    return float(u[0])


def _dop853(u0, T):
    sol = solve_ivp(lambda t, y: [float(_force(y[0]))], (0.0, T), [u0], method="DOP853",
                    rtol=1e-12, atol=1e-14)
    return sol.y[0, -1]


def _rk4(u0, T, n):
    u, dt = u0, T / n
    for _ in range(n):
        k1 = _force(u)
        k2 = _force(u + 0.5 * dt * k1)
        k3 = _force(u + 0.5 * dt * k2)
        k4 = _force(u + dt * k3)
        u = u + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return float(u)


def test_implicit_branch_second_order_against_dop853_and_rk4():
    u0, T = 10.0, 2.0e-3            # drag time u/|F| ~ 1e-3 R*/c here
    ref = _dop853(u0, T)
    ref_rk4 = _rk4(u0, T, 20000)
    assert ref == pytest.approx(ref_rk4, rel=1e-10)
    assert ref < 0.8 * u0            # a substantial deceleration
    errs = []
    for h in (2e-4, 1e-4, 5e-5):
        st = {}
        n_half = int(round(T / (0.5 * h)))
        errs.append(abs(_run(u0, h, n_half, tau_hat=1e-7, stats=st) - ref))
        assert st["limited"] == 0 and st["newton_unconverged"] == 0
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.1)


def test_damping_branch_is_exact_relaxation():
    # when the limiter trips, each half step relaxes towards p_tilde = mu/sqrt(1-mu^2)
    # with time constant tau_min: compare with an ODE solution of dp/dt = -(p - p_tilde)/tau.
    u0, h, tau = 10.0, 1e-4, 1e-2   # tau_min much longer than the drag time -> limiter trips
    st = {}
    n_half = 60
    u = _run(u0, h, n_half, tau_hat=tau, stats=st)
    assert st["limited"] == n_half
    pt = MU / np.sqrt(1 - MU * MU)
    sol = solve_ivp(lambda t, y: [-(y[0] - pt) / tau], (0.0, n_half * 0.5 * h), [u0],
                    method="DOP853", rtol=1e-13, atol=1e-15)
    assert u == pytest.approx(sol.y[0, -1], rel=1e-10)


def test_limiter_switch_point():
    # implicit iff |F(p0)| tau_min <= |p0|
    u0 = 10.0
    F0 = abs(float(_force(u0)))
    tau_switch = u0 / F0
    st = {}
    drag.half_step(np.array([u0]), _force, _dforce, 1e-6, 0.999 * tau_switch, np.array([MU]), stats=st)
    assert st["limited"] == 0
    st = {}
    drag.half_step(np.array([u0]), _force, _dforce, 1e-6, 1.001 * tau_switch, np.array([MU]), stats=st)
    assert st["limited"] == 1


def test_zero_force_leaves_particle_alone():
    # a particle far from resonance (y beyond the cutoff) is untouched, also at rest
    u = np.array([0.0, 0.3, -2.0])
    z = lambda v: np.zeros_like(v)
    out = drag.half_step(u, z, z, 1e-3, 1e3, np.array([0.4, 0.4, 0.4]))
    np.testing.assert_array_equal(out, u)


def test_attractor_is_fixed_point():
    pt = MU / np.sqrt(1 - MU * MU)
    out = drag.half_step(np.array([pt]), _force, _dforce, 1e-4, 1e-7, np.array([MU]))
    assert out[0] == pytest.approx(pt, rel=1e-12)
