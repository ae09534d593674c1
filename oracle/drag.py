"""Semi-implicit RICS drag half step (Sec. 3, the limiter inequality, Eq. implicit
and the exponential damping that follows it).

The paper applies the continuous drag by Strang splitting: a drag update over
dt/2, the Lorentz push over dt, a second drag update over dt/2.  Each half
step starts from p0 and
  * if |F_hat(p0)| dt/(2|p0|) < dt/(2 tau_min), i.e. |F_hat(p0)| tau_min < |p0|,
    solves the implicit midpoint equation p1 = p0 + (dt/2) (F(p0) + F(p1))/2
    by Newton-Raphson;
  * otherwise relaxes p1 = p_tilde + (p0 - p_tilde) exp(-dt/(2 tau_min)) with
    the attractor p_tilde = mu / (1 - mu^2)^(1/2).
Readings of what the paper leaves open: the limiter is tested with
F evaluated at p0 and with "<=" so that a particle at rest with zero force
stays where it is; Newton stops at |delta| <= 1e-14 (1 + |p1|) or after 50
iterations.  Times are in R*/c (dt = h per step, tau_min in the same unit).

Pins (tests/test_oracle_drag.py): the damping branch equals the exact solution
of dp/dt = -(p - p_tilde)/tau_min; the implicit branch converges at second
order in h to an RK4 reference and to scipy's DOP853 of dp/dt = F(p).
"""
import numpy as np

NEWTON_TOL = 1e-14
NEWTON_MAX = 50


def attractor(mu):
    """p_tilde = mu / (1 - mu^2)^(1/2): the momentum with beta = mu (Sec. 2.2, Sec. 3)."""
    return mu / np.sqrt(1.0 - mu * mu)


def half_step(u0, force, dforce, h, tau_hat, mu, stats=None):
    """One drag update over h/2.

    u0        momenta (float64 array)
    force     callable u -> F_hat(u) for these particles (same shape)
    dforce    callable u -> dF_hat/du
    h         step length in R*/c (scalar)
    tau_hat   tau_min in R*/c (scalar)
    mu        photon cosine at the particles (for the attractor)
    stats     optional dict receiving 'limited', 'newton_iter_max', 'newton_unconverged'
    """
    u0 = np.asarray(u0, dtype=np.float64)
    F0 = force(u0)
    implicit = np.abs(F0) * tau_hat <= np.abs(u0)

    # Implicit midpoint p1 = p0 + (h/4)(F0 + F(p1)), Newton on G(p1) = 0.
    u1 = u0 + 0.5 * h * F0
    active = implicit.copy()
    it_max = 0
    for it in range(NEWTON_MAX):
        if not active.any():
            break
        G = u1 - u0 - 0.25 * h * (F0 + force(u1))
        dG = 1.0 - 0.25 * h * dforce(u1)
        delta = G / dG
        u1 = np.where(active, u1 - delta, u1)
        done = np.abs(delta) <= NEWTON_TOL * (1.0 + np.abs(u1))
        active &= ~done
        it_max = it + 1
    unconverged = int(active.sum())

    pt = attractor(mu)
    damped = pt + (u0 - pt) * np.exp(-0.5 * h / tau_hat)
    out = np.where(implicit, u1, damped)
    if stats is not None:
        stats['limited'] = stats.get('limited', 0) + int((~implicit).sum())
        stats['newton_iter_max'] = max(stats.get('newton_iter_max', 0), it_max)
        stats['newton_unconverged'] = stats.get('newton_unconverged', 0) + unconverged
    return out
