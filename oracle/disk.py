"""RICS from a finite stellar disk instead of the radial beam (Sec. 5; Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2.2 writes the scattering rate (Eq. scatteringNdot) as an integral over
the directions of the thermal photons, and evaluates it for photons that stream
radially from the star, subtending pi/x^2 steradian: that is the radial beam
behind Eq. contdrag.  Sec. 5 notes that the real radiation field differs from
that idealisation.  The first correction is the finite size of the star: at
x = r/R*, the blackbody surface (uniform intensity, no limb darkening) fills a
cone of half-angle theta_d, sin(theta_d) = 1/x, around the radial direction.
A photon in the cone at polar angle t from the radial direction and azimuth phi
about it crosses the field direction at the cosine

    mu' = mu cos t + (1 - mu^2)^(1/2) sin t cos phi,

mu the cosine between the radial direction and the field (the radial beam's
photon cosine).  The resonance of each direction sits at
y(mu') = b / (Theta gamma (1 - beta mu')), and the rate and the force
(F = Ndot DeltaP with DeltaP = gamma (mu' - beta)/(1 - beta mu') hbar omega_B / c
per direction, Sec. 2.2) become cone integrals:

    Ndot_hat = A_N / (pi gamma) * integral dOmega  y^2 / (e^y - 1)
    F_hat    = A_F / pi * integral dOmega  gamma (mu' - beta) y^3 / (e^y - 1)

with the prefactors A_F, A_N of oracle/rics.py (whose pi/x^2 is the radial
beam's solid angle).  Replacing the cone by pi/x^2 directions all at mu' = mu
gives back Eqs. scatteringNdot and contdrag.

The quadrature rule is part of this photon-field model (the library's table is
built with the same rule): Gauss-Legendre in c = cos t over [cos theta_d, 1]
with n_c nodes, and in phi over [0, pi] with n_phi nodes (the integrand is even
in phi), the solid angle being dOmega = dc dphi.

Pins (tests/test_oracle_disk.py): for a particle at rest the resonance does not
depend on the direction, and the cone integrals have closed forms -- the force
equals the radial beam's exactly (the mean of mu' over the cone is mu times the
radial beam's solid angle), the rate is the radial beam's times
2 / (1 + cos theta_d); far from the star both approach the radial beam as x^-2;
the Gauss-Legendre rule converges to an adaptive two-dimensional quadrature of
the same integrals.
"""
import numpy as np

from . import rics

N_C = 24          # Gauss-Legendre nodes in cos(t)
N_PHI = 24        # Gauss-Legendre nodes in phi over [0, pi]


def cone_rule(x, n_c=N_C, n_phi=N_PHI):
    """Nodes (cos t, phi) and weights (dc dphi, the [0, pi] half doubled) of the
    product rule over the stellar disk seen from x = r/R* (x >= 1)."""
    x = float(x)
    cd = np.sqrt(max(1.0 - 1.0 / (x * x), 0.0))        # cos(theta_d)
    gc, wc = np.polynomial.legendre.leggauss(n_c)
    gp, wp = np.polynomial.legendre.leggauss(n_phi)
    c = 0.5 * (1.0 - cd) * gc + 0.5 * (1.0 + cd)
    w_c = 0.5 * (1.0 - cd) * wc
    phi = 0.5 * np.pi * (gp + 1.0)
    w_p = 0.5 * np.pi * wp * 2.0                       # the phi in [pi, 2 pi] half mirrors it
    C, P = np.meshgrid(c, phi, indexing="ij")
    W = np.outer(w_c, w_p)
    return C.ravel(), P.ravel(), W.ravel()


def photon_cosines(mu, c, phi):
    """mu' of the directions (c = cos t, phi) for a field at cosine mu to the radial direction."""
    s = np.sqrt(np.maximum(1.0 - c * c, 0.0))
    return mu * c + np.sqrt(np.maximum(1.0 - mu * mu, 0.0)) * s * np.cos(phi)


def _cone(u, b, mu, x, kT_keV, n_c, n_phi):
    """(F_hat, Ndot_hat) of one particle (scalars) by the product rule."""
    A_F, A_N = rics.prefactors(kT_keV)
    gam, beta = rics.lorentz(u)
    c, phi, w = cone_rule(x, n_c, n_phi)
    mup = photon_cosines(mu, c, phi)
    y = b / (rics.theta_of_kT(kT_keV) * gam * (1.0 - beta * mup))
    big = y > rics.Y_CUTOFF
    ys = np.where(big, 1.0, y)
    em1 = np.expm1(ys)
    f2 = np.where(big, 0.0, ys * ys / em1)
    f3 = np.where(big, 0.0, ys ** 3 / em1)
    F = A_F / np.pi * np.sum(w * gam * (mup - beta) * f3)
    N = A_N / (np.pi * gam) * np.sum(w * f2)
    return F, N


def disk_rics(u, b, mu, x, kT_keV, n_c=N_C, n_phi=N_PHI):
    """(F_hat, Ndot_hat) of the finite stellar disk at momenta u and local geometry
    (b, mu, x); arrays broadcast together."""
    u, b, mu, x = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (u, b, mu, x)))
    F = np.empty(u.shape)
    N = np.empty(u.shape)
    for idx in np.ndindex(u.shape):
        F[idx], N[idx] = _cone(u[idx], b[idx], mu[idx], x[idx], kT_keV, n_c, n_phi)
    return F, N


def build_table(geom_at, n_lg, n_s, L_cells, kT_keV, n_c=N_C, n_phi=N_PHI):
    """F_hat and Ndot_hat of the finite disk for u >= 0 on the (log10 gamma, s) table
    grid of rics.table_axes; shape (n_lg, n_s).  Looked up by rics.table_lookup."""
    lg, s = rics.table_axes(n_lg, n_s, L_cells)
    b, mu, x = geom_at(s)
    gam = 10.0 ** lg
    u = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    F = np.empty((n_lg, n_s))
    N = np.empty((n_lg, n_s))
    for j in range(n_s):
        F[:, j], N[:, j] = disk_rics(u, b[j], mu[j], x[j], kT_keV, n_c, n_phi)
    return F, N
