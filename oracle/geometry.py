"""Dipole field-line geometry along the arc length s (Appendix B.2 of the paper).

The paper models one closed dipole field line r = r_eq sin^2(theta) with
footpoints on the star at colatitude theta_0 = arcsin((R*/r_eq)^(1/2)) and
feeds the RICS kernel the field strength B_d(l), the photon-field cosine
mu(l) = B^r / B_d and the radius r(l) along the line (Appendix B.2, the dipole
field formula and the footpoint colatitude).  The curvature radius is not in
the paper; it is the textbook curvature of the same curve and is only used by
the curvature conversion rule of the pair-injection step.

Units: lengths in R*, s = 0 at the northern footpoint (theta = theta_0),
s = L at the southern one.  R = r_eq / R* ("R_max").

Pins (tests/test_oracle_geometry.py): the line length against the paper's
cell count N_x = 3.84e5 at dl/R* = 6.67e-5 for r_eq = 10 (Sec. 3 and 4.2),
B at the pole surface = B*, mirror symmetry about the equator, mu = 0 and
R_curv = R/3 at the equator, and a brute-force polyline arc length;
interp_nodes against numpy's piecewise-linear interp, at nodes and midpoints
(tests/test_oracle_circuit_gravity.py).
"""
import numpy as np


def _phi(u):
    """Antiderivative helper: Phi(u) = u sqrt(1+3u^2) + asinh(sqrt(3) u)/sqrt(3).

    ds = R sin(theta) sqrt(1 + 3 cos^2 theta) dtheta along r = R sin^2 theta,
    so with u = cos(theta), s(u) = (R/2) [Phi(u0) - Phi(u)].
    """
    u = np.asarray(u, dtype=np.float64)
    return u * np.sqrt(1.0 + 3.0 * u * u) + np.arcsinh(np.sqrt(3.0) * u) / np.sqrt(3.0)


def footpoint_cos(R):
    """cos(theta_0) with sin^2(theta_0) = R*/r_eq (Appendix B.2, footpoint colatitude)."""
    return np.sqrt(1.0 - 1.0 / R)


def line_length(R):
    """Total arc length L/R* of the field line r = R sin^2(theta) between its footpoints."""
    u0 = footpoint_cos(R)
    return R * _phi(u0)


def s_of_cos(R, u):
    """Arc length s/R* from the northern footpoint to the point with cos(theta) = u."""
    u0 = footpoint_cos(R)
    return 0.5 * R * (_phi(u0) - _phi(u))


def cos_of_s(R, s):
    """Invert s(u) by bisection on u in [-u0, u0] (s decreases monotonically in u).

    100 halvings of an interval of width < 2 reach the float64 resolution.
    """
    s = np.asarray(s, dtype=np.float64)
    u0 = footpoint_cos(R)
    lo = np.full_like(s, -u0)   # s(lo) = L
    hi = np.full_like(s, u0)    # s(hi) = 0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        beyond = s_of_cos(R, mid) > s      # mid lies north of the target: move hi down
        hi = np.where(beyond, hi, mid)
        lo = np.where(beyond, mid, lo)
    return 0.5 * (lo + hi)


def field_b(b_pole, R, u):
    """b = B/B_QED of the dipole at (r, theta) on the line (Appendix B.2, B_d formula).

    B_d = B* R*^3 / (2 r^3) sqrt(3 cos^2 theta + 1) with r = R (1 - u^2) in R*.
    """
    r = R * (1.0 - u * u)
    return b_pole / (2.0 * r ** 3) * np.sqrt(1.0 + 3.0 * u * u)


def photon_mu(u):
    """mu = B^r / B_d = 2 cos(theta) / sqrt(1 + 3 cos^2 theta) (Appendix B.2).

    Photons stream radially out of the star; mu is the cosine between their
    direction and the field direction +s (positive in the northern half).
    """
    return 2.0 * u / np.sqrt(1.0 + 3.0 * u * u)


def radius(R, u):
    """x = r/R* = R sin^2(theta) along the line."""
    return R * (1.0 - u * u)


def curvature_radius(R, u):
    """Curvature radius of r = R sin^2(theta) in R* (textbook polar-curve curvature).

    kappa = |r^2 + 2 r'^2 - r r''| / (r^2 + r'^2)^(3/2) gives
    R_curv = R sin(theta) (1 + 3 cos^2 theta)^(3/2) / (3 (1 + cos^2 theta)).
    """
    sin_t = np.sqrt(np.maximum(1.0 - u * u, 0.0))
    return R * sin_t * (1.0 + 3.0 * u * u) ** 1.5 / (3.0 * (1.0 + u * u))


def node_tables(R, n_cells, b_pole):
    """Geometry at the n_cells+1 grid nodes s_i = i L / n_cells.

    Returns a dict of float64 arrays: s (R*), cos (cos theta), b, mu, x (r/R*),
    rc (curvature radius in R*), plus the scalars L and ds (cell length in R*).
    """
    L = line_length(R)
    s = np.arange(n_cells + 1, dtype=np.float64) * (L / n_cells)
    u = cos_of_s(R, s)
    u[0] = footpoint_cos(R)
    u[-1] = -footpoint_cos(R)
    return dict(L=L, ds=L / n_cells, s=s, cos=u,
                b=field_b(b_pole, R, u), mu=photon_mu(u),
                x=radius(R, u), rc=curvature_radius(R, u))


def interp_nodes(table, xcell):
    """Linear interpolation of a node array at particle positions xcell (in cells).

    The geometry seen by a particle is the straight line between the values at
    the two nodes bounding its cell (the grid carries the geometry, as in any
    PIC code).  xcell must lie in [0, n_cells].
    """
    n = table.shape[0] - 1
    i = np.clip(np.floor(xcell).astype(np.int64), 0, n - 1)
    f = xcell - i
    return table[i] * (1.0 - f) + table[i + 1] * f
