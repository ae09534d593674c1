"""One PIC step of the 1D field-line model, plain FP64 (Sec. 3 and Appendix B).

Code units (the paper gives only the ratios, Sec. 3; the rest are readings):
  * one cell = one length unit, one step = one time unit; the speed of light
    is the CFL factor C = c0/c = 0.5 cells/step;
  * the fiducial skin depth d0 = 48 cells, so omega_p0 = C/d0 per step;
  * n0 is `ppc0` macro-particles per cell per species; a lepton carries charge
    +-Q and mass Q, an ion +Q and mass Q m_i/m_e, with Q = omega_p0^2/(4 pi ppc0)
    so that 4 pi n0 Q^2/M_e = omega_p0^2;
  * the twist current j_psi = (j_psi/n0 e c) * ppc0 * Q * C, uniform (Sec. 3);
  * one step is h = C ds/R* in units of R*/c, ds the cell length in R*;
  * tau_min = eta_min (n_psi/n0)^(1/2) / omega_p0 steps with n_psi/n0 = |j_psi/(n0 e c)|
    (Sec. 3, the definition of eta_min).

State of a line: per species the positions x (cells, float64), momenta
u = gamma beta (float64) and 64-bit ids; the field E on the n cell centres
(faces k+1/2); the step counter.  Species: 0 e- pair, 1 e+ pair,
2 atmospheric e-, 3 ion.  RICS acts on the leptons (species 0-2) only.

One step (Sec. 3; the order inside the stochastic regime -- kick, draw on the
post-kick momentum, recoil, move -- is a reading, the paper being silent):
  1. gather E at x^n (linear between cell centres, constant beyond the outer ones);
  2. geometry b, mu, x=r/R*, R_curv at x^n (linear between nodes);
  3. continuous regime (lepton, b < b_thr): drag h/2, Lorentz kick, drag h/2;
     stochastic regime (lepton, b >= b_thr): kick, then an event with
     probability min(Ndot_hat h, 1) drawn from Philox keyed by (step, id);
     an event emits eps = gamma (1 - (1+2b)^-1/2) and leaves gamma - eps;
     ions: kick only.  Gravity T/h towards the nearest wall inside the layer;
  4. move x^{n+1} = x^n + C u/gamma;
  5. charge-conserving deposit j_{k+1/2} += q |[x^n, x^{n+1}] cap [k, k+1]| (signed),
     path clipped to the domain [0, n];
  6. absorb particles with x^{n+1} outside [0, n);
  7. photons with eps >= 2 convert at s' (immediately at x^n, or where the
     straight photon path leaves the curved line by arcsin(2/eps)) into an
     e-/e+ pair at gamma = eps/2 each, if s' is inside and the start-of-step
     count of all particles in that cell is below n_max;
  8. atmosphere: refill the layer cells to the hydrostatic profile with
     co-located (e-, ion) pairs;
  9. pair annihilation at the density limit n_max (see `annihilate`);
 10. Ampere  E_{k+1/2} -= 4 pi (j_{k+1/2} - j_psi).

Pins:
  * tests/test_oracle_pic.py: hyperbolic motion, Gauss's law to roundoff, the
    energy ledger with drag off, the cold two-stream growth rate;
  * tests/test_oracle_annihilation.py: the current of one annihilated pair in
    closed form, Gauss's law, the count left in a cell, independence of the
    particle order;
  * tests/test_oracle_atmosphere_events.py: the refill's Maxwellian momenta,
    uniform offsets and hydrostatic targets; energy conservation through an
    event and its pair; the event and pair yield against Binomial(N, Ndot h).
  * tests/test_oracle_circuit_gravity.py: the circuit potential V_c against the
    energy a test lepton gains crossing a frozen-field line (sign and 1/c^2), and
    the layer gravity against relativistic free fall under a constant force
    towards the nearer wall (fall time from rest, apex of a thrown particle, no
    force outside the layer).
Parity unpinned: which e-/e+ of an over-full cell annihilate (the smallest Philox
keys) is a reading of a step the paper leaves open; it is pinned only by its
independence of the particle order, not by anything the paper fixes.
The photon energy eps is pinned in tests/test_oracle_rics.py by explicit
four-momenta (resonant absorption, perpendicular decay, boost back);
energy conservation through an event pins what the step does with it.
The angle-resolved events (option 'emission': 'isotropic' or 'dipole' rest-frame
patterns, the cosine drawn from the other words of the event's Philox block) are
pinned in tests/test_oracle_emission.py by the printed E_gamma(theta), 60-digit
Lorentz boosts, the rest-frame mass shell, the paper's bounds on E_gamma and the
patterns' distribution functions; the patterns themselves are readings.
"""
import math

import numpy as np

from . import disk, drag, geometry, mlp, philox, rics

N_SPECIES = 4
SPECIES_SIGN = (-1.0, +1.0, -1.0, +1.0)
SPECIES_LEPTON = (True, True, True, False)


def species_mass(s, mass_ratio):
    return mass_ratio if s == 3 else 1.0


DEFAULTS = dict(
    b_pole=10.0, cfl=0.5, d0_cells=48.0, ppc0=64.0, j_twist=0.5, kT_keV=0.5,
    eta_min=1.0e3, b_thr=0.1, mass_ratio=100.0, rics="table", table_nlg=256,
    table_ns=512, pairs=False, conversion="immediate", nmax_over_n0=0.0,
    atmosphere=False, atm_a0=0.0, atm_h_cells=0.0, atm_T=0.01, atm_cut=0.01,
    gravity=True, frozen_field=False, seed=0, lines=None, mlp_params=None, mlp_norm=None, mlp_fallback_tol=0.0,
    annihilation=True, photon_field="radial", emission="perpendicular",
)


class Line:
    """Derived constants and node tables of one field line (FP64)."""

    def __init__(self, cfg, line_index, line_cfg, cell_base):
        self.cfg = cfg
        self.index = line_index
        self.cell_base = cell_base
        self.R = float(line_cfg['r_eq'])
        self.n = int(line_cfg['n_cells'])
        self.line_cfg = line_cfg
        C = cfg['cfl']
        self.C = C
        geo = geometry.node_tables(self.R, self.n, cfg['b_pole'])
        self.geo = geo
        self.L_rstar = geo['L']
        self.ds = geo['ds']                      # cell length in R*
        self.h = C * self.ds                     # step in R*/c
        self.wp0 = C / cfg['d0_cells']           # per step
        self.Q = self.wp0 ** 2 / (4.0 * math.pi * cfg['ppc0'])
        self.j_tw = cfg['j_twist'] * cfg['ppc0'] * self.Q * C
        npsi = abs(cfg['j_twist'])
        self.tau_steps = cfg['eta_min'] * math.sqrt(npsi) / self.wp0 if npsi > 0 else cfg['eta_min'] / self.wp0
        self.tau_hat = self.tau_steps * self.h
        nmax = cfg['nmax_over_n0'] if cfg['nmax_over_n0'] > 0 else cfg['d0_cells'] ** 2
        self.n_max = nmax * cfg['ppc0']
        # atmosphere (Appendix B.1, Eq. densprofile)
        a0 = cfg['atm_a0'] if cfg['atm_a0'] > 0 else 18.0 * npsi
        if a0 <= 0.0:
            a0 = cfg['atm_cut']          # no atmosphere without a twist current
        hat = cfg['atm_h_cells'] if cfg['atm_h_cells'] > 0 else 3.0 * cfg['d0_cells'] / math.sqrt(a0)
        self.atm_a0, self.atm_h = a0, hat
        self.atm_depth = hat * math.log(a0 / cfg['atm_cut']) if a0 > cfg['atm_cut'] else 0.0
        k = np.arange(self.n)
        d = np.minimum(k + 0.5, self.n - k - 0.5)
        prof = a0 * np.exp(-d / hat)
        self.atm_target = np.where(prof >= cfg['atm_cut'],
                                   np.floor(prof * cfg['ppc0']), 0.0).astype(np.int64)
        # the surrogate's error estimate on this line and, above the tolerance, the
        # table as its source (mlp_fallback_tol > 0)
        fallback = cfg['rics'] == 'mlp' and cfg['mlp_fallback_tol'] > 0.0
        self.mlp_error = None
        self.use_table = cfg['rics'] == 'table'
        if cfg['rics'] == 'table' or fallback:
            def geom_at(sc):
                u = geometry.cos_of_s(self.R, sc * self.ds)
                return (geometry.field_b(cfg['b_pole'], self.R, u), geometry.photon_mu(u),
                        geometry.radius(self.R, u))
            build = disk.build_table if cfg['photon_field'] == 'disk' else rics.build_table
            self.F_tab, self.N_tab = build(geom_at, cfg['table_nlg'], cfg['table_ns'], float(self.n), cfg['kT_keV'])
        if fallback:
            _, s_rows = rics.table_axes(cfg['table_nlg'], cfg['table_ns'], float(self.n))
            b_r, mu_r, x_r = geom_at(s_rows)
            nm = np.asarray(cfg['mlp_norm'], dtype=np.float64).reshape(2, 3)
            self.mlp_error = mlp.line_error_estimate(np.asarray(cfg['mlp_params'], dtype=np.float64),
                                                     (nm[0], nm[1]), b_r, mu_r, x_r, cfg['table_nlg'],
                                                     cfg['kT_keV'], self.h)
            self.use_table = self.mlp_error > cfg['mlp_fallback_tol']

    def geometry_at(self, xc):
        g = self.geo
        return (geometry.interp_nodes(g['b'], xc), geometry.interp_nodes(g['mu'], xc),
                geometry.interp_nodes(g['x'], xc), geometry.interp_nodes(g['rc'], xc))

    def rics_funcs(self, xc, b, mu, xr):
        """(force(u), dforce(u), rate(u)) closures for particles at xc."""
        cfg = self.cfg
        kT = cfg['kT_keV']
        mode = cfg['rics']
        if cfg['photon_field'] == 'disk' and mode not in ('table', 'off'):
            raise ValueError("the finite-disk photon field is tabulated (rics='table') only")
        if mode == 'exact':
            return (lambda u: rics.drag_force(u, b, mu, xr, kT),
                    lambda u: rics.drag_force_du(u, b, mu, xr, kT),
                    lambda u: rics.scatter_rate(u, b, mu, xr, kT))
        if mode == 'table' or (mode == 'mlp' and self.use_table):
            L = float(self.n)
            return (lambda u: rics.table_lookup(self.F_tab, self.N_tab, u, xc, L)[0],
                    lambda u: rics.table_lookup(self.F_tab, self.N_tab, u, xc, L)[2],
                    lambda u: rics.table_lookup(self.F_tab, self.N_tab, u, xc, L)[1])
        if mode == 'off':
            z = lambda u: np.zeros_like(np.asarray(u, dtype=np.float64))
            return z, z, z
        if mode == 'mlp':
            # the surrogate network (oracle/mlp.py), fed the arc-length fraction of the
            # particle (u >= 0) or of its mirror point (u < 0)
            P = np.asarray(cfg['mlp_params'], dtype=np.float64)
            nm = np.asarray(cfg['mlp_norm'], dtype=np.float64).reshape(2, 3)
            norm = (nm[0], nm[1])
            sl = xc / self.n

            def args(u):
                u = np.asarray(u, dtype=np.float64)
                return u, np.where(u >= 0, sl, 1.0 - sl), b, mu, xr, kT
            return (lambda u: mlp.surrogate_rics(P, norm, *args(u))[0],
                    lambda u: mlp.surrogate_force_du(P, norm, *args(u)),
                    lambda u: mlp.surrogate_rics(P, norm, *args(u))[1])
        raise ValueError(f"unknown rics mode {mode!r}")


def make_config(**kw):
    cfg = dict(DEFAULTS)
    cfg.update(kw)
    if not cfg['lines']:
        raise ValueError("config needs at least one line")
    return cfg


class State:
    """Particles and fields of all lines."""

    def __init__(self, cfg):
        if cfg['emission'] not in rics.EMISSION_PATTERNS:
            raise ValueError(f"emission must be one of {rics.EMISSION_PATTERNS}")
        self.cfg = cfg
        self.lines = []
        base = 0
        for i, lc in enumerate(cfg['lines']):
            # a line taken out of a batch keeps its global cell numbering (the
            # atmosphere's draws are keyed by global cell) through 'cell_base'
            base = int(lc.get('cell_base', base))
            self.lines.append(Line(cfg, i, lc, base))
            base += int(lc['n_cells'])
        self.step = 0
        # per line: list over species of dict(x, u, id); E; counters; pair rate
        self.parts = [[_empty() for _ in range(N_SPECIES)] for _ in self.lines]
        self.E = [np.zeros(l.n) for l in self.lines]
        self.j_last = [np.zeros(l.n) for l in self.lines]
        self.pair_rate = [np.zeros(l.n, dtype=np.int64) for l in self.lines]
        self.counters = [_zero_counters() for _ in self.lines]
        self.energy_twist = [0.0 for _ in self.lines]
        self.energy_walls = [0.0 for _ in self.lines]


def _empty():
    return dict(x=np.zeros(0), u=np.zeros(0), id=np.zeros(0, dtype=np.uint64))


COUNTER_NAMES = ('events', 'pairs_created', 'photons_escaped', 'absorbed',
                 'psc_clipped', 'limited', 'newton_unconverged', 'atm_injected', 'annihilated')


def _zero_counters():
    return {k: 0 for k in COUNTER_NAMES}


def init_state(cfg):
    """Initial state: ppc_init co-located e-/e+ pairs per cell (Sec. 3, the homogeneous pair plasma).

    Pair i of a line sits in cell i // ppc_init at offset U24(w0) of the Philox
    block (0, i, line, STREAM_INIT); its momentum is 0 ("cold"), +-gamma beta0
    ("stream", e+ along the twist current) or, for "hot", gamma log-uniform in
    [1, gamma_max] from w1 with the sign from the top bit of w2 (same for both
    members).  Ids: line * 2^40 + 2 i (e-) and + 1 (e+).
    """
    st = State(cfg)
    k0, k1 = philox.seed_key(cfg['seed'])
    for li, ln in enumerate(st.lines):
        lc = ln.line_cfg
        ppc = int(lc.get('ppc_init', 0))
        npair = ppc * ln.n
        if npair == 0:
            continue
        i = np.arange(npair, dtype=np.uint64)
        w = philox.philox4x32_10(0, i, li, philox.STREAM_INIT, k0, k1)
        x = (i // np.uint64(ppc)).astype(np.float64) + philox.uniform24(w[0])
        mode = lc.get('init', 'cold')
        if mode == 'cold':
            u = np.zeros(npair)
            ue, up = u, u.copy()
        elif mode == 'hot':
            gmax = float(lc.get('init_gamma_max', 1.0e4))
            gam = 10.0 ** (philox.uniform24(w[1]) * math.log10(gmax))
            sgn = np.where((w[2] >> np.uint32(31)) == 1, -1.0, 1.0)
            u = sgn * np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
            ue, up = u, u.copy()
        elif mode == 'stream':
            b0 = float(lc.get('init_beta', 0.1))
            us = b0 / math.sqrt(1.0 - b0 * b0) * (1.0 if cfg['j_twist'] >= 0 else -1.0)
            up = np.full(npair, us)
            ue = np.full(npair, -us)
        else:
            raise ValueError(mode)
        base = np.uint64(li) << np.uint64(40)
        st.parts[li][0] = dict(x=x.copy(), u=ue.astype(np.float64), id=base + 2 * i)
        st.parts[li][1] = dict(x=x.copy(), u=up.astype(np.float64), id=base + 2 * i + 1)
    return st


def gather_E(E, xc):
    """E at positions xc, linear between cell centres k+1/2, constant beyond the outer ones."""
    n = E.shape[0]
    xs = np.clip(xc - 0.5, 0.0, n - 1.0)
    k = np.minimum(np.floor(xs).astype(np.int64), n - 2)
    w = xs - k
    return E[k] * (1.0 - w) + E[k + 1] * w


def deposit(j, q, x0, x1, n):
    """Add q times the signed overlap of [x0, x1] (clipped to [0, n]) with every cell."""
    a = np.clip(x0, 0.0, float(n))
    b = np.clip(x1, 0.0, float(n))
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    sgn = np.sign(b - a)
    k0 = np.minimum(np.floor(lo).astype(np.int64), n - 1)
    k1 = np.minimum(np.floor(hi).astype(np.int64), n - 1)
    same = k0 == k1
    w0 = np.where(same, b - a, sgn * (k1 - lo))
    w1 = np.where(same, 0.0, sgn * (hi - k1))
    j += q * np.bincount(k0, weights=w0, minlength=n)
    j += q * np.bincount(k1, weights=w1, minlength=n)


def cell_counts(ln, parts, species=None, use_key='x'):
    """Per-cell counts of live particles (all species or the given ones)."""
    n = ln.n
    tot = np.zeros(n, dtype=np.int64)
    for s in (range(N_SPECIES) if species is None else species):
        xc = parts[s][use_key]
        if xc.size:
            tot += np.bincount(np.floor(xc).astype(np.int64), minlength=n)
    return tot


def annihilation_keys(step, ids, k0, k1):
    """64-bit ranking keys of the annihilation draw: words 1 (high) and 0 (low) of
    the Philox block (step, id low, id high, STREAM_ANNIH)."""
    lo, hi = philox.split_id(ids)
    w = philox.philox4x32_10(step, lo, hi, philox.STREAM_ANNIH, k0, k1)
    return (w[1].astype(np.uint64) << np.uint64(32)) | w[0].astype(np.uint64)


def annihilate(ln, parts, nstep, k0, k1, j, counters):
    """Pair annihilation at the density limit (Sec. 3: pairs annihilate where the
    total density approaches n_max, so that the skin depth stays resolved; the
    paper gives no mechanics, so these are readings):

      * a cell whose count N of all particles (after the step's push, pair
        creation and atmosphere refill) exceeds n_max loses
        k = min(N-, N+, ceil((N - n_max)/2)) secondary pairs, N-/N+ its e-/e+
        (species 0/1) counts; atmospheric electrons and ions do not annihilate;
      * the annihilating e- and e+ are the k of each species in the cell with the
        smallest (key, id), key = `annihilation_keys` -- a choice independent of
        where the particles sit in memory;
      * charge conservation: each pair annihilates as if its positron first moved
        to its electron, which deposits +Q (x- - x+) on the cell's face current;
        summed over the cell's pairs that is Q (sum x- - sum x+), whatever the
        pairing, and the neutral pair then leaves no charge behind.

    Returns the new per-species particle dicts; adds the current to j.
    """
    n = ln.n
    counts = cell_counts(ln, parts)
    over = counts > ln.n_max
    if not over.any():
        return parts
    ne = cell_counts(ln, parts, species=(0,))
    npos = cell_counts(ln, parts, species=(1,))
    need = np.ceil((counts - ln.n_max) / 2.0)
    k = np.where(over, np.minimum(np.minimum(ne, npos), need), 0).astype(np.int64)
    out = list(parts)
    xsum = []
    for s in (0, 1):
        P = parts[s]
        if P['x'].size == 0:
            xsum.append(np.zeros(n))
            continue
        cell = np.floor(P['x']).astype(np.int64)
        key = annihilation_keys(nstep, P['id'], k0, k1)
        order = np.lexsort((P['id'], key, cell))       # by cell, then key, then id
        cs = cell[order]
        rank = np.arange(cs.size) - np.searchsorted(cs, cs, side='left')
        remove = np.zeros(cs.size, dtype=bool)
        remove[order] = rank < k[cs]
        xsum.append(np.bincount(cell[remove], weights=P['x'][remove], minlength=n))
        out[s] = dict(x=P['x'][~remove], u=P['u'][~remove], id=P['id'][~remove])
    j += ln.Q * (xsum[0] - xsum[1])
    counters['annihilated'] += int(k.sum())
    return out


def step(st, stats=None):
    """Advance every line by one step."""
    for li in range(len(st.lines)):
        _step_line(st, li, stats)
    st.step += 1


def _step_line(st, li, stats):
    cfg = st.cfg
    ln = st.lines[li]
    n, C = ln.n, ln.C
    E = st.E[li]
    parts = st.parts[li]
    cnt = st.counters[li]
    nstep = st.step
    k0, k1 = philox.seed_key(cfg['seed'])
    j = np.zeros(n)
    counts_start = cell_counts(ln, parts)
    events = []          # per species: (x^n, direction, eps, parent id, R_curv)
    new_parts = []

    for s in range(N_SPECIES):
        P = parts[s]
        if P['x'].size == 0:
            new_parts.append(P)
            continue
        x0, u, pid = P['x'], P['u'].copy(), P['id']
        qm = SPECIES_SIGN[s] / species_mass(s, cfg['mass_ratio'])
        Ep = gather_E(E, x0)
        kick = qm * Ep / C
        if cfg['atmosphere'] and cfg['gravity'] and ln.atm_depth > 0:
            dwall = np.minimum(x0, n - x0)
            towards = np.where(x0 < 0.5 * n, -1.0, 1.0)
            g = cfg['atm_T'] / species_mass(s, cfg['mass_ratio']) * C / ln.atm_h
            kick = kick + np.where(dwall <= ln.atm_depth, towards * g, 0.0)
        if SPECIES_LEPTON[s] and cfg['rics'] != 'off':
            b, mu, xr, rc = ln.geometry_at(x0)
            cont = b < cfg['b_thr']
            ic = np.nonzero(cont)[0]
            isr = np.nonzero(~cont)[0]
            unew = np.empty_like(u)
            if ic.size:
                # continuous regime: Strang splitting drag h/2, kick, drag h/2
                force, dforce, _ = ln.rics_funcs(x0[ic], b[ic], mu[ic], xr[ic])
                v = drag.half_step(u[ic], force, dforce, ln.h, ln.tau_hat, mu[ic], stats=cnt)
                v = v + kick[ic]
                v = drag.half_step(v, force, dforce, ln.h, ln.tau_hat, mu[ic], stats=cnt)
                unew[ic] = v
            if isr.size:
                # stochastic regime: kick, draw, recoil
                _, _, rate = ln.rics_funcs(x0[isr], b[isr], mu[isr], xr[isr])
                us = u[isr] + kick[isr]
                lam = rate(us) * ln.h
                p = np.minimum(lam, 1.0)
                cnt['psc_clipped'] += int((lam > 1.0).sum())
                lo, hi = philox.split_id(pid[isr])
                w = philox.philox4x32_10(nstep, lo, hi, philox.STREAM_RICS, k0, k1)
                ev = philox.uniform24(w[0]) < p
                if cfg['emission'] == 'perpendicular':
                    gam = np.sqrt(1.0 + us * us)
                    eps = rics.photon_energy(us, b[isr])
                    gnew = gam - eps
                    dirn = np.where(us >= 0.0, 1.0, -1.0)
                    urec = dirn * np.sqrt(np.maximum(gnew * gnew - 1.0, 0.0))
                else:
                    # rest-frame emission cosine from the event's other Philox words
                    mu_r = rics.emission_cosine(w[1], w[2], w[3], cfg['emission'])
                    eps, urec, dirn = rics.emission(us, b[isr], mu_r)
                unew[isr] = np.where(ev, urec, us)
                if ev.any():
                    cnt['events'] += int(ev.sum())
                    sel = isr[ev]
                    events.append((x0[sel], dirn[ev], eps[ev], pid[sel], rc[sel]))
            u = unew
        else:
            u = u + kick
        gam = np.sqrt(1.0 + u * u)
        x1 = x0 + C * u / gam
        deposit(j, SPECIES_SIGN[s] * ln.Q, x0, x1, n)
        alive = (x1 >= 0.0) & (x1 < n)
        nabs = int((~alive).sum())
        if nabs:
            cnt['absorbed'] += nabs
            m = species_mass(s, cfg['mass_ratio']) * ln.Q
            st.energy_walls[li] += float(np.sum(m * C * C * (gam[~alive] - 1.0)))
        new_parts.append(dict(x=x1[alive], u=u[alive], id=pid[alive]))

    # photon conversion into pairs (Sec. 3: inject immediately, limited by n_max)
    if events:
        ex = np.concatenate([e[0] for e in events])
        ed = np.concatenate([e[1] for e in events])
        ee = np.concatenate([e[2] for e in events])
        ei = np.concatenate([e[3] for e in events])
        er = np.concatenate([e[4] for e in events])
        conv = (ee >= 2.0) if cfg['pairs'] else np.zeros(ee.shape, dtype=bool)
        if cfg['conversion'] == 'immediate':
            sp = ex.copy()
        elif cfg['conversion'] == 'curvature':
            sp = ex + ed * (er / ln.ds) * np.arcsin(np.minimum(2.0 / np.maximum(ee, 2.0), 1.0))
        else:
            raise ValueError(cfg['conversion'])
        inside = (sp >= 0.0) & (sp < n)
        cell = np.where(inside, np.floor(np.where(inside, sp, 0.0)), 0).astype(np.int64)
        make = conv & inside & (counts_start[cell] < ln.n_max)
        cnt['photons_escaped'] += int((~make).sum())
        cnt['pairs_created'] += int(make.sum())
        if make.any():
            gp = 0.5 * ee[make]
            up = ed[make] * np.sqrt(np.maximum(gp * gp - 1.0, 0.0))
            lo, hi = philox.split_id(ei[make])
            w = philox.philox4x32_10(nstep, lo, hi, philox.STREAM_CHILD, k0, k1)
            st.pair_rate[li] += np.bincount(cell[make], minlength=n)
            for s, ids in ((0, philox.id_from_words(w[0], w[1])), (1, philox.id_from_words(w[2], w[3]))):
                P = new_parts[s]
                new_parts[s] = dict(x=np.concatenate([P['x'], sp[make]]),
                                    u=np.concatenate([P['u'], up]),
                                    id=np.concatenate([P['id'], ids]))

    # atmosphere (Sec. 3 and Appendix B.1): refill to the hydrostatic profile
    if cfg['atmosphere']:
        ne = np.zeros(n, dtype=np.int64)
        ni = np.zeros(n, dtype=np.int64)
        if new_parts[2]['x'].size:
            ne = np.bincount(np.floor(new_parts[2]['x']).astype(np.int64), minlength=n)
        if new_parts[3]['x'].size:
            ni = np.bincount(np.floor(new_parts[3]['x']).astype(np.int64), minlength=n)
        deficit = np.maximum(ln.atm_target - np.minimum(ne, ni), 0)
        cells = np.nonzero(deficit)[0]
        if cells.size:
            cc = np.repeat(cells, deficit[cells])
            kk = np.concatenate([np.arange(d) for d in deficit[cells]]).astype(np.uint64)
            gc = (cc + ln.cell_base).astype(np.uint64)
            wa = philox.philox4x32_10(nstep, gc, kk, philox.STREAM_ATM_A, k0, k1)
            wb = philox.philox4x32_10(nstep, gc, kk, philox.STREAM_ATM_B, k0, k1)
            wc = philox.philox4x32_10(nstep, gc, kk, philox.STREAM_ATM_ID, k0, k1)
            xa = cc.astype(np.float64) + philox.uniform24(wa[0])
            T = cfg['atm_T']
            ue = math.sqrt(T) * np.sqrt(-2.0 * np.log(philox.uniform24_open0(wa[1]))) * \
                np.cos(2.0 * math.pi * philox.uniform24(wa[2]))
            ui = math.sqrt(T / cfg['mass_ratio']) * np.sqrt(-2.0 * np.log(philox.uniform24_open0(wb[0]))) * \
                np.cos(2.0 * math.pi * philox.uniform24(wb[1]))
            for s, uu, ids in ((2, ue, philox.id_from_words(wc[0], wc[1])),
                               (3, ui, philox.id_from_words(wc[2], wc[3]))):
                P = new_parts[s]
                new_parts[s] = dict(x=np.concatenate([P['x'], xa]), u=np.concatenate([P['u'], uu]),
                                    id=np.concatenate([P['id'], ids]))
            cnt['atm_injected'] += int(cc.size)

    if cfg['annihilation']:
        new_parts = annihilate(ln, new_parts, nstep, k0, k1, j, cnt)

    st.parts[li] = new_parts
    st.j_last[li] = j
    if not cfg['frozen_field']:
        Enew = E - 4.0 * math.pi * (j - ln.j_tw)
        # work done by the twist current on the field, time-centred (energy ledger)
        st.energy_twist[li] += float(np.sum(0.5 * (E + Enew) * ln.j_tw))
        st.E[li] = Enew


# ---------------------------------------------------------------------------
# Moments (Sec. 3 results: densities, currents, V_c; Sec. 5: 1D Gauss law)
# ---------------------------------------------------------------------------

def charge_density(st, li):
    """rho on the n+1 nodes from cloud-in-cell weights (charge per cell length)."""
    ln = st.lines[li]
    rho = np.zeros(ln.n + 1)
    for s in range(N_SPECIES):
        xc = st.parts[li][s]['x']
        if xc.size == 0:
            continue
        i = np.floor(xc).astype(np.int64)
        f = xc - i
        q = SPECIES_SIGN[s] * ln.Q
        rho += q * np.bincount(i, weights=1.0 - f, minlength=ln.n + 1)
        rho += q * np.bincount(i + 1, weights=f, minlength=ln.n + 1)
    return rho


def gauss_residual(st, li):
    """max over interior nodes of |E_{i+1/2} - E_{i-1/2} - 4 pi rho_i| / (4 pi Q ppc0)."""
    ln = st.lines[li]
    rho = charge_density(st, li)
    E = st.E[li]
    r = E[1:] - E[:-1] - 4.0 * math.pi * rho[1:-1]
    return float(np.max(np.abs(r))) / (4.0 * math.pi * ln.Q * st.cfg['ppc0']) if r.size else 0.0


def circuit_potential(st, li):
    """e V_c / (m_e c^2) = -sum_k E_k / C^2 (the line integral of E along the line, Sec. 2)."""
    ln = st.lines[li]
    return -float(np.sum(st.E[li])) / (ln.C * ln.C)


def energies(st, li):
    """(kinetic, field) energy of a line in code units."""
    ln = st.lines[li]
    K = 0.0
    for s in range(N_SPECIES):
        u = st.parts[li][s]['u']
        if u.size:
            m = species_mass(s, st.cfg['mass_ratio']) * ln.Q
            K += float(np.sum(m * ln.C ** 2 * (np.sqrt(1.0 + u * u) - 1.0)))
    U = float(np.sum(st.E[li] ** 2)) / (8.0 * math.pi)
    return K, U


# ---------------------------------------------------------------------------
# State exchange with other implementations (positions as int32 cell + float32
# offset, momenta float32) for per-step comparisons
# ---------------------------------------------------------------------------

def load_particles(st, li, s, cell, off, u, pid):
    """Replace species s of line li by the given state, promoted exactly to float64."""
    st.parts[li][s] = dict(x=np.asarray(cell, dtype=np.float64) + np.asarray(off, dtype=np.float64),
                           u=np.asarray(u, dtype=np.float64),
                           id=np.asarray(pid, dtype=np.uint64).copy())
