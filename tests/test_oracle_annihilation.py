"""Pins of the oracle's pair annihilation at the density limit (oracle/pic.py,
`annihilate`): what charge conservation and the count rule fix, independently of
how the oracle writes them."""
import math

import numpy as np

from oracle import pic


def _cfg(n_cells=16, **kw):
    d = dict(lines=[dict(r_eq=4.0, n_cells=n_cells, ppc_init=0, init="cold")], rics="off", j_twist=0.0,
             ppc0=1.0, nmax_over_n0=3.0)
    d.update(kw)
    return pic.make_config(**d)


def _load(st, s, x, ids, u=None):
    x = np.asarray(x, dtype=np.float64)
    cell = np.floor(x).astype(np.int32)
    pic.load_particles(st, 0, s, cell, x - cell, np.zeros(x.size) if u is None else u,
                       np.asarray(ids, dtype=np.uint64))


def _gauss_change(st, E0, rho0):
    """max |dE_{i+1/2} - dE_{i-1/2} - 4 pi drho_i| over interior nodes since (E0, rho0)."""
    rho = pic.charge_density(st, 0)
    dE = st.E[0] - E0
    return np.max(np.abs(dE[1:] - dE[:-1] - 4.0 * math.pi * (rho - rho0)[1:-1]))


def test_one_pair_current_in_closed_form():
    # four particles at rest in cell 5, n_max = 3: exactly one pair annihilates.  With
    # no motion and no twist current the only current is the annihilation's, so
    # Ampere gives E_5 = -4 pi Q (x_e- - x_e+) for the removed pair and 0 elsewhere,
    # and the change of E matches the change of the charge density (Gauss's law).
    st = pic.init_state(_cfg())
    xe, xp = np.array([5.2, 5.7]), np.array([5.4, 5.9])
    _load(st, 0, xe, [10, 12])
    _load(st, 1, xp, [11, 13])
    E0, rho0 = st.E[0].copy(), pic.charge_density(st, 0)
    pic.step(st)
    ln = st.lines[0]
    ke = set(int(i) for i in st.parts[0][0]["id"])
    kp = set(int(i) for i in st.parts[0][1]["id"])
    assert len(ke) == 1 and len(kp) == 1
    xe_gone = float(xe[[10, 12].index(({10, 12} - ke).pop())])
    xp_gone = float(xp[[11, 13].index(({11, 13} - kp).pop())])
    E = st.E[0]
    expect = np.zeros(ln.n)
    expect[5] = -4.0 * math.pi * ln.Q * (xe_gone - xp_gone)
    assert np.allclose(E, expect, rtol=0, atol=1e-15)
    assert st.counters[0]["annihilated"] == 1
    assert _gauss_change(st, E0, rho0) < 1e-15


def test_no_annihilation_at_or_below_the_limit():
    st = pic.init_state(_cfg())
    _load(st, 0, [5.2, 6.5], [10, 12])
    _load(st, 1, [5.4, 6.6], [11, 13])
    pic.step(st)
    assert st.parts[0][0]["x"].size == 2 and st.parts[0][1]["x"].size == 2
    assert np.all(st.E[0] == 0.0)


def _hot_overdense(seed=3, n_cells=40, per_cell=30, nmax=11.0, atmosphere_like=0):
    rng = np.random.default_rng(seed)
    cfg = _cfg(n_cells=n_cells, nmax_over_n0=nmax, j_twist=0.3)
    st = pic.init_state(cfg)
    m = n_cells * per_cell
    for s in (0, 1):
        x = rng.uniform(0.0, n_cells, m)
        u = rng.normal(0.0, 0.3, m)
        _load(st, s, x, np.arange(m, dtype=np.uint64) * 4 + s, u)
    if atmosphere_like:
        x = rng.uniform(0.0, n_cells, atmosphere_like)
        _load(st, 2, x, np.arange(atmosphere_like, dtype=np.uint64) * 4 + 2)
        _load(st, 3, x, np.arange(atmosphere_like, dtype=np.uint64) * 4 + 3)
    return st


def test_gauss_law_holds_through_annihilation():
    # the initial field is zero while the charge density is not: check the change
    # of E against the change of the charge density over four steps
    st = _hot_overdense()
    E0 = st.E[0].copy()
    rho0 = pic.charge_density(st, 0)
    for _ in range(4):
        pic.step(st)
    ln = st.lines[0]
    assert st.counters[0]["annihilated"] > 100
    assert _gauss_change(st, E0, rho0) < 1e-9 * 4.0 * math.pi * ln.Q


def test_count_left_in_each_cell():
    # every cell holds ~60 > n_max = 40: after one step a cell that keeps both
    # species holds N - 2 ceil((N - n_max)/2), i.e. 39 or 40 particles; a cell still
    # over the limit has run out of one species (k = min(N-, N+, ...)), its excess
    # being atmospheric particles that do not annihilate
    st = _hot_overdense(nmax=40.0, atmosphere_like=50)
    ln = st.lines[0]
    pic.step(st)
    counts = pic.cell_counts(ln, st.parts[0])
    ne = pic.cell_counts(ln, st.parts[0], species=(0,))
    npos = pic.cell_counts(ln, st.parts[0], species=(1,))
    both = (ne > 0) & (npos > 0)
    assert both.sum() >= 35
    assert np.all((counts[both] == 39) | (counts[both] == 40))
    assert np.all((ne[counts > 40] == 0) | (npos[counts > 40] == 0))
    # the atmosphere species are never removed
    assert st.parts[0][2]["x"].size == 50 and st.parts[0][3]["x"].size == 50


def test_equal_numbers_removed_per_cell_and_only_where_over_the_limit():
    st = _hot_overdense(n_cells=30, per_cell=8, nmax=14.0)
    ln = st.lines[0]
    ref = pic.init_state(st.cfg)
    ref.parts = [[dict(P) for P in st.parts[0]]]
    ref.cfg = dict(st.cfg, annihilation=False)
    pic.step(st)
    pic.step(ref)
    # same motion with annihilation off: the removed ones are exactly the difference
    kept = [set(int(i) for i in st.parts[0][s]["id"]) for s in range(4)]
    moved = [dict(zip((int(i) for i in ref.parts[0][s]["id"]), ref.parts[0][s]["x"])) for s in range(4)]
    counts = pic.cell_counts(ln, ref.parts[0])
    removed = [{i: x for i, x in moved[s].items() if i not in kept[s]} for s in (0, 1)]
    assert len(removed[0]) > 0
    for c in range(ln.n):
        ke = sum(1 for x in removed[0].values() if math.floor(x) == c)
        kp = sum(1 for x in removed[1].values() if math.floor(x) == c)
        assert ke == kp
        if counts[c] <= ln.n_max:
            assert ke == 0
    assert ref.parts[0][0]["x"].size == st.parts[0][0]["x"].size + len(removed[0])


def test_independent_of_particle_order():
    a = _hot_overdense(seed=5)
    b = _hot_overdense(seed=5)
    rng = np.random.default_rng(9)
    for s in (0, 1):
        P = b.parts[0][s]
        perm = rng.permutation(P["x"].size)
        b.parts[0][s] = {k: v[perm] for k, v in P.items()}
    for _ in range(2):
        pic.step(a)
        pic.step(b)
    for s in (0, 1):
        assert set(int(i) for i in a.parts[0][s]["id"]) == set(int(i) for i in b.parts[0][s]["id"])
    assert np.allclose(a.E[0], b.E[0], rtol=1e-12, atol=1e-15)
