"""The combined cascade configuration (many lines of 32,768 cells with R_max in
[10, 100], a hot pair seed cascading to n_max, the surface atmosphere with ions at
m_i/m_e = 100, curvature conversion, pair annihilation over n_max) with fewer
lines, and the surrogate network as the RICS source with each line's table as its
fallback where the network's error estimate on the line exceeds 1e-3."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2609_17661_amd import Pic1D, workloads

from . import parity

pytestmark = pytest.mark.gpu

N_LINES = 4
TOL = 1e-3


def _print(*a):
    print(*a, flush=True)


def _network(seed):
    """Random weights of the network's shape and the oracle sample stream's target normalisation."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (o, i) in enumerate(omlp.LAYERS):
        s = 0.15 if li == len(omlp.LAYERS) - 1 else 1.0
        parts.append((rng.uniform(-1, 1, (o, i)) * s * omlp.glorot_bound(o, i), rng.uniform(-0.1, 0.1, o)))
    p = omlp.pack(parts).astype(np.float32).astype(np.float64)
    _, O, _ = omlp.training_samples(seed=seed, n=4096)
    mean, std = omlp.normalisation(O)
    return p, np.concatenate([mean, std]).astype(np.float32).astype(np.float64)


def _line_oracle_config(cfg, li):
    """One line of the batch for the oracle, keeping its global cell numbering."""
    base = sum(l["n_cells"] for l in cfg["lines"][:li])
    return parity.oracle_config(dict(cfg, lines=[dict(cfg["lines"][li], cell_base=base)]))


def _snap(sim, li):
    m = sim.moments(li)
    return dict(lines=[dict(parts=[sim.get_particles(li, s) for s in range(4)], E=sim.get_field(li))],
                step=m["step"]), m


def test_cfg5_fewer_lines_fallback_ledger_and_sampled_parity():
    """Four lines of the cascade configuration, replayed from 100-step HIP graphs until
    the cascade presses on n_max.  Every line's fallback decision and error estimate
    match the oracle's; in one step every line keeps Gauss's law, its particle-count
    ledger and the density rule (no cell above n_max unless it ran out of e- or e+),
    and three lines (the shortest R_max, the median, the longest) are compared with
    the oracle on a sample, with the couplings through the whole line's cell counts
    (the pair gate at n_max, annihilation) taken from the whole line."""
    from oracle import pic
    cfg = workloads.cfg5(n_lines=N_LINES, seed=3)
    p, norm = _network(61)
    cfg.update(rics="mlp", mlp_params=p, mlp_norm=norm, mlp_fallback_tol=TOL)
    n_max = cfg["nmax_over_n0"] * cfg["ppc0"]
    radii = [l["r_eq"] for l in cfg["lines"]]
    _print("cfg5 lines", radii)
    sim = Pic1D(cfg)
    for li in range(N_LINES):
        e_g, tab_g = sim.rics_line_info(li)
        ln = pic.State(_line_oracle_config(cfg, li)).lines[0]
        _print(f"  line {li}: estimate GPU {e_g:.6g} oracle {ln.mlp_error:.6g}, table {tab_g} / {ln.use_table}")
        assert tab_g == ln.use_table
        assert abs(e_g - ln.mlp_error) <= 1e-3 * ln.mlp_error + 1e-6
    sim.set_graph(100)
    for c in range(3):
        sim.step(100)
        _print("  steps", (c + 1) * 100, [sum(sim.moments(li)["count"]) for li in range(N_LINES)])
    order = np.argsort(radii, kind="stable")
    pick = [int(order[0]), int(order[N_LINES // 2]), int(order[-1])]
    m0 = [sim.moments(li) for li in range(N_LINES)]
    before = {li: _snap(sim, li)[0] for li in pick}
    sim.step(1)
    annihilated = 0
    for li in range(N_LINES):
        m1 = sim.moments(li)
        d = {k: m1["counters"][k] - m0[li]["counters"][k] for k in m1["counters"]}
        grown = 2 * (d["pairs_created"] + d["atm_injected"] - d["annihilated"]) - d["absorbed"]
        assert sum(m1["count"]) - sum(m0[li]["count"]) == grown, (li, d)
        assert m1["gauss_residual"] <= 1e-6
        annihilated += d["annihilated"]
        n = sim.n_cells(li)
        per = [np.bincount(sim.get_particles(li, s)["cell"], minlength=n) for s in range(4)]
        N = per[0] + per[1] + per[2] + per[3]
        assert not ((N > n_max) & (per[0] > 0) & (per[1] > 0)).any()
        _print(f"  line {li}: {d} count {sum(m1['count'])} residual {m1['gauss_residual']:.2e} "
               f"cells at the limit {int((N >= n_max - 1).sum())}")
    assert annihilated > 0
    for li in pick:
        after = _snap(sim, li)[0]
        rep, _ = parity.sampled_compare(_line_oracle_config(cfg, li), before[li], after, 40000,
                                        np.random.default_rng(li), n_max=n_max)
        _print(f"  sampled line {li} (R_max {radii[li]:.1f}):", rep)
        assert rep["compared"] > 5000
        assert rep["excused"] <= max(3, 1e-3 * rep["compared"])
    sim.close()
