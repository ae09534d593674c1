"""The batched path: many ragged lines in one state, HIP-graph replay and the autotuner."""
import numpy as np
import pytest

from paper_2609_17661_amd import Pic1D, workloads

from . import parity

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _ragged(n_lines=6, seed=3, **kw):
    """Lines of uneven length and particle count, hot plasma, pairs and atmosphere."""
    rng = np.random.default_rng(seed)
    lines = []
    for i in range(n_lines):
        n = int(rng.integers(40, 200))
        p = int(rng.integers(3, 14))
        lines.append(dict(r_eq=float(2.0 * 15.0 ** rng.random()), n_cells=n, ppc_init=p, init="hot",
                          init_gamma_max=2e3, capacity=[200_000, 200_000, 40_000, 40_000]))
    cfg = dict(rics="exact", kT_keV=0.5, j_twist=0.5, ppc0=8.0, seed=seed, pairs=True, conversion="curvature",
               atmosphere=True, sort_interval=3, lines=lines)
    cfg.update(kw)
    return cfg


def _state(sim):
    """Every line's particles sorted by id, E, counts and counters."""
    out = []
    for li in range(sim.n_lines):
        parts = []
        for s in range(4):
            p = sim.get_particles(li, s)
            o = np.argsort(p["id"])
            parts.append({k: v[o] for k, v in p.items()})
        m = sim.moments(li)
        out.append(dict(parts=parts, E=sim.get_field(li), count=m["count"], counters=m["counters"], step=m["step"]))
    return out


def _assert_same(a, b):
    for la, lb in zip(a, b):
        assert la["step"] == lb["step"]
        assert la["count"] == lb["count"]
        assert la["counters"] == lb["counters"]
        assert np.array_equal(la["E"], lb["E"])
        for pa, pb in zip(la["parts"], lb["parts"]):
            for k in pa:
                assert np.array_equal(pa[k], pb[k]), k


@pytest.mark.parametrize("emission", ["perpendicular", "dipole"])
def test_ragged_lines_step_parity(emission):
    cfg = _ragged(emission=emission)
    ocfg = parity.oracle_config(cfg)
    sim = Pic1D(cfg)
    _print("ragged lines", emission, [(l["r_eq"], l["n_cells"], l["ppc_init"]) for l in cfg["lines"]])
    for k in range(3):
        before = parity.snapshot(sim)
        sim.step(1)
        after = parity.snapshot(sim)
        rep, _ = parity.compare_step(ocfg, before, after)
        _print(f"  step {k}: {rep}")
        assert rep["excused"] <= max(3, 1e-3 * rep["compared"])
        sim.step(2)
    for li in range(sim.n_lines):
        assert sim.moments(li)["gauss_residual"] <= 1e-6


def test_graph_replay_equals_eager_stepping():
    cfg = _ragged(seed=5)
    eager = Pic1D(cfg)
    graph = Pic1D(cfg)
    graph.set_graph(6)               # 6 steps per graph: two sorts (interval 3) per replay
    done = 0
    # calls that start off the graph boundary, span several replays and end inside one;
    # eager moments, particle reads and synchronisations between the replays
    for n in (4, 7, 12, 1, 13):
        eager.step(n)
        graph.step(n)
        done += n
        _print("steps", done)
        _assert_same(_state(eager), _state(graph))


def test_graph_replay_without_sorting():
    cfg = _ragged(seed=6, sort_interval=0, pairs=False)
    eager = Pic1D(cfg)
    graph = Pic1D(cfg)
    graph.set_graph(5)
    for n in (5, 10, 3):
        eager.step(n)
        graph.step(n)
        _assert_same(_state(eager), _state(graph))


def test_autotune_changes_speed_not_results():
    cfg = _ragged(seed=7)
    ref = Pic1D(cfg)
    tuned = Pic1D(cfg)
    out = tuned.autotune(trial_steps=4)
    _print("autotune", out)
    assert out["n_trials"] >= 3
    assert out["push_blocks_per_cu"] in (1, 2, 3, 4, 6, 8)
    assert out["push_ppt"] in (4, 8, 16) and out["deposit_window"] in (32, 64)
    assert out["sort_granularity"] in (8, 16, 32)
    assert out["ms_per_step_after"] <= out["ms_per_step_before"]
    steps = tuned.moments(0)["step"]
    ref.step(steps)
    _assert_same(_state(ref), _state(tuned))
    tuned.set_graph(out["sort_interval"])
    tuned.step(2 * out["sort_interval"] + 1)
    ref.step(2 * out["sort_interval"] + 1)
    _assert_same(_state(ref), _state(tuned))


def test_many_lines_conserve_charge_per_line():
    """64 lines of the batched workload's shape (scaled down): Gauss per line after graph replays."""
    cfg = workloads.cfg3(n_lines=64, seed=1)
    for ln in cfg["lines"]:
        ln["n_cells"] = max(256, ln["n_cells"] // 16)
        ln["ppc_init"] = max(4, ln["ppc_init"] // 8)
        ln["capacity"] = [ln["n_cells"] * ln["ppc_init"] * 2, ln["n_cells"] * ln["ppc_init"] * 2, 0, 0]
    cfg["lines"] = [dict(l, init="hot", init_gamma_max=1e3) for l in cfg["lines"]]
    cfg["ppc0"] = 16.0
    cfg["sort_interval"] = 10
    cfg["pairs"] = False          # a hot plasma on these lines cascades past any fixed capacity
    sim = Pic1D(cfg)
    sim.set_graph(20)
    sim.step(45)
    worst = 0.0
    for li in range(sim.n_lines):
        m = sim.moments(li)
        worst = max(worst, m["gauss_residual"])
        assert m["step"] == 45
    _print("64 lines: worst Gauss residual", worst)
    assert worst <= 1e-6


def _line_snapshot(sim, li):
    m = sim.moments(li)
    return dict(lines=[dict(parts=[sim.get_particles(li, s) for s in range(4)], E=sim.get_field(li))],
                step=m["step"]), m


def test_cfg3_full_size_sampled_lines_and_ledger():
    """The 256-line batched workload at full size (about 2.3e6 cells and 6.6e8
    particles) in the autotuned launch shape, replayed from 100-step HIP graphs as in
    the timed benchmark.  After 100 replayed steps, one step is compared on the
    shortest, the median and the longest line, each on a sample (every particle of a
    line with at most 40,000 per species, else 40,000 e- and 40,000 e+, and the pair
    members they can make) against a one-line oracle configuration: a line's step
    does not depend on its place in the batch (event and pair draws are keyed by
    step and particle id).  Every line is checked through Gauss's law and its
    particle-count ledger."""
    cfg = workloads.cfg3()
    sim = Pic1D(cfg)
    tune = sim.autotune(trial_steps=5)
    _print("cfg3 autotune", tune)
    sim.set_graph(100)
    sim.step(100)
    n = sim.n_lines
    cells = np.array([l["n_cells"] for l in cfg["lines"]])
    order = np.argsort(cells, kind="stable")
    pick = [int(order[0]), int(order[n // 2]), int(order[-1])]
    m0 = [sim.moments(li) for li in range(n)]
    before = {li: _line_snapshot(sim, li)[0] for li in pick}
    sim.step(1)
    after = {}
    worst = 0.0
    for li in range(n):
        if li in pick:
            after[li], m1 = _line_snapshot(sim, li)
        else:
            m1 = sim.moments(li)
        d = {k: m1["counters"][k] - m0[li]["counters"][k] for k in m1["counters"]}
        grown = 2 * (d["pairs_created"] - d["annihilated"]) - d["absorbed"]
        assert sum(m1["count"]) - sum(m0[li]["count"]) == grown, (li, d)
        assert m1["step"] == m0[li]["step"] + 1
        worst = max(worst, m1["gauss_residual"])
    _print("cfg3 worst Gauss residual", worst)
    assert worst <= 1e-6
    for li in pick:
        ocfg = parity.oracle_config(dict(cfg, lines=[cfg["lines"][li]]))
        rep, _ = parity.sampled_compare(ocfg, before[li], after[li], 40000, np.random.default_rng(li))
        _print("cfg3 line", li, cfg["lines"][li]["n_cells"], "cells:", rep)
        assert rep["compared"] > 2000
        assert rep["excused"] <= max(3, 1e-3 * rep["compared"])


SHAPES = {"exact": [(4, 32), (8, 32), (16, 32), (8, 64)], "table": [(4, 128), (8, 128), (16, 128), (8, 64)]}


@pytest.mark.parametrize("rics", ["exact", "table"])
def test_every_push_shape_gives_the_same_results(rics):
    """Every tile shape the autotuner can pick (4, 8 or 16 particles per lane, both
    deposit windows, several block counts), set at the start and changed between
    steps (which re-plans the tiles of the live particles), gives the same
    particles, field and counters as the default shape, bit for bit."""
    cfg = _ragged(seed=11, rics=rics)
    ref = Pic1D(cfg)
    ref.step(7)
    want = _state(ref)
    ref.close()
    shapes = SHAPES[rics]
    for k, (ppt, ww) in enumerate(shapes):
        sim = Pic1D(cfg)
        sim.set_push_shape(1 + k, ppt, ww)
        sim.step(3)
        nxt = shapes[(k + 1) % len(shapes)]
        sim.set_push_shape(2, nxt[0], nxt[1])
        sim.step(4)
        _print(rics, "shape", (ppt, ww), "then", nxt)
        _assert_same(want, _state(sim))
        sim.close()
    sim = Pic1D(cfg)
    with pytest.raises(RuntimeError):
        sim.set_push_shape(4, 8, 48)
    sim.close()
