"""Long-run statistics of the HIP path against the oracle.

Float32 and float64 trajectories separate over time, so long runs are compared
statistically:
  * time-averaged profiles of the species densities, the current and E on the
    R_max = 4 line (512 cells, 64 e-/e+ per cell) over steps 200-999, within
    2% in the relative L2 norm ||<f>_gpu - <f>_oracle||_2 / max(||<f>_oracle||_2,
    floor), with floors sqrt(N) n0 for the densities, |j_psi| sqrt(N) for the
    current and 4 pi Q ppc0 d0 sqrt(N) for E (one n0 of charge over a skin depth);
  * the same averages on the hot cascading line over steps 100-399 (drag,
    events, pairs, annihilation), and its pairs created per cell per step
    against the oracle's run-to-run spread;
  * event, pair and annihilation yields of the hot line within 3 sigma
    (Poisson), over several seeds.
"""
import math

import numpy as np
import pytest

from oracle import pic
from paper_2609_17661_amd import Pic1D, workloads

from . import parity

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _rel_l2(a, b, floor):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor))


def test_time_averaged_profiles_match_oracle():
    steps, avg_start = 1000, 200
    cfg = dict(workloads.CFG1, avg_start_step=avg_start)
    sim = Pic1D(cfg)
    sim.step(steps)
    m = sim.moments(0, average=True)
    assert m["avg_steps"] == steps - avg_start

    ocfg = parity.oracle_config(cfg)
    st = pic.init_state(ocfg)
    ln = st.lines[0]
    n = ln.n
    ppc0 = ocfg["ppc0"]
    sums = dict(n=np.zeros((4, n)), j=np.zeros(n), E=np.zeros(n))
    for k in range(steps):
        pic.step(st)
        if k >= avg_start:
            for s in range(4):
                x = st.parts[0][s]["x"]
                if x.size:
                    sums["n"][s] += np.bincount(np.floor(x).astype(np.int64), minlength=n)
            sums["j"] += st.j_last[0]
            sums["E"] += st.E[0]
        if k % 200 == 0:
            _print("oracle step", k)
    navg = steps - avg_start
    n_o = sums["n"] / navg / ppc0
    j_o = sums["j"] / navg / (ppc0 * ln.Q * ln.C)
    E_o = sums["E"] / navg
    rn = [_rel_l2(m["n"][s], n_o[s], math.sqrt(n)) for s in (0, 1)]
    rj = _rel_l2(m["j"], j_o, abs(ocfg["j_twist"]) * math.sqrt(n))
    rE = _rel_l2(m["E"], E_o, 4 * math.pi * ln.Q * ppc0 * ocfg["d0_cells"] * math.sqrt(n))
    _print("relative L2: n_e", rn[0], "n_p", rn[1], "j", rj, "E", rE)
    assert max(rn) <= 0.02 and rj <= 0.02 and rE <= 0.02


def _oracle_averages(cfg, steps, avg_start):
    """Time averages of the oracle over steps avg_start..steps-1: species densities
    (n0), current (n0 e c), E and pairs made per cell per step; and its counters."""
    ocfg = parity.oracle_config(cfg)
    st = pic.init_state(ocfg)
    ln = st.lines[0]
    n = ln.n
    ppc0 = ocfg["ppc0"]
    sums = dict(n=np.zeros((4, n)), j=np.zeros(n), E=np.zeros(n), p=np.zeros(n))
    for k in range(steps):
        p_before = st.pair_rate[0].copy()
        pic.step(st)
        if k >= avg_start:
            for s in range(4):
                x = st.parts[0][s]["x"]
                if x.size:
                    sums["n"][s] += np.bincount(np.floor(x).astype(np.int64), minlength=n)
            sums["j"] += st.j_last[0]
            sums["E"] += st.E[0]
            sums["p"] += st.pair_rate[0] - p_before
        if k % 100 == 0:
            _print("oracle step", k, "seed", ocfg["seed"])
    navg = steps - avg_start
    return dict(n=sums["n"] / navg / ppc0, j=sums["j"] / navg / (ppc0 * ln.Q * ln.C), E=sums["E"] / navg,
                p=sums["p"] / navg, counters=st.counters[0], ln=ln, ocfg=ocfg)


def test_time_averaged_profiles_of_a_cascading_line_match_oracle():
    """The hot R_max = 4 line (gamma log-uniform to 1e4): RICS drag on both branches,
    scattering events, immediate pair creation capped by n_max = 3 n0 and pair
    annihilation act throughout.  Time averages over steps 100-399 of the species
    densities, the current and E against the oracle's within 2% relative L2 with the
    floors above.  The pairs created per cell per step (Sec. 4.1, Figs. 2-3) come in
    bursts (one energetic lepton converts photons in one cell over several steps), a
    few hundred per cell over the window: their profile is as close to the oracle's
    as the oracle's own run from another seed is (the GPU shares the oracle's draws;
    the bar is the oracle's run-to-run spread).  The yields of the whole run agree
    within 3 sigma."""
    steps, avg_start = 400, 100
    cfg = dict(workloads.CFG1_HOT, nmax_over_n0=3.0, avg_start_step=avg_start)
    sim = Pic1D(cfg)
    sim.step(steps)
    m = sim.moments(0, average=True)
    assert m["avg_steps"] == steps - avg_start
    c_gpu = m["counters"]
    o = _oracle_averages(cfg, steps, avg_start)
    o1 = _oracle_averages(dict(cfg, seed=1), steps, avg_start)
    ln, ocfg = o["ln"], o["ocfg"]
    n = ln.n
    c_o = o["counters"]
    _print("counters gpu", {k: c_gpu[k] for k in ("events", "pairs_created", "annihilated", "limited", "newton")},
           "oracle", {k: c_o[k] for k in ("events", "pairs_created", "annihilated", "limited")})
    assert c_o["pairs_created"] > 1e5 and c_o["annihilated"] > 1e5 and c_o["limited"] > 1e5
    assert o["p"].sum() > 10.0          # pairs still made in the averaging window
    rn = [_rel_l2(m["n"][s], o["n"][s], math.sqrt(n)) for s in (0, 1)]
    rj = _rel_l2(m["j"], o["j"], abs(ocfg["j_twist"]) * math.sqrt(n))
    rE = _rel_l2(m["E"], o["E"], 4 * math.pi * ln.Q * ocfg["ppc0"] * ocfg["d0_cells"] * math.sqrt(n))
    _print("relative L2: n_e", rn[0], "n_p", rn[1], "j", rj, "E", rE)
    assert max(rn) <= 0.02 and rj <= 0.02 and rE <= 0.02
    rp_gpu = _rel_l2(m["pair_rate"], o["p"], 0.0)
    rp_seed = _rel_l2(o1["p"], o["p"], 0.0)
    _print("pair rate per cell: relative L2 gpu-oracle", rp_gpu, "; oracle seed 1 - seed 0", rp_seed)
    assert rp_gpu <= rp_seed
    # the yields of the whole run
    for key in ("events", "pairs_created", "annihilated"):
        assert abs(c_gpu[key] - c_o[key]) <= 3.0 * math.sqrt(c_o[key]), key


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pair_and_event_yields_over_seeds_within_three_sigma(seed):
    """Event and pair yields of the hot line (n_max = 3 n0) over 30 steps, per seed."""
    cfg = dict(workloads.CFG1_HOT, nmax_over_n0=3.0, seed=seed)
    sim = Pic1D(cfg)
    ocfg = parity.oracle_config(cfg)
    st = pic.init_state(ocfg)
    steps = 30
    sim.step(steps)
    for _ in range(steps):
        pic.step(st)
    g = sim.moments(0)["counters"]
    o = st.counters[0]
    _print("seed", seed, "gpu", {k: g[k] for k in ("events", "pairs_created", "annihilated")},
           "oracle", {k: o[k] for k in ("events", "pairs_created", "annihilated")})
    for key in ("events", "pairs_created", "annihilated"):
        assert o[key] > 100
        assert abs(g[key] - o[key]) <= 3.0 * math.sqrt(o[key]), key


def test_pair_yield_matches_oracle_within_three_sigma():
    # the hot line cascades (every lepton with gamma >~ 10 scatters each step at this
    # resolution); n_max = 3 n0 per cell caps it at ~1e5 particles
    cfg = dict(workloads.CFG1_HOT, nmax_over_n0=3.0)
    sim = Pic1D(cfg)
    ocfg = parity.oracle_config(cfg)
    st = pic.init_state(ocfg)
    steps = 8
    sim.step(steps)
    for _ in range(steps):
        pic.step(st)
    g = sim.moments(0)["counters"]["pairs_created"]
    o = st.counters[0]["pairs_created"]
    e_g = sim.moments(0)["counters"]["events"]
    e_o = st.counters[0]["events"]
    _print("pairs gpu", g, "oracle", o, "events gpu", e_g, "oracle", e_o)
    assert o > 100
    assert abs(g - o) <= 3.0 * math.sqrt(o)
    assert abs(e_g - e_o) <= 3.0 * math.sqrt(e_o)


def test_cold_two_stream_growth_rate_on_the_gpu():
    """Linear theory, not the oracle: the symmetric cold two-stream instability of e+ at
    +v0 and e- at -v0 (carrying the twist current exactly) grows at w_b/(2 gamma0^(3/2))
    near k v0 = (sqrt 3/2) w_b/gamma0^(3/2)."""
    beta, ppc, n = 0.2, 64, 1024
    cfg = dict(rics="off", ppc0=float(ppc), j_twist=2 * beta, seed=3,
               lines=[dict(r_eq=4.0, n_cells=n, ppc_init=ppc, init="stream", init_beta=beta)])
    sim = Pic1D(cfg)
    C, d0 = 0.5, 48.0
    wb = C / d0
    g0 = 1 / math.sqrt(1 - beta ** 2)
    v0 = beta * C
    gth = wb / (2 * g0 ** 1.5)
    kth = math.sqrt(3) / 2 * wb / g0 ** 1.5 / v0
    win = np.hanning(n - 400)
    A, T = [], []
    for i in range(0, 1001, 20):
        if i >= 400:
            A.append(np.abs(np.fft.rfft(sim.get_field(0)[200:n - 200] * win)))
            T.append(i)
        sim.step(20)
    A, T = np.array(A), np.array(T)
    k = 2 * np.pi * np.fft.rfftfreq(n - 400)
    rates = np.polyfit(T, np.log(A + 1e-300), 1)[0]
    band = (k > 0.5 * kth) & (k < 1.5 * kth)
    _print("two-stream growth", rates[band].max(), "theory", gth)
    assert rates[band].max() == pytest.approx(gth, rel=0.10)
