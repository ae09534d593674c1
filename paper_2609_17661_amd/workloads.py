"""Synthetic workloads (plain parameter dictionaries; no arithmetic of the method).

Each workload is a config dict accepted by the library binding; tests also hand
the same dict to the oracle.  The shapes follow the paper's setup (Sec. 3 and
Appendix B: one dipole line, CFL 0.5, 48 cells per skin depth, B*/B_QED = 10)
at the sizes of the benchmark configurations:

* CFG1      one line, R_max = 4, 512 cells, 64 e-/e+ per cell each (65,536),
            cold start, TABLE 256 x 512 at kT = 0.5 keV, pairs off, 1000 steps.
* CFG1_HOT  CFG1 with gamma log-uniform in [1, 1e4] and pairs on (exercises
            the drag branches, the stochastic events and pair injection).
* CFG2      one line, R_max = 30, 65,536 cells, 200 e-/e+ per cell each,
            surface atmosphere with ions at m_i/m_e = 100, pairs on with
            curvature conversion, capacity for 1e8 particles, 20,000 steps.
* CFG4      the surrogate comparison: the R_max = 4 line of the network's
            training geometry at the particle count of CFG2 (65,536 cells,
            200 e-/e+ per cell each), gamma log-uniform in [1, 1e4] so that
            the drag and the scattering events are active, pairs on up to
            n_max = 3 n0 per cell (at this resolution almost every lepton with
            gamma >~ 1e3 in the b >= 0.1 region scatters each step, and the
            cascade is held by n_max).  Sorted every 5 steps: pair creation
            appends unsorted particles every step (the autotuner's choice).
* cfg3()    the batched path: 256 lines with R_max log-uniform in [2, 100]
            (seeded draw), 1,024 to 32,768 cells per line (a power law in
            R_max through those endpoints, rounded to multiples of 256),
            32-256 e-/e+ per cell per line (uniform integers), cold start,
            TABLE RICS, pairs on with curvature conversion.
* cfg5()    the combined cascade run: 64 lines with R_max log-uniform in
            [10, 100], 32,768 cells each, a hot pair seed of 64 e-/e+ per cell
            cascading up to n_max = 6 n0 (n0 = 32 per cell: about 4e8
            particles over all lines), the surface atmosphere with ions at
            m_i/m_e = 100, pairs on with curvature conversion, TABLE RICS.
"""
import numpy as np

CFG1 = dict(
    rics="table", table_nlg=256, table_ns=512, kT_keV=0.5, j_twist=0.5, ppc0=64.0, pairs=False,
    atmosphere=False, seed=0,
    lines=[dict(r_eq=4.0, n_cells=512, ppc_init=64, init="cold")],
)
CFG1_STEPS = 1000

CFG1_HOT = dict(CFG1, pairs=True, conversion="immediate",
                lines=[dict(r_eq=4.0, n_cells=512, ppc_init=64, init="hot", init_gamma_max=1.0e4,
                            capacity=[400000, 400000, 0, 0])])

CFG2 = dict(
    rics="table", table_nlg=256, table_ns=512, kT_keV=0.5, j_twist=0.5, ppc0=200.0, pairs=True,
    conversion="curvature", atmosphere=True, mass_ratio=100.0, seed=0, sort_interval=50,
    lines=[dict(r_eq=30.0, n_cells=65536, ppc_init=200, init="cold",
                capacity=[46_000_000, 46_000_000, 4_000_000, 4_000_000])],
)
CFG2_STEPS = 20000

CFG4 = dict(
    rics="table", table_nlg=256, table_ns=512, kT_keV=0.5, j_twist=0.5, ppc0=200.0, pairs=True,
    conversion="immediate", nmax_over_n0=3.0, seed=0, sort_interval=5,
    lines=[dict(r_eq=4.0, n_cells=65536, ppc_init=200, init="hot", init_gamma_max=1.0e4,
                capacity=[40_000_000, 40_000_000, 0, 0])],
)


def cfg3(n_lines=256, seed=0, rics="table", headroom=1.05):
    """The batched many-line workload (about 2.3e6 cells and 6.6e8 particles at 256 lines)."""
    rng = np.random.default_rng(seed)
    R = 2.0 * 50.0 ** rng.random(n_lines)
    expo = np.log(32.0) / np.log(50.0)                   # 1,024 cells at R_max = 2, 32,768 at 100
    cells = np.clip(np.round(1024.0 * (R / 2.0) ** expo / 256.0) * 256.0, 1024, 32768).astype(int)
    ppc = rng.integers(32, 257, n_lines)
    lines = []
    for r, n, p in zip(R, cells, ppc):
        cap = int(headroom * p * n) + 4096
        lines.append(dict(r_eq=float(r), n_cells=int(n), ppc_init=int(p), init="cold", capacity=[cap, cap, 0, 0]))
    return dict(rics=rics, table_nlg=256, table_ns=512, kT_keV=0.5, j_twist=0.5, ppc0=float(np.mean(ppc)),
                pairs=True, conversion="curvature", seed=seed, sort_interval=50, lines=lines)


def cfg5(n_lines=64, seed=0, rics="table", n_cells=32768, ppc=84, nmax_over_n0=11.0, ppc0=32.0):
    """The combined cascade run: 64 lines with R_max log-uniform in [10, 100], 32,768
    cells each, a hot pair seed (gamma log-uniform to 1e4) cascading up to
    n_max = nmax_over_n0 * ppc0 particles per cell, the surface atmosphere with ions
    at m_i/m_e = 100, pairs with curvature conversion.  The resident count levels
    off where pair creation and annihilation over n_max balance; with a seed of 84
    pairs per cell and n_max = 11 n0 that is about 4e8 particles over 64 lines."""
    rng = np.random.default_rng(seed)
    R = 10.0 * 10.0 ** rng.random(n_lines)
    nmax = nmax_over_n0 * ppc0
    cap_pair = int(0.6 * nmax * n_cells) + ppc * n_cells + 4096
    cap_atm = 16 * n_cells
    lines = [dict(r_eq=float(r), n_cells=n_cells, ppc_init=ppc, init="hot", init_gamma_max=1.0e4,
                  capacity=[cap_pair, cap_pair, cap_atm, cap_atm]) for r in R]
    return dict(rics=rics, table_nlg=256, table_ns=512, kT_keV=0.5, j_twist=0.5, ppc0=ppc0, pairs=True,
                conversion="curvature", nmax_over_n0=nmax_over_n0, atmosphere=True, mass_ratio=100.0,
                seed=seed, sort_interval=50, lines=lines)


def small(r_eq=4.0, n_cells=96, ppc=16, init="hot", **kw):
    """A small line for per-step parity tests (the oracle steps it in well under a second)."""
    line = dict(r_eq=r_eq, n_cells=n_cells, ppc_init=ppc, init=init, init_gamma_max=kw.pop("gamma_max", 1.0e3),
                capacity=kw.pop("capacity", [400_000, 400_000, 200_000, 200_000]))
    cfg = dict(rics="exact", kT_keV=0.5, j_twist=0.5, ppc0=float(ppc), seed=kw.pop("seed", 7), lines=[line])
    cfg.update(kw)
    return cfg
