"""Configuration dictionaries of the pic1d library (names follow the paper's notation).

A config is a plain dict; `complete_config` fills in the defaults below.  Lines
are dicts with r_eq (R_max/R*), n_cells, ppc_init, init ("cold", "hot",
"stream", "empty"), init_gamma_max, init_beta and optional capacity[4].
"""
import copy

RICS = {"off": 0, "exact": 1, "table": 2, "mlp": 3}
CONVERSION = {"immediate": 0, "curvature": 1}
PHOTON_FIELD = {"radial": 0, "disk": 1}
EMISSION = {"perpendicular": 0, "isotropic": 1, "dipole": 2}
INIT = {"cold": 0, "hot": 1, "stream": 2, "empty": 3}
SPECIES = {"e_pair": 0, "p_pair": 1, "e_atm": 2, "ion": 3}

DEFAULTS = dict(
    b_pole=10.0,        # B*/B_QED (Sec. 3)
    cfl=0.5,            # c0/c (Sec. 3)
    d0_cells=48.0,      # cells per skin depth at n0 (Sec. 3)
    ppc0=64.0,          # macro-particles per cell per species at n0
    j_twist=0.5,        # j_psi/(n0 e c)
    kT_keV=0.5,
    eta_min=1.0e3,      # tau_min w_p = eta_min (n_psi/n0)^(1/2) (Sec. 3)
    b_thr=0.1,          # stochastic regime above (Sec. 3)
    mass_ratio=100.0,
    rics="table",
    table_nlg=256,
    table_ns=512,
    pairs=False,
    conversion="immediate",
    nmax_over_n0=0.0,   # 0: (d0_cells)^2
    atmosphere=False,
    atm_a0=0.0,         # 0: 18 |j_twist|
    atm_h_cells=0.0,    # 0: 3 d0 / a0^(1/2)
    atm_T=0.01,         # T/m_e c^2 (Sec. 3)
    atm_cut=0.01,
    gravity=True,
    frozen_field=False,
    annihilation=True,  # e-/e+ pairs annihilate in cells over n_max (Sec. 3)
    photon_field="radial",  # "radial": the radial beam (Sec. 2.2); "disk": the finite stellar disk (Sec. 5)
    emission="perpendicular",   # rest-frame photon direction of an event (Appendix A.2-A.3):
                                # "perpendicular" (Eq. perpemit), "isotropic", "dipole"
    seed=0,
    sort_interval=0,
    avg_start_step=-1,
    lines=None,
    mlp_params=None,    # RICS "mlp": the network's 50,563 parameters (float32 values)
    mlp_norm=None,      # RICS "mlp": output mean[3] and std[3]
    mlp_fallback_tol=0.0,   # RICS "mlp": > 0, lines where the network's error estimate exceeds it use a table
)


def complete_config(cfg):
    out = copy.deepcopy(DEFAULTS)
    for k, v in cfg.items():
        if k not in DEFAULTS:
            raise KeyError(f"unknown config key {k!r}")
        out[k] = copy.deepcopy(v)
    if not out["lines"]:
        raise ValueError("config needs at least one line")
    return out
