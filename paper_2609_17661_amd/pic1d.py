"""Python binding of libpic1d.so (argument marshalling only).

Every step of the PIC path runs in the HIP kernels of the library; this module
builds the C config struct, allocates the device workspace as a torch uint8
tensor, passes torch's current HIP stream, and copies results in and out.  It
raises if the library has not been built: there is no fallback.
"""
import ctypes
import os

import numpy as np

from .config import CONVERSION, EMISSION, INIT, PHOTON_FIELD, RICS, SPECIES, complete_config

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpic1d.so")
_lib = None

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ECAPACITY", -4: "EDEVICE", -5: "ENONFINITE",
          -6: "ESTATE"}


class Pic1dError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pic1d {STATUS.get(code, code)}: {msg}")
        self.code = code


class CLine(ctypes.Structure):
    _fields_ = [("r_eq", ctypes.c_double), ("n_cells", ctypes.c_int32), ("ppc_init", ctypes.c_int32),
                ("init_mode", ctypes.c_int32), ("pad0", ctypes.c_int32), ("init_gamma_max", ctypes.c_double),
                ("init_beta", ctypes.c_double), ("capacity", ctypes.c_int64 * 4)]


class CConfig(ctypes.Structure):
    _fields_ = [("n_lines", ctypes.c_int32), ("emission", ctypes.c_int32), ("lines", ctypes.POINTER(CLine)),
                ("b_pole", ctypes.c_double), ("cfl", ctypes.c_double), ("d0_cells", ctypes.c_double),
                ("ppc0", ctypes.c_double), ("j_twist", ctypes.c_double), ("kT_keV", ctypes.c_double),
                ("eta_min", ctypes.c_double), ("b_thr", ctypes.c_double), ("mass_ratio", ctypes.c_double),
                ("rics_backend", ctypes.c_int32), ("table_nlg", ctypes.c_int32), ("table_ns", ctypes.c_int32),
                ("pairs", ctypes.c_int32), ("conversion", ctypes.c_int32), ("atmosphere", ctypes.c_int32),
                ("gravity", ctypes.c_int32), ("frozen_field", ctypes.c_int32),
                ("annihilation", ctypes.c_int32), ("photon_field", ctypes.c_int32),
                ("nmax_over_n0", ctypes.c_double), ("atm_a0", ctypes.c_double), ("atm_h_cells", ctypes.c_double),
                ("atm_T", ctypes.c_double), ("atm_cut", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("sort_interval", ctypes.c_int32), ("avg_start_step", ctypes.c_int32),
                ("mlp_weights", ctypes.c_void_p), ("mlp_norm", ctypes.c_void_p),
                ("mlp_fallback_tol", ctypes.c_double), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p)]


class CMoments(ctypes.Structure):
    _fields_ = [("n_cell", ctypes.POINTER(ctypes.c_double) * 4), ("j", ctypes.POINTER(ctypes.c_double)),
                ("E", ctypes.POINTER(ctypes.c_double)), ("pair_rate", ctypes.POINTER(ctypes.c_double)),
                ("gauss_residual", ctypes.c_double), ("v_circuit", ctypes.c_double),
                ("energy_kinetic", ctypes.c_double), ("energy_field", ctypes.c_double),
                ("count", ctypes.c_int64 * 4), ("counters", ctypes.c_int64 * 16), ("step", ctypes.c_int64),
                ("avg_steps", ctypes.c_int64)]


COUNTER_NAMES = ("events", "pairs_created", "photons_escaped", "absorbed", "psc_clipped", "limited",
                 "newton", "atm_injected", "pushed", "draws", "mlp_evals", "annihilated", "pushed_ions",
                 "mlp_needed")


class CProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_int64 * 8)]


KERNELS = ("push", "append", "field", "plan", "sort", "annihilate")


class CTuneOut(ctypes.Structure):
    _fields_ = [("push_blocks_per_cu", ctypes.c_int32), ("xcd_walk", ctypes.c_int32), ("sort_interval", ctypes.c_int32),
                ("n_trials", ctypes.c_int32), ("ms_per_step_before", ctypes.c_double),
                ("ms_per_step_after", ctypes.c_double), ("push_ppt", ctypes.c_int32),
                ("deposit_window", ctypes.c_int32), ("sort_granularity", ctypes.c_int32)]


class CMlpTrainConfig(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_samples", ctypes.c_int64), ("batch", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("lr", ctypes.c_double), ("lr_final", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("init_params", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p)]


class CMlpTrainResult(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("norm", ctypes.c_void_p), ("loss", ctypes.c_void_p),
                ("n_loss", ctypes.c_int32), ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("seconds", ctypes.c_double)]

class CTpConfig(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_double), ("kT_keV", ctypes.c_double), ("b_pole", ctypes.c_double),
                ("b_pp", ctypes.c_double), ("t_max", ctypes.c_double), ("dt_max", ctypes.c_double),
                ("tol", ctypes.c_double), ("tol_stiff", ctypes.c_double), ("max_steps", ctypes.c_int64)]


class CTpResult(ctypes.Structure):
    _fields_ = [("gamma_min", ctypes.c_double), ("s_first", ctypes.c_double), ("s_b", ctypes.c_double),
                ("l_pp", ctypes.c_double), ("L", ctypes.c_double), ("crossed", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("steps", ctypes.c_int64)]


P = ctypes.c_void_p
_SIGS = {
    "pic1d_workspace_size": (ctypes.c_int, [ctypes.POINTER(CConfig), ctypes.POINTER(ctypes.c_size_t)]),
    "pic1d_init": (ctypes.c_int, [ctypes.POINTER(CConfig), ctypes.POINTER(P)]),
    "pic1d_step": (ctypes.c_int, [P, ctypes.c_int32]),
    "pic1d_moments": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(CMoments)]),
    "pic1d_free": (None, [P]),
    "pic1d_last_error": (ctypes.c_char_p, [P]),
    "pic1d_get_particles": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64), P, P, P, P]),
    "pic1d_set_particles": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P, P, P, P]),
    "pic1d_get_field": (ctypes.c_int, [P, ctypes.c_int32, P]),
    "pic1d_set_field": (ctypes.c_int, [P, ctypes.c_int32, P]),
    "pic1d_set_step": (ctypes.c_int, [P, ctypes.c_int64]),
    "pic1d_rics_eval": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int64, P, P, P, P, P]),
    "pic1d_rics_line_info": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "pic1d_profile": (ctypes.c_int, [P, ctypes.c_int32]),
    "pic1d_profile_read": (ctypes.c_int, [P, ctypes.POINTER(CProfile)]),
    "pic1d_set_graph": (ctypes.c_int, [P, ctypes.c_int32]),
    "pic1d_autotune": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(CTuneOut)]),
    "pic1d_set_push_shape": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "pic1d_set_sort_granularity": (ctypes.c_int, [P, ctypes.c_int32]),
    "pic1d_testparticle_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "pic1d_testparticle_sweep": (ctypes.c_int, [ctypes.POINTER(CTpConfig), ctypes.c_int32, P, P, P, ctypes.c_size_t,
                                                P]),
    "pic1d_mlp_param_count": (ctypes.c_int, []),
    "pic1d_mlp_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "pic1d_mlp_samples": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, P, P, P, ctypes.c_size_t,
                                         P]),
    "pic1d_mlp_forward": (ctypes.c_int, [P, ctypes.c_int64, P, P, P, ctypes.c_size_t, P]),
    "pic1d_mlp_loss_grad": (ctypes.c_int, [P, ctypes.c_int64, P, P, P, ctypes.POINTER(ctypes.c_double), P,
                                           ctypes.c_size_t, P]),
    "pic1d_mlp_loss_grad_static": (ctypes.c_int, [P, ctypes.c_int64, P, P, P, ctypes.POINTER(ctypes.c_double), P]),
    "pic1d_mlp_adam": (ctypes.c_int, [P, P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, P]),
    "pic1d_mlp_train": (ctypes.c_int, [ctypes.POINTER(CMlpTrainConfig), ctypes.POINTER(CMlpTrainResult)]),
}

EXPORTED = tuple(_SIGS)


def lib_path():
    return _LIB_PATH


def load():
    """Load libpic1d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_2609_17661_amd.build.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def make_cconfig(cfg):
    """C config struct (and the line array it points to) from a complete config dict."""
    lines = cfg["lines"]
    arr = (CLine * len(lines))()
    for i, ln in enumerate(lines):
        arr[i].r_eq = float(ln["r_eq"])
        arr[i].n_cells = int(ln["n_cells"])
        arr[i].ppc_init = int(ln.get("ppc_init", 0))
        arr[i].init_mode = INIT[ln.get("init", "cold")]
        arr[i].init_gamma_max = float(ln.get("init_gamma_max", 1.0e4))
        arr[i].init_beta = float(ln.get("init_beta", 0.0))
        cap = ln.get("capacity", [0, 0, 0, 0])
        for s in range(4):
            arr[i].capacity[s] = int(cap[s])
    c = CConfig()
    c.n_lines = len(lines)
    c.lines = arr
    for k in ("b_pole", "cfl", "d0_cells", "ppc0", "j_twist", "kT_keV", "eta_min", "b_thr", "mass_ratio",
              "nmax_over_n0", "atm_a0", "atm_h_cells", "atm_T", "atm_cut"):
        setattr(c, k, float(cfg[k]))
    c.rics_backend = RICS[cfg["rics"]]
    c.table_nlg = int(cfg["table_nlg"])
    c.table_ns = int(cfg["table_ns"])
    c.pairs = int(bool(cfg["pairs"]))
    c.conversion = CONVERSION[cfg["conversion"]]
    c.atmosphere = int(bool(cfg["atmosphere"]))
    c.gravity = int(bool(cfg["gravity"]))
    c.frozen_field = int(bool(cfg["frozen_field"]))
    c.annihilation = int(bool(cfg["annihilation"]))
    c.photon_field = PHOTON_FIELD[cfg["photon_field"]]
    c.emission = EMISSION[cfg["emission"]]
    c.seed = int(cfg["seed"]) & 0xFFFFFFFFFFFFFFFF
    c.sort_interval = int(cfg["sort_interval"])
    c.mlp_fallback_tol = float(cfg["mlp_fallback_tol"])
    c.avg_start_step = int(cfg["avg_start_step"])
    return c, arr


def workspace_size(cfg):
    lib = load()
    c, keep = make_cconfig(complete_config(cfg))
    n = ctypes.c_size_t(0)
    rc = lib.pic1d_workspace_size(ctypes.byref(c), ctypes.byref(n))
    if rc != 0:
        raise Pic1dError(rc, lib.pic1d_last_error(None).decode())
    return n.value


class Pic1D:
    """One simulation state on the current HIP device (all lines of a config)."""

    def __init__(self, cfg, device="cuda", mlp_weights=None, mlp_norm=None):
        import torch

        self._torch = torch
        self.lib = load()
        self.cfg = complete_config(cfg)
        c, self._lines_keep = make_cconfig(self.cfg)
        n = ctypes.c_size_t(0)
        rc = self.lib.pic1d_workspace_size(ctypes.byref(c), ctypes.byref(n))
        if rc != 0:
            raise Pic1dError(rc, self.lib.pic1d_last_error(None).decode())
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.workspace.device)
        c.workspace = ctypes.c_void_p(self.workspace.data_ptr())
        c.workspace_bytes = n.value
        c.stream = ctypes.c_void_p(self.stream.cuda_stream)
        if mlp_weights is None:
            mlp_weights = self.cfg.get("mlp_params")
        if mlp_norm is None:
            mlp_norm = self.cfg.get("mlp_norm")
        if mlp_weights is not None:
            self._mlp = np.ascontiguousarray(mlp_weights, dtype=np.float32)
            c.mlp_weights = ctypes.c_void_p(self._mlp.ctypes.data)
        if mlp_norm is not None:
            self._mlp_norm = np.ascontiguousarray(mlp_norm, dtype=np.float32).reshape(6)
            c.mlp_norm = ctypes.c_void_p(self._mlp_norm.ctypes.data)
        h = ctypes.c_void_p()
        rc = self.lib.pic1d_init(ctypes.byref(c), ctypes.byref(h))
        if rc != 0:
            raise Pic1dError(rc, self.lib.pic1d_last_error(None).decode())
        self.h = h
        self.n_lines = len(self.cfg["lines"])

    def _check(self, rc):
        if rc != 0:
            raise Pic1dError(rc, self.lib.pic1d_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.pic1d_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(self.lib.pic1d_step(self.h, int(n)))

    def n_cells(self, line=0):
        return int(self.cfg["lines"][line]["n_cells"])

    def moments(self, line=0, average=False, reset=False):
        n = self.n_cells(line)
        out = CMoments()
        arrs = {f"n{s}": np.zeros(n) for s in range(4)}
        arrs.update(j=np.zeros(n), E=np.zeros(n), pair_rate=np.zeros(n))
        for s in range(4):
            out.n_cell[s] = arrs[f"n{s}"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        out.j = arrs["j"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        out.E = arrs["E"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        out.pair_rate = arrs["pair_rate"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        flags = (1 if average else 0) | (2 if reset else 0)
        self._check(self.lib.pic1d_moments(self.h, int(line), flags, ctypes.byref(out)))
        res = dict(n=np.stack([arrs[f"n{s}"] for s in range(4)]), j=arrs["j"], E=arrs["E"],
                   pair_rate=arrs["pair_rate"], gauss_residual=out.gauss_residual, v_circuit=out.v_circuit,
                   energy_kinetic=out.energy_kinetic, energy_field=out.energy_field,
                   count=[int(x) for x in out.count], step=int(out.step), avg_steps=int(out.avg_steps))
        res["counters"] = {k: int(out.counters[i]) for i, k in enumerate(COUNTER_NAMES)}
        return res

    def get_particles(self, line=0, species=0):
        cnt = ctypes.c_int64(0)
        # a zero-capacity call reports the live count (and fails with EINVAL if it is non-zero)
        self.lib.pic1d_get_particles(self.h, line, species, 0, ctypes.byref(cnt), None, None, None, None)
        n = cnt.value
        cell = np.zeros(n, dtype=np.int32)
        off = np.zeros(n, dtype=np.float32)
        u = np.zeros(n, dtype=np.float32)
        pid = np.zeros(n, dtype=np.uint64)
        self._check(self.lib.pic1d_get_particles(self.h, line, species, n, ctypes.byref(cnt), _ptr(cell), _ptr(off),
                                                 _ptr(u), _ptr(pid)))
        return dict(cell=cell, off=off, u=u, id=pid)

    def set_particles(self, line, species, cell, off, u, pid):
        cell = np.ascontiguousarray(cell, dtype=np.int32)
        off = np.ascontiguousarray(off, dtype=np.float32)
        u = np.ascontiguousarray(u, dtype=np.float32)
        pid = np.ascontiguousarray(pid, dtype=np.uint64)
        self._check(self.lib.pic1d_set_particles(self.h, line, species, cell.size, _ptr(cell), _ptr(off), _ptr(u),
                                                 _ptr(pid)))

    def get_field(self, line=0):
        E = np.zeros(self.n_cells(line))
        self._check(self.lib.pic1d_get_field(self.h, line, _ptr(E)))
        return E

    def set_field(self, line, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.n_cells(line)
        self._check(self.lib.pic1d_set_field(self.h, line, _ptr(E)))

    def profile(self, enable=True):
        self._check(self.lib.pic1d_profile(self.h, int(bool(enable))))

    def profile_read(self):
        out = CProfile()
        self._check(self.lib.pic1d_profile_read(self.h, ctypes.byref(out)))
        return {k: dict(ms=out.ms[i], launches=int(out.launches[i])) for i, k in enumerate(KERNELS)}

    def set_step(self, step):
        self._check(self.lib.pic1d_set_step(self.h, int(step)))

    def set_graph(self, steps_per_graph):
        """Replay the step sequence from captured HIP graphs of this many steps (0: eager)."""
        self._check(self.lib.pic1d_set_graph(self.h, int(steps_per_graph)))

    def autotune(self, trial_steps=5):
        """Pick the launch shape by timing real steps; returns the choice and the timings."""
        out = CTuneOut()
        self._check(self.lib.pic1d_autotune(self.h, int(trial_steps), ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in CTuneOut._fields_}

    def set_push_shape(self, blocks_per_cu, ppt, window):
        """Launch shape of the particle kernel: blocks per CU, particles per lane, deposit window (cells)."""
        self._check(self.lib.pic1d_set_push_shape(self.h, int(blocks_per_cu), int(ppt), int(window)))

    def set_sort_granularity(self, bins_per_cell):
        """Sort bins per cell (a power of two, 1 to 32); the results do not depend on it."""
        self._check(self.lib.pic1d_set_sort_granularity(self.h, int(bins_per_cell)))

    def rics_line_info(self, line=0):
        """(surrogate error estimate on the line, whether the line uses its table)."""
        err = ctypes.c_double(0.0)
        tab = ctypes.c_int32(0)
        self._check(self.lib.pic1d_rics_line_info(self.h, int(line), ctypes.byref(err), ctypes.byref(tab)))
        return err.value, bool(tab.value)

    def rics_eval(self, line, s_cells, u):
        """F_hat, Ndot_hat, eps of the configured backend at device tensors s_cells, u (float32)."""
        torch = self._torch
        s_cells = s_cells.to(device=self.workspace.device, dtype=torch.float32).contiguous()
        u = u.to(device=self.workspace.device, dtype=torch.float32).contiguous()
        n = s_cells.numel()
        F = torch.empty_like(s_cells)
        N = torch.empty_like(s_cells)
        eps = torch.empty_like(s_cells)
        self._check(self.lib.pic1d_rics_eval(self.h, int(line), n, ctypes.c_void_p(s_cells.data_ptr()),
                                             ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                             ctypes.c_void_p(N.data_ptr()), ctypes.c_void_p(eps.data_ptr())))
        return F, N, eps


# ---------------------------------------------------------------------------
# test-particle map (Appendix A.4)
# ---------------------------------------------------------------------------

def testparticle_sweep(r_eq, gamma0=1000.0, kT_keV=1.0, b_pole=10.0, b_pp=0.1, t_max=4.0, dt_max=1e-2, tol=1e-3,
                       tol_stiff=0.3, max_steps=100_000_000, device="cuda"):
    """gamma_min, s_first, s_b, l_pp, L, crossed and steps of test leptons on lines r_eq
    (one device thread per line); dict of numpy arrays."""
    import torch
    r = np.ascontiguousarray(r_eq, dtype=np.float64)
    n = r.size
    lib = load()
    nb = ctypes.c_size_t(0)
    _raise_global(lib.pic1d_testparticle_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
    c = CTpConfig(gamma0, kT_keV, b_pole, b_pp, t_max, dt_max, tol, tol_stiff, max_steps)
    out = (CTpResult * n)()
    _raise_global(lib.pic1d_testparticle_sweep(ctypes.byref(c), n, _ptr(r), ctypes.cast(out, ctypes.c_void_p),
                                               _dev_ptr(ws), ws.numel(), _stream(ws.device)))
    res = {k: np.array([getattr(o, k) for o in out]) for k, _ in CTpResult._fields_ if k != "pad"}
    res["crossed"] = res["crossed"].astype(bool)
    return res


# ---------------------------------------------------------------------------
# RICS surrogate network (pic1d_mlp_*): device tensors are torch float32
# ---------------------------------------------------------------------------

def _raise_global(rc):
    if rc != 0:
        raise Pic1dError(rc, load().pic1d_last_error(None).decode())


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


MLP_SAMPLES_WORKSPACE = 256     # bytes of device workspace of pic1d_mlp_samples (its error word)


def mlp_param_count():
    return load().pic1d_mlp_param_count()


def _mlp_workspace(batch, n_pool, device):
    import torch
    n = ctypes.c_size_t(0)
    _raise_global(load().pic1d_mlp_workspace_size(int(batch), int(n_pool), ctypes.byref(n)))
    return torch.empty(n.value, dtype=torch.uint8, device=device)


def mlp_samples(seed, first, n, device="cuda"):
    """Inputs (n x 4) and float32 targets (n x 4: o1, o2, o3, 0) of the seeded sample stream."""
    import torch
    x = torch.empty((max(n, 1), 4), dtype=torch.float32, device=device)
    o = torch.empty((max(n, 1), 4), dtype=torch.float32, device=device)
    ws = torch.empty(MLP_SAMPLES_WORKSPACE, dtype=torch.uint8, device=x.device)
    _raise_global(load().pic1d_mlp_samples(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first), int(n), _dev_ptr(x),
                                           _dev_ptr(o), _dev_ptr(ws), ws.numel(), _stream(x.device)))
    return x[:n], o[:n]


def mlp_forward(params, x):
    """Network outputs (normalised targets, n x 3) for raw inputs x (n x 4); params: float32 device tensor."""
    import torch
    n = x.shape[0]
    out = torch.empty((max(n, 1), 3), dtype=torch.float32, device=x.device)
    ws = _mlp_workspace(1, 0, x.device)
    _raise_global(load().pic1d_mlp_forward(_dev_ptr(params.contiguous()), n, _dev_ptr(x.contiguous()), _dev_ptr(out),
                                           _dev_ptr(ws), ws.numel(), _stream(x.device)))
    return out[:n]


def mlp_loss_grad(params, x, t):
    """(loss, gradient) of the mean squared error against normalised targets t (n x 3)."""
    import torch
    n = x.shape[0]
    grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=x.device)
    ws = _mlp_workspace(n, 0, x.device)
    loss = ctypes.c_double(0.0)
    _raise_global(load().pic1d_mlp_loss_grad(_dev_ptr(params.contiguous()), n, _dev_ptr(x.contiguous()),
                                             _dev_ptr(t.contiguous()), _dev_ptr(grad), ctypes.byref(loss),
                                             _dev_ptr(ws), ws.numel(), _stream(x.device)))
    return loss.value, grad


def mlp_loss_grad_static(params, x, t):
    """mlp_loss_grad through the allocation-free entry point (n <= 2048); the
    gradient tensor is the caller's."""
    import torch
    n = x.shape[0]
    grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=x.device)
    loss = ctypes.c_double(0.0)
    _raise_global(load().pic1d_mlp_loss_grad_static(_dev_ptr(params.contiguous()), n, _dev_ptr(x.contiguous()),
                                                    _dev_ptr(t.contiguous()), _dev_ptr(grad), ctypes.byref(loss),
                                                    _stream(x.device)))
    return loss.value, grad


def mlp_adam(params, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on float32 device tensors."""
    _raise_global(load().pic1d_mlp_adam(_dev_ptr(params), _dev_ptr(m), _dev_ptr(v), _dev_ptr(grad), int(t),
                                        float(lr), float(beta1), float(beta2), float(eps), _stream(params.device)))


def mlp_train(seed=0, n_samples=1 << 22, batch=8192, steps=20000, lr=2e-3, lr_final=1e-5, init_params=None,
              n_loss=50, device="cuda"):
    """Train the surrogate on the GPU; returns dict(params, norm, loss, loss_first, loss_last, seconds)."""
    ws = _mlp_workspace(batch, n_samples, device)
    c = CMlpTrainConfig()
    c.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    c.n_samples = int(n_samples)
    c.batch = int(batch)
    c.steps = int(steps)
    c.lr = float(lr)
    c.lr_final = float(lr_final)
    keep = None
    if init_params is not None:
        keep = np.ascontiguousarray(init_params, dtype=np.float32)
        c.init_params = ctypes.c_void_p(keep.ctypes.data)
    c.workspace = _dev_ptr(ws)
    c.workspace_bytes = ws.numel()
    c.stream = _stream(ws.device)
    params = np.zeros(mlp_param_count(), dtype=np.float32)
    norm = np.zeros(6, dtype=np.float32)
    loss = np.zeros(max(n_loss, 1), dtype=np.float64)
    r = CMlpTrainResult()
    r.params = ctypes.c_void_p(params.ctypes.data)
    r.norm = ctypes.c_void_p(norm.ctypes.data)
    r.loss = ctypes.c_void_p(loss.ctypes.data)
    r.n_loss = int(n_loss)
    _raise_global(load().pic1d_mlp_train(ctypes.byref(c), ctypes.byref(r)))
    del keep
    return dict(params=params, norm=norm, loss=loss[:r.n_loss].copy(), loss_first=r.loss_first,
                loss_last=r.loss_last, seconds=r.seconds)
