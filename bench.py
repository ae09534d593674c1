"""Benchmark: particle-steps/s of the 1D PIC hot path (push + RICS drag + deposit +
pairs + atmosphere + Ampere) on one MI355X, with the push kernel's roofline, the
surrogate-network path beside the table and exact paths, and the FP64 oracle
timed on the host as a CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--backend table|exact|off]
                    [--workload cfg2|cfg1|cfg4] [--no-cpu-baseline] [--no-surrogate]
                    [--push-shape BPC,PPT,WINDOW] [--launch eager|graph]
    python bench.py --copy-calibration     # plain 256 MiB device copy, for HBM counters
    python bench.py --cascade              # the combined cascade run (cfg5) on its own

Plain path (the headline `value`): the R_max = 30 line with 65,536 cells, 200
e-/e+ per cell each (2.6e7 particles), surface atmosphere with ions at
m_i/m_e = 100, pairs on with curvature conversion, capacity for 1e8 particles,
TABLE RICS backend.  Launch shape and sort interval from the library's
autotuner; the timed region is the workload's whole run of 20,000 steps (after
the tuner's trial steps and the warm-up), whose step time rises about threefold
after the first two thousand steps as the line heats (`along_the_run`, per 2000
steps); the timed steps are launched eagerly or replayed from 100-step HIP
graphs, whichever a 200-step trial of each finds faster (`launch`).  The
per-kernel breakdown and the push kernel's roofline come from HIP events around
every launch in a profiled window of eagerly launched steps that follows the
timed region (events cannot bracket kernels inside a replayed graph).

Batched path (`batched`): 256 dipole lines of uneven length and particle count
(about 7.7e8 particles) in one state, launch shape picked by the library's
autotuner, eager launches or 100-step HIP graphs as on the plain path; per-line
Gauss residuals.

Surrogate path (`surrogate_vs_table`): the network is trained on the GPU by the
library (outside the timed region), then the R_max = 4 line of its training
geometry at the same particle count (65,536 cells x 200 hot e-/e+ per cell) is
stepped with the TABLE, EXACT and MLP backends in turn.  The network's error is
judged against the library's EXACT backend at the workload's particles.

Cascade run (`cascade`; `--cascade` runs it alone): 64 lines of 32,768
cells whose hot pair seed cascades up to n_max (about 4e8 particles), stepped
from 100-step graphs in chunks; wall time, particle count and pairs created per
chunk, the pair multiplicity M = n e c / j_psi at the end, and k_push's HBM rate
at the final count.  The RICS source is the
surrogate network (trained first on the GPU) with each line's table as its
fallback where the network's error estimate on the line exceeds 1e-3; the
line count on each source is reported.

Inputs are synthetic (Philox initial plasma) and resident in HBM before each
timed region.  One JSON line is printed.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
BF16_PEAK = 2.5e15         # MI355X dense bf16 MFMA, FLOP/s
# algorithmic bytes of the particle kernel per particle-step: a lepton reads cell,
# offset, momentum and id (16 B) and writes cell, offset, momentum (12 B); an ion
# needs no id (no draws)
BYTES_PER_LEPTON = 28
BYTES_PER_ION = 24
BYTES_PER_CREATED = 16     # a created particle written by the append kernel
# the stricter count of what the kernel must move: the id is read only for a draw
BYTES_PER_PARTICLE = 24    # cell, offset, u: read 12 B + write 12 B
BYTES_PER_DRAW = 8         # 64-bit id read for a Philox event draw
MLP_FLOP_PER_EVAL = 2 * (4 * 128 + 3 * 128 * 128 + 128 * 3)   # multiply-adds of one network evaluation, x2
MLP_MFMA_PER_GROUP = 308   # v_mfma_f32_16x16x32_bf16 per 16 evaluations (three bfloat16 terms per activation)
PROFILE_HBM = os.path.join(ROOT, "profiles", "k_push_cfg2_table_hbm.md")
CAL_BYTES = 256 << 20      # bytes read (and written) by one calibration copy


KERNEL_SOURCES = ("kernels.hip", "kernels.h", "pic1d_dev.h", "rics_dev.h", "mlp_dev.h")


def sources_digest():
    """sha256 over the sources that define the particle kernel: HBM counters are
    only reported for the kernel they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_17661_amd", "csrc")
    files = [os.path.join(csrc, f) for f in KERNEL_SOURCES]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(backend, workload):
    """HBM bytes per k_push launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (calibrated against a plain copy), or None if it was taken on another
    kernel source, backend or workload."""
    if not os.path.exists(PROFILE_HBM):
        return None
    kv = {}
    with open(PROFILE_HBM) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    try:
        if kv.get("sources_sha256") != sources_digest() or kv.get("backend") != backend or \
                kv.get("workload") != workload:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device-to-device copy of CAL_BYTES, three times: the known traffic
    that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.ones(CAL_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": CAL_BYTES, "bytes_written": CAL_BYTES, "copies": 3}),
          flush=True)


def _oracle_run(cfg, sample_ppc, steps, seed):
    """Step the oracle (one thread of numpy) on the workload's first line with
    sample_ppc pairs per cell; returns (particle-steps, seconds, particles at start)."""
    from threadpoolctl import threadpool_limits

    from oracle import pic
    from tests import parity

    c = dict(cfg, seed=seed)
    c["lines"] = [dict(cfg["lines"][0], ppc_init=sample_ppc)]
    ocfg = parity.oracle_config(c)
    st = pic.init_state(ocfg)
    n0 = sum(p["x"].size for p in st.parts[0])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pushed = 0
        for _ in range(steps):
            pushed += sum(p["x"].size for p in st.parts[0])
            pic.step(st)
        dt = time.perf_counter() - t0
    return pushed, dt, n0


def _oracle_worker(args):
    import threadpoolctl  # noqa: F401  (imported before numpy spins up its pools)
    cfg, sample_ppc, steps, seed = args
    return _oracle_run(cfg, sample_ppc, steps, seed)


def cpu_baseline(cfg, sample_ppc=40, steps=6):
    """The oracle (FP64 numpy) on the same line with fewer particles per cell: one
    process on one core, then one process per host core, each stepping its own
    copy of the line (different seeds; lines are independent), timed together."""
    import multiprocessing as mp

    pushed, dt, n0 = _oracle_run(cfg, sample_ppc, steps, cfg.get("seed", 0))
    single = dict(value=pushed / dt, unit="particle-steps/s", cores=1, kind="oracle",
                  sample=f"R_max=30 line, 65,536 cells, {sample_ppc} e-/e+ per cell ({n0} particles) "
                         f"+ atmosphere and pairs as in the workload, {steps} steps, numpy float64, one thread",
                  seconds=dt)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(cfg, sample_ppc, steps, 1000 + k) for k in range(cores)])
    wall = time.perf_counter() - t0
    # timed from the slowest worker's own clock (process start-up excluded)
    tot = sum(r[0] for r in res)
    slowest = max(r[1] for r in res)
    single["all_cores"] = dict(value=tot / slowest, unit="particle-steps/s", cores=cores, kind="oracle",
                               sample=f"{cores} processes, each the single-thread sample on its own copy of "
                                      f"the line (seeds 1000+k)", seconds=slowest, wall_seconds=wall)
    single["host"] = _host_cpu()
    return single


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def _counters(sim):
    tot = None
    for li in range(sim.n_lines):
        c = sim.moments(li)["counters"]
        tot = dict(c) if tot is None else {k: tot[k] + c[k] for k in tot}
    return tot


def timed_run(sim, steps, warmup, profile=True, chunk=None):
    """Warm up, then time `steps` steps with HIP events on the library's stream;
    with profile, per-kernel event timing (pic1d_profile) is on during the timed
    steps (profiled steps are launched eagerly, never from a captured graph).
    With `chunk`, an event every `chunk` steps also gives the step time along the
    run (no host synchronisation inside the timed region)."""
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    m0 = sim.moments(0)
    c0 = _counters(sim)
    sim.profile(profile)
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    marks = []
    if chunk:
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            sim.step(n)
            done += n
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            marks.append((done, e))
    else:
        sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    along = []
    prev_e, prev_n = ev0, 0
    for n, e in marks:
        along.append({"steps": [m0["step"] + prev_n, m0["step"] + n], "ms_per_step": prev_e.elapsed_time(e) / (n - prev_n)})
        prev_e, prev_n = e, n
    prof = sim.profile_read()
    sim.profile(False)
    m1 = sim.moments(0)
    c1 = _counters(sim)
    cnt = {k: c1[k] - c0[k] for k in c1}
    push = prof["push"]
    push_avg_s = push["ms"] / max(push["launches"], 1) * 1e-3
    return dict(ms=ms, value=cnt["pushed"] / (ms * 1e-3), ms_per_step=ms / steps, counters=cnt, along=along,
                push_avg_s=push_avg_s, launches=push["launches"],
                kernels_ms={k: v["ms"] / max(v["launches"], 1) for k, v in prof.items() if v["launches"]},
                m0=m0, m1=m1)


def pick_launch(sim, trial_steps=200, graph_steps=100, force=None):
    """Eager launches or replays of `graph_steps`-step HIP graphs, whichever runs
    the same steps faster here (the results are identical either way): time
    trial_steps real steps each way and keep the faster.  The graph trial first
    steps twice the graph length, so that the graphs of both particle buffer
    sets are captured before the timed steps."""
    sim.set_graph(0)
    eager = timed_run(sim, trial_steps, 0, profile=False)["ms_per_step"]
    sim.set_graph(graph_steps)
    graph = timed_run(sim, trial_steps, 2 * graph_steps, profile=False)["ms_per_step"]
    mode = "graph" if graph < eager else "eager"
    if force:
        mode = force
    sim.set_graph(graph_steps if mode == "graph" else 0)
    return {"mode": mode, "graph_steps": graph_steps if mode == "graph" else 0,
            "trial_steps": trial_steps, "trial_ms_per_step": {"eager": eager, "graph": graph},
            **({"set_by_flag": True} if force else {})}


def hbm_bytes_per_launch(r):
    """Algorithmic bytes of one particle-kernel launch: 28 B per lepton-step, 24 B
    per ion-step."""
    c = r["counters"]
    ions = c["pushed_ions"]
    return (BYTES_PER_LEPTON * (c["pushed"] - ions) + BYTES_PER_ION * ions) / max(r["launches"], 1)


def strict_bytes_per_launch(r):
    """What the kernel must move at the least: cell, offset and momentum both ways,
    the id only where a draw needs it."""
    c = r["counters"]
    return (BYTES_PER_PARTICLE * c["pushed"] + BYTES_PER_DRAW * c["draws"]) / max(r["launches"], 1)


def window_bytes(r):
    """Algorithmic bytes of all steps of a window: the particle kernel's plus 16 B
    per created particle (pair members and atmosphere particles)."""
    c = r["counters"]
    ions = c["pushed_ions"]
    created = 2 * c["pairs_created"] + 2 * c["atm_injected"]
    return BYTES_PER_LEPTON * (c["pushed"] - ions) + BYTES_PER_ION * ions + BYTES_PER_CREATED * created


def push_roofline(r):
    b = hbm_bytes_per_launch(r)
    achieved = b / r["push_avg_s"]
    strict = strict_bytes_per_launch(r)
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "kernel": "k_push", "avg_ms": r["push_avg_s"] * 1e3,
            "launches": r["launches"], "bytes_per_launch": b,
            "bytes_rule": "28 B per lepton-step, 24 B per ion-step",
            "strict_bytes_per_launch": strict, "strict_frac": strict / r["push_avg_s"] / HBM_PEAK,
            "strict_rule": "24 B per particle-step + 8 B per Philox draw (id read only for a draw)"}


def surrogate_comparison(steps, warmup, mlp_steps):
    """Train the network, then step the CFG4 line with the table, exact and MLP backends."""
    import numpy as np
    import torch

    from paper_2609_17661_amd import Pic1D, pic1d, workloads

    t0 = time.perf_counter()
    tr = pic1d.mlp_train(seed=0, n_samples=1 << 22, batch=8192, steps=mlp_steps, lr=2e-3, lr_final=2e-6, n_loss=10)
    out = {"training": {"steps": mlp_steps, "batch": 8192, "pool": 1 << 22, "seconds": tr["seconds"],
                        "loss_first": tr["loss_first"], "loss_last": tr["loss_last"]}}
    print(f"# surrogate trained in {time.perf_counter() - t0:.1f} s, loss {tr['loss_last']:.3g}", file=sys.stderr,
          flush=True)
    res = {}
    for backend in ("table", "exact", "mlp"):
        cfg = dict(workloads.CFG4)
        cfg["rics"] = backend
        if backend == "mlp":
            cfg["mlp_params"] = tr["params"]
            cfg["mlp_norm"] = tr["norm"]
        sim = Pic1D(cfg, device="cuda:0")
        # the same steps for every backend: the cascade reaches the density limit within
        # its first tens of steps, and the warm-up puts the timed steps there (sorted
        # every 5 steps, the autotuner's choice on this line)
        r = timed_run(sim, steps, warmup)
        c = r["counters"]
        entry = {"value": r["value"], "ms_per_step": r["ms_per_step"], "k_push_ms": r["push_avg_s"] * 1e3,
                 "kernels_ms": r["kernels_ms"], "events_per_step": c["events"] / steps,
                 "pairs_created_per_step": c["pairs_created"] / steps,
                 "annihilated_per_step": c["annihilated"] / steps, "particles_end": sum(r["m1"]["count"]),
                 "step_window": [r["m0"]["step"], r["m1"]["step"]]}
        if backend != "mlp":
            entry["roofline"] = push_roofline(r)
        if backend == "mlp":
            launches = max(r["launches"], 1)
            needed = c["mlp_needed"] / launches
            lanes = c["mlp_evals"] / launches
            achieved = needed * MLP_FLOP_PER_EVAL / r["push_avg_s"]
            executed = lanes / 16 * MLP_MFMA_PER_GROUP * (16 * 16 * 32 * 2) / r["push_avg_s"]
            entry["roofline"] = {"bound": "mfma", "achieved": achieved / 1e12, "peak": BF16_PEAK / 1e12,
                                 "unit": "TFLOP/s", "frac": achieved / BF16_PEAK, "kernel": "k_push<mlp>",
                                 "evals_needed_per_launch": needed, "flop_per_eval": MLP_FLOP_PER_EVAL,
                                 "rule": "evaluations the step needs: 2 per continuous-regime lepton step "
                                         "plus its refinements, 1 per stochastic-regime step",
                                 "lane_evals_executed_per_launch": lanes,
                                 "executed_mfma_tflops": executed / 1e12, "executed_frac": executed / BF16_PEAK}
            # network error against the library's exact backend at this workload's particles
            p = sim.get_particles(0, 0)
            n = min(200000, p["cell"].size)
            s = torch.from_numpy((p["cell"][:n] + p["off"][:n]).astype(np.float32))
            u = torch.from_numpy(p["u"][:n].astype(np.float32))
            Fm, Nm, _ = (t.cpu().numpy().astype(np.float64) for t in sim.rics_eval(0, s, u))
            ecfg = dict(workloads.CFG4)
            ecfg["rics"] = "exact"
            ecfg["lines"] = [dict(ecfg["lines"][0], init="empty", ppc_init=0, capacity=[256, 256, 0, 0])]
            esim = Pic1D(ecfg, device="cuda:0")
            Fe, Ne, _ = (t.cpu().numpy().astype(np.float64) for t in esim.rics_eval(0, s, u))
            esim.close()
            h = cfg["cfl"] if "cfl" in cfg else 0.5
            h *= 9.004239 / cfg["lines"][0]["n_cells"]        # one step in R*/c on the R_max = 4 line
            uu = np.abs(u.numpy().astype(np.float64))
            sig = np.abs(Fe) * h >= 1e-9 * np.maximum(uu, 1e-30)
            eF = np.abs(Fm - Fe)[sig] / np.abs(Fe)[sig]
            sigN = Ne * h > 1e-9
            eN = np.abs(Nm - Ne)[sigN] / Ne[sigN]
            # the drag half's branch (damping where |F| tau_min > |u|) taken from the network
            # and from the exact force at the same momenta: tau_min = eta_min (n_psi)^(1/2) / w_p
            # steps (Sec. 3), w_p = C / d0 per step, one step = h in R*/c
            cfl = cfg.get("cfl", 0.5)
            tau_hat = cfg.get("eta_min", 1.0e3) * abs(cfg["j_twist"]) ** 0.5 / (cfl / cfg.get("d0_cells", 48.0)) * h
            flip = (np.abs(Fm) * tau_hat > uu) != (np.abs(Fe) * tau_hat > uu)
            entry["error_vs_exact"] = {
                "limiter_branch_flip_rate": float(flip.mean()),
                "F_median": float(np.median(eF)), "F_p99": float(np.quantile(eF, 0.99)), "F_max": float(eF.max()),
                "Ndot_median": float(np.median(eN)) if eN.size else None,
                "Ndot_p99": float(np.quantile(eN, 0.99)) if eN.size else None,
                "sample": f"{n} e- of the workload after the timed steps, where |F| h >= 1e-9 |u|"}
        res[backend] = entry
        sim.close()
        del sim
        torch.cuda.empty_cache()
        print(f"# {backend}: {entry['value']:.3g} particle-steps/s", file=sys.stderr, flush=True)
    out.update(res)
    out["workload"] = ("cfg4: R_max=4 line (the network's training geometry), 65536 cells, 200 hot e-/e+ per cell "
                       "(gamma log-uniform to 1e4), pairs (immediate) held by n_max = 3 n0, sorted every 5 steps; "
                       "every backend timed over the same steps after the same warm-up")
    out["mlp_over_table"] = res["mlp"]["value"] / res["table"]["value"]
    return out


def batched_path(steps, warmup):
    """The 256-line workload: autotuned launch shape, eager launches or 100-step HIP
    graphs (the faster), per-line conservation."""
    import torch

    from paper_2609_17661_amd import Pic1D, workloads

    t0 = time.perf_counter()
    cfg = workloads.cfg3()
    sim = Pic1D(cfg, device="cuda:0")
    t_init = time.perf_counter() - t0
    tune = sim.autotune(trial_steps=5)
    launch = pick_launch(sim)
    r = timed_run(sim, steps, warmup, profile=False)
    rp = timed_run(sim, 10, 0, profile=True)         # kernel breakdown (eager launches)
    gauss = [sim.moments(li)["gauss_residual"] for li in range(sim.n_lines)]
    counts = sum(sum(sim.moments(li)["count"]) for li in range(sim.n_lines))
    out = {"workload": f"cfg3: {sim.n_lines} lines, R_max log-uniform in [2, 100], "
                       f"{sum(l['n_cells'] for l in cfg['lines'])} cells, 32-256 e-/e+ per cell per line, "
                       "cold, table RICS, pairs (curvature), sort every 50 steps (tuned)",
           "value": r["value"], "ms_per_step": r["ms_per_step"], "steps": steps, "launch": launch,
           "particles": counts, "autotune": tune, "init_seconds": t_init,
           "eager_ms_per_step": rp["ms_per_step"], "kernels_ms": rp["kernels_ms"],
           "roofline": push_roofline(rp),
           "gauss_residual_max_over_lines": max(gauss)}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    print(f"# batched: {out['value']:.3g} particle-steps/s", file=sys.stderr, flush=True)
    return out


def cascade_run(chunks, chunk_steps, profile_steps, mlp_train_steps=0, fallback_tol=1e-3):
    """The combined cascade run (cfg5): 64 lines of 32,768 cells whose hot pair seed
    cascades up to n_max, stepped in chunks replayed from graphs; wall time, particle
    count and pairs created per chunk, the pair multiplicity M = n e c / j_psi at the
    end, then a profiled window for k_push's HBM
    rate at the final particle count.  With mlp_train_steps > 0 the RICS source is
    the surrogate network, trained on the GPU first, with each line's table as its
    fallback where the network's error estimate on the line exceeds fallback_tol."""
    import numpy as np
    import torch

    from paper_2609_17661_amd import Pic1D, pic1d, workloads

    def live(sim):
        return sum(sum(sim.moments(li)["count"]) for li in range(sim.n_lines))

    cfg = workloads.cfg5()
    training = None
    if mlp_train_steps > 0:
        tr = pic1d.mlp_train(seed=0, n_samples=1 << 22, batch=8192, steps=mlp_train_steps, lr=2e-3,
                             lr_final=2e-6, n_loss=10)
        training = {"steps": mlp_train_steps, "seconds": tr["seconds"], "loss_last": tr["loss_last"]}
        print(f"# cascade surrogate trained: {training}", file=sys.stderr, flush=True)
        cfg.update(rics="mlp", mlp_params=tr["params"], mlp_norm=tr["norm"], mlp_fallback_tol=fallback_tol)
    t0 = time.perf_counter()
    sim = Pic1D(cfg, device="cuda:0")
    t_init = time.perf_counter() - t0
    rics_src = {"backend": cfg["rics"]}
    if training:
        info = [sim.rics_line_info(li) for li in range(sim.n_lines)]
        est = np.array([e for e, _ in info])
        rics_src.update(training=training, fallback_tol=fallback_tol,
                        lines_on_table=int(sum(t for _, t in info)), lines_on_network=int(sum(not t for _, t in info)),
                        estimate_min=float(est.min()), estimate_median=float(np.median(est)),
                        estimate_max=float(est.max()))
        print(f"# cascade RICS source: {rics_src}", file=sys.stderr, flush=True)
    seed_pairs = sum(l["ppc_init"] * l["n_cells"] for l in cfg["lines"])
    n_start = live(sim)
    sim.set_graph(100)          # the seed evolves fastest at first: no launch trials before it
    rows, pairs, annihilated, wall = [], 0, 0, 0.0
    for c in range(chunks):
        r = timed_run(sim, chunk_steps, 0, profile=False)
        pairs += r["counters"]["pairs_created"]
        annihilated += r["counters"]["annihilated"]
        wall += r["ms"] * 1e-3
        rows.append({"steps_done": (c + 1) * chunk_steps, "ms_per_step": r["ms_per_step"],
                     "particle_steps_per_s": r["value"], "particles": live(sim), "pairs_created": pairs,
                     "pairs_annihilated": annihilated})
        print(f"# cascade chunk {c}: {rows[-1]}", file=sys.stderr, flush=True)
    rp = timed_run(sim, profile_steps, 0, profile=True)
    bytes_per_launch = hbm_bytes_per_launch(rp)
    moms = [sim.moments(li) for li in range(sim.n_lines)]
    gauss = max(m["gauss_residual"] for m in moms)
    # the paper's pair multiplicity M = n e c / j_psi per cell (Sec. 4.3), n the e-/e+
    # pair density in units of n0 and j_psi = j_twist n0 e c
    M = [(m["n"][0] + m["n"][1]) / abs(cfg["j_twist"]) for m in moms]
    Mall = np.concatenate(M)
    multiplicity = {"definition": "M = n e c / j_psi per cell, n the e-/e+ pair density",
                    "mean": float(Mall.mean()), "median": float(np.median(Mall)),
                    "p99": float(np.quantile(Mall, 0.99)), "max": float(Mall.max()),
                    "line_mean_min": float(min(x.mean() for x in M)),
                    "line_mean_max": float(max(x.mean() for x in M))}
    src = ("surrogate network with per-line table fallback" if training else "TABLE") + " RICS"
    out = {"workload": f"cfg5: {sim.n_lines} lines, R_max log-uniform in [10, 100], 32768 cells each, hot pair "
                       f"seed {cfg['lines'][0]['ppc_init']} e-/e+ per cell (gamma to 1e4), "
                       f"n_max = {cfg['nmax_over_n0']:g} n0 (n0 = {cfg['ppc0']:g}), atmosphere with ions at "
                       f"m_i/m_e = 100, pairs (curvature), pair annihilation over n_max, {src}, 100-step graphs",
           "rics": rics_src, "init_seconds": t_init, "wall_seconds": wall, "steps": chunks * chunk_steps,
           "particles_start": n_start, "particles_end": rows[-1]["particles"],
           "pairs_created_per_seed_pair": pairs / seed_pairs, "multiplicity": multiplicity,
           "pairs_annihilated": annihilated, "chunks": rows,
           "kernels_ms_at_end": rp["kernels_ms"],
           "k_push_ms_at_end": rp["push_avg_s"] * 1e3,
           "hbm_GBps_at_end": bytes_per_launch / rp["push_avg_s"] / 1e9,
           "roofline_frac_at_end": bytes_per_launch / rp["push_avg_s"] / HBM_PEAK,
           "gauss_residual_max_over_lines": gauss}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def plain_path(cfg, steps, warmup, profile_steps, chunk=None, push_shape=None, launch_mode=None):
    """Autotune, pick eager or graph launches, time `steps` steps after `warmup`,
    then a profiled window of eager launches for the kernel breakdown.  With
    push_shape (blocks per CU, particles per lane, window), that tile shape replaces
    the tuner's (so that separate counter runs all profile the same kernel)."""
    from paper_2609_17661_amd import Pic1D

    sim = Pic1D(cfg, device="cuda:0")
    print(f"# init done: {cfg['lines'][0]}", file=sys.stderr, flush=True)
    tune = sim.autotune(trial_steps=10)        # launch shape and sort interval (results do not depend on them)
    if push_shape:
        sim.set_push_shape(*push_shape)
        tune = dict(tune, push_blocks_per_cu=push_shape[0], push_ppt=push_shape[1], deposit_window=push_shape[2],
                    shape_set_by_flag=True)
    print(f"# autotuned: {tune}", file=sys.stderr, flush=True)
    launch = pick_launch(sim, force=launch_mode)
    print(f"# launch: {launch}", file=sys.stderr, flush=True)
    r = timed_run(sim, steps, warmup, profile=False, chunk=chunk)
    # kernel breakdown and roofline: events around every launch, eager launches
    rp = timed_run(sim, profile_steps, 0, profile=True)
    sim.close()
    del sim
    return r, rp, tune, launch


def whole_step(r, steps):
    """Algorithmic bytes of whole steps (particle kernel plus created particles) over
    the timed window's step time: the roofline of the step, sorts and all."""
    b = window_bytes(r) / steps
    t = r["ms_per_step"] * 1e-3
    return {"bytes_per_step": b, "achieved": b / t / 1e9, "unit": "GB/s", "frac": b / t / HBM_PEAK}


ACTIVE_STEPS = 300     # timed steps of the hot-start leg


def active_phase(cfg, steps, warmup, profile_steps):
    """The headline line with a hot pair plasma (gamma log-uniform to 1e4): RICS
    events, drag on both branches and pair creation act in every timed step."""
    c = dict(cfg)
    c["lines"] = [dict(cfg["lines"][0], init="hot", init_gamma_max=1.0e4)]
    r, rp, tune, launch = plain_path(c, steps, warmup, profile_steps)
    cnt = r["counters"]
    out = {"workload": "cfg2 line (R_max=30, 65536 cells, 200 ppc, atmosphere, pairs by curvature conversion), "
                       "hot start: gamma log-uniform in [1, 1e4]",
           "value": r["value"], "unit": "particle-steps/s", "ms_per_step": r["ms_per_step"],
           "step_window": [r["m0"]["step"], r["m1"]["step"]],
           "events_per_step": cnt["events"] / steps, "pairs_created_per_step": cnt["pairs_created"] / steps,
           "draws_per_step": cnt["draws"] / steps, "newton_per_step": cnt["newton"] / steps,
           "particles_end": sum(r["m1"]["count"]), "roofline": push_roofline(rp),
           "whole_step": whole_step(r, steps), "kernels_ms": rp["kernels_ms"], "autotune": tune, "launch": launch,
           "gauss_residual": r["m1"]["gauss_residual"]}
    print(f"# active phase: {out['value']:.3g} particle-steps/s", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: cfg2's whole run of 20,000 steps; 300 for the other workloads)")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--profile-steps", type=int, default=100,
                    help="eager steps with per-kernel events after the timed region")
    ap.add_argument("--backend", default="table", choices=["table", "exact", "off"])
    ap.add_argument("--workload", default="cfg2", choices=["cfg2", "cfg1", "cfg4"])
    ap.add_argument("--init", default=None, choices=["cold", "hot"],
                    help="initial plasma of the line instead of the workload's (hot: gamma log-uniform to 1e4)")
    ap.add_argument("--no-active", action="store_true", help="skip the hot-start leg of the headline line")
    ap.add_argument("--eta-min", type=float, default=None,
                    help="drag-time variant: eta_min instead of the workload's 1e3 (App. C uses 1e2)")
    ap.add_argument("--mass-ratio", type=float, default=None,
                    help="mass-ratio variant: m_i/m_e instead of the workload's 100")
    ap.add_argument("--push-shape", default=None,
                    help="BPC,PPT,WINDOW: the particle kernel's tile shape instead of the tuner's (for counter runs)")
    ap.add_argument("--launch", default=None, choices=["eager", "graph"],
                    help="launch mode of the timed steps instead of the faster of the two trials "
                         "(counter runs: eager)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cascade", action="store_true", help="skip the combined cascade run (cfg5) leg")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate comparison (for profiling its kernels)")
    ap.add_argument("--surrogate-steps", type=int, default=10)
    ap.add_argument("--mlp-train-steps", type=int, default=200000)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--cascade", action="store_true",
                    help="only the combined cascade run (cfg5), as its own JSON line")
    ap.add_argument("--cascade-chunks", type=int, default=6)
    ap.add_argument("--cascade-mlp-train-steps", type=int, default=20000,
                    help="training steps of the cascade run's surrogate (0: the table alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures the hot path on one GPU only (requested --gpus {args.gpus}); "
              f"field lines would shard across GPUs without per-step communication", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    from paper_2609_17661_amd import Pic1D, workloads

    if args.cascade:
        print(json.dumps({"cascade": cascade_run(args.cascade_chunks, 100, 20, args.cascade_mlp_train_steps)}),
              flush=True)
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate_vs_table": surrogate_comparison(args.surrogate_steps, 30, args.mlp_train_steps)}),
              flush=True)
        return
    steps = args.steps if args.steps is not None else (workloads.CFG2_STEPS if args.workload == "cfg2" else 300)
    cfg = dict({"cfg2": workloads.CFG2, "cfg1": workloads.CFG1, "cfg4": workloads.CFG4}[args.workload])
    cfg["rics"] = args.backend
    variant = ""
    if args.eta_min is not None:
        cfg["eta_min"] = args.eta_min
        variant += f", eta_min={args.eta_min:g}"
    if args.mass_ratio is not None:
        cfg["mass_ratio"] = args.mass_ratio
        variant += f", m_i/m_e={args.mass_ratio:g}"
    if args.init is not None:
        cfg["lines"] = [dict(cfg["lines"][0], init=args.init, init_gamma_max=1.0e4)]
        variant += f", {args.init} start" + (" (gamma log-uniform to 1e4)" if args.init == "hot" else "")
    # the step time changes along the run (the line heats after a couple of thousand
    # steps): long runs also report it per 2000 steps
    shape = tuple(int(x) for x in args.push_shape.split(",")) if args.push_shape else None
    r, rp, tune, launch = plain_path(cfg, steps, args.warmup, args.profile_steps,
                                     chunk=2000 if steps >= 4000 else None, push_shape=shape,
                                     launch_mode=args.launch)
    roof = push_roofline(rp)
    # HBM bytes per k_push launch (rocprofv3), measured on the unmodified workload only
    traffic = measured_traffic(args.backend, args.workload) if not variant else None
    roof["traffic"] = traffic
    roof["traffic_unit"] = "bytes/launch"
    roof["traffic_over_algorithmic"] = traffic / roof["bytes_per_launch"] if traffic else None
    m0, m1 = r["m0"], r["m1"]
    names = {"cfg2": "cfg2: one dipole line R_max=30, 65536 cells, 200 ppc e-/e+, atmosphere ions m_i/m_e=100, "
                     f"pairs (curvature), {args.backend} RICS",
             "cfg1": f"cfg1: R_max=4, 512 cells, 64 ppc, {args.backend} RICS",
             "cfg4": f"cfg4: R_max=4, 65536 cells, 200 hot ppc e-/e+, pairs (immediate), n_max = 3 n0, "
                     f"{args.backend} RICS"}
    res = {
        "metric": "particle-steps/s (push+RICS drag+deposit+pairs)",
        "value": r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 particles / f64 field",
        "data": "synthetic",
        "config": {"workload": names[args.workload] + variant,
                   "particles_start": sum(m0["count"]), "particles_end": sum(m1["count"]),
                   "step_window": [m0["step"], m1["step"]], "parallelism": "single GPU"},
        "roofline": roof,
        "whole_step": whole_step(r, steps),
        "along_the_run": r["along"],
        "launch": launch,
        "profiled_ms_per_step": rp["ms_per_step"],
        "kernels_ms": rp["kernels_ms"],
        "autotune": tune,
        "counters": r["counters"],
        "gauss_residual": m1["gauss_residual"],
    }
    torch.cuda.empty_cache()
    if args.workload == "cfg2" and not variant and not args.no_active:
        res["active_phase"] = active_phase(cfg, min(steps, ACTIVE_STEPS), args.warmup, args.profile_steps)
    if not args.no_batched:
        res["batched"] = batched_path(100, 5)
    if not args.no_surrogate:
        res["surrogate_vs_table"] = surrogate_comparison(args.surrogate_steps, 30, args.mlp_train_steps)
    if not args.no_cascade:
        res["cascade"] = cascade_run(args.cascade_chunks, 100, 20, args.cascade_mlp_train_steps)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
