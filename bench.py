"""Benchmark: particle-steps/s of the 1D PIC hot path (push + RICS drag + deposit +
pairs + atmosphere + Ampere) on one MI355X, with the push kernel's roofline, the
surrogate-network path beside the table and exact paths, and the FP64 oracle
timed on the host as a CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--backend table|exact|off]
                    [--workload cfg2|cfg1] [--no-cpu-baseline] [--no-surrogate]
    python bench.py --copy-calibration     # plain 256 MiB device copy, for HBM counters
    python bench.py --cascade              # the combined cascade run (cfg5) on its own

Plain path (the headline `value`): the R_max = 30 line with 65,536 cells, 200
e-/e+ per cell each (2.6e7 particles), surface atmosphere with ions at
m_i/m_e = 100, pairs on with curvature conversion, capacity for 1e8 particles,
TABLE RICS backend.  Launch shape and sort interval from the library's
autotuner; the timed steps are launched eagerly or replayed from 100-step HIP
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

Cascade run (`--cascade`, not part of the default line): 64 lines of 32,768
cells whose hot pair seed cascades up to n_max (about 4e8 particles), stepped
from 100-step graphs in chunks; wall time, particle count and pair multiplicity
per chunk, and k_push's HBM rate at the final count.

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
BYTES_PER_PARTICLE = 24    # cell, offset, u: read 12 B + write 12 B
BYTES_PER_DRAW = 8         # 64-bit id read for a Philox event draw
BYTES_PER_CHILD = 20       # appended particle: cell, offset, u, id
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


def cpu_baseline(cfg, sample_ppc=40, steps=6):
    """The oracle (FP64 numpy, single thread) on the same line with fewer particles per cell."""
    from threadpoolctl import threadpool_limits

    from oracle import pic
    from tests import parity

    c = dict(cfg)
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
    return dict(value=pushed / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"R_max=30 line, 65,536 cells, {sample_ppc} e-/e+ per cell ({n0} particles) "
                       f"+ atmosphere and pairs as in the workload, {steps} steps, numpy float64, one thread",
                seconds=dt)


def _counters(sim):
    tot = None
    for li in range(sim.n_lines):
        c = sim.moments(li)["counters"]
        tot = dict(c) if tot is None else {k: tot[k] + c[k] for k in tot}
    return tot


def timed_run(sim, steps, warmup, profile=True):
    """Warm up, then time `steps` steps with HIP events on the library's stream;
    with profile, per-kernel event timing (pic1d_profile) is on during the timed
    steps (profiled steps are launched eagerly, never from a captured graph)."""
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
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = sim.profile_read()
    sim.profile(False)
    m1 = sim.moments(0)
    c1 = _counters(sim)
    cnt = {k: c1[k] - c0[k] for k in c1}
    push = prof["push"]
    push_avg_s = push["ms"] / max(push["launches"], 1) * 1e-3
    return dict(ms=ms, value=cnt["pushed"] / (ms * 1e-3), ms_per_step=ms / steps, counters=cnt,
                push_avg_s=push_avg_s, launches=push["launches"],
                kernels_ms={k: v["ms"] / max(v["launches"], 1) for k, v in prof.items() if v["launches"]},
                m0=m0, m1=m1)


def pick_launch(sim, trial_steps=200, graph_steps=100):
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
    sim.set_graph(graph_steps if mode == "graph" else 0)
    return {"mode": mode, "graph_steps": graph_steps if mode == "graph" else 0,
            "trial_steps": trial_steps, "trial_ms_per_step": {"eager": eager, "graph": graph}}


def hbm_bytes_per_launch(r):
    c = r["counters"]
    return (BYTES_PER_PARTICLE * c["pushed"] + BYTES_PER_DRAW * c["draws"] +
            BYTES_PER_CHILD * 2 * c["pairs_created"]) / max(r["launches"], 1)


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
        r = timed_run(sim, steps, warmup)
        entry = {"value": r["value"], "ms_per_step": r["ms_per_step"], "k_push_ms": r["push_avg_s"] * 1e3,
                 "kernels_ms": r["kernels_ms"], "events": r["counters"]["events"],
                 "pairs_created": r["counters"]["pairs_created"]}
        if backend == "mlp":
            evals = r["counters"]["mlp_evals"] / max(r["launches"], 1)
            achieved = evals * MLP_FLOP_PER_EVAL / r["push_avg_s"]
            executed = evals / 16 * MLP_MFMA_PER_GROUP * (16 * 16 * 32 * 2) / r["push_avg_s"]
            entry["roofline"] = {"bound": "mfma", "achieved": achieved / 1e12, "peak": BF16_PEAK / 1e12,
                                 "unit": "TFLOP/s", "frac": achieved / BF16_PEAK, "kernel": "k_push<mlp>",
                                 "evals_per_launch": evals, "flop_per_eval": MLP_FLOP_PER_EVAL,
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
            entry["error_vs_exact"] = {
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
                       "(gamma log-uniform to 1e4), pairs (immediate)")
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
    bytes_per_launch = hbm_bytes_per_launch(rp)
    out = {"workload": f"cfg3: {sim.n_lines} lines, R_max log-uniform in [2, 100], "
                       f"{sum(l['n_cells'] for l in cfg['lines'])} cells, 32-256 e-/e+ per cell per line, "
                       "cold, table RICS, pairs (curvature), sort every 50 steps (tuned)",
           "value": r["value"], "ms_per_step": r["ms_per_step"], "steps": steps, "launch": launch,
           "particles": counts, "autotune": tune, "init_seconds": t_init,
           "eager_ms_per_step": rp["ms_per_step"], "kernels_ms": rp["kernels_ms"],
           "roofline": {"bound": "hbm", "achieved": bytes_per_launch / rp["push_avg_s"] / 1e9,
                        "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": bytes_per_launch / rp["push_avg_s"] / HBM_PEAK, "kernel": "k_push"},
           "gauss_residual_max_over_lines": max(gauss)}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    print(f"# batched: {out['value']:.3g} particle-steps/s", file=sys.stderr, flush=True)
    return out


def cascade_run(chunks, chunk_steps, profile_steps):
    """The combined cascade run (cfg5): 64 lines of 32,768 cells whose hot pair seed
    cascades up to n_max, stepped in chunks replayed from graphs; wall time, particle
    count and pair multiplicity per chunk, then a profiled window for k_push's HBM
    rate at the final particle count."""
    import torch

    from paper_2609_17661_amd import Pic1D, workloads

    def live(sim):
        return sum(sum(sim.moments(li)["count"]) for li in range(sim.n_lines))

    t0 = time.perf_counter()
    cfg = workloads.cfg5()
    sim = Pic1D(cfg, device="cuda:0")
    t_init = time.perf_counter() - t0
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
    gauss = max(sim.moments(li)["gauss_residual"] for li in range(sim.n_lines))
    out = {"workload": f"cfg5: {sim.n_lines} lines, R_max log-uniform in [10, 100], 32768 cells each, hot pair "
                       f"seed {cfg['lines'][0]['ppc_init']} e-/e+ per cell (gamma to 1e4), n_max = 6 n0 (n0 = 32), atmosphere with ions at "
                       f"m_i/m_e = 100, pairs (curvature), pair annihilation over n_max, TABLE RICS, 100-step graphs",
           "init_seconds": t_init, "wall_seconds": wall, "steps": chunks * chunk_steps,
           "particles_start": n_start, "particles_end": rows[-1]["particles"],
           "pair_multiplicity": pairs / seed_pairs, "pairs_annihilated": annihilated, "chunks": rows,
           "kernels_ms_at_end": rp["kernels_ms"],
           "k_push_ms_at_end": rp["push_avg_s"] * 1e3,
           "hbm_GBps_at_end": bytes_per_launch / rp["push_avg_s"] / 1e9,
           "roofline_frac_at_end": bytes_per_launch / rp["push_avg_s"] / HBM_PEAK,
           "gauss_residual_max_over_lines": gauss}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--profile-steps", type=int, default=100,
                    help="eager steps with per-kernel events after the timed region")
    ap.add_argument("--backend", default="table", choices=["table", "exact", "off"])
    ap.add_argument("--workload", default="cfg2", choices=["cfg2", "cfg1"])
    ap.add_argument("--eta-min", type=float, default=None,
                    help="drag-time variant: eta_min instead of the workload's 1e3 (App. C uses 1e2)")
    ap.add_argument("--mass-ratio", type=float, default=None,
                    help="mass-ratio variant: m_i/m_e instead of the workload's 100")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate comparison (for profiling its kernels)")
    ap.add_argument("--surrogate-steps", type=int, default=10)
    ap.add_argument("--mlp-train-steps", type=int, default=200000)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--cascade", action="store_true",
                    help="only the combined cascade run (cfg5), as its own JSON line")
    ap.add_argument("--cascade-chunks", type=int, default=6)
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
        print(json.dumps({"cascade": cascade_run(args.cascade_chunks, 100, 20)}), flush=True)
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate_vs_table": surrogate_comparison(args.surrogate_steps, 3, args.mlp_train_steps)}),
              flush=True)
        return
    cfg = dict(workloads.CFG2 if args.workload == "cfg2" else workloads.CFG1)
    cfg["rics"] = args.backend
    variant = ""
    if args.eta_min is not None:
        cfg["eta_min"] = args.eta_min
        variant += f", eta_min={args.eta_min:g}"
    if args.mass_ratio is not None:
        cfg["mass_ratio"] = args.mass_ratio
        variant += f", m_i/m_e={args.mass_ratio:g}"
    sim = Pic1D(cfg, device="cuda:0")
    print(f"# init done: {cfg['lines'][0]}", file=sys.stderr, flush=True)
    tune = sim.autotune(trial_steps=10)        # launch shape and sort interval (results do not depend on them)
    print(f"# autotuned: {tune}", file=sys.stderr, flush=True)
    launch = pick_launch(sim)
    print(f"# launch: {launch}", file=sys.stderr, flush=True)
    r = timed_run(sim, args.steps, args.warmup, profile=False)
    # kernel breakdown and roofline: events around every launch, eager launches
    rp = timed_run(sim, args.profile_steps, 0, profile=True)
    bytes_per_launch = hbm_bytes_per_launch(rp)
    achieved = bytes_per_launch / rp["push_avg_s"]
    # HBM bytes per k_push launch (rocprofv3), measured on the unmodified workload only
    traffic = measured_traffic(args.backend, args.workload) if not variant else None
    m0, m1 = r["m0"], r["m1"]
    res = {
        "metric": "particle-steps/s (push+RICS drag+deposit+pairs)",
        "value": r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 particles / f64 field",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: one dipole line R_max=30, 65536 cells, 200 ppc e-/e+, "
                                f"atmosphere ions m_i/m_e=100, pairs (curvature), {args.backend} RICS"
                                if args.workload == "cfg2" else f"cfg1: R_max=4, 512 cells, 64 ppc, {args.backend} RICS")
                               + variant,
                   "particles_start": sum(m0["count"]), "particles_end": sum(m1["count"]),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK,
                     "traffic": traffic,
                     "kernel": "k_push", "avg_ms": rp["push_avg_s"] * 1e3, "launches": rp["launches"],
                     "bytes_per_launch": bytes_per_launch, "traffic_unit": "bytes/launch",
                     "traffic_over_algorithmic": traffic / bytes_per_launch if traffic else None},
        "launch": launch,
        "profiled_ms_per_step": rp["ms_per_step"],
        "kernels_ms": rp["kernels_ms"],
        "autotune": tune,
        "counters": r["counters"],
        "gauss_residual": m1["gauss_residual"],
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_batched:
        res["batched"] = batched_path(100, 5)
    if not args.no_surrogate:
        res["surrogate_vs_table"] = surrogate_comparison(args.surrogate_steps, 3, args.mlp_train_steps)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
