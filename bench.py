"""Benchmark: particle-steps/s of the 1D PIC hot path (push + RICS drag + deposit +
pairs + atmosphere + Ampere) on one MI355X, with the push kernel's HBM roofline
and the FP64 oracle timed on the host as a CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--backend table|exact|off]
                    [--workload cfg2|cfg1] [--no-cpu-baseline]
    python bench.py --copy-calibration     # plain 256 MiB device copy, for HBM counters

Workload (default): the R_max = 30 line with 65,536 cells, 200 e-/e+ per cell
each (2.6e7 particles), surface atmosphere with ions at m_i/m_e = 100, pairs on
with curvature conversion, capacity for 1e8 particles, TABLE RICS backend.
Inputs are synthetic (Philox initial plasma) and resident in HBM before the
timed region.  One JSON line is printed.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
BYTES_PER_PARTICLE = 24    # cell, offset, u: read 12 B + write 12 B
BYTES_PER_DRAW = 8         # 64-bit id read for a Philox event draw
BYTES_PER_CHILD = 20       # appended particle: cell, offset, u, id
PROFILE_HBM = os.path.join(ROOT, "profiles", "k_push_cfg2_table_hbm.md")
CAL_BYTES = 256 << 20      # bytes read (and written) by one calibration copy


def sources_digest():
    """sha256 over the library sources: HBM counters are only reported for the
    kernel they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_17661_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)) + [os.path.join(ROOT, "include", "pic1d.h")]
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


def cpu_baseline(cfg, sample_ppc=20, steps=3):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--backend", default="table", choices=["table", "exact", "off"])
    ap.add_argument("--workload", default="cfg2", choices=["cfg2", "cfg1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build measures the single-GPU hot path "
              f"(requested --gpus {args.gpus}); lines would shard across GPUs without per-step "
              f"communication, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    from paper_2609_17661_amd import Pic1D, workloads

    cfg = dict(workloads.CFG2 if args.workload == "cfg2" else workloads.CFG1)
    cfg["rics"] = args.backend
    sim = Pic1D(cfg, device="cuda:0")
    print(f"# init done: {cfg['lines'][0]}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    m0 = sim.moments(0)
    sim.profile(True)
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = sim.profile_read()
    sim.profile(False)
    m1 = sim.moments(0)
    c0, c1 = m0["counters"], m1["counters"]
    pushed = c1["pushed"] - c0["pushed"]
    draws = c1["draws"] - c0["draws"]
    children = 2 * (c1["pairs_created"] - c0["pairs_created"])
    value = pushed / (ms * 1e-3)
    push = prof["push"]
    push_avg_s = push["ms"] / max(push["launches"], 1) * 1e-3
    bytes_per_launch = (BYTES_PER_PARTICLE * pushed + BYTES_PER_DRAW * draws + BYTES_PER_CHILD * children) / max(
        push["launches"], 1)
    achieved = bytes_per_launch / push_avg_s
    traffic = measured_traffic(args.backend, args.workload)     # HBM bytes per k_push launch (rocprofv3)
    res = {
        "metric": "particle-steps/s (push+RICS drag+deposit+pairs)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 particles / f64 field",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: one dipole line R_max=30, 65536 cells, 200 ppc e-/e+, "
                               f"atmosphere ions m_i/m_e=100, pairs (curvature), {args.backend} RICS"
                   if args.workload == "cfg2" else f"cfg1: R_max=4, 512 cells, 64 ppc, {args.backend} RICS",
                   "particles_start": sum(m0["count"]), "particles_end": sum(m1["count"]),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK,
                     "traffic": traffic,
                     "kernel": "k_push", "avg_ms": push_avg_s * 1e3,
                     "bytes_per_launch": bytes_per_launch, "traffic_unit": "bytes/launch",
                     "traffic_over_algorithmic": traffic / bytes_per_launch if traffic else None},
        "kernels_ms": {k: v["ms"] / max(v["launches"], 1) for k, v in prof.items() if v["launches"]},
        "counters": {k: c1[k] - c0[k] for k in c1},
        "gauss_residual": m1["gauss_residual"],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
