"""Parity of the surrogate-network kernels (bfloat16 MFMA) with the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2609_17661_amd import pic1d

pytestmark = pytest.mark.gpu

# The forward pass carries activations as three bfloat16 terms (24 significant
# bits) with float32 accumulation over at most 128 products per layer, so the
# outputs agree with the float64 evaluation of the same bfloat16 weights to a
# few float32 ulps of the accumulated magnitudes: OUT_TOL absolute on outputs of
# order one.  Gradients: GRAD_TOL relative in the 2-norm of each layer's block.
OUT_TOL = 2e-6
GRAD_TOL = 2e-6


def _print(*a):
    print(*a, flush=True)


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in omlp.LAYERS:
        parts.append((rng.uniform(-1, 1, (o, i)) * scale * omlp.glorot_bound(o, i), rng.uniform(-0.2, 0.2, o)))
    return omlp.pack(parts)


def _torch():
    import torch
    return torch


def _box_inputs(seed, n):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, 8, n), rng.uniform(0, 1, n), rng.uniform(-2, 3, n),
                     rng.uniform(0.3, 1, n)], axis=1).astype(np.float32)


def test_sample_stream_matches_oracle():
    torch = _torch()
    first, n = 123456789012, 4001
    _print("mlp samples", first, n)
    x, o = pic1d.mlp_samples(11, first, n)
    X, O, used = omlp.training_samples(seed=11, n=n, first=first)
    xg = x.cpu().numpy()
    og = o.cpu().numpy().astype(np.float64)
    assert np.array_equal(xg, X), "inputs are 24-bit uniforms mapped in float64 and stored float32: bit-exact"
    # targets: float64 on both sides, stored float32 on the GPU (half an ulp of |o| <= 32)
    err = np.abs(og[:, :3] - O)
    assert np.all(err <= 2.0 ** -24 * np.maximum(np.abs(O), 1.0) + 1e-9), err.max()
    assert np.all(og[:, 3] == 0.0)
    _print("attempts used up to", used.max(), "max target error", err.max())
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 16, 1001])
def test_forward_matches_oracle(n):
    torch = _torch()
    p = _params(21, 1.5)
    X = _box_inputs(22, n)
    _print("mlp forward n", n)
    out = pic1d.mlp_forward(torch.from_numpy(p.astype(np.float32)).cuda(), torch.from_numpy(X).cuda())
    ref, _ = omlp.forward(p.astype(np.float32).astype(np.float64), omlp.normalize_inputs(X.astype(np.float64)))
    got = out.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    _print("max |out - oracle|", err.max(), "max |out|", np.abs(ref).max())
    assert np.all(err <= OUT_TOL * np.maximum(1.0, np.abs(ref)))


def test_loss_and_gradient_match_oracle():
    torch = _torch()
    n = 777          # ragged against the 16-sample groups and the 256-sample gradient chunks
    p = _params(31, 1.5).astype(np.float32).astype(np.float64)
    X = _box_inputs(32, n)
    T = np.random.default_rng(33).standard_normal((n, 3)).astype(np.float32)
    _print("mlp loss_grad n", n)
    loss, g = pic1d.mlp_loss_grad(torch.from_numpy(p.astype(np.float32)).cuda(), torch.from_numpy(X).cuda(),
                                  torch.from_numpy(T).cuda())
    L, gref = omlp.loss_and_grad(p, omlp.normalize_inputs(X.astype(np.float64)), T.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - L) <= 1e-5 * L
    k = 0
    for o, i in omlp.LAYERS:
        for size in (o * i, o):
            a, b = g[k:k + size], gref[k:k + size]
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            _print("block", o, i, size, "relative error", rel)
            assert rel <= GRAD_TOL
            k += size


def test_adam_step_matches_oracle():
    torch = _torch()
    rng = np.random.default_rng(41)
    n = omlp.N_PARAM
    th = rng.standard_normal(n).astype(np.float32)
    m = (rng.standard_normal(n) * 1e-2).astype(np.float32)
    v = (rng.uniform(0, 1e-3, n)).astype(np.float32)
    g = (rng.standard_normal(n) * 1e-2).astype(np.float32)
    t, lr = 5, 1e-3
    dt = [torch.from_numpy(a.copy()).cuda() for a in (th, m, v, g)]
    pic1d.mlp_adam(dt[0], dt[1], dt[2], dt[3], t, lr)
    ref, mref, vref = omlp.adam_step(th.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                                     g.astype(np.float64), t, lr)
    # the new parameter is rounded to float32: one ulp of theta plus float32 arithmetic on the step
    got = dt[0].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-5 * np.abs(ref - th))
    # moments: float32 rounding of the constants and of the two terms of each update (they may cancel)
    mb = 2.0 ** -21 * (0.9 * np.abs(m) + 0.1 * np.abs(g))
    vb = 2.0 ** -21 * (0.999 * v + 0.001 * g.astype(np.float64) ** 2)
    assert np.all(np.abs(dt[1].cpu().numpy() - mref) <= mb)
    assert np.all(np.abs(dt[2].cpu().numpy() - vref) <= vb)


def test_training_on_the_gpu_reduces_the_loss():
    _print("mlp train small")
    r = pic1d.mlp_train(seed=5, n_samples=1 << 16, batch=2048, steps=300, lr=2e-3, lr_final=1e-4, n_loss=10)
    _print("loss", r["loss_first"], "->", r["loss_last"], "in", r["seconds"], "s")
    assert np.all(np.isfinite(r["params"]))
    assert r["loss_last"] < 0.05 * r["loss_first"]
    # the normalisation is the mean and standard deviation of the pool's targets (oracle, float64)
    X, O, _ = omlp.training_samples(seed=5, n=1 << 16)
    mean, std = omlp.normalisation(O)
    assert np.allclose(r["norm"][:3], mean, rtol=1e-5, atol=1e-5)
    assert np.allclose(r["norm"][3:], std, rtol=1e-5)


# ---------------------------------------------------------------------------
# the surrogate inside the pusher (RICS backend "mlp")
# ---------------------------------------------------------------------------
def _pusher_network(seed):
    """Random weights (float32 values) with a small output layer, and the target
    normalisation of the oracle's sample stream: drag of physical size, both
    branches of the limiter and stochastic events all occur."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (o, i) in enumerate(omlp.LAYERS):
        s = 0.15 if li == len(omlp.LAYERS) - 1 else 1.0
        parts.append((rng.uniform(-1, 1, (o, i)) * s * omlp.glorot_bound(o, i), rng.uniform(-0.1, 0.1, o)))
    p = omlp.pack(parts).astype(np.float32).astype(np.float64)
    _, O, _ = omlp.training_samples(seed=seed, n=4096)
    mean, std = omlp.normalisation(O)
    norm = np.concatenate([mean, std]).astype(np.float32).astype(np.float64)
    return p, norm


def _mlp_cfg(seed, **kw):
    from paper_2609_17661_amd import workloads
    p, norm = _pusher_network(seed)
    cfg = workloads.small(r_eq=4.0, rics="mlp", **kw)
    cfg["mlp_params"] = p
    cfg["mlp_norm"] = norm
    return cfg


def test_rics_eval_of_the_surrogate_matches_oracle():
    import torch
    from oracle import pic
    from paper_2609_17661_amd import Pic1D

    from . import parity
    cfg = _mlp_cfg(51, n_cells=400, ppc=1, init="empty")
    sim = Pic1D(cfg)
    st = pic.State(parity.oracle_config(cfg))
    ln = st.lines[0]
    rng = np.random.default_rng(52)
    n = 5001
    s = rng.uniform(0, 400, n).astype(np.float32)
    lg = rng.uniform(0, 6, n)
    u = (np.where(rng.random(n) < 0.5, -1.0, 1.0) * np.sqrt(np.maximum(10 ** (2 * lg) - 1, 0))).astype(np.float32)
    _print("mlp rics_eval", n)
    F, N, eps = (t.cpu().numpy().astype(np.float64) for t in sim.rics_eval(0, torch.from_numpy(s), torch.from_numpy(u)))
    xs = s.astype(np.float64)
    uu = u.astype(np.float64)
    b, mu, xr, _ = ln.geometry_at(xs)
    force, _, rate = ln.rics_funcs(xs, b, mu, xr)
    Fo, No = force(uu), rate(uu)
    # network outputs agree to ~OUT_TOL; 10^(mean + std out) turns that into a relative error of
    # ln(10) std OUT_TOL; float32 inputs, exp2 of arguments up to ~100 and the factor
    # (gamma mu - u) (condition number cond, as for the closed form) add a few float32 ulps each
    gam = np.sqrt(1 + uu * uu)
    cond = (gam * np.abs(mu) + np.abs(uu)) / np.maximum(np.abs(gam * mu - uu), 1e-300)
    tolF = np.log(10) * cfg["mlp_norm"][3] * OUT_TOL + 1e-5 + 2e-7 * cond
    tolN = np.log(10) * cfg["mlp_norm"][4] * OUT_TOL + 1e-5
    nz = Fo != 0
    relF = np.abs(F - Fo)[nz] / np.abs(Fo)[nz]
    relN = np.abs(N - No)[No > 0] / No[No > 0]
    _print("F rel max", relF.max(), "N rel max", relN.max(), "zeros", np.sum(~nz))
    assert np.all(relF <= tolF[nz])
    assert np.all(relN <= tolN)
    assert np.array_equal(F[~nz], Fo[~nz])          # beyond the Planck cutoff both are exactly zero


@pytest.mark.parametrize("kw", [dict(init="hot", gamma_max=3e3, pairs=True),
                                dict(init="cold", pairs=False, ppc=24),
                                # tau_min = 68 steps: the implicit midpoint's fixed-point
                                # refinement runs (Eq. implicit)
                                dict(init="hot", gamma_max=1e4, pairs=True, eta_min=1.0, ppc=16),
                                # angle-resolved events (dipole pattern) with the surrogate's Ndot
                                dict(init="hot", gamma_max=1e4, pairs=True, conversion="curvature",
                                     emission="dipole")])
def test_step_parity_with_the_surrogate(kw):
    from paper_2609_17661_amd import Pic1D

    from . import parity
    args = dict(n_cells=96, ppc=12)
    args.update(kw)
    cfg = _mlp_cfg(61, **args)
    ocfg = parity.oracle_config(cfg)
    sim = Pic1D(cfg)
    _print("mlp step parity", kw)
    total = dict(compared=0, excused=0)
    for k in range(3):
        before = parity.snapshot(sim)
        sim.step(1)
        after = parity.snapshot(sim)
        rep, st = parity.compare_step(ocfg, before, after)
        _print(f"  step {k}: {rep} {st.counters[0]}")
        total["compared"] += rep["compared"]
        total["excused"] += rep["excused"]
        sim.step(2)
    assert total["compared"] > 0
    assert total["excused"] <= max(3, 1e-3 * total["compared"])
    assert sim.moments(0)["gauss_residual"] <= 1e-6
    if kw.get("eta_min", 1e3) < 10.0:
        n_refined = sim.moments(0)["counters"]["newton"]
        _print("  drag halves refined:", n_refined)
        assert n_refined > 0


# ---------------------------------------------------------------------------
# what the trained network gains
# ---------------------------------------------------------------------------
def _continued_targets(X):
    """o1, o2, o3 of the oracle's definitions, continued past the Planck cutoff in log
    form (finite for every y) so that a table can hold them at every node."""
    from oracle import rics
    X = np.asarray(X, dtype=np.float64)
    lg, sl, lb, kT = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
    gam = 10.0 ** lg
    u = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    b = 10.0 ** lb
    mu, x = omlp.line_geometry(sl)
    y = rics.resonance_y(u, b, mu, kT)
    A_F, A_N = rics.prefactors(kT)
    lp = -np.log10(-np.expm1(-y)) - y / np.log(10.0)          # log10 of 1/(e^y - 1)
    o1 = np.log10(A_F / (x * x)) + 3.0 * np.log10(y) + lp
    o2 = np.log10(A_N / (x * x * gam)) + 2.0 * np.log10(y) + lp
    return np.stack([o1, o2, np.log10(rics.photon_energy(u, b))], axis=1)


def _multilinear_table_error(n, X, O):
    """Relative errors of a 4D multilinear table with n nodes per input axis over the network's box."""
    axes = [np.linspace(lo, hi, n) for lo, hi in zip(omlp.IN_LO, omlp.IN_HI)]
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 4)
    V = _continued_targets(grid).reshape(n, n, n, n, 3)
    f = (X - omlp.IN_LO) / (omlp.IN_HI - omlp.IN_LO) * (n - 1)
    i0 = np.clip(np.floor(f).astype(int), 0, n - 2)
    w = f - i0
    out = np.zeros((X.shape[0], 3))
    for corner in range(16):
        wt = np.ones(X.shape[0])
        idx = []
        for d in range(4):
            bit = (corner >> d) & 1
            wt = wt * (w[:, d] if bit else 1.0 - w[:, d])
            idx.append(i0[:, d] + bit)
        out += wt[:, None] * V[idx[0], idx[1], idx[2], idx[3]]
    return np.abs(out - O) * np.log(10.0)


def test_trained_network_beats_a_table_of_equal_storage():
    """The network (50,563 parameters) against a 4D multilinear table holding more values
    (12^4 nodes x 3 outputs = 62,208) over the same inputs, on held-out samples of the
    sample stream scored against the oracle's exact targets: errors of 10^o, relative."""
    import torch
    _print("mlp training for the comparison")
    r = pic1d.mlp_train(seed=3, n_samples=1 << 20, batch=8192, steps=20000, lr=2e-3, lr_final=2e-6, n_loss=5)
    _print("loss", r["loss_first"], "->", r["loss_last"], "in", r["seconds"], "s")
    X, O, _ = omlp.training_samples(seed=3, n=20000, first=1 << 40)
    out = pic1d.mlp_forward(torch.from_numpy(r["params"]).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    o = out.astype(np.float64) * r["norm"][3:].astype(np.float64) + r["norm"][:3].astype(np.float64)
    e_net = np.abs(o - O) * np.log(10.0)
    e_tab = _multilinear_table_error(12, X.astype(np.float64), O)
    for k, name in enumerate(("F/(gamma mu - u)", "Ndot", "eps")):
        _print(f"{name}: network median {np.median(e_net[:, k]):.3e} p99 {np.quantile(e_net[:, k], 0.99):.3e}; "
               f"table median {np.median(e_tab[:, k]):.3e} p99 {np.quantile(e_tab[:, k], 0.99):.3e}")
    for k in (0, 1):
        assert np.median(e_net[:, k]) < 0.5 * np.median(e_tab[:, k])
        assert np.quantile(e_net[:, k], 0.99) < 0.1 * np.quantile(e_tab[:, k], 0.99)


# ---------------------------------------------------------------------------
# the table as the network's fallback, per line
# ---------------------------------------------------------------------------
def _fallback_cfg(tol, radii, n_cells=96, ppc=12):
    p, norm = _pusher_network(61)
    lines = [dict(r_eq=r, n_cells=n_cells, ppc_init=ppc, init="hot", init_gamma_max=3e3,
                  capacity=[200_000, 200_000, 50_000, 50_000]) for r in radii]
    return dict(rics="mlp", kT_keV=0.5, j_twist=0.5, ppc0=float(ppc), seed=7, pairs=True, table_nlg=64, table_ns=48,
                mlp_params=p, mlp_norm=norm, mlp_fallback_tol=tol, lines=lines)


def _oracle_estimates(cfg):
    from oracle import pic

    from . import parity
    st = pic.State(parity.oracle_config(cfg))
    return [ln.mlp_error for ln in st.lines], [ln.use_table for ln in st.lines]


def test_fallback_estimates_match_oracle():
    """Per-line error estimates of the network (largest relative error of F and Ndot on the
    table nodes) from the GPU's bfloat16 network against the oracle's float64 one."""
    from paper_2609_17661_amd import Pic1D
    radii = [4.0, 10.0, 40.0]
    cfg = _fallback_cfg(1e30, radii)
    e_o, _ = _oracle_estimates(cfg)
    _print("fallback estimates, oracle", e_o)
    sim = Pic1D(cfg)
    info = [sim.rics_line_info(li) for li in range(len(radii))]
    _print("fallback estimates, GPU", info)
    for (e, tab), eo in zip(info, e_o):
        assert not tab
        # network outputs within OUT_TOL (relative ln(10) std OUT_TOL after 10^o), float32
        # geometry and the factor (gamma mu - u) near the attractor: 1e-3 relative is ample
        assert abs(e - eo) <= 1e-3 * eo + 1e-6, (e, eo)
    sim.close()


def test_mixed_step_parity_with_table_fallback():
    """Two lines, a tolerance between their estimates: one steps with the network, the
    other with its table, in the same launch, each matched against the oracle."""
    from paper_2609_17661_amd import Pic1D

    from . import parity
    radii = [4.0, 40.0]
    e_o, _ = _oracle_estimates(_fallback_cfg(1e30, radii))
    assert e_o[0] != e_o[1]
    tol = math.sqrt(e_o[0] * e_o[1])
    cfg = _fallback_cfg(tol, radii)
    ocfg = parity.oracle_config(cfg)
    _, use_o = _oracle_estimates(cfg)
    sim = Pic1D(cfg)
    use_g = [sim.rics_line_info(li)[1] for li in range(len(radii))]
    _print("fallback tol", tol, "tables (oracle, GPU)", use_o, use_g)
    assert use_g == use_o and sorted(use_g) == [False, True]
    total = dict(compared=0, excused=0)
    for k in range(3):
        before = parity.snapshot(sim)
        sim.step(1)
        after = parity.snapshot(sim)
        rep, st = parity.compare_step(ocfg, before, after)
        _print(f"  step {k}: {rep}")
        total["compared"] += rep["compared"]
        total["excused"] += rep["excused"]
        sim.step(2)
    assert total["compared"] > 0
    assert total["excused"] <= max(3, 1e-3 * total["compared"])
    for li in range(len(radii)):
        assert sim.moments(li)["gauss_residual"] <= 1e-6
    sim.close()


def test_precision_ablation_of_the_trained_network():
    """Which precision sets the trained surrogate's error floor.  The network is trained
    on the GPU (float32 master weights; the forward pass with bfloat16 weights and
    three-term bfloat16 activations), then the force factor 10^o1 = |F|/|gamma mu - u|
    and the rate 10^o2 are scored against the exact targets on held-out samples for
      (a) the GPU forward,
      (b) the FP64 oracle forward with the same bfloat16-rounded weights,
      (c) the FP64 oracle forward with the float32 master weights (no rounding).
    (a) matches (b) to the forward's tolerance.  (c) against (b) is the ablation: the
    error the bfloat16 weights add on top of the fit."""
    import torch
    r = pic1d.mlp_train(seed=5, n_samples=1 << 20, batch=8192, steps=20000, lr=2e-3, lr_final=2e-6, n_loss=5)
    X, O, _ = omlp.training_samples(seed=5, n=20000, first=1 << 41)
    P = r["params"].astype(np.float64)
    mean = r["norm"][:3].astype(np.float64)
    std = r["norm"][3:].astype(np.float64)
    out_a = pic1d.mlp_forward(torch.from_numpy(r["params"]).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    Xn = omlp.normalize_inputs(X.astype(np.float64))
    out_b = omlp.forward(P, Xn, round_weights=True)[0]
    out_c = omlp.forward(P, Xn, round_weights=False)[0]

    def rel(out):
        o = out.astype(np.float64) * std + mean
        return np.abs(10.0 ** (o - O) - 1.0)
    res = {}
    for name, out in (("a GPU bf16", out_a), ("b FP64, bf16 weights", out_b), ("c FP64, fp32 weights", out_c)):
        e = rel(out)
        res[name] = e
        _print(f"{name}: F factor median {np.median(e[:, 0]):.3e} p99 {np.quantile(e[:, 0], 0.99):.3e} "
               f"max {e[:, 0].max():.3e}; Ndot median {np.median(e[:, 1]):.3e} p99 {np.quantile(e[:, 1], 0.99):.3e} "
               f"max {e[:, 1].max():.3e}")
    ea, eb, ec = res["a GPU bf16"], res["b FP64, bf16 weights"], res["c FP64, fp32 weights"]
    # (a) and (b): the same network to the forward's tolerance (relative ln(10) std OUT_TOL)
    for k in (0, 1):
        assert np.max(np.abs(ea[:, k] - eb[:, k]) / (1.0 + eb[:, k])) <= 10 * np.log(10) * std[k] * OUT_TOL
    # the bfloat16 weights move the outputs by about their 2^-9 relative rounding; the
    # fit's own error sits on top of that either way
    _print("median ratio bf16 / fp32 weights:", np.median(eb[:, 0]) / np.median(ec[:, 0]),
           np.median(eb[:, 1]) / np.median(ec[:, 1]))
