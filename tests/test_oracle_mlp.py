"""Pins of the surrogate-network oracle (oracle/mlp.py) against independent facts."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp, philox, rics


def test_parameter_count_is_the_stated_architecture():
    # 4 -> 128 x 4 hidden (SiLU) -> 3 has 50,563 weights and biases
    assert mlp.N_PARAM == 50563
    p = np.arange(mlp.N_PARAM, dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_bf16_rounding_ties_and_torch():
    # hand-worked ties: the bfloat16 ulp at 1 is 2^-7
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0                      # tie -> even (down)
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6       # tie -> even (up)
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7
    assert mlp.bf16_round(np.float32(-1.5)) == -1.5
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-30, 30, 100000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_silu_and_its_derivative():
    z = np.linspace(-30, 30, 2001)
    assert mlp.silu(0.0) == 0.0 and mlp.silu_grad(0.0) == 0.5
    assert np.allclose(mlp.silu(z), z / (1.0 + np.exp(-z)), rtol=1e-14, atol=1e-300)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(z))) < 1e-8


def test_sparse_network_is_a_known_composition():
    """Neuron 3 <- input 2 <- ... -> output 2: out_2 = silu^4(x_2); a transposed or reordered layer breaks it."""
    layers = [(np.zeros((o, i)), np.zeros(o)) for o, i in mlp.LAYERS]
    layers[0][0][3, 2] = 1.0
    layers[1][0][5, 3] = 1.0
    layers[2][0][7, 5] = 1.0
    layers[3][0][1, 7] = 1.0 + 2.0 ** -9          # rounds to 1 in bfloat16
    layers[4][0][2, 1] = -2.0
    layers[4][1][0] = 0.25
    p = mlp.pack(layers)
    X = np.random.default_rng(2).uniform(-1, 1, (50, 4))
    out, _ = mlp.forward(p, X)
    s = mlp.silu
    assert np.allclose(out[:, 2], -2.0 * s(s(s(s(X[:, 2])))), rtol=1e-15, atol=0)
    assert np.all(out[:, 0] == 0.25) and np.all(out[:, 1] == 0.0)
    out_unrounded, _ = mlp.forward(p, X, round_weights=False)
    assert np.allclose(out_unrounded[:, 2], -2.0 * s((1 + 2.0 ** -9) * s(s(s(X[:, 2])))), rtol=1e-15)


def _random_params(rng, scale=1.0):
    parts = []
    for o, i in mlp.LAYERS:
        parts.append((rng.uniform(-1, 1, (o, i)) * scale * mlp.glorot_bound(o, i), rng.uniform(-0.1, 0.1, o)))
    return mlp.pack(parts)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    p = _random_params(rng, 1.5)
    X = rng.uniform(-1, 1, (7, 4))
    T = rng.standard_normal((7, 3))
    L, g = mlp.loss_and_grad(p, X, T, round_weights=False)
    idx = np.concatenate([rng.choice(mlp.N_PARAM, 300, replace=False), np.arange(mlp.N_PARAM - 387, mlp.N_PARAM)])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, X, T, round_weights=False)[0] -
              mlp.loss_and_grad(p - e, X, T, round_weights=False)[0]) / (2 * h)
        # central-difference truncation is O(h^2); its roundoff is about L eps / h ~ 1e-10 L
        assert abs(fd - g[k]) <= 1e-7 * abs(g[k]) + 1e-9 * max(L, 1.0), (k, fd, g[k])


def test_gradient_uses_the_rounded_weights():
    rng = np.random.default_rng(4)
    p = _random_params(rng)
    X = rng.uniform(-1, 1, (5, 4))
    T = rng.standard_normal((5, 3))
    pr = mlp.pack(mlp.forward_weights(p))
    assert np.allclose(mlp.loss_and_grad(p, X, T)[1], mlp.loss_and_grad(pr, X, T, round_weights=False)[1],
                       rtol=1e-13, atol=1e-16)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are exactly g and g^2,
    # so every step moves theta by lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 8):
        new, m, v = mlp.adam_step(th, m, v, g, t, lr, eps=eps)
        assert np.allclose(th - new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
        th = new


def test_targets_equal_the_rics_definitions():
    rng = np.random.default_rng(5)
    X = np.stack([rng.uniform(0, 8, 3000), rng.uniform(0, 1, 3000), rng.uniform(-2, 3, 3000),
                  rng.uniform(0.3, 1, 3000)], axis=1)
    o1, o2, o3, y = mlp.targets(X)
    gam = 10.0 ** X[:, 0]
    u = np.sqrt(gam * gam - 1.0)
    b = 10.0 ** X[:, 2]
    mu, x = mlp.line_geometry(X[:, 1])
    ok = (y <= rics.Y_CUTOFF) & (np.abs(gam * mu - u) > 1e-6 * gam)
    F = rics.drag_force(u, b, mu, x, X[:, 3])
    N = rics.scatter_rate(u, b, mu, x, X[:, 3])
    assert np.allclose(10.0 ** o1[ok] * (gam * mu - u)[ok], F[ok], rtol=1e-9, atol=0)
    assert np.allclose(10.0 ** o2[ok], N[ok], rtol=1e-9, atol=0)
    assert np.allclose(10.0 ** o3, rics.photon_energy(u, b), rtol=1e-12)
    assert np.all(N[y > rics.Y_CUTOFF] == 0.0)


def test_sample_stream_follows_the_philox_definition():
    X, O, used = mlp.training_samples(seed=11, n=4000, first=123456789012)
    k0, k1 = philox.seed_key(11)
    idx = np.arange(123456789012, 123456789012 + 4000, dtype=np.uint64)
    lo = (idx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (idx >> np.uint64(32)).astype(np.uint32)
    for a in range(int(used.max()) + 1):
        w = philox.philox4x32_10(lo, hi, a, mlp.STREAM_MLP_SAMPLE, k0, k1)
        u24 = [philox.uniform24(w[j]) for j in range(4)]
        cand = np.stack([np.float32(8.0 * u24[0]), np.float32(u24[1]), np.float32(-2.0 + 5.0 * u24[2]),
                         np.float32(0.3 + 0.7 * u24[3])], axis=1).astype(np.float32)
        sel = used == a
        assert np.array_equal(X[sel], cand[sel])
        # every earlier attempt of these samples was beyond the Planck cutoff
        later = used > a
        assert np.all(mlp.targets(cand[later].astype(np.float64))[3] > rics.Y_CUTOFF)
    assert np.all(mlp.targets(X.astype(np.float64))[3] <= rics.Y_CUTOFF)
    # the accepted fraction of first attempts is the measure of the box inside the cutoff (~0.77)
    assert 0.73 < np.mean(used == 0) < 0.81
    o = np.stack(mlp.targets(X.astype(np.float64))[:3], axis=1)
    assert np.array_equal(o, O)


def test_surrogate_sign_mirror_and_cutoff():
    # a network with zero weights outputs its biases: F = (gamma mu - u) 10^(mean + std b)
    layers = [(np.zeros((o, i)), np.zeros(o)) for o, i in mlp.LAYERS]
    layers[4][1][:] = [0.5, -0.25, 0.125]
    p = mlp.pack(layers)
    mean, std = np.array([-1.0, -2.0, 3.0]), np.array([4.0, 5.0, 2.0])
    u = np.array([3.0, -3.0, 0.0, 200.0])
    b, mu, x, kT = 0.05, 0.6, 1.5, 0.5
    F, N, eps = mlp.surrogate_rics(p, (mean, std), u, np.array([0.3, 0.7, 0.3, 0.3]), b, mu, x, kT)
    G = 10.0 ** (mean[0] + std[0] * 0.5)
    gam = np.sqrt(1 + u * u)
    y = rics.resonance_y(u, b, mu, kT)
    expect = np.where(y <= rics.Y_CUTOFF, (gam * mu - u) * G, 0.0)
    assert np.allclose(F, expect, rtol=1e-14, atol=0)
    assert F[0] < 0 < F[1]              # beyond the attractor (beta > mu) the force decelerates
    assert np.allclose(N[y <= 80], 10.0 ** (mean[1] - std[1] * 0.25), rtol=1e-14)
    assert np.allclose(eps, 10.0 ** (mean[2] + std[2] * 0.125), rtol=1e-14)


def test_input_gradient_matches_central_differences():
    rng = np.random.default_rng(6)
    p = _random_params(rng, 1.5)
    X = rng.uniform(-1, 1, (6, 4))
    J = mlp.input_grad(p, X)
    h = 1e-6
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        fd = (mlp.forward(p, X + e)[0] - mlp.forward(p, X - e)[0]) / (2 * h)
        assert np.allclose(fd, J[:, :, j], rtol=1e-7, atol=1e-9)


def test_surrogate_force_derivative_matches_central_differences():
    rng = np.random.default_rng(7)
    p = _random_params(rng, 0.5)
    norm = (np.array([-1.0, -2.0, 3.0]), np.array([0.3, 0.5, 0.2]))
    b, mu, x, kT, sl = 0.03, 0.4, 2.0, 0.5, 0.35
    u = np.array([0.3, 2.0, 40.0, -0.3, -2.0, -40.0])
    sle = np.where(u >= 0, sl, 1 - sl)
    dF = mlp.surrogate_force_du(p, norm, u, sle, b, mu, x, kT)
    h = 1e-6 * np.maximum(1.0, np.abs(u))
    Fp = mlp.surrogate_rics(p, norm, u + h, sle, b, mu, x, kT)[0]
    Fm = mlp.surrogate_rics(p, norm, u - h, sle, b, mu, x, kT)[0]
    assert np.allclose((Fp - Fm) / (2 * h), dF, rtol=1e-6, atol=1e-12 * np.max(np.abs(Fp)))


def test_pic_step_with_the_surrogate_conserves_charge():
    from oracle import pic
    rng = np.random.default_rng(8)
    params = _random_params(rng, 0.3)
    cfg = pic.make_config(rics="mlp", mlp_params=params, mlp_norm=(np.array([0.0, 1.0, 2.0]),
                                                                    np.array([1.0, 1.0, 1.0])),
                          ppc0=8.0, lines=[dict(r_eq=4.0, n_cells=64, ppc_init=8, init="hot",
                                                init_gamma_max=1e3)])
    st = pic.init_state(cfg)
    stats = {}
    for _ in range(4):
        pic.step(st, stats)
    assert pic.gauss_residual(st, 0) < 1e-12
    assert st.counters[0]['events'] > 0


# ---------------------------------------------------------------------------
# the surrogate's error estimate on a line (the decision for its table fallback)
# ---------------------------------------------------------------------------
def _line_rows(R, b_pole, n_s):
    from oracle import geometry
    L = geometry.line_length(R)
    c = geometry.cos_of_s(R, (np.arange(n_s) + 0.5) / n_s * L)
    return geometry.field_b(b_pole, R, c), geometry.photon_mu(c), geometry.radius(R, c)


def _exact(scale_F=1.0, scale_N=1.0):
    def f(u, sl, b, mu, x, kT):
        return scale_F * rics.drag_force(u, b, mu, x, kT), scale_N * rics.scatter_rate(u, b, mu, x, kT)
    return f


def test_error_estimate_of_scaled_definitions_is_the_scale():
    b, mu, x = _line_rows(10.0, 10.0, 16)
    kw = dict(n_lg=64, kT=0.5, h=1e-3)
    assert mlp.line_error_estimate(None, None, b, mu, x, surrogate=_exact(), **kw) == 0.0
    e = mlp.line_error_estimate(None, None, b, mu, x, surrogate=_exact(1.0 + 3e-3, 1.0 - 1e-3), **kw)
    assert abs(e - 3e-3) < 1e-12
    e = mlp.line_error_estimate(None, None, b, mu, x, surrogate=_exact(1.0, 1.0 + 7e-3), **kw)
    assert abs(e - 7e-3) < 1e-12
    # a force of the wrong sign is off by 2
    assert abs(mlp.line_error_estimate(None, None, b, mu, x, surrogate=_exact(-1.0), **kw) - 2.0) < 1e-12


def test_error_estimate_counts_significant_nodes_only():
    b, mu, x = _line_rows(10.0, 10.0, 16)
    # with a vanishing step no node moves u or scatters enough to count
    assert mlp.line_error_estimate(None, None, b, mu, x, 64, 0.5, 1e-40, surrogate=_exact(5.0, 5.0)) == 0.0
    # non-finite output: no trust
    def nan_at_top(u, sl, bj, muj, xj, kT):
        F, N = _exact()(u, sl, bj, muj, xj, kT)
        return np.where(u == u.max(), np.nan, F), N
    e = mlp.line_error_estimate(None, None, b, mu, x, 64, 0.5, 1e3, surrogate=nan_at_top)
    assert e == np.inf


def test_error_estimate_feeds_each_row_its_own_arc_fraction():
    """A surrogate that rebuilds the geometry from s/L alone (the R_max = 4 line) is exact
    on that line's rows, and far off when the rows are handed in reversed."""
    from oracle import geometry
    R, bp, n_s = mlp.R_TRAIN, 10.0, 24

    def from_sl(u, sl, bj, muj, xj, kT):
        c = geometry.cos_of_s(R, sl * geometry.line_length(R))
        bb, mm, xx = geometry.field_b(bp, R, c), geometry.photon_mu(c), geometry.radius(R, c)
        return rics.drag_force(u, bb, mm, xx, kT), rics.scatter_rate(u, bb, mm, xx, kT)
    b, mu, x = _line_rows(R, bp, n_s)
    assert mlp.line_error_estimate(None, None, b, mu, x, 48, 0.5, 1e-3, surrogate=from_sl) < 1e-9
    e = mlp.line_error_estimate(None, None, b[::-1], mu[::-1], x[::-1], 48, 0.5, 1e-3, surrogate=from_sl)
    assert e > 0.5


def test_fallback_decision_per_line():
    """With a tolerance between two lines' estimates, the line above it takes its table."""
    from oracle import pic
    rng = np.random.default_rng(4)
    parts = []
    for li, (o, i) in enumerate(mlp.LAYERS):
        s = 0.15 if li == len(mlp.LAYERS) - 1 else 1.0
        parts.append((rng.uniform(-1, 1, (o, i)) * s * mlp.glorot_bound(o, i), rng.uniform(-0.1, 0.1, o)))
    p = mlp.pack(parts)
    _, O, _ = mlp.training_samples(seed=4, n=2048)
    mean, std = mlp.normalisation(O)
    base = dict(rics="mlp", mlp_params=p, mlp_norm=np.concatenate([mean, std]), table_nlg=32, table_ns=16,
                lines=[dict(r_eq=4.0, n_cells=64), dict(r_eq=40.0, n_cells=64)])
    st = pic.State(pic.make_config(mlp_fallback_tol=1e30, **base))
    e = [ln.mlp_error for ln in st.lines]
    assert all(np.isfinite(v) and v > 0 for v in e) and e[0] != e[1]
    assert not any(ln.use_table for ln in st.lines)
    tol = math.sqrt(e[0] * e[1])
    st = pic.State(pic.make_config(mlp_fallback_tol=tol, **base))
    assert [ln.use_table for ln in st.lines] == [v > tol for v in e]
    assert [ln.mlp_error for ln in st.lines] == e
    # without a tolerance no estimate is made and every line uses the network
    st = pic.State(pic.make_config(**base))
    assert all(ln.mlp_error is None and not ln.use_table for ln in st.lines)
