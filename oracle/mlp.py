"""FP64 oracle of the RICS surrogate network: forward, backward, Adam, targets.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper evaluates the RICS drag force and scattering rate from their
definitions (Sec. 2.2, Eqs. scatteringNdot and contdrag) and proposes no
surrogate; the network here is an addition whose targets are those
definitions.  What it computes:

  inputs   (log10 gamma, s/L, log10 b, kT/keV) on the box
           [0, 8] x [0, 1] x [-2, 3] x [0.3, 1], mapped affinely to [-1, 1];
           s/L is the arc-length fraction along the R_max = 4 dipole line
           (Appendix B.2), which fixes mu and x = r/R*; b is an independent
           field strength, so the network covers a family of B_pole values;
  network  4 -> 128 -> 128 -> 128 -> 128 -> 3, SiLU after each hidden layer
           (z/(1+e^-z)), linear output; 50,563 parameters; the forward pass
           uses the weights rounded to bfloat16 (round to nearest even) and the
           biases in full precision;
  outputs  normalised targets t_k = (o_k - mean_k)/std_k of
             o1 = log10(|F_hat| / |gamma mu - u|) = log10(A_F g(y) / x^2)
             o2 = log10(Ndot_hat)
             o3 = log10(eps),  eps = gamma (1 - (1+2b)^-1/2)   (Appendix A.3)
           for u >= 0; F_hat = (gamma mu - u) 10^o1 carries its exact sign, and
           u < 0 uses the mirror F(-u, s) = -F(u, L - s).  Where the resonance
           parameter y exceeds the Planck cutoff the definitions are exactly
           zero and the network is not used;
  loss     mean over samples and outputs of the squared error of t;
  Adam     Kingma & Ba (2015), Algorithm 1, with bias correction.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss
against the backward pass; Adam's closed-form step for a constant gradient;
bfloat16 rounding against torch's conversion and hand-worked ties; a sparse
network whose output is a known composition of SiLUs (catches transposed or
reordered layers); the targets against rics.drag_force, rics.scatter_rate and
rics.photon_energy; the sample generator's inputs against the Philox
definition.
"""
import math

import numpy as np

from . import geometry, philox, rics

N_IN = 4
N_OUT = 3
WIDTH = 128
LAYERS = ((WIDTH, N_IN), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (N_OUT, WIDTH))   # (out, in)
N_PARAM = sum(o * i + o for o, i in LAYERS)          # 50,563
IN_LO = np.array([0.0, 0.0, -2.0, 0.3])
IN_HI = np.array([8.0, 1.0, 3.0, 1.0])
R_TRAIN = 4.0                                        # dipole line of the training geometry
STREAM_MLP_SAMPLE = 7
MAX_ATTEMPTS = 64


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def unpack(params):
    """Flat vector -> [(W (out x in), b (out)), ...] in layer order (row-major W, then b)."""
    params = np.asarray(params, dtype=np.float64)
    if params.shape != (N_PARAM,):
        raise ValueError(f"expected {N_PARAM} parameters, got {params.shape}")
    out, k = [], 0
    for o, i in LAYERS:
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16_round(x):
    """Round float32 values to bfloat16 (8-bit significand), nearest even; returned as float64.

    NaN is passed through; finite values that round past the largest bfloat16
    become infinities, as IEEE rounding prescribes.
    """
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    r = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def forward_weights(params, round_weights=True):
    """Weights as the forward pass uses them: W rounded (via float32) to bfloat16, b unrounded."""
    if not round_weights:
        return [(W.copy(), b.copy()) for W, b in unpack(params)]
    return [(bf16_round(W), b.copy()) for W, b in unpack(params)]


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def sigmoid(z):
    """1/(1+e^-z), evaluated without cancellation for either sign of z."""
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def normalize_inputs(X):
    """(log10 gamma, s/L, log10 b, kT) -> [-1, 1]^4."""
    X = np.asarray(X, dtype=np.float64)
    return 2.0 * (X - IN_LO) / (IN_HI - IN_LO) - 1.0


def forward(params, Xn, round_weights=True):
    """Network output (normalised targets) for normalised inputs Xn (n x 4), and the cache."""
    a = np.asarray(Xn, dtype=np.float64)
    layers = forward_weights(params, round_weights)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = silu(z) if li < len(layers) - 1 else z
    return a, cache


def loss_and_grad(params, Xn, T, round_weights=True):
    """Mean squared error over the n x 3 outputs and its gradient (flat, same packing).

    The gradient is taken with respect to the weights the forward pass uses
    (the bfloat16 values), which is the gradient applied to the master weights.
    """
    T = np.asarray(T, dtype=np.float64)
    out, cache = forward(params, Xn, round_weights)
    n = out.shape[0]
    diff = out - T
    L = float(np.sum(diff * diff)) / (n * N_OUT)
    layers = forward_weights(params, round_weights)
    d = 2.0 * diff / (n * N_OUT)             # dL/dz of the output layer
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        a_in, z = cache[li]
        W, _ = layers[li]
        if li < len(layers) - 1:
            d = d * silu_grad(z)
        grads[li] = (d.T @ a_in, d.sum(axis=0))
        d = d @ W
    return L, pack(grads)


def input_grad(params, Xn):
    """d(output_k)/d(Xn_j) of the network at normalised inputs Xn: array n x 3 x 4."""
    out, cache = forward(params, Xn)
    layers = forward_weights(params)
    n = out.shape[0]
    J = np.zeros((n, N_OUT, N_IN))
    for k in range(N_OUT):
        d = np.zeros((n, N_OUT))
        d[:, k] = 1.0
        for li in range(len(layers) - 1, -1, -1):
            _, z = cache[li]
            if li < len(layers) - 1:
                d = d * silu_grad(z)
            d = d @ layers[li][0]
        J[:, k, :] = d
    return J


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); t counts from 1.  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# targets and the surrogate RICS functions
# ---------------------------------------------------------------------------

def line_geometry(s_over_L, R=R_TRAIN):
    """(mu, x) at the arc-length fraction s/L of the dipole line r = R sin^2 theta."""
    L = geometry.line_length(R)
    c = geometry.cos_of_s(R, np.asarray(s_over_L, dtype=np.float64) * L)
    return geometry.photon_mu(c), geometry.radius(R, c)


def targets(X, R=R_TRAIN):
    """(o1, o2, o3, y) of inputs X = (log10 gamma, s/L, log10 b, kT), u >= 0."""
    X = np.asarray(X, dtype=np.float64)
    lg, sl, lb, kT = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
    gam = 10.0 ** lg
    u = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    b = 10.0 ** lb
    mu, x = line_geometry(sl, R)
    y = rics.resonance_y(u, b, mu, kT)
    A_F, A_N = rics.prefactors(kT)
    f2, f3 = rics._planck_factors(y)
    with np.errstate(divide="ignore"):
        o1 = np.log10(A_F * f3 / (x * x))
        o2 = np.log10(A_N * f2 / (x * x * gam))
        o3 = np.log10(rics.photon_energy(u, b))
    return o1, o2, o3, y


def training_samples(seed, n, first=0, R=R_TRAIN):
    """Inputs and exact targets of samples first .. first+n-1 of the seeded sample stream.

    Sample i takes the first attempt a = 0, 1, ... whose Philox block
    (counter (i_lo, i_hi, a, STREAM_MLP_SAMPLE), key = seed) gives y within the
    Planck cutoff; the four words map to log10 gamma = 8 U0, s/L = U1,
    log10 b = -2 + 5 U2 and kT = 0.3 + 0.7 U3 (U = 24-bit uniforms), each
    formed in float64 and stored as float32.  Returns (X float32 n x 4,
    O float64 n x 3, attempts used).
    """
    k0, k1 = philox.seed_key(seed)
    idx = np.arange(first, first + n, dtype=np.uint64)
    lo = (idx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (idx >> np.uint64(32)).astype(np.uint32)
    X = np.zeros((n, N_IN), dtype=np.float32)
    O = np.zeros((n, N_OUT))
    used = np.full(n, -1, dtype=np.int64)
    todo = np.arange(n)
    for a in range(MAX_ATTEMPTS):
        if todo.size == 0:
            break
        w = philox.philox4x32_10(lo[todo], hi[todo], a, STREAM_MLP_SAMPLE, k0, k1)
        cand = np.stack([
            (8.0 * philox.uniform24(w[0])).astype(np.float32),
            philox.uniform24(w[1]).astype(np.float32),
            (-2.0 + 5.0 * philox.uniform24(w[2])).astype(np.float32),
            (0.3 + 0.7 * philox.uniform24(w[3])).astype(np.float32)], axis=1)
        o1, o2, o3, y = targets(cand.astype(np.float64), R)
        ok = y <= rics.Y_CUTOFF
        sel = todo[ok]
        X[sel] = cand[ok]
        O[sel] = np.stack([o1[ok], o2[ok], o3[ok]], axis=1)
        used[sel] = a
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("sample stream exhausted its attempts")
    return X, O, used


def surrogate_rics(params, norm, u, s_over_L_eff, b, mu, x, kT):
    """(F_hat, Ndot_hat, eps) of the surrogate at momenta u for particles with geometry (b, mu, x).

    s_over_L_eff is the arc-length fraction of the particle for u >= 0 and of its
    mirror point (1 - s/L) for u < 0.  norm = (mean[3], std[3]).  Beyond the
    Planck cutoff F and Ndot are exactly zero, as in the definitions.
    """
    u = np.asarray(u, dtype=np.float64)
    ua = np.abs(u)
    gam = np.sqrt(1.0 + ua * ua)
    mean, std = norm
    X = np.stack([np.log10(gam), np.asarray(s_over_L_eff, dtype=np.float64) * np.ones_like(u),
                  np.log10(b) * np.ones_like(u), kT * np.ones_like(u)], axis=1)
    out, _ = forward(params, normalize_inputs(X))
    o = out * std + mean
    y = rics.resonance_y(u, b, mu, kT)
    inside = y <= rics.Y_CUTOFF
    F = np.where(inside, (gam * mu - u) * 10.0 ** o[:, 0], 0.0)
    N = np.where(inside, 10.0 ** o[:, 1], 0.0)
    eps = 10.0 ** o[:, 2]
    return F, N, eps


def surrogate_force_du(params, norm, u, s_over_L_eff, b, mu, x, kT):
    """dF_hat/du of the surrogate force (u of either sign), by the chain rule through the network.

    F = w G with w = gamma mu - u and G = 10^(o1(log10 gamma)):
    dF/du = -(1 - beta mu) G + w G ln(10) (do1/dlog10 gamma) (dlog10 gamma/du) for u >= 0,
    with dlog10 gamma/du = beta/(gamma ln 10) and do1/dlog10 gamma = std_1 (d out_1/d Xn_0) 2/8.
    For u < 0, F(u, s) = -F(|u|, L - s) with mu(L - s) = -mu(s), so dF/du(u) equals the
    u >= 0 derivative at |u| with mu replaced by -mu.
    """
    u = np.asarray(u, dtype=np.float64)
    ua = np.abs(u)
    gam = np.sqrt(1.0 + ua * ua)
    beta_a = ua / gam
    mean, std = norm
    X = np.stack([np.log10(gam), np.asarray(s_over_L_eff, dtype=np.float64) * np.ones_like(u),
                  np.log10(b) * np.ones_like(u), kT * np.ones_like(u)], axis=1)
    Xn = normalize_inputs(X)
    out, _ = forward(params, Xn)
    G = 10.0 ** (out[:, 0] * std[0] + mean[0])
    dO1 = input_grad(params, Xn)[:, 0, 0] * std[0] * 2.0 / (IN_HI[0] - IN_LO[0])
    # evaluate the u >= 0 form at |u| with the mirrored geometry mu_eff = sign(u) mu
    mu_eff = np.where(u >= 0, mu, -mu)
    w = gam * mu_eff - ua
    dFa = -(1.0 - beta_a * mu_eff) * G + w * G * dO1 * beta_a / gam
    y = rics.resonance_y(u, b, mu, kT)
    return np.where(y <= rics.Y_CUTOFF, dFa, 0.0)


def line_error_estimate(params, norm, b, mu, x, n_lg, kT, h, surrogate=None):
    """Largest relative error of the surrogate against the definitions on one line's table nodes.

    The nodes are those of the line's RICS table (log10 gamma_i = 8 i/(n_lg - 1),
    rows at arc-length fractions (j + 1/2)/n_s with geometry (b, mu, x)[j]), u >= 0;
    the definitions are Eqs. contdrag and scatteringNdot.  A node counts for the
    force where the exact force moves u by at least 1e-9 max(u, 1) in one step of
    length h (R*/c), for the rate where it gives at least 1e-9 scatterings a step.  A
    non-finite network output counts as an infinite error.  surrogate(u, s/L, b,
    mu, x, kT) -> (F_hat, Ndot_hat) replaces the network (for the pins).
    """
    if surrogate is None:
        def surrogate(u, sl, bj, muj, xj, kT_):
            F, N, _ = surrogate_rics(params, norm, u, sl, bj, muj, xj, kT_)
            return F, N
    b, mu, x = (np.asarray(a, dtype=np.float64) for a in (b, mu, x))
    n_s = b.shape[0]
    gam = 10.0 ** (8.0 * np.arange(n_lg, dtype=np.float64) / (n_lg - 1))
    u = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    worst = 0.0
    for j in range(n_s):
        F, N = surrogate(u, (j + 0.5) / n_s, b[j], mu[j], x[j], kT)
        Fe = rics.drag_force(u, b[j], mu[j], x[j], kT)
        Ne = rics.scatter_rate(u, b[j], mu[j], x[j], kT)
        sf = (np.abs(Fe) * h >= 1e-9 * np.maximum(u, 1.0)) & (Fe != 0.0)
        sn = Ne * h >= 1e-9
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            ef = np.abs(F[sf] - Fe[sf]) / np.abs(Fe[sf])
            en = np.abs(N[sn] - Ne[sn]) / Ne[sn]
        e = np.concatenate([ef, en])
        if e.size:
            e = np.where(np.isfinite(e), e, np.inf)
            worst = max(worst, float(e.max()))
    return worst


def normalisation(O):
    """Per-output mean and standard deviation of a sample set (the normalisation of the targets)."""
    O = np.asarray(O, dtype=np.float64)
    mean = O.mean(axis=0)
    std = np.sqrt(np.mean((O - mean) ** 2, axis=0))
    return mean, std


def mlp_flops_per_eval():
    """Multiply-adds x 2 of one evaluation."""
    return 2 * sum(o * i for o, i in LAYERS)


def glorot_bound(fan_out, fan_in):
    return math.sqrt(6.0 / (fan_in + fan_out))
