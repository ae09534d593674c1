"""The finite stellar disk's RICS table (Sec. 5), built on the GPU by the cone
quadrature, against the oracle's table of the same rule (oracle/disk.py)."""
import numpy as np
import pytest

from oracle import pic, rics
from paper_2609_17661_amd import Pic1D, workloads

from . import parity

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("r_eq,n_cells", [(4.0, 128), (30.0, 200)])
def test_disk_table_matches_oracle_at_nodes_and_between(r_eq, n_cells):
    import torch
    nlg, ns = 48, 40
    cfg = workloads.small(r_eq=r_eq, n_cells=n_cells, ppc=1, init="empty", rics="table", table_nlg=nlg,
                          table_ns=ns, photon_field="disk")
    cfg["lines"][0]["capacity"] = [256, 256, 0, 0]
    _print("disk table", r_eq, n_cells)
    sim = Pic1D(cfg)
    ln = pic.Line(parity.oracle_config(cfg), 0, cfg["lines"][0], 0)
    rng = np.random.default_rng(5)
    # the table nodes (row centres, log10 gamma nodes), then random points, both signs of u
    lg, s_rows = rics.table_axes(nlg, ns, float(n_cells))
    S, G = np.meshgrid(s_rows, 10.0 ** lg, indexing="ij")
    s_pts = np.concatenate([S.ravel(), rng.uniform(0, n_cells, 20000)])
    g_pts = np.concatenate([G.ravel(), 10.0 ** rng.uniform(0, 8, 20000)])
    u = np.sqrt(np.maximum(g_pts ** 2 - 1.0, 0.0)) * np.where(rng.random(g_pts.size) < 0.5, -1.0, 1.0)
    s32 = s_pts.astype(np.float32)
    u32 = u.astype(np.float32)
    F, N, _ = (t.cpu().numpy().astype(np.float64) for t in sim.rics_eval(0, torch.from_numpy(s32),
                                                                       torch.from_numpy(u32)))
    Fo, No, _ = rics.table_lookup(ln.F_tab, ln.N_tab, u32.astype(np.float64), s32.astype(np.float64), float(n_cells))
    # float32 table values and a float32 column and row weight: the error is a few
    # ulps of the largest of the four corners the bilinear lookup reads (near the
    # Planck cutoff the next column can be 1e5 times the interpolated value, and a
    # weight off by 1e-6 of a column moves the result by 1e-6 of that corner)
    def corner_max(T, uu, xs):
        neg = uu < 0.0
        ua = np.abs(uu)
        sx = np.where(neg, float(n_cells) - xs, xs)
        fi = np.clip(np.log10(np.sqrt(1.0 + ua * ua)) * ((nlg - 1) / 8.0), 0.0, nlg - 1)
        fj = np.clip(sx * (ns / float(n_cells)) - 0.5, 0.0, ns - 1)
        i0 = np.minimum(np.floor(fi).astype(np.int64), nlg - 2)
        j0 = np.minimum(np.floor(fj).astype(np.int64), ns - 2)
        A = np.abs(T)
        return np.maximum.reduce([A[i0, j0], A[i0 + 1, j0], A[i0, j0 + 1], A[i0 + 1, j0 + 1]])

    uu = u32.astype(np.float64)
    xs = s32.astype(np.float64)
    cF = corner_max(ln.F_tab, uu, xs)
    cN = corner_max(ln.N_tab, uu, xs)
    nzF = cF > 0
    nzN = cN > 0
    errF = np.abs(F - Fo)[nzF] / cF[nzF]
    errN = np.abs(N - No)[nzN] / cN[nzN]
    _print("  F err (of the largest corner) median/99%/max", np.median(errF), np.quantile(errF, 0.99), errF.max(),
           "N max", errN.max(), "points", nzF.sum())
    assert nzF.sum() > 10000 and nzN.sum() > 10000
    assert errF.max() < 1e-5 and errN.max() < 1e-5
    np.testing.assert_array_equal(F[~nzF], 0.0)
    np.testing.assert_array_equal(N[~nzN], 0.0)
    # and the disk differs from the radial beam (the model is switched on)
    rad = dict(cfg, photon_field="radial")
    ln_r = pic.Line(parity.oracle_config(rad), 0, rad["lines"][0], 0)
    assert np.abs(ln_r.N_tab - ln.N_tab).max() > 1e-3 * np.abs(ln.N_tab).max()
