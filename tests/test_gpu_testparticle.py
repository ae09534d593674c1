"""The test-particle map of Appendix A.4 (Fig. 6) on the GPU against the oracle's
Radau integration of the same equations (oracle/testparticle.py)."""
import numpy as np
import pytest

from oracle import testparticle as tp
from paper_2609_17661_amd import pic1d

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


RADII = (1.5, 2.0, 3.0, 4.0, 6.0, 10.0, 30.0, 100.0)


def test_sweep_matches_oracle_line_by_line():
    _print("GPU sweep of", len(RADII), "lines")
    g = pic1d.testparticle_sweep(np.array(RADII))
    for k, R in enumerate(RADII):
        o = tp.sweep_line(R)
        _print(f"R={R}: gpu gmin {g['gamma_min'][k]:.9g} s1 {g['s_first'][k]:.7g} lpp {g['l_pp'][k]:.7g} "
               f"crossed {g['crossed'][k]} steps {g['steps'][k]}; oracle gmin {o['gamma_min']:.9g} "
               f"s1 {o['s_first']} lpp {o['l_pp']:.7g} crossed {o['crossed']}")
        assert g["L"][k] == pytest.approx(o["L"], rel=1e-13)
        assert bool(g["crossed"][k]) == o["crossed"]
        if o["crossed"]:
            assert g["gamma_min"][k] == pytest.approx(o["gamma_min"], rel=1e-5)
        else:
            assert g["gamma_min"][k] - 1.0 < 1e-3 and abs(g["gamma_min"][k] - o["gamma_min"]) < 1e-4
        assert o["s_first"] is not None
        assert g["s_first"][k] == pytest.approx(o["s_first"], abs=2e-4)
        if o["s_b"] is None:
            assert g["s_b"][k] == -1.0
        else:
            assert g["s_b"][k] == pytest.approx(o["s_b"], abs=1e-10)
        assert g["l_pp"][k] == pytest.approx(o["l_pp"], abs=4e-4)


def test_sweep_over_the_magnetosphere_shows_the_papers_regions():
    """64 lines from r_eq = 1.2 to 40 R* (Fig. 6's test-particle map): the pair zone
    grows over the shortest lines, then falls to about 2 R*; gamma_min > 1 on the
    short lines and ~1 beyond a critical radius."""
    R = np.geomspace(1.2, 40.0, 64)
    g = pic1d.testparticle_sweep(R)
    k_peak = int(np.argmax(g["l_pp"]))
    crit = R[np.argmax(~g["crossed"])] if (~g["crossed"]).any() else None
    _print("l_pp peak", g["l_pp"][k_peak], "at r_eq", R[k_peak], "; first line stopped at the equator:", crit)
    _print("r_eq, gamma_min, l_pp:", list(zip(np.round(R, 3), np.round(g["gamma_min"], 4), np.round(g["l_pp"], 3))))
    assert 0 < k_peak < 63
    assert np.all(np.diff(g["l_pp"][:k_peak + 1]) > -1e-9)
    # the sharp fall right after the peak, to about 2 R* (Fig. 6 top), then a slow decline
    after = g["l_pp"][k_peak + 1:k_peak + 12]
    assert after.max() < 0.5 * g["l_pp"][k_peak] and np.all((after > 1.8) & (after < 2.7))
    assert np.all(np.diff(g["l_pp"][k_peak + 1:]) < 1e-9)
    assert crit is not None and 3.0 < crit < 8.0
    assert np.all(g["gamma_min"][R < 3.0] > 2.0)
    assert np.all(g["gamma_min"][(R > 6.0) & (R < 30.0)] - 1.0 < 1e-3)
