"""CPU checks of the C ABI: the library loads and exports every declared symbol;
host-only calls validate configs.  No kernel is launched."""
import ctypes
import os
import re

import pytest

import paper_2609_17661_amd as pkg
from paper_2609_17661_amd import pic1d, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pic1d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic1d_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pic1d.lib_path()):
        pytest.fail("libpic1d.so is not built (run __graft_entry__.build())")
    return pic1d.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "pic1d_init" in names and "pic1d_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(pic1d.EXPORTED) | set(getattr(pic1d, "EXPORTED_EXTRA", ()))


def test_workspace_size_of_benchmark_configs(lib):
    small = pkg.workspace_size(workloads.CFG1)
    big = pkg.workspace_size(workloads.CFG2)
    assert 1e6 < small < 1e8
    # two SoA copies of 20-byte particles for 1e8 slots dominate
    assert 3.5e9 < big < 6e9


@pytest.mark.parametrize("bad", [
    dict(cfl=0.7), dict(ppc0=0.0), dict(rics="table", table_nlg=1),
    dict(lines=[dict(r_eq=0.5, n_cells=64)]), dict(lines=[dict(r_eq=4.0, n_cells=1)]),
    dict(mass_ratio=0.5),
])
def test_invalid_configs_are_rejected(lib, bad):
    cfg = dict(workloads.CFG1)
    cfg.update(bad)
    with pytest.raises(pic1d.Pic1dError) as ei:
        pkg.workspace_size(cfg)
    assert ei.value.code == -1


def test_unknown_emission_pattern_is_rejected(lib):
    c, keep = pic1d.make_cconfig(pic1d.complete_config(dict(workloads.CFG1, emission="dipole")))
    n = ctypes.c_size_t(0)
    assert lib.pic1d_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
    c.emission = 3
    assert lib.pic1d_workspace_size(ctypes.byref(c), ctypes.byref(n)) == -1
    assert b"emission" in lib.pic1d_last_error(None)
    with pytest.raises(KeyError):
        pkg.workspace_size(dict(workloads.CFG1, emission="beamed"))


def test_null_state_calls_fail_cleanly(lib):
    assert lib.pic1d_step(None, 1) == -1
    lib.pic1d_free(None)
    assert isinstance(lib.pic1d_last_error(None), bytes)
