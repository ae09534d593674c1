"""Pins of oracle/philox.py: published known-answer vectors and rocRAND's
independent open-source Philox4x32-10, built for the host by the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(t, 16) for t in line.split()])
    return rows


def test_known_answer_vectors():
    for r in _kat():
        out = philox.philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(o) for o in out] == r[6:10]


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe,
                    os.path.join(HERE, "philox_rocrand_ref.cpp")],
                   check=True, capture_output=True, cwd="/tmp")
    return exe


def test_against_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(12345)
    n = 2000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctr[:10, 1:] = 0           # small counters as used by the method
    inp = "\n".join(" ".join(f"{int(v):x}" for v in list(c) + list(k)) for c, k in zip(ctr, key))
    res = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(t, 16) for t in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    for i in range(n):
        out = philox.philox4x32_10(ctr[i, 0], ctr[i, 1], ctr[i, 2], ctr[i, 3], key[i, 0], key[i, 1])
        assert [int(o) for o in out] == [int(v) for v in ref[i]]


def test_vectorised_matches_scalar_and_uniform_range():
    c1 = np.arange(1000, dtype=np.uint64)
    w = philox.philox4x32_10(7, c1, 3, philox.STREAM_RICS, 11, 0)
    for i in (0, 1, 500, 999):
        s = philox.philox4x32_10(7, int(c1[i]), 3, philox.STREAM_RICS, 11, 0)
        assert [int(x[i]) for x in w] == [int(x) for x in s]
    U = philox.uniform24(w[0])
    assert U.min() >= 0.0 and U.max() < 1.0
    assert np.all(U * 2 ** 24 == np.floor(U * 2 ** 24))
    V = philox.uniform24_open0(w[1])
    assert V.min() > 0.0 and V.max() <= 1.0
    assert abs(U.mean() - 0.5) < 0.05


def test_ids_are_tagged_and_split_roundtrip():
    pid = philox.id_from_words(np.uint32(0x89abcdef), np.uint32(0x01234567))
    assert int(pid) == (1 << 63) | 0x0123456789abcdef
    lo, hi = philox.split_id(pid)
    assert int(lo) == 0x89abcdef and int(hi) == (0x01234567 | 0x80000000)
