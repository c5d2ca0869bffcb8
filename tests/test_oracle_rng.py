"""Pins of the oracle's random numbers: Philox4x32-10 against its published
known-answer vectors and against rocRAND's independent implementation; the
shuffle-key and pair-uniform definitions; the open-interval uniform mapping."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], tuple(v[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(oracle_mod, ctr, key, expect):
    assert oracle_mod.philox4x32_10(ctr, key) == expect


@pytest.fixture(scope="module")
def rocrand_ref():
    src = os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")
    out_dir = os.path.join(HERE, "helpers", "_build")
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "librocrand_philox_ref.so")
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available to build the rocRAND reference")
        subprocess.check_call([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-fPIC", "-shared",
                               "-o", lib, src])
    L = ctypes.CDLL(lib)
    L.rocrand_philox_ref.argtypes = [ctypes.c_void_p] * 3
    L.rocrand_philox_ref.restype = None
    return L


def test_philox_matches_rocrand(oracle_mod, rocrand_ref):
    g = np.random.default_rng(7)
    for _ in range(3000):
        c = g.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        k = g.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        out = np.zeros(4, np.uint32)
        rocrand_ref.rocrand_philox_ref(c.ctypes.data, k.ctypes.data, out.ctypes.data)
        assert oracle_mod.philox4x32_10(c, k) == tuple(int(x) for x in out)


def test_shuffle_key_is_word_of_counter_block(oracle_mod):
    seed = 0x0123456789ABCDEF
    for cell, step in [(0, 0), (5, 17), (2 ** 32 - 1, 2 ** 32 - 1)]:
        for s in range(12):
            w = oracle_mod.philox4x32_10([s // 4, cell, step, 0],
                                         [seed & 0xFFFFFFFF, seed >> 32])
            assert oracle_mod.shuffle_key(seed, cell, step, s) == w[s % 4]


def test_pair_uniform_definition_and_range(oracle_mod):
    seed = 987654321
    for m in range(8):
        w = oracle_mod.philox4x32_10([m // 2, 3, 9, 1], [seed & 0xFFFFFFFF, seed >> 32])
        hi, lo = w[2 * (m % 2)], w[2 * (m % 2) + 1]
        k = ((hi << 32) | lo) >> 12
        u = oracle_mod.pair_uniform(seed, 3, 9, m)
        assert u == (2 * k + 1) / 2.0 ** 53
        assert 0.0 < u < 1.0


def test_uniform_extremes_stay_open():
    # the mapping (2k+1) 2^-53 with k in [0, 2^52) is exact and never 0 or 1
    lo = (2 * 0 + 1) / 2.0 ** 53
    hi = (2 * (2 ** 52 - 1) + 1) / 2.0 ** 53
    assert lo > 0.0 and hi < 1.0
    assert float(2 * (2 ** 52 - 1) + 1) == 2 ** 53 - 1      # exactly representable


def test_uniforms_look_uniform(oracle_mod):
    us = np.array([oracle_mod.pair_uniform(42, c, 0, m) for c in range(50) for m in range(40)])
    # Kolmogorov-Smirnov against U(0,1)
    from scipy import stats
    assert stats.kstest(us, "uniform").pvalue > 1e-3


def test_philox_range_is_the_single_call(oracle_mod):
    """The counter-range form (used to check the device on 2^30 counters) is the
    single Philox call on counter (c0 + lo32(i), c1 + hi32(i), c2, c3), words
    modulo 2^32 (across the wrap of the first word as well)."""
    for ctr, key in (([5, 7, 9, 11], [3, 4]), ([0xFFFFFFF0, 0xFFFFFFFF, 1, 2], [0xFFFFFFFF, 0])):
        out = oracle_mod.philox_range(1000, ctr, key, threads=3)
        for i in (0, 1, 15, 16, 17, 500, 999):
            c = [(ctr[0] + i) & 0xFFFFFFFF, ctr[1], ctr[2], ctr[3]]
            assert tuple(int(v) for v in out[i]) == oracle_mod.philox4x32_10(c, key), (ctr, i)
