"""The device arithmetic of the bit-exact path, pinned element by element on large
random samples through the C ABI:

* the step's square root (terminal velocity above 600 um) and its division
  (eq. (P_ij)) against numpy's IEEE-754 binary64 results (correctly rounded), on
  2^30 inputs: half with random bit patterns over every positive finite binary64
  (all exponents, subnormals included), half in the ranges the method meets
  (radii and probability numerators over many decades, cell volumes 1e-3..1e7);
* Philox4x32-10 on 2^30 counters (all four counter words and the key varied
  between chunks) against the oracle's implementation.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

CHUNK = 1 << 26
CHUNKS = 16          # 2^30 elements in all


def _random_positive_finite(g, n):
    bits = g.integers(1, 0x7FEFFFFFFFFFFFFF, n, dtype=np.uint64, endpoint=True)
    return bits.view(np.float64)


def _log_uniform(g, lo, hi, n):
    return np.exp(g.uniform(np.log(lo), np.log(hi), n))


def test_sqrt_and_division_2e30(sdm_mod):
    g = np.random.default_rng(20251203)
    for c in range(CHUNKS):
        if c % 2 == 0:
            a = _random_positive_finite(g, CHUNK)
            b = _random_positive_finite(g, CHUNK)
        else:
            a = _log_uniform(g, 1e-30, 1e10, CHUNK)
            b = _log_uniform(g, 1e-3, 1e7, CHUNK)
        at = torch.from_numpy(a).cuda()
        bt = torch.from_numpy(b).cuda()
        sq, q = sdm_mod.debug_sqrt_div(at, bt)
        sq = sq.cpu().numpy()
        q = q.cpu().numpy()
        with np.errstate(over="ignore", under="ignore"):
            sq_ref = np.sqrt(a)
            q_ref = a / b
        bad_s = np.count_nonzero(sq.view(np.uint64) != sq_ref.view(np.uint64))
        bad_q = np.count_nonzero(q.view(np.uint64) != q_ref.view(np.uint64))
        assert bad_s == 0, f"chunk {c}: {bad_s} square roots differ"
        assert bad_q == 0, f"chunk {c}: {bad_q} quotients differ"
        del at, bt
    torch.cuda.empty_cache()


def test_philox_2e30_counters(sdm_mod, oracle_mod):
    g = np.random.default_rng(777)
    out = torch.empty((CHUNK, 4), dtype=torch.int32, device="cuda")
    for c in range(CHUNKS):
        ctr = [int(v) for v in g.integers(0, 1 << 32, 4, dtype=np.uint64)]
        key = [int(v) for v in g.integers(0, 1 << 32, 2, dtype=np.uint64)]
        if c == 0:
            ctr, key = [0, 0, 0, 0], [0, 0]
        elif c == 1:
            ctr, key = [0xFFFFFFFF - (CHUNK // 2)] + [0xFFFFFFFF] * 3, [0xFFFFFFFF] * 2
        dev = sdm_mod.debug_philox_range(CHUNK, ctr, key, out).cpu().numpy().view(np.uint32)
        ref = oracle_mod.philox_range(CHUNK, ctr, key, threads=16)
        bad = np.count_nonzero(np.any(dev != ref, axis=1))
        assert bad == 0, f"chunk {c} (counter {ctr}, key {key}): {bad} calls differ"
