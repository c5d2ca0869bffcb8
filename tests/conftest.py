"""Shared fixtures.  GPU tests carry ``@pytest.mark.gpu``; everything else runs on CPU."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libsdm.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def sdm_mod():
    """The HIP binding; GPU tests only."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a HIP device")
    from paper_1310_1905_amd import sdm
    sdm.lib()
    return sdm


def _moments_close(got, exp, slots_per_cell):
    """Per-cell moments from the device against the oracle's plain in-order sum.

    Both sides form the same non-negative terms xi r^k (k products left to right)
    and divide by the same rho_d dV; only the order of the additions differs.  Any
    order of recursive summation of n non-negative terms lies within
    (n-1) 2^-53 (1 + O(n 2^-53)) of the exact sum, relative, so two orders differ by
    at most 2(n-1) 2^-53 of it, and each side's division adds 2^-53: a cell of n
    slots must agree to (2n + 4) 2^-53 relative.  A cell with no term is 0 on both
    sides exactly."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    n = np.asarray(slots_per_cell, dtype=np.float64)
    assert got.shape == exp.shape
    tol = (2.0 * n + 4.0) * 2.0 ** -53 * np.abs(exp)
    bad = np.nonzero(~(np.abs(got - exp) <= tol))[0]
    assert bad.size == 0, (f"{bad.size} cells outside (2n+4) 2^-53; first {bad[:5]}: "
                           f"{got[bad[:5]]} vs {exp[bad[:5]]}")
    assert np.array_equal(got == 0.0, exp == 0.0)


@pytest.fixture(scope="session")
def moments_close():
    return _moments_close
