"""Pins of the oracle's gridded diagnostics and collision-probability probe.

Moments follow the definition M^[k] = (rho_d dV)^-1 sum N_i r_i^k over the
super-droplets of a cell whose radius lies in [r_min, r_max] (Sect. 5.2,
diagnostics of the particle-based scheme); the super-droplet concentration is
the number of live super-droplets per cell.  The probe returns the largest
P_ij (eq. P_ij) over the pairs one step would test.  Checks here are exact
integer sums, compensated (fsum) sums, brute-force range filters and closed
forms of P_ij for cells where every pairing gives the same probability.
"""
import math

import numpy as np
import pytest

from paper_1310_1905_amd import synth


def _state(oracle_mod, seed=3, n_cells=9, max_per_cell=300):
    pop = synth.tiny_cells(seed=seed, n_cells=n_cells, max_per_cell=max_per_cell)
    st = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    return pop, st


def _cells(st):
    off = st.offsets.astype(np.int64)
    return [(int(off[c]), int(off[c + 1])) for c in range(st.n_cells)]


def test_zeroth_moment_is_exact_multiplicity_sum(oracle_mod):
    _, st = _state(oracle_mod)
    m0 = st.moments(0)
    for c, (b, e) in enumerate(_cells(st)):
        total = sum(int(v) for v in st.xi[b:e])   # exact integer arithmetic
        assert total < 2**53
        assert m0[c] == float(total) / st.dV[c]


@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_moments_match_compensated_sum(oracle_mod, k):
    _, st = _state(oracle_mod, seed=5)
    mk = st.moments(k)
    for c, (b, e) in enumerate(_cells(st)):
        # r ** k as k products left to right, as the definition's r^k is formed
        terms = []
        for x, r in zip(st.xi[b:e], st.r[b:e]):
            rk = 1.0
            for _ in range(k):
                rk = rk * float(r)
            terms.append(float(x) * rk)
        exact = math.fsum(terms)
        # a plain left-to-right sum of n non-negative terms is within
        # (n - 1) 2^-53 (1 + O(n 2^-53)) of the exact sum; the division adds 2^-53
        n = e - b
        assert mk[c] == pytest.approx(exact / st.dV[c], rel=(n + 2) * 2.0 ** -53, abs=0.0)
        # and it is the sum taken in ascending slot order, term by term
        run = 0.0
        for t in terms:
            run = run + t
        assert mk[c] == run / st.dV[c]


def test_radius_range_is_inclusive_brute_force(oracle_mod):
    _, st = _state(oracle_mod, seed=7)
    # take bounds equal to radii present in the data so both ends are hit exactly
    r_sorted = np.sort(st.r[st.xi > 0])
    r_min, r_max = float(r_sorted[len(r_sorted) // 4]), float(r_sorted[3 * len(r_sorted) // 4])
    m3 = st.moments(3, r_min, r_max)
    for c, (b, e) in enumerate(_cells(st)):
        ref = math.fsum(float(x) * float(r) ** 3 for x, r in zip(st.xi[b:e], st.r[b:e])
                        if x > 0 and r_min <= r <= r_max)
        assert m3[c] == pytest.approx(ref / st.dV[c], rel=1e-13, abs=0.0)
    # an empty range gives exact zeros
    assert np.all(st.moments(3, 1.0, 2.0) == 0.0)
    # a reversed range is empty as well
    assert np.all(st.moments(0, r_max, r_min) == 0.0)


def test_dry_air_density_divides(oracle_mod):
    _, st = _state(oracle_mod, seed=9)
    rho = np.linspace(0.9, 1.2, st.n_cells)
    m0 = st.moments(0, rho_d=rho)
    for c, (b, e) in enumerate(_cells(st)):
        total = sum(int(v) for v in st.xi[b:e])
        assert m0[c] == float(total) / (rho[c] * st.dV[c])


def test_dead_super_droplets_are_ignored(oracle_mod):
    pop, st = _state(oracle_mod, seed=11)
    xi = st.xi.copy()
    xi[::3] = 0
    st.xi[:] = xi
    conc = st.sd_conc()
    m0 = st.moments(0)
    for c, (b, e) in enumerate(_cells(st)):
        assert conc[c] == int(np.count_nonzero(xi[b:e]))
        assert m0[c] == float(sum(int(v) for v in xi[b:e])) / st.dV[c]


def test_empty_cells(oracle_mod):
    st = oracle_mod.SlotState(np.array([2, 2], dtype=np.uint32), np.array([5, 7], dtype=np.uint64),
                              np.array([1e-5, 2e-5]), np.array([1.0, 2.0, 3.0, 4.0]))
    assert list(st.sd_conc()) == [0, 0, 2, 0]
    m = st.moments(3)
    assert m[0] == 0.0 and m[1] == 0.0 and m[3] == 0.0
    assert m[2] == pytest.approx((5 * 1e-15 + 7 * 8e-15) / 3.0, rel=1e-15)


def test_probe_closed_form_two_droplets(oracle_mod):
    """n = 2: one pair, upscale factor 1, P = max(N) b (v1 + v2) dt / dV."""
    b = oracle_mod.DEFAULT_PARAMS[0]
    r1, r2, x1, x2, dV, dt = 11e-6, 23e-6, 3_000_000, 1_000, 1e6, 2.0
    st = oracle_mod.SlotState(np.array([0, 0], dtype=np.uint32), np.array([x1, x2], dtype=np.uint64),
                              np.array([r1, r2]), np.array([dV]))
    v = lambda r: 4.0 / 3.0 * math.pi * r ** 3
    expect = max(x1, x2) * b * (v(r1) + v(r2)) * dt / dV
    got = st.max_probability(dt, oracle_mod.GOLOVIN, 1, 0)
    assert got == pytest.approx(expect, rel=1e-14)
    # P is linear in dt
    assert st.max_probability(3 * dt, oracle_mod.GOLOVIN, 1, 0) == pytest.approx(3 * got, rel=1e-14)


@pytest.mark.parametrize("n", [3, 4, 9, 64, 101])
def test_probe_closed_form_identical_droplets(oracle_mod, n):
    """Identical droplets: every pairing has the same P = N b 2v dt/dV n(n-1)/2/floor(n/2)."""
    b = oracle_mod.DEFAULT_PARAMS[0]
    r, x, dV, dt = 15e-6, 12345, 10.0, 1.0
    st = oracle_mod.SlotState(np.zeros(n, dtype=np.uint32), np.full(n, x, dtype=np.uint64),
                              np.full(n, r), np.array([dV]))
    v = 4.0 / 3.0 * math.pi * r ** 3
    expect = x * b * 2 * v * dt / dV * (n * (n - 1) / 2) / (n // 2)
    assert st.max_probability(dt, oracle_mod.GOLOVIN, 7, 3) == pytest.approx(expect, rel=1e-14)


def test_probe_is_max_over_the_steps_pairs(oracle_mod):
    """Brute force over the pairing the step draws (its order is pinned elsewhere)."""
    pop, st = _state(oracle_mod, seed=13, n_cells=5, max_per_cell=40)
    seed, step, dt = 99, 4, 0.7
    best = 0.0
    for c, (b, e) in enumerate(_cells(st)):
        order = oracle_mod.cell_order(st.xi[b:e], seed, c, step)
        n = len(order)
        for m in range(n // 2):
            ia, ib = b + int(order[2 * m]), b + int(order[2 * m + 1])
            xj = max(int(st.xi[ia]), int(st.xi[ib]))
            K = oracle_mod.kernel(oracle_mod.GEOMETRIC, float(st.r[ia]), float(st.r[ib]))
            best = max(best, xj * K * dt / st.dV[c] * (n * (n - 1) / 2) / (n // 2))
    got = st.max_probability(dt, oracle_mod.GEOMETRIC, seed, step)
    assert got == pytest.approx(best, rel=1e-14)
    # the probe leaves the state alone
    xi0, r0 = st.xi.copy(), st.r.copy()
    st.max_probability(dt, oracle_mod.GEOMETRIC, seed, step)
    assert np.array_equal(xi0, st.xi) and np.array_equal(r0, st.r)


def test_third_moment_conserved_over_golovin_run(oracle_mod):
    """Coalescence conserves liquid volume: M^[3] over the whole box stays put."""
    pop = synth.box_golovin(seed=synth.SEEDS[0])
    st = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    m3_0 = st.moments(3)[0]
    m0_0 = st.moments(0)[0]
    for t in range(200):
        st.step(pop.dt, oracle_mod.GOLOVIN, pop.seed, t)
    assert st.moments(3)[0] == pytest.approx(m3_0, rel=1e-12)
    assert st.moments(0)[0] < m0_0
    assert st.sd_conc()[0] == np.count_nonzero(st.xi)


def test_probe_per_cell_maxima(oracle_mod):
    """Per-cell maxima by brute force over each cell's pairing; 0 below two live SDs."""
    pop, st = _state(oracle_mod, seed=17, n_cells=6, max_per_cell=50)
    seed, step, dt = 5, 2, 1.3
    g, cm = st.max_probability(dt, oracle_mod.GOLOVIN, seed, step, per_cell=True)
    assert g == cm.max()
    for c, (b, e) in enumerate(_cells(st)):
        order = oracle_mod.cell_order(st.xi[b:e], seed, c, step)
        n = len(order)
        best = 0.0
        for m in range(n // 2):
            ia, ib = b + int(order[2 * m]), b + int(order[2 * m + 1])
            xj = max(int(st.xi[ia]), int(st.xi[ib]))
            K = oracle_mod.kernel(oracle_mod.GOLOVIN, float(st.r[ia]), float(st.r[ib]))
            best = max(best, xj * K * dt / st.dV[c] * (n * (n - 1) / 2) / (n // 2))
        assert cm[c] == pytest.approx(best, rel=1e-14, abs=0.0)
