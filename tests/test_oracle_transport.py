"""Pins of the oracle's particle transport (Sect. 5.1: advection by the
backward-Euler scheme with its analytic solution on an Arakawa-C grid, periodic
in x; sedimentation by explicit Euler; particles leaving the domain flagged with
zero multiplicity) and of the stable re-sort by cell that follows it.

Checks: the uniform-flow and linear-flow closed forms of backward Euler, the
use of the time-level-n cell, periodic wrap, the fall of small drops at
k1 r^2, leaving through the bottom, stability and completeness of the re-sort,
and exact conservation of the number of droplets under the incompressible eddy.
"""
import numpy as np
import pytest

from paper_1310_1905_amd import synth


def test_uniform_flow_is_a_shift(oracle_mod):
    for x, i, c in [(5.0, 0, 0.1), (37.5, 1, -0.3), (1499.0, 74, 0.25)]:
        assert oracle_mod.advect_1d(x, 20.0, i, c, c) == x + 20.0 * c


@pytest.mark.parametrize("a,b", [(0.3, 0.01), (-0.5, 0.02), (0.2, -0.03)])
def test_linear_flow_matches_backward_euler(oracle_mod, a, b):
    """u(x) = a + b x inside the cell: x' = x + dt u(x') gives x' = (x + a dt) / (1 - b dt)."""
    d, dt = 20.0, 1.0
    g = np.random.default_rng(1)
    for _ in range(100):
        i = int(g.integers(0, 50))
        x = (i + float(g.random())) * d
        cl = (a + b * i * d) * dt / d
        cr = (a + b * (i + 1) * d) * dt / d
        got = oracle_mod.advect_1d(x, d, i, cl, cr)
        exp = (x + a * dt) / (1.0 - b * dt)
        assert got == pytest.approx(exp, rel=1e-12, abs=1e-12)


def _one(oracle_mod, x, z, xi, r, nx=4, nz=3, d=10.0):
    cell = np.array([min(int(v // d), nx - 1) + nx * min(int(w // d), nz - 1)
                     for v, w in zip(x, z)], dtype=np.uint32)
    st = oracle_mod.SlotState(cell, np.array(xi, dtype=np.uint64), np.array(r, dtype=np.float64),
                              np.full(nx * nz, 1.0))
    st.set_positions(x, z, nx, nz, d, d)
    return st


def test_cell_of_time_level_n_and_periodic_wrap(oracle_mod):
    nx, nz, d = 4, 3, 10.0
    cx = np.zeros(nz * nx)
    cx[1 * nx + 3] = 0.5      # left edge of cell (3, 1)
    cx[1 * nx + 0] = 0.9      # edge 0 of row 1 == right edge of cell (3, 1)
    st = _one(oracle_mod, [38.0], [15.0], [7], [1e-5])
    st.transport(cx, None, 1.0, sediment=False)
    # x' = (38 + 10 (0.5 - 3 * 0.4)) / (1 - 0.4) = 51.666..., wrapped by 40
    exp = (38.0 + 10.0 * (0.5 - 3.0 * 0.4)) / (1.0 - 0.4) - 40.0
    assert st.x[0] == exp and st.z[0] == 15.0
    assert list(st.offsets[1:] - st.offsets[:-1]).index(1) == 1 + nx * 1   # cell (1, 1)
    # negative motion wraps the other way
    cx2 = np.full(nz * nx, -0.3)
    st = _one(oracle_mod, [1.0], [5.0], [7], [1e-5])
    st.transport(cx2, None, 1.0, sediment=False)
    assert st.x[0] == 1.0 + 10.0 * -0.3 + 40.0


def test_sedimentation_and_leaving_the_domain(oracle_mod):
    k1 = oracle_mod.DEFAULT_PARAMS[1]
    r = [10e-6, 30e-6, 20e-6]
    st = _one(oracle_mod, [5.0, 15.0, 25.0], [0.01, 25.0, 29.0], [3, 4, 5], r)
    st.transport(None, None, 2.0, sediment=True)
    x, z = st.positions_input_order()
    xi, _ = st.input_order()
    # first drop: 0.1 - k1 r^2 dt < 0 -> leaves through the bottom
    assert 0.01 - k1 * r[0] ** 2 * 2.0 < 0.0
    assert xi[0] == 0 and z[0] == 0.0
    assert z[1] == 25.0 - k1 * r[1] ** 2 * 2.0 and xi[1] == 4
    assert z[2] == 29.0 - k1 * r[2] ** 2 * 2.0 and xi[2] == 5
    # leaving through the top is also flagged
    cz = np.full(4 * 4, 0.9)
    st = _one(oracle_mod, [5.0], [29.5], [3], [1e-5])
    st.transport(None, cz, 1.0, sediment=False)
    xi, _ = st.input_order()
    assert xi[0] == 0 and st.z[0] == 20.0


def test_resort_is_stable_and_complete(oracle_mod):
    g = np.random.default_rng(3)
    nx, nz, d = 8, 6, 20.0
    n = 3000
    cell = g.integers(0, nx * nz, n).astype(np.uint32)
    pop = synth.Population("t", cell, g.integers(1, 9, n).astype(np.uint64),
                           g.uniform(1e-6, 1e-4, n), np.full(nx * nz, 1.0), "golovin", 1.0, 1, 0)
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=4)
    st = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    st.set_positions(x, z, nx, nz, d, d)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 5.0, w_max=2.0)
    before = st.id.copy()
    pos_before = {int(i): s for s, i in enumerate(before)}
    st.transport(cx, cz, 5.0, sediment=False)
    assert sorted(st.id.tolist()) == list(range(n))
    off = st.offsets.astype(np.int64)
    for c in range(nx * nz):
        ids = st.id[off[c]:off[c + 1]]
        prev = [pos_before[int(i)] for i in ids]
        assert prev == sorted(prev)          # old storage order kept within a cell
        i = np.clip(np.floor(st.x[off[c]:off[c + 1]] / d), 0, nx - 1)
        k = np.clip(np.floor(st.z[off[c]:off[c + 1]] / d), 0, nz - 1)
        assert np.all(i + nx * k == c)


def test_eddy_is_divergence_free(oracle_mod):
    nx, nz, d = 75, 75, 20.0
    cx, cz = synth.eddy_courant(nx, nz, d, d, 1.0)
    cx = cx.reshape(nz, nx)
    cz = cz.reshape(nz + 1, nx)
    div = (np.roll(cx, -1, axis=1) - cx) + (cz[1:] - cz[:-1])
    assert np.abs(div).max() < 1e-15
    assert np.all(cz[0] == 0.0) and np.abs(cz[-1]).max() < 1e-15
    assert np.abs(cx).max() < 0.1


def test_eddy_conserves_droplets_and_keeps_uniform_density(oracle_mod):
    pop = synth.domain_2d(seed=synth.SEEDS[2], nx=20, ny=20, per_cell=32)
    nx = nz = 20
    d = 20.0
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=5)
    st = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    st.set_positions(x, z, nx, nz, d, d)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 2.0, w_max=1.0)
    total = int(st.xi.sum())
    for _ in range(60):
        st.transport(cx, cz, 2.0, sediment=False)
    assert int(st.xi.sum()) == total
    counts = (st.offsets[1:] - st.offsets[:-1]).astype(np.float64)
    # incompressible flow keeps the density uniform: Poisson-like spread around 32
    assert abs(counts.mean() - 32.0) < 1e-9
    assert counts.std() < 3.0 * np.sqrt(32.0)
