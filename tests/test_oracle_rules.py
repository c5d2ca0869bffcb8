"""Pins of the oracle's release-rule mode and recycling (Sect. 5.1.4).

Release rule: a collision happens when the uniform deviate is below P_ij and
then exactly one event takes place; equal multiplicities collide by the same
scheme and leave the larger (first) particle with multiplicity zero.
Recycling (at the start of a step, within each cell): zero-multiplicity
particles take the radius and half the multiplicity of the live particles with
the highest multiplicities.

Checks: hand-worked outcomes, number and volume bookkeeping, a worked
recycling example, invariants of recycling on random cells (multiplicity per
radius value conserved exactly, donors are the top-ranked particles), the
coincidence of the two rule sets when P_ij < 1 and no multiplicities are equal,
and the Golovin analytic number decay with the release rule plus recycling.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_1310_1905_amd import synth


def test_gamma_release_rule(oracle_mod):
    assert oracle_mod.gamma_fidelity(0.3, 0.2) == 1
    assert oracle_mod.gamma_fidelity(0.3, 0.3) == 0      # strictly below
    assert oracle_mod.gamma_fidelity(0.3, 0.7) == 0
    assert oracle_mod.gamma_fidelity(7.5, 0.999) == 1    # never more than one event
    assert oracle_mod.gamma_fidelity(0.0, 2.0 ** -53) == 0


def test_release_outcomes_hand_worked(oracle_mod):
    cbrt9 = oracle_mod.cbrt_rn(9.0)
    # unequal: j loses xi_k, k takes the merged radius, r_j unchanged
    assert oracle_mod.collide_pair_fidelity(1, 10, 1.0, 3, 2.0) == (7, 1.0, 3, cbrt9)
    # equal: j is left with zero multiplicity
    assert oracle_mod.collide_pair_fidelity(1, 5, 1.0, 5, 2.0) == (0, 1.0, 5, cbrt9)
    # no event
    assert oracle_mod.collide_pair_fidelity(0, 5, 1.0, 5, 2.0) == (5, 1.0, 5, 2.0)


def test_release_outcome_conserves_volume(oracle_mod):
    g = np.random.default_rng(1)
    for _ in range(200):
        xk = int(g.integers(1, 10 ** 6))
        xj = xk + int(g.integers(0, 10 ** 6))
        rj, rk = float(g.uniform(1e-6, 1e-3)), float(g.uniform(1e-6, 1e-3))
        a, ra, b, rb = oracle_mod.collide_pair_fidelity(1, xj, rj, xk, rk)
        assert a + b == xj    # xi_k droplets disappear into the merged ones
        v0 = xj * rj ** 3 + xk * rk ** 3
        assert abs(a * ra ** 3 + b * rb ** 3 - v0) <= 1e-14 * v0


def test_recycle_worked_example(oracle_mod):
    # dead slots 0, 3, 5; live ranked by multiplicity: slot 6 (8), 1 (5), 2 (3), 4 (1).
    # The three top donors in slot order (1, 2, 6) feed dead slots (0, 3, 5).
    xi, r, n = oracle_mod.recycle_cell([0, 5, 3, 0, 1, 0, 8], [1., 2., 3., 4., 5., 6., 7.])
    assert n == 3
    assert list(xi) == [2, 3, 2, 1, 1, 4, 4]
    assert list(r) == [2., 2., 3., 3., 5., 7., 7.]


def test_recycle_limits(oracle_mod):
    # donors with multiplicity 1 cannot be split
    xi, r, n = oracle_mod.recycle_cell([0, 1, 0, 1], [1., 2., 3., 4.])
    assert n == 0 and list(xi) == [0, 1, 0, 1]
    # more dead than live: only as many as there are donors
    xi, r, n = oracle_mod.recycle_cell([0, 0, 0, 9, 0], [1., 2., 3., 4., 5.])
    assert n == 1 and list(xi) == [4, 0, 0, 5, 0] and r[0] == 4.0
    # ties in multiplicity go to the lower slot
    xi, r, n = oracle_mod.recycle_cell([6, 0, 6, 6], [1., 2., 3., 4.])
    assert n == 1 and list(xi) == [3, 3, 6, 6] and r[1] == 1.0
    # nothing dead or nothing alive
    assert oracle_mod.recycle_cell([3, 4], [1., 2.])[2] == 0
    assert oracle_mod.recycle_cell([0, 0], [1., 2.])[2] == 0
    assert oracle_mod.recycle_cell([], [])[2] == 0


@pytest.mark.parametrize("seed", range(6))
def test_recycle_invariants(oracle_mod, seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 300))
    xi0 = g.integers(1, 20, n).astype(np.uint64)
    xi0[g.random(n) < g.uniform(0.0, 0.8)] = 0
    r0 = np.round(g.uniform(1, 50, n))   # few distinct radii, so donors share them
    xi1, r1, nrec = oracle_mod.recycle_cell(xi0, r0)
    # multiplicity carried by each radius value is unchanged (exact integers)
    for v in np.unique(r0):
        assert int(xi0[r0 == v].sum()) == int(xi1[r1 == v].sum())
    dead0 = np.nonzero(xi0 == 0)[0]
    live0 = np.nonzero(xi0 > 0)[0]
    take = min(len(dead0), len(live0))
    ranked = sorted(live0, key=lambda s: (-int(xi0[s]), s))[:take]
    donors = sorted(s for s in ranked if xi0[s] >= 2)
    assert nrec == len(donors)
    for d, t in zip(donors, dead0[:nrec]):
        assert xi1[t] == xi0[d] // 2 and xi1[d] == xi0[d] - xi0[d] // 2 and r1[t] == r0[d]
    untouched = np.setdiff1d(np.arange(n), np.concatenate([donors, dead0[:nrec]]).astype(int))
    assert np.array_equal(xi1[untouched], xi0[untouched])


def test_rules_coincide_without_ties_and_below_one(oracle_mod):
    """With P_ij < 1 and all multiplicities distinct, both rule sets agree exactly."""
    g = np.random.default_rng(5)
    n_cells, per = 40, 60
    cell = np.repeat(np.arange(n_cells, dtype=np.uint32), per)
    xi = g.permutation(np.arange(1000, 1000 + n_cells * per)).astype(np.uint64) * 1000
    r = np.exp(g.uniform(np.log(5e-6), np.log(1e-4), cell.size))
    dV = np.full(n_cells, 1.5)
    a = oracle_mod.SlotState(cell, xi, r, dV)
    b = oracle_mod.SlotState(cell, xi, r, dV)
    assert a.max_probability(0.2, oracle_mod.GEOMETRIC, 3, 0) < 1.0
    a.step(0.2, oracle_mod.GEOMETRIC, 3, 0)
    b.step(0.2, oracle_mod.GEOMETRIC, 3, 0, rules=oracle_mod.RULE_FIDELITY)
    assert a.stats[1] > 100
    assert np.array_equal(a.xi, b.xi) and np.array_equal(a.r, b.r)


def _run_release(oracle_mod, seed, rules):
    pop = synth.box_golovin(seed=seed)
    st = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    snaps = {}
    for t in range(2400):
        st.step(pop.dt, oracle_mod.GOLOVIN, pop.seed, t, rules=rules)
        if t + 1 in (1200, 2400):
            snaps[t + 1] = (st.xi.copy(), st.r.copy())
    return pop, snaps


def test_release_rules_golovin_number_decay(oracle_mod):
    """The release rule with recycling follows N(t) = N0 exp(-b N0 v0 t) while P_ij
    stays mostly below one, conserving volume; recycling keeps few slots dead."""
    rules = oracle_mod.RULE_FIDELITY | oracle_mod.RULE_RECYCLE
    with ThreadPoolExecutor(8) as ex:
        runs = list(ex.map(lambda s: _run_release(oracle_mod, s, rules), synth.SEEDS[:8]))
    pop = runs[0][0]
    N0, v0, b = pop.meta["N0"], pop.meta["v0"], pop.meta["b"]
    B = b * N0 * v0
    for t in (1200, 2400):
        ratios = [sn[t][0].astype(np.float64).sum() / float(pop.dV[0]) / (N0 * np.exp(-B * t))
                  for _, sn in runs]
        assert abs(float(np.mean(ratios)) - 1.0) < 0.03, (t, ratios)
        for p, sn in runs:
            xi, r = sn[t]
            v_init = float(np.sum(p.xi.astype(np.float64) * p.r ** 3))
            assert abs(float(np.sum(xi.astype(np.float64) * r ** 3)) - v_init) <= 1e-12 * v_init
            assert np.count_nonzero(xi == 0) < 0.01 * xi.size
