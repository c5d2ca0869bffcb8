"""Parity of the gridded diagnostics, the collision-probability probe and the
sub-stepping entry points with the FP64 oracle, through the C ABI.

Bar: super-droplet concentrations and sub-step counts exact; probabilities
bit-exact (both sides evaluate eq. (P_ij) in the same order without
contraction); moments within (2n + 4) 2^-53 relative of the oracle's plain
in-order sum for a cell of n slots (the device adds in a wavefront-parallel
order; see the moments_close fixture); states after fixed or adaptive
sub-stepping bit-exact.  Cases span all three kernel tiers (cells of a few,
hundreds and tens of thousands of storage slots), empty, single-SD and dead-SD
cells, radius ranges hitting data values, dry-air density, and the large
domain at full size (1024 x 1024 cells, ~134M SDs).
"""
import math

import numpy as np
import pytest
import torch

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu


def _pair(sdm_mod, oracle_mod, pop, dV_scale=1.0):
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV * dV_scale)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV * dV_scale)
    return ctx, ref


def _bits_equal(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _assert_state(ctx, ref, what):
    xi_g, r_g = ctx.state_numpy()
    xi_o, r_o = ref.input_order()
    assert np.array_equal(xi_g, xi_o), what
    assert _bits_equal(r_g, r_o), what


CASES = [(60, 200), (600, 120), (40000, 3)]   # (max slots per cell, cells): wave, block, grid tiers


@pytest.mark.parametrize("max_per_cell,n_cells", CASES)
def test_sd_conc_and_moments(sdm_mod, oracle_mod, moments_close, max_per_cell, n_cells):
    pop = synth.tiny_cells(seed=900 + max_per_cell, n_cells=n_cells, max_per_cell=max_per_cell,
                           dead_fraction=0.2)
    ctx, ref = _pair(sdm_mod, oracle_mod, pop)
    assert np.array_equal(ctx.sd_conc().cpu().numpy().astype(np.uint32), ref.sd_conc())
    r_live = np.sort(ref.r[ref.xi > 0])
    r_lo, r_hi = float(r_live[len(r_live) // 5]), float(r_live[4 * len(r_live) // 5])
    rho = np.linspace(0.8, 1.25, n_cells)
    for k, lo, hi, dens in [(0, 0.0, math.inf, None), (1, 0.0, math.inf, None),
                            (3, 0.0, math.inf, rho), (6, r_lo, r_hi, None), (2, r_lo, r_hi, rho),
                            (3, r_hi, r_lo, None), (16, 0.0, math.inf, None)]:
        got = ctx.moments(k, lo, hi, rho_d=dens).cpu().numpy()
        exp = ref.moments(k, lo, hi, rho_d=dens)
        moments_close(got, exp, np.diff(ref.offsets))


def test_moments_follow_the_state(sdm_mod, oracle_mod, moments_close):
    pop = synth.tiny_cells(seed=77, n_cells=300, max_per_cell=300, xi_max=50)
    ctx, ref = _pair(sdm_mod, oracle_mod, pop, dV_scale=1e-4)
    for t in range(25):
        ctx.step(2.0, "geometric", pop.seed, t)
        ref.step(2.0, oracle_mod.GEOMETRIC, pop.seed, t)
    for k in (0, 3):
        moments_close(ctx.moments(k).cpu().numpy(), ref.moments(k), np.diff(ref.offsets))
    assert np.array_equal(ctx.sd_conc().cpu().numpy().astype(np.uint32), ref.sd_conc())


@pytest.mark.parametrize("max_per_cell,n_cells", CASES)
@pytest.mark.parametrize("kernel", ["geometric", "golovin"])
def test_probe_matches_oracle(sdm_mod, oracle_mod, kernel, max_per_cell, n_cells):
    kind = oracle_mod.GOLOVIN if kernel == "golovin" else oracle_mod.GEOMETRIC
    pop = synth.tiny_cells(seed=910 + max_per_cell, n_cells=n_cells, max_per_cell=max_per_cell,
                           dead_fraction=0.15)
    ctx, ref = _pair(sdm_mod, oracle_mod, pop)
    xi0, r0 = ctx.state_numpy()
    for step in (0, 5, 2 ** 32 - 1):
        g, cm = ctx.probe(1.5, kernel, 4242, step, per_cell=True)
        g_o, cm_o = ref.max_probability(1.5, kind, 4242, step, per_cell=True)
        assert _bits_equal(cm.cpu().numpy(), cm_o), step
        assert _bits_equal([g], [g_o]), step
        assert g == float(cm_o.max())
    xi1, r1 = ctx.state_numpy()
    assert np.array_equal(xi0, xi1) and _bits_equal(r0, r1)
    # a step after probing is the plain step
    ctx.step(1.5, kernel, 4242, 5)
    ref.step(1.5, kind, 4242, 5)
    _assert_state(ctx, ref, "step after probe")


def test_probe_of_empty_and_dead_cells(sdm_mod, oracle_mod):
    cell = np.array([1, 1, 3, 3, 3], dtype=np.uint32)
    xi = np.array([0, 5, 0, 0, 0], dtype=np.uint64)
    r = np.array([1e-5, 2e-5, 3e-5, 4e-5, 5e-5])
    dV = np.ones(5)
    ctx = sdm_mod.Context(cell, xi, r, dV)
    g, cm = ctx.probe(1.0, "golovin", 1, 0, per_cell=True)
    assert g == 0.0 and np.all(cm.cpu().numpy() == 0.0)
    assert list(ctx.sd_conc().cpu().numpy()) == [0, 1, 0, 0, 0]


@pytest.mark.parametrize("n_sub", [1, 4, 10])
def test_fixed_substeps(sdm_mod, oracle_mod, n_sub):
    pop = synth.tiny_cells(seed=31, n_cells=150, max_per_cell=700, xi_max=40)
    ctx, ref = _pair(sdm_mod, oracle_mod, pop, dV_scale=1e-4)
    ctx.substeps(4.0, n_sub, "geometric", pop.seed, 100)
    h = 4.0 / n_sub
    for i in range(n_sub):
        ref.step(h, oracle_mod.GEOMETRIC, pop.seed, 100 + i)
    _assert_state(ctx, ref, f"substeps {n_sub}")
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1]))


def test_adaptive_substeps(sdm_mod, oracle_mod):
    pop = synth.tiny_cells(seed=41, n_cells=200, max_per_cell=500, xi_max=1000)
    ctx, ref = _pair(sdm_mod, oracle_mod, pop)
    step, seen = 0, set()
    for dt, p_limit in [(0.02, 0.5), (0.5, 0.5), (2.0, 0.5), (50.0, 0.2), (1e-6, 0.5), (1.0, 0.1)]:
        n = ctx.adaptive(dt, p_limit, 64, "geometric", pop.seed, step)
        pmax = ref.max_probability(dt, oracle_mod.GEOMETRIC, pop.seed, step)
        n_exp = 1 if not pmax > p_limit else min(64, math.ceil(pmax / p_limit))
        assert n == n_exp, (dt, p_limit, pmax)
        for i in range(n):
            ref.step(dt / n, oracle_mod.GEOMETRIC, pop.seed, step + i)
        step += n
        seen.add(n)
        _assert_state(ctx, ref, f"adaptive dt={dt}")
    assert 1 in seen and 64 in seen and len(seen) >= 4
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1]))


def test_invalid_arguments(sdm_mod):
    pop = synth.tiny_cells(seed=3, n_cells=10, max_per_cell=20)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    with pytest.raises(sdm_mod.SdmError):
        ctx.moments(17)
    with pytest.raises(sdm_mod.SdmError):
        ctx.moments(3, float("nan"), 1.0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.substeps(1.0, 0, "golovin", 1, 0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.substeps(1.0, 3, "golovin", 1, 2 ** 32 - 2)
    with pytest.raises(sdm_mod.SdmError):
        ctx.adaptive(1.0, 0.0, 4, "golovin", 1, 0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.adaptive(1.0, 0.5, 0, "golovin", 1, 0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.probe(-1.0, "golovin", 1, 0)


def test_full_size_domain(sdm_mod, oracle_mod, moments_close):
    """1024 x 1024 cells, ~134M SDs."""
    pop = synth.large_domain(seed=synth.SEEDS[0])
    kind = oracle_mod.GOLOVIN if pop.kernel == "golovin" else oracle_mod.GEOMETRIC
    ctx, ref = _pair(sdm_mod, oracle_mod, pop)
    ctx.autotune(pop.dt, pop.kernel, seed=pop.seed ^ 0x5A5A, reps=3)   # as bench.py selects it
    moments_close(ctx.moments(3).cpu().numpy(), ref.moments(3), np.diff(ref.offsets))
    assert np.array_equal(ctx.sd_conc().cpu().numpy().astype(np.uint32), ref.sd_conc())
    g = ctx.probe(pop.dt, pop.kernel, pop.seed, 0)
    g_o = ref.max_probability(pop.dt, kind, pop.seed, 0)
    assert _bits_equal([g], [g_o])
    del ctx
    torch.cuda.empty_cache()
