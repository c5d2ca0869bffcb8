"""Parity of the split tier (a workgroup-tier cell spread over 2^block_split
workgroups by the top key bits; changed SDs written at once, multiplicities that
drop to zero once every workgroup of the cell has read) with the FP64 oracle,
through the C ABI.

Bar: pairing order, multiplicities, radii, dry attributes, counters and the
per-cell probe maxima all bit-exact.  Cases: cells of 65 to 8192 slots with dead
slots and every split from 2 to 32 workgroups (so that digits with no live SD,
and cells where one workgroup holds every live SD, occur); the release rules
with dry attributes, where equal multiplicities leave slots empty within the
step; the 8192-SD Golovin box over many steps; the rule that batches take no
split; and the time-out path of the wait, forced from the host.
"""
import numpy as np
import pytest

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu

RELEASE = 1


def _bits_equal(a, b):
    return np.array_equal(np.ascontiguousarray(a, np.float64).view(np.uint64),
                          np.ascontiguousarray(b, np.float64).view(np.uint64))


def _assert_same(ctx, ref, what):
    xi_g, r_g = ctx.state_numpy()
    xi_o, r_o = ref.input_order()
    assert np.array_equal(xi_g, xi_o), what
    assert _bits_equal(r_g, r_o), what
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1])), what


def _cells(g, sizes, dead=0.05, xi_hi=40):
    cell = np.repeat(np.arange(len(sizes), dtype=np.uint32), sizes)
    n = cell.size
    xi = g.integers(1, xi_hi, n).astype(np.uint64)
    xi[g.random(n) < dead] = 0
    r = np.exp(g.uniform(np.log(5e-6), np.log(2e-3), n))
    dV = g.uniform(1e-3, 1.0, len(sizes))
    return cell, xi, r, dV


@pytest.mark.parametrize("split", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("kernel", ["geometric", "golovin"])
def test_split_cells(sdm_mod, oracle_mod, kernel, split):
    g = np.random.default_rng(900 + split)
    sizes = [65, 100, 513, 2047, 2049, 3000, 8191, 8192, 40, 600, 64, 4000]
    cell, xi, r, dV = _cells(g, sizes)
    xi[np.repeat(np.arange(len(sizes)), sizes) == 11] = 0      # a dead cell
    xi[np.flatnonzero(cell == 3)[:2040]] = 0                   # 7 live SDs in 2047 slots
    kind = oracle_mod.GOLOVIN if kernel == "golovin" else oracle_mod.GEOMETRIC
    ctx = sdm_mod.Context(cell, xi, r, dV)
    ctx.set_launch_config(group_slots=64, block_slots=8192, block_split=split)
    assert ctx.launch_config().block_split == split
    assert ctx.plan()[1:] == (2, 10, 0)
    ref = oracle_mod.SlotState(cell, xi, r, dV)
    order, nlive = ctx.permutation(seed=11, step=4)
    order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
    off = ref.offsets.astype(np.int64)
    for c in range(len(sizes)):
        exp = oracle_mod.cell_order(ref.xi[off[c]:off[c] + sizes[c]], 11, c, 4)
        assert nlive[c] == exp.size, c
        assert np.array_equal(order[off[c]:off[c] + exp.size], exp), (sizes[c], split)
    gmax, cm = ctx.probe(2.0, kernel, 11, 3, per_cell=True)
    gref, cref = ref.max_probability(2.0, kind, 11, 3, per_cell=True)
    assert _bits_equal(cm.cpu().numpy(), cref)
    assert _bits_equal([gmax], [gref])
    for t in range(4):
        ctx.step(2.0, kernel, 11, t)
        ref.step_parallel(2.0, kind, 11, t, threads=8)
    _assert_same(ctx, ref, f"split {split} {kernel}")
    assert ref.stats[1] > 0


@pytest.mark.parametrize("split", [1, 3, 5])
def test_split_release_rules_with_dry_attributes(sdm_mod, oracle_mod, split):
    """Multiplicities of 1..3 make equal pairs common: under the release rules
    they leave one member empty within the step."""
    g = np.random.default_rng(77 + split)
    sizes = [300, 1000, 5000, 8192]
    cell, xi, r, dV = _cells(g, sizes, dead=0.02, xi_hi=4)
    dV = dV * 1e-6
    rd3 = (r * g.uniform(0.05, 0.2, r.size)) ** 3
    kappa = g.uniform(0.1, 1.3, r.size)
    ctx = sdm_mod.Context(cell, xi, r, dV)
    ctx.attach_dry(rd3, kappa)
    ctx.set_rules(RELEASE)
    ctx.set_launch_config(group_slots=256, block_slots=8192, block_split=split)
    ref = oracle_mod.SlotState(cell, xi, r, dV)
    ref.set_dry(rd3, kappa)
    for t in range(6):
        ctx.step(1.0, "geometric", 5, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, 5, t, rules=oracle_mod.RULE_FIDELITY)
    _assert_same(ctx, ref, f"release + dry, split {split}")
    rd3_g, k_g = ctx.dry()
    rd3_o, k_o = ref.dry_input_order()
    assert _bits_equal(rd3_g.cpu().numpy(), rd3_o)
    assert _bits_equal(k_g.cpu().numpy(), k_o)
    assert np.count_nonzero(ref.input_order()[0] == 0) > np.count_nonzero(xi == 0)


def test_split_golovin_box_many_steps(sdm_mod, oracle_mod):
    """The 8192-SD Golovin box, 300 steps with 8 workgroups, against the oracle."""
    pop = synth.box_golovin(seed=synth.SEEDS[0])
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.set_launch_config(group_slots=64, block_slots=8192, block_split=3)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    for t in range(300):
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
        ref.step(pop.dt, oracle_mod.GOLOVIN, pop.seed, t)
    _assert_same(ctx, ref, "box")


def test_split_rejected_where_it_does_not_apply(sdm_mod):
    pop = synth.tiny_cells(seed=3, n_cells=10, max_per_cell=20)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    for bad in (dict(block_split=6), dict(block_slots=0, group_slots=512, block_split=1)):
        with pytest.raises(sdm_mod.SdmError) as e:
            ctx.set_launch_config(**bad)
        assert e.value.status == -1
    b = sdm_mod.Batch(1000, 16, 4)
    with pytest.raises(sdm_mod.SdmError) as e:
        b.set_launch_config(block_split=1)
    assert e.value.status == -1
    assert b.launch_config().block_split == 0
    b.close()


def test_split_wait_time_out_is_reported(sdm_mod, oracle_mod):
    """The time-out path of the zero-multiplicity wait, forced from the host: the
    context's split-step count is skewed so that the wait's target is never met,
    with a poll limit of 64.  Steps still finish (every wait gives up), the writes
    happen anyway, so the state equals the oracle's here (all workgroups had in fact
    read long before), and sdm_get_stats reports the time-outs as an error."""
    g = np.random.default_rng(31)
    sizes = [3000, 5000]
    cell, xi, r, dV = _cells(g, sizes, dead=0.0, xi_hi=2)      # all xi = 1: zeros every step
    dV = dV * 1e-7
    ctx = sdm_mod.Context(cell, xi, r, dV)
    ctx.set_rules(RELEASE)
    ctx.set_launch_config(group_slots=256, block_slots=8192, block_split=2)
    ref = oracle_mod.SlotState(cell, xi, r, dV)
    ctx.step(1.0, "geometric", 9, 0)
    ref.step(1.0, oracle_mod.GEOMETRIC, 9, 0, rules=oracle_mod.RULE_FIDELITY)
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1]))   # no time-out yet
    ctx.debug_split_wait(64, epoch_skew=1000)
    for t in range(1, 3):
        ctx.step(1.0, "geometric", 9, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, 9, t, rules=oracle_mod.RULE_FIDELITY)
    with pytest.raises(sdm_mod.SdmError) as e:
        ctx.stats()
    assert e.value.status == -3 and "timed out" in str(e.value)
    xi_g, r_g = ctx.state_numpy()
    xi_o, r_o = ref.input_order()
    assert np.array_equal(xi_g, xi_o) and _bits_equal(r_g, r_o)
    assert np.count_nonzero(xi_o == 0) > 0
