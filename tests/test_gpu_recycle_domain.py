"""Parity of the domain-wide recycling (the recycling procedure of Sect. 5.1.4
over all cells, leavers of Sect. 5.1.5 included) with the FP64 oracle, through
the C ABI.

Bar: storage layout (offsets and slot -> input index), positions, multiplicities,
radii, dry attributes and the recycled-slot count all bit-exact.  Cases: one cell
without positions (stepped under the release rules: the per-cell procedure),
explicit recycling of random domains with positions (dead fractions from a few to
most slots, tied and 40-bit multiplicities so that the radix selection of the
threshold takes several passes, donors of multiplicity one), transport with
sedimentation and dry attributes stepped under the release rules with
domain-wide recycling, and the rule checks.
"""
import numpy as np
import pytest

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu

RELEASE, RECYCLE, RECYCLE_DOMAIN = 1, 2, 4


def _bits_equal(a, b):
    return np.array_equal(np.ascontiguousarray(a, np.float64).view(np.uint64),
                          np.ascontiguousarray(b, np.float64).view(np.uint64))


def _assert_same(ctx, ref, what, positions=True, dry=False):
    if positions:
        off, idx = ctx.layout()
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), ref.offsets), what
        assert np.array_equal(idx.cpu().numpy().astype(np.uint64), ref.id), what
        xg, zg = ctx.positions()
        xo, zo = ref.positions_input_order()
        assert _bits_equal(xg.cpu().numpy(), xo), what
        assert _bits_equal(zg.cpu().numpy(), zo), what
    xi_g, r_g = ctx.state_numpy()
    xi_o, r_o = ref.input_order()
    assert np.array_equal(xi_g, xi_o), what
    assert _bits_equal(r_g, r_o), what
    if dry:
        rd3_g, k_g = ctx.dry()
        rd3_o, k_o = ref.dry_input_order()
        assert _bits_equal(rd3_g.cpu().numpy(), rd3_o), what
        assert _bits_equal(k_g.cpu().numpy(), k_o), what
    assert ctx.recycled() == int(getattr(ref, "recycled", 0)), what


def test_one_cell_steps(sdm_mod, oracle_mod):
    """A Golovin box under the release rules with domain-wide recycling, 80 steps."""
    pop = synth.box_golovin(seed=synth.SEEDS[4], n_sd=2 ** 12)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.set_rules(RELEASE | RECYCLE_DOMAIN)
    for t in range(80):
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
        ref.step(pop.dt, oracle_mod.GOLOVIN, pop.seed, t,
                 rules=oracle_mod.RULE_FIDELITY | oracle_mod.RULE_RECYCLE_DOMAIN)
    _assert_same(ctx, ref, "box", positions=False)
    assert ctx.recycled() > 0
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1]))


@pytest.mark.parametrize("case", range(10))
def test_explicit_recycling_random_domains(sdm_mod, oracle_mod, case):
    g = np.random.default_rng(7000 + case)
    nx, nz, d = int(g.integers(1, 9)), int(g.integers(1, 9)), 10.0
    n = int(g.integers(2, 12000)) if case < 8 else 150000
    x = g.uniform(0, nx * d, n)
    z = g.uniform(0, nz * d, n)
    if case % 3 == 0:
        xi = g.integers(1, 6, n).astype(np.uint64)                 # many ties, some ones
    elif case % 3 == 1:
        xi = g.integers(1, 1 << 40, n, dtype=np.uint64)            # several radix passes
    else:
        xi = (g.integers(1, 50, n) * 1000003).astype(np.uint64)    # few distinct, large
    xi[g.random(n) < g.uniform(0.02, 0.8)] = 0
    r = np.round(g.uniform(1, 60, n)) * 1e-6
    cell = (np.floor(x / d) + nx * np.floor(z / d)).astype(np.uint32)
    print(f"case {case}: {n} SDs, {nx} x {nz} cells", flush=True)
    ctx = sdm_mod.Context(cell, xi, r, np.ones(nx * nz))
    ref = oracle_mod.SlotState(cell, xi, r, np.ones(nx * nz))
    ctx.attach_transport(x, z, nx, nz, d, d)
    ref.set_positions(x, z, nx, nz, d, d)
    ctx.recycle_domain()
    ref.recycle_domain()
    _assert_same(ctx, ref, f"case {case}")
    # a second pass: fewer (or no) dead slots left
    ctx.recycle_domain()
    ref.recycle_domain()
    _assert_same(ctx, ref, f"case {case}, second pass")


def test_transport_with_domain_recycling_and_dry_attributes(sdm_mod, oracle_mod):
    """Sedimentation sends particles out of the domain (multiplicity zero); each step
    recycles them over the whole domain before the pairing, under the release rules,
    with dry attributes carried along."""
    nx, nz, d = 16, 8, 5.0
    g = np.random.default_rng(13)
    n = 6000
    cell = g.integers(0, nx * nz, n).astype(np.uint32)
    r = np.exp(g.uniform(np.log(5e-6), np.log(1.5e-3), n))
    pop = synth.Population("sedi", cell, g.integers(1, 40, n).astype(np.uint64), r,
                           np.full(nx * nz, 1e-3), "geometric", 1.0, 1, 13)
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=14)
    rd3 = (r * g.uniform(0.05, 0.2, n)) ** 3
    kappa = g.uniform(0.1, 1.3, n)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.attach_dry(rd3, kappa)
    ref.set_dry(rd3, kappa)
    ctx.attach_transport(x, z, nx, nz, d, d)
    ref.set_positions(x, z, nx, nz, d, d)
    ctx.set_rules(RELEASE | RECYCLE_DOMAIN)
    rules = oracle_mod.RULE_FIDELITY | oracle_mod.RULE_RECYCLE_DOMAIN
    cx, cz = synth.eddy_courant(nx, nz, d, d, 1.0, w_max=0.5)
    for t in range(12):
        ctx.transport(cx, cz, 1.0, sediment=True)
        ref.transport(cx, cz, 1.0, sediment=True)
        ctx.step(1.0, "geometric", 77, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, 77, t, rules=rules)
    _assert_same(ctx, ref, "transport + domain recycling", dry=True)
    assert ctx.recycled() > 0 and ref.stats[1] > 0
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1]))


def test_domain_2d_transport_and_domain_recycling(sdm_mod, oracle_mod):
    """The 2D domain (75 x 75 cells, 64 SDs each) in the eddy with sedimentation,
    release rules and domain-wide recycling, 25 steps."""
    pop = synth.domain_2d(seed=synth.SEEDS[5])
    nx = nz = 75
    d = 20.0
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=3)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV * 1e-3)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV * 1e-3)
    ctx.attach_transport(x, z, nx, nz, d, d)
    ref.set_positions(x, z, nx, nz, d, d)
    ctx.set_rules(RELEASE | RECYCLE_DOMAIN)
    rules = oracle_mod.RULE_FIDELITY | oracle_mod.RULE_RECYCLE_DOMAIN
    cx, cz = synth.eddy_courant(nx, nz, d, d, 1.0, w_max=2.0)
    for t in range(25):
        ctx.transport(cx, cz, 1.0, sediment=True)
        ref.transport(cx, cz, 1.0, sediment=True)
        ctx.step(1.0, "geometric", pop.seed, t)
        ref.step_parallel(1.0, oracle_mod.GEOMETRIC, pop.seed, t, rules=rules)
    _assert_same(ctx, ref, "2D domain + domain recycling")
    assert ctx.recycled() > 0


def test_rule_checks(sdm_mod):
    pop = synth.tiny_cells(seed=3, n_cells=10, max_per_cell=20)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    for bad in (8, RECYCLE | RECYCLE_DOMAIN):
        with pytest.raises(sdm_mod.SdmError) as e:
            ctx.set_rules(bad)
        assert e.value.status == -1
    with pytest.raises(sdm_mod.SdmError) as e:       # several cells, no positions
        ctx.set_rules(RECYCLE_DOMAIN)
    assert e.value.status == -4
    with pytest.raises(sdm_mod.SdmError) as e:
        ctx.recycle_domain()
    assert e.value.status == -4
    assert ctx.rules() == 0
