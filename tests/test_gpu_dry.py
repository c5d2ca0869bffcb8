"""The optional dry attributes (r_d^3 summed, kappa averaged on coalescence,
Sect. 5.1.4) through the C ABI against the oracle.

Bar: r_d^3 and kappa bit-exact, with multiplicities and radii bit-exact as in
the other parity tests.  Cases: attach/get round trip and invalid inputs; both
tiers (wavefront groups, one- and many-chunk grid cells) under the default
rules and under the release rules with recycling; the 128 x 128 large domain;
transport with the attributes attached before and after the positions; dry
moments.
"""
import numpy as np
import pytest

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def _dry_inputs(n, seed):
    g = np.random.default_rng(seed)
    rd3 = np.exp(g.uniform(np.log(1e-24), np.log(1e-18), n))
    kappa = g.uniform(0.0, 1.3, n)
    return rd3, kappa


def _assert_same(ctx, ref, what):
    xi_g, r_g = ctx.state_numpy()
    xi_o, r_o = ref.input_order()
    assert np.array_equal(xi_g, xi_o), what
    assert np.array_equal(_bits(r_g), _bits(r_o)), what
    rd3_g, k_g = (t.cpu().numpy() for t in ctx.dry())
    rd3_o, k_o = ref.dry_input_order()
    bad = np.nonzero(_bits(rd3_g) != _bits(rd3_o))[0]
    assert bad.size == 0, f"{what}: {bad.size} r_d^3 differ, first at {bad[:5]}"
    assert np.array_equal(_bits(k_g), _bits(k_o)), what
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1])), what


def test_attach_roundtrip_and_errors(sdm_mod):
    pop = synth.tiny_cells(seed=3, n_cells=20, max_per_cell=50)
    rd3, kappa = _dry_inputs(pop.n_sd, 3)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    for call in (lambda: ctx.dry(), lambda: ctx.dry_moments(0)):
        with pytest.raises(sdm_mod.SdmError) as e:
            call()
        assert e.value.status == -4                     # nothing attached
    for bad_rd3, bad_k in ((0.0, 0.5), (-1e-20, 0.5), (np.nan, 0.5), (np.inf, 0.5),
                           (1e-20, -0.1), (1e-20, np.nan)):
        r2, k2 = rd3.copy(), kappa.copy()
        r2[7], k2[7] = bad_rd3, bad_k
        with pytest.raises(sdm_mod.SdmError) as e:
            ctx.attach_dry(r2, k2)
        assert e.value.status == -1
    ctx.attach_dry(rd3, kappa)
    a, b = (t.cpu().numpy() for t in ctx.dry())
    assert np.array_equal(_bits(a), _bits(rd3)) and np.array_equal(_bits(b), _bits(kappa))
    with pytest.raises(sdm_mod.SdmError) as e:
        ctx.attach_dry(rd3, kappa)
    assert e.value.status == -4                         # already attached


CASES = [(60, 200), (600, 120), (40000, 3)]   # wave tier; one- and many-chunk grid cells


@pytest.mark.parametrize("max_per_cell,n_cells", CASES)
@pytest.mark.parametrize("rules", [0, 3])
def test_dry_parity_both_tiers(sdm_mod, oracle_mod, max_per_cell, n_cells, rules):
    pop = synth.tiny_cells(seed=800 + max_per_cell + rules, n_cells=n_cells,
                           max_per_cell=max_per_cell, xi_max=8, dead_fraction=0.1)
    rd3, kappa = _dry_inputs(pop.n_sd, max_per_cell + rules)
    dV = pop.dV * (1e-4 if max_per_cell < 1000 else 1e-6)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, dV)
    ctx.attach_dry(rd3, kappa)
    ctx.set_rules(rules)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, dV)
    ref.set_dry(rd3, kappa)
    for t in range(5):
        ctx.step(3.0, "geometric", pop.seed, t)
        ref.step_parallel(3.0, oracle_mod.GEOMETRIC, pop.seed, t, threads=8, rules=rules)
    assert ref.stats[1] > 0
    _assert_same(ctx, ref, f"dry {max_per_cell} rules {rules}")


def test_dry_large_domain_reduced(sdm_mod, oracle_mod):
    pop = synth.large_domain(seed=synth.SEEDS[3], nx=128, ny=128, shuffle=True)
    rd3, kappa = _dry_inputs(pop.n_sd, 17)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.set_launch_config(group_slots=256, groups_per_wave=8, waves_per_block=1)
    ctx.attach_dry(rd3, kappa)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ref.set_dry(rd3, kappa)
    for t in range(4):
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
        ref.step_parallel(pop.dt, oracle_mod.GEOMETRIC, pop.seed, t, threads=16)
    _assert_same(ctx, ref, "large domain 128x128 with dry attributes")


@pytest.mark.parametrize("dry_first", [True, False])
def test_dry_with_transport(sdm_mod, oracle_mod, dry_first):
    nx, nz, d = 24, 20, 20.0
    pop = synth.domain_2d(seed=synth.SEEDS[5], nx=nx, ny=nz, per_cell=40)
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=4)
    rd3, kappa = _dry_inputs(pop.n_sd, 21)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ref.set_dry(rd3, kappa)
    ref.set_positions(x, z, nx, nz, d, d)
    if dry_first:
        ctx.attach_dry(rd3, kappa)
        ctx.attach_transport(x, z, nx, nz, d, d)
    else:
        ctx.attach_transport(x, z, nx, nz, d, d)
        ctx.attach_dry(rd3, kappa)
    ctx.set_rules(3)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 2.0, w_max=3.0)
    for t in range(12):
        ctx.transport(cx, cz, 2.0, sediment=True)
        ref.transport(cx, cz, 2.0, sediment=True)
        ctx.step(2.0, "geometric", pop.seed, t)
        ref.step(2.0, oracle_mod.GEOMETRIC, pop.seed, t, rules=3)
    assert ref.stats[1] > 0
    _assert_same(ctx, ref, f"transport, dry attached {'first' if dry_first else 'second'}")


def test_dry_moments(sdm_mod, oracle_mod, moments_close):
    pop = synth.tiny_cells(seed=44, n_cells=300, max_per_cell=700, xi_max=50)
    rd3, kappa = _dry_inputs(pop.n_sd, 44)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.attach_dry(rd3, kappa)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ref.set_dry(rd3, kappa)
    rho = np.random.default_rng(2).uniform(0.8, 1.2, pop.n_cells)
    for k, lo, hi, rh in ((0, 0.0, np.inf, None), (1, 2e-8, 8e-7, None), (3, 0.0, np.inf, rho),
                          (6, 1e-7, 1e-6, rho)):
        g = ctx.dry_moments(k, lo, hi, rh).cpu().numpy()
        o = ref.dry_moments(k, lo, hi, rh)
        moments_close(g, o, np.diff(ref.offsets))


@pytest.mark.parametrize("max_per_cell,n_cells", [(60, 200), (600, 60)])
def test_autotune_with_dry_attributes(sdm_mod, oracle_mod, max_per_cell, n_cells):
    """The autotuner's candidate steps merge r_d^3 and kappa and recycle; it must
    put them back, so a tuned context continues exactly as one never tuned."""
    pop = synth.tiny_cells(seed=850 + max_per_cell, n_cells=n_cells, max_per_cell=max_per_cell,
                           xi_max=8, dead_fraction=0.1)
    rd3, kappa = _dry_inputs(pop.n_sd, 850 + max_per_cell)
    dV = pop.dV * 1e-4
    tuned = sdm_mod.Context(pop.cell, pop.xi, pop.r, dV)
    plain = sdm_mod.Context(pop.cell, pop.xi, pop.r, dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, dV)
    ref.set_dry(rd3, kappa)
    for c in (tuned, plain):
        c.attach_dry(rd3, kappa)
        c.set_rules(3)   # release rules + recycling
    tuned.autotune(3.0, "geometric", seed=pop.seed ^ 0x77, reps=2)
    a, b = (t.cpu().numpy() for t in tuned.dry())
    assert np.array_equal(_bits(a), _bits(rd3)) and np.array_equal(_bits(b), _bits(kappa))
    assert tuned.stats() == (0, 0)
    for t in range(6):
        for c in (tuned, plain):
            c.step(3.0, "geometric", pop.seed, t)
        ref.step(3.0, oracle_mod.GEOMETRIC, pop.seed, t, rules=3)
    assert ref.stats[1] > 0
    _assert_same(tuned, ref, "autotuned, dry attached")
    _assert_same(plain, ref, "never tuned, dry attached")
