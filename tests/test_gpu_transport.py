"""Parity of particle transport (Sect. 5.1: backward-Euler advection on an
Arakawa-C grid, periodic in x; explicit-Euler sedimentation; leavers flagged
with zero multiplicity) and of the per-step re-sort by cell with the FP64
oracle, through the C ABI.

Bar: positions bit-exact, storage layout (offsets and slot -> input index)
identical, multiplicities and radii bit-exact after transport interleaved with
coalescence steps (the re-sort fixes the storage slots both sides key their
random numbers by).  Cases: attachment (re-sort by the cells of the positions),
the single-eddy flow alone, sedimentation with particles leaving the domain,
recycling of the leavers under the release rules, a 2D-domain run of 60 steps
with all processes, steps in which nobody or nearly everybody changes cell, the
device launch plan against the host's (also over many chunks), invalid inputs,
and one step of the large domain at full size (1024 x 1024 cells, ~134M SDs).
"""
import numpy as np
import pytest
import torch

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu


def _bits_equal(a, b):
    return np.array_equal(np.ascontiguousarray(a, np.float64).view(np.uint64),
                          np.ascontiguousarray(b, np.float64).view(np.uint64))


def _setup(sdm_mod, oracle_mod, pop, nx, nz, d, seed=5):
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=seed)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.attach_transport(x, z, nx, nz, d, d)
    ref.set_positions(x, z, nx, nz, d, d)
    return ctx, ref


def _assert_same(ctx, ref, what, stats=True):
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
    if stats:
        assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1])), what


def test_attach_resorts_by_position(sdm_mod, oracle_mod):
    nx = nz = 12
    d = 20.0
    pop = synth.domain_2d(seed=synth.SEEDS[3], nx=nx, ny=nz, per_cell=16)
    # positions drawn in other cells than pop.cell: attachment moves every SD
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=7)
    x = np.roll(x, 5)
    z = np.roll(z, 11)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.attach_transport(x, z, nx, nz, d, d)
    ref.set_positions(x, z, nx, nz, d, d)
    _assert_same(ctx, ref, "attach")


def test_eddy_advection(sdm_mod, oracle_mod):
    nx = nz = 30
    d = 20.0
    pop = synth.domain_2d(seed=synth.SEEDS[4], nx=nx, ny=nz, per_cell=24)
    ctx, ref = _setup(sdm_mod, oracle_mod, pop, nx, nz, d)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 4.0, w_max=2.0)
    for t in range(15):
        ctx.transport(cx, cz, 4.0, sediment=False)
        ref.transport(cx, cz, 4.0, sediment=False)
    _assert_same(ctx, ref, "eddy")
    assert int(ref.xi.sum()) == int(pop.xi.sum())


def test_sedimentation_leavers_and_recycling(sdm_mod, oracle_mod):
    nx, nz, d = 16, 8, 5.0
    g = np.random.default_rng(11)
    n = 5000
    cell = g.integers(0, nx * nz, n).astype(np.uint32)
    r = np.exp(g.uniform(np.log(5e-6), np.log(1.5e-3), n))     # all terminal-velocity branches
    pop = synth.Population("sedi", cell, g.integers(1, 40, n).astype(np.uint64), r,
                           np.full(nx * nz, 1e-3), "geometric", 1.0, 1, 11)
    ctx, ref = _setup(sdm_mod, oracle_mod, pop, nx, nz, d, seed=12)
    rules = oracle_mod.RULE_FIDELITY | oracle_mod.RULE_RECYCLE
    ctx.set_rules(rules)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 1.0, w_max=0.5)
    for t in range(10):
        ctx.transport(cx, cz, 1.0, sediment=True)
        ref.transport(cx, cz, 1.0, sediment=True)
        ctx.step(1.0, "geometric", 99, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, 99, t, rules=rules)
    _assert_same(ctx, ref, "sedimentation")
    assert np.count_nonzero(ref.xi == 0) > 0          # leavers not all recycled
    assert ctx.recycled() > 0 and ref.stats[1] > 0


def test_domain_2d_all_processes(sdm_mod, oracle_mod):
    """The 2D domain (75 x 75 cells of 20 m, 64 SDs per cell) in the single-eddy flow with
    sedimentation and coalescence, 60 steps of 1 s."""
    pop = synth.domain_2d(seed=synth.SEEDS[0])
    nx = nz = 75
    d = 20.0
    ctx, ref = _setup(sdm_mod, oracle_mod, pop, nx, nz, d)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 1.0)
    for t in range(60):
        ctx.transport(cx, cz, 1.0, sediment=True)
        ref.transport(cx, cz, 1.0, sediment=True)
        ctx.step(1.0, "geometric", pop.seed, t)
        ref.step_parallel(1.0, oracle_mod.GEOMETRIC, pop.seed, t)
    _assert_same(ctx, ref, "domain 2d")
    assert ref.stats[1] > 0


def test_no_movers_and_mass_movement(sdm_mod, oracle_mod):
    """Steps without flow or fall (nobody changes cell: the storage stays as it is),
    then a uniform flow of Courant number 0.9 in x and z, under which nine in ten
    particles change cell every step and those leaving the top are flagged; each
    transport step is followed by a coalescence step, both sides bit-exact."""
    nx, nz, d = 24, 16, 20.0
    pop = synth.domain_2d(seed=synth.SEEDS[4], nx=nx, ny=nz, per_cell=30)
    ctx, ref = _setup(sdm_mod, oracle_mod, pop, nx, nz, d)
    off0, idx0 = (a.cpu().numpy().copy() for a in ctx.layout())
    for t in range(2):
        ctx.transport(None, None, 1.0, sediment=False)
        ref.transport(None, None, 1.0, sediment=False)
    off1, idx1 = (a.cpu().numpy() for a in ctx.layout())
    assert np.array_equal(off0, off1) and np.array_equal(idx0, idx1)
    _assert_same(ctx, ref, "no movers")
    cx = np.full(nz * nx, 0.9)
    cz = np.full((nz + 1) * nx, 0.9)
    for t in range(4):
        ctx.transport(cx, cz, 1.0, sediment=False)
        ref.transport(cx, cz, 1.0, sediment=False)
        ctx.step(1.0, "geometric", pop.seed, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, pop.seed, t)
        _assert_same(ctx, ref, f"uniform flow step {t}")
    assert (ctx.state_numpy()[0] == 0).sum() > 0      # some left through the top


@pytest.mark.parametrize("slots", [256, 512])
def test_device_plan_equals_host_plan(sdm_mod, oracle_mod, slots):
    """After a transport step the launch plan is built on the device; it must match
    the host's greedy packing (group count, cells in groups) and give the same results."""
    nx = nz = 40
    d = 20.0
    pop = synth.domain_2d(seed=synth.SEEDS[6], nx=nx, ny=nz, per_cell=100)
    ctx, ref = _setup(sdm_mod, oracle_mod, pop, nx, nz, d)
    ctx.set_launch_config(group_slots=slots)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 2.0, w_max=3.0)
    for t in range(5):
        ctx.transport(cx, cz, 2.0, sediment=True)
        ref.transport(cx, cz, 2.0, sediment=True)
        ctx.step(1.0, "geometric", 5, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, 5, t)
    dev = ctx.plan()
    other = 512 if slots == 256 else 256
    ctx.set_launch_config(group_slots=other)
    ctx.set_launch_config(group_slots=slots)      # host plan from the same offsets
    host = ctx.plan()
    assert dev == host
    _assert_same(ctx, ref, "device plan")


def test_device_plan_many_chunks(sdm_mod):
    """A grid of 320 x 256 cells: the device plan walks 80 chunks of 1024 cells and
    chains their exit tables in two runs; after each transport step its group count
    equals that of the host's greedy packing of the same offsets."""
    nx, nz, d = 320, 256, 20.0
    pop = synth.domain_2d(seed=synth.SEEDS[6], nx=nx, ny=nz, per_cell=60)
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=3)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.set_launch_config(group_slots=256)
    ctx.attach_transport(x, z, nx, nz, d, d)
    cx, cz = synth.eddy_courant(nx, nz, d, d, 2.0, w_max=3.0)
    for _ in range(3):
        ctx.transport(cx, cz, 2.0, sediment=True)
        dev = ctx.plan()
        ctx.set_launch_config(group_slots=512)
        ctx.set_launch_config(group_slots=256)     # host plan from the same offsets
        host = ctx.plan()
        assert dev == host and dev[1] == nx * nz and dev[2] == dev[3] == 0


def test_transport_errors(sdm_mod):
    nx = nz = 4
    d = 10.0
    pop = synth.domain_2d(seed=synth.SEEDS[5], nx=nx, ny=nz, per_cell=8)
    x, z = synth.positions_in_cells(pop, nx, nz, d, d, seed=1)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    with pytest.raises(sdm_mod.SdmError) as e:
        ctx.transport(None, None, 1.0)
    assert e.value.status == -4                        # no transport attached
    with pytest.raises(sdm_mod.SdmError):
        ctx.attach_transport(x, z, 3, 5, d, d)         # grid does not match n_cells
    bad = z.copy()
    bad[3] = nz * d                                    # outside [0, nz dz)
    with pytest.raises(sdm_mod.SdmError):
        ctx.attach_transport(x, bad, nx, nz, d, d)
    ctx.attach_transport(x, z, nx, nz, d, d)
    with pytest.raises(sdm_mod.SdmError) as e:
        ctx.attach_transport(x, z, nx, nz, d, d)
    assert e.value.status == -4
    cx = np.zeros(nz * nx)
    cx[5] = -1.5                                       # C_r - C_l = 1.5 in cell (1, 1)
    with pytest.raises(sdm_mod.SdmError):
        ctx.transport(cx, None, 1.0)
    cz = np.zeros((nz + 1) * nx)
    cz[2] = np.nan
    with pytest.raises(sdm_mod.SdmError):
        ctx.transport(None, cz, 1.0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.transport(None, None, 0.0)
    # the failed calls left the state alone
    xi_g, _ = ctx.state_numpy()
    assert np.array_equal(np.sort(xi_g), np.sort(pop.xi))


def test_large_domain_one_transport_step(sdm_mod, oracle_mod):
    """1024 x 1024 cells of 20 m, ~134M SDs: one eddy + sedimentation step, then the
    layout, positions and multiplicities of every SD compared."""
    pop = synth.large_domain(seed=synth.SEEDS[0])
    nx = nz = 1024
    d = 20.0
    ctx, ref = _setup(sdm_mod, oracle_mod, pop, nx, nz, d)
    ctx.autotune(pop.dt, pop.kernel, seed=pop.seed ^ 0x5A5A, reps=3)   # as bench.py selects it
    cx, cz = synth.eddy_courant(nx, nz, d, d, pop.dt, w_max=2.0)
    ctx.transport(cx, cz, pop.dt, sediment=True)
    ref.transport(cx, cz, pop.dt, sediment=True)
    _assert_same(ctx, ref, "large domain transport", stats=False)
    del ctx
    torch.cuda.empty_cache()
