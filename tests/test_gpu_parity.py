"""Parity of the HIP coalescence step with the FP64 oracle, through the C ABI.

Bar: multiplicities and shuffle permutations bit-exact;
radii within 1e-12 relative -- and since both sides round the cube root
correctly and evaluate eq. (P_ij) in the same order without contraction, the
radii are checked bit-exact as well.

Cases: ragged cells of both kernel tiers (wavefront groups up to 256 or 512
storage slots, the grid tier above, including a cell of 2^23 slots whose digit
buckets overflow LDS), empty / single-SD / dead-SD cells, both collection
kernels, many steps; the 2D domain (75 x 75 x 64 SDs, 600 steps); the Golovin box
(8192 SDs in one cell); the large domain at reduced size in full and at full size
(1024 x 1024 cells, ~134M SDs, in the launch configuration the benchmark times) on
sampled cells, which the oracle advances one by one.
"""
import numpy as np
import pytest
import torch

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu


def _assert_same(ctx, ref, what):
    xi_g, r_g = ctx.state_numpy()
    xi_o, r_o = ref.input_order()
    bad = np.nonzero(xi_g != xi_o)[0]
    assert bad.size == 0, f"{what}: {bad.size} multiplicities differ, first at {bad[:5]}"
    rel = np.abs(r_g - r_o) / r_o
    assert rel.max() <= 1e-12, f"{what}: radius rel. error {rel.max()}"
    nbits = int(np.count_nonzero(r_g.view(np.uint64) != r_o.view(np.uint64)))
    assert nbits == 0, f"{what}: {nbits} radii differ in the last bits"
    assert ctx.stats() == (int(ref.stats[0]), int(ref.stats[1])), what


def _run_pair(sdm_mod, oracle_mod, pop, steps, dt, kernel, dV_scale=1.0, threads=8):
    kind = oracle_mod.GOLOVIN if kernel == "golovin" else oracle_mod.GEOMETRIC
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV * dV_scale)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV * dV_scale)
    for t in range(steps):
        ctx.step(dt, kernel, pop.seed, t)
        ref.step_parallel(dt, kind, pop.seed, t, threads=threads)
    return ctx, ref


@pytest.mark.parametrize("kernel", ["geometric", "golovin"])
@pytest.mark.parametrize("max_per_cell", [3, 40, 256, 257, 512, 513, 900])
def test_ragged_cells(sdm_mod, oracle_mod, kernel, max_per_cell):
    pop = synth.tiny_cells(seed=100 + max_per_cell, n_cells=150, max_per_cell=max_per_cell,
                           xi_max=60)
    ctx, ref = _run_pair(sdm_mod, oracle_mod, pop, 12, 3.0, kernel, dV_scale=1e-4)
    _assert_same(ctx, ref, f"ragged {kernel} {max_per_cell}")
    assert ref.stats[1] > 0


@pytest.mark.parametrize("max_per_cell", [40, 300, 700])
def test_permutation_bit_exact(sdm_mod, oracle_mod, max_per_cell):
    pop = synth.tiny_cells(seed=7, n_cells=120, max_per_cell=max_per_cell, dead_fraction=0.3)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV)
    off = ref.offsets.astype(np.int64)
    for step in (0, 1, 99, 2 ** 32 - 1):
        order, nlive = ctx.permutation(seed=31337, step=step)
        order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
        for c in range(ref.n_cells):
            exp = oracle_mod.cell_order(ref.xi[off[c]:off[c + 1]], 31337, c, step)
            assert nlive[c] == exp.size
            assert np.array_equal(order[off[c]:off[c] + exp.size], exp), (step, c)


@pytest.mark.parametrize("shape", [
    dict(group_slots=256, groups_per_wave=1, waves_per_block=1, xcd_remap=0),
    dict(group_slots=256, groups_per_wave=3, waves_per_block=4, xcd_remap=1),
    dict(group_slots=512, groups_per_wave=1, waves_per_block=2, xcd_remap=0),
    dict(group_slots=512, groups_per_wave=8, waves_per_block=4, xcd_remap=1),
])
def test_launch_shapes_give_identical_results(sdm_mod, oracle_mod, shape):
    pop = synth.tiny_cells(seed=55, n_cells=700, max_per_cell=600, xi_max=40)
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV * 1e-4)
    ctx.set_launch_config(**shape)
    ref = oracle_mod.SlotState(pop.cell, pop.xi, pop.r, pop.dV * 1e-4)
    for t in range(6):
        ctx.step(3.0, "geometric", pop.seed, t)
        ref.step_parallel(3.0, oracle_mod.GEOMETRIC, pop.seed, t, threads=8)
    _assert_same(ctx, ref, f"shape {shape}")
    order, nlive = ctx.permutation(seed=3, step=7)
    off = ref.offsets.astype(np.int64)
    order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
    for c in range(0, ref.n_cells, 7):
        exp = oracle_mod.cell_order(ref.xi[off[c]:off[c + 1]], 3, c, 7)
        assert nlive[c] == exp.size and np.array_equal(order[off[c]:off[c] + exp.size], exp)


def test_many_cells_per_group(sdm_mod, oracle_mod):
    """Runs of tiny and empty cells: groups reach the 64-cell limit."""
    pop = synth.tiny_cells(seed=8, n_cells=3000, max_per_cell=4, xi_max=9, dead_fraction=0.2)
    ctx, ref = _run_pair(sdm_mod, oracle_mod, pop, 8, 5.0, "golovin", dV_scale=1e-9)
    _assert_same(ctx, ref, "tiny cells")
    groups, wave_cells, block_cells, grid_cells = ctx.plan()
    assert wave_cells == pop.n_cells and block_cells == grid_cells == 0
    assert groups <= pop.n_cells // 64 + 60


@pytest.mark.parametrize("kernel", ["geometric", "golovin"])
def test_grid_tier_cells(sdm_mod, oracle_mod, kernel):
    """Cells of up to 60000 storage slots, spread over many workgroups."""
    pop = synth.tiny_cells(seed=91, n_cells=6, max_per_cell=60000, xi_max=30, dead_fraction=0.2)
    sizes = np.bincount(pop.cell, minlength=pop.n_cells)
    assert (sizes > 16384).sum() >= 3
    ctx, ref = _run_pair(sdm_mod, oracle_mod, pop, 4, 3.0, kernel, dV_scale=1e-6, threads=6)
    _assert_same(ctx, ref, f"grid tier {kernel}")
    assert ref.stats[1] > 0
    order, nlive = ctx.permutation(seed=17, step=3)
    order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
    off = ref.offsets.astype(np.int64)
    for c in range(ref.n_cells):
        exp = oracle_mod.cell_order(ref.xi[off[c]:off[c + 1]], 17, c, 3)
        assert nlive[c] == exp.size
        assert np.array_equal(order[off[c]:off[c] + exp.size], exp), c


def test_grid_tier_plan_transitions(sdm_mod, oracle_mod):
    """Grid cells at the sizes where the digit bits or the slot-chunk size of the
    grid tier change (257, 1024/1025, 2048/2049, 4097, 65537, 700001 and 2^20 + 1
    slots; 700001 has the most digits, 1024, that chunks placed through LDS take, and
    a partial last chunk; 2^20 + 1 has 4096-slot chunks placed directly), with dead
    slots: pairing order and two steps bit-exact."""
    g = np.random.default_rng(77)
    sizes = [257, 1024, 1025, 2048, 2049, 4097, 65537, 700001, (1 << 20) + 1, 100]
    cell = np.repeat(np.arange(len(sizes), dtype=np.uint32), sizes)
    n = cell.size
    xi = g.integers(1, 40, n).astype(np.uint64)
    xi[g.random(n) < 0.05] = 0
    r = np.exp(g.uniform(np.log(5e-6), np.log(2e-3), n))
    dV = np.array([1e-2, 1e-1, 1e-1, 1.0, 1.0, 1.0, 10.0, 5e2, 1e3, 1e-3])
    ctx = sdm_mod.Context(cell, xi, r, dV)
    ctx.set_launch_config(group_slots=256, block_slots=0)
    assert ctx.plan()[1:] == (1, 0, len(sizes) - 1)
    ref = oracle_mod.SlotState(cell, xi, r, dV)
    order, nlive = ctx.permutation(seed=5, step=2)
    order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
    off = ref.offsets.astype(np.int64)
    for c in range(len(sizes)):
        exp = oracle_mod.cell_order(ref.xi[off[c]:off[c + 1]], 5, c, 2)
        assert nlive[c] == exp.size
        assert np.array_equal(order[off[c]:off[c] + exp.size], exp), sizes[c]
    for t in range(2):
        ctx.step(2.0, "geometric", 9, t)
        ref.step_parallel(2.0, oracle_mod.GEOMETRIC, 9, t, threads=10)
    _assert_same(ctx, ref, "grid plan transitions")
    assert ref.stats[1] > 0


@pytest.mark.parametrize("kernel", ["geometric", "golovin"])
def test_block_tier_cells(sdm_mod, oracle_mod, kernel):
    """Cells of the workgroup tier (one workgroup per cell, the sort in LDS): 513 to
    8192 storage slots, with the neighbours of its limits (512/513 against the
    wavefront groups, 2048/2049 between its 256- and 1024-thread workgroups,
    8192/8193 against the grid tier) and dead slots: the plan splits as stated,
    the pairing order and three steps are bit-exact; with the tier limited to
    2048 slots, and switched off, the results are the same."""
    g = np.random.default_rng(4242)
    sizes = [513, 700, 1500, 2047, 2048, 2049, 3000, 5000, 8191, 8192, 8193, 40, 600, 512]
    cell = np.repeat(np.arange(len(sizes), dtype=np.uint32), sizes)
    n = cell.size
    xi = g.integers(1, 40, n).astype(np.uint64)
    xi[g.random(n) < 0.05] = 0
    r = np.exp(g.uniform(np.log(5e-6), np.log(2e-3), n))
    dV = g.uniform(1e-3, 1.0, len(sizes))
    kind = oracle_mod.GOLOVIN if kernel == "golovin" else oracle_mod.GEOMETRIC
    states = []
    for block_slots, plan in ((8192, (2, 11, 1)), (2048, (2, 6, 6)), (0, (2, 0, 12))):
        ctx = sdm_mod.Context(cell, xi, r, dV)
        ctx.set_launch_config(group_slots=512, block_slots=block_slots)
        assert ctx.plan()[1:] == plan, block_slots
        ref = oracle_mod.SlotState(cell, xi, r, dV)
        order, nlive = ctx.permutation(seed=11, step=4)
        order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
        off = ref.offsets.astype(np.int64)
        for c in range(len(sizes)):
            exp = oracle_mod.cell_order(ref.xi[off[c]:off[c] + sizes[c]], 11, c, 4)
            assert nlive[c] == exp.size
            assert np.array_equal(order[off[c]:off[c] + exp.size], exp), sizes[c]
        for t in range(3):
            ctx.step(2.0, kernel, 11, t)
            ref.step_parallel(2.0, kind, 11, t, threads=8)
        _assert_same(ctx, ref, f"block tier {kernel} limit {block_slots}")
        assert ref.stats[1] > 0
        states.append(ctx.state_numpy())
    for xs, rs in states[1:]:
        assert np.array_equal(xs, states[0][0])
        assert np.array_equal(rs.view(np.uint64), states[0][1].view(np.uint64))


def test_grid_tier_huge_cell(sdm_mod, oracle_mod):
    """One cell of 2^23 + 1000 storage slots next to a 700-slot one: its 4096
    digit buckets hold about 2048 live entries each, so buckets within and beyond
    the LDS capacity of the bucket sort both occur; the pairing order and two
    steps are bit-exact."""
    g = np.random.default_rng(2323)
    n_big = (1 << 23) + 1000
    cell = np.concatenate([np.zeros(n_big, np.uint32), np.ones(700, np.uint32)])
    n = cell.size
    xi = g.integers(1, 31, n).astype(np.uint64)
    xi[g.random(n) < 0.01] = 0
    r = np.exp(g.uniform(np.log(5e-6), np.log(2e-3), n))
    dV = np.array([1e3, 1e-3])
    ctx = sdm_mod.Context(cell, xi, r, dV)
    assert ctx.plan()[1:] == (0, 1, 1)
    ref = oracle_mod.SlotState(cell, xi, r, dV)
    order, nlive = ctx.permutation(seed=99, step=5)
    order, nlive = order.cpu().numpy(), nlive.cpu().numpy()
    off = ref.offsets.astype(np.int64)
    for c in range(2):
        exp = oracle_mod.cell_order(ref.xi[off[c]:off[c + 1]], 99, c, 5)
        assert nlive[c] == exp.size
        assert np.array_equal(order[off[c]:off[c] + exp.size], exp), c
    for t in range(2):
        ctx.step(1.0, "geometric", 7, t)
        ref.step(1.0, oracle_mod.GEOMETRIC, 7, t)
    _assert_same(ctx, ref, "huge grid cell")
    assert ref.stats[1] > 0


def test_empty_and_degenerate_inputs(sdm_mod, oracle_mod):
    # no SDs at all, a single cell with one SD, and a cell with only dead SDs
    ctx = sdm_mod.Context(np.zeros(0, np.uint32), np.zeros(0, np.uint64), np.zeros(0),
                          np.ones(3))
    ctx.step(1.0, "geometric", 1, 0)
    assert ctx.stats() == (0, 0)
    ctx = sdm_mod.Context(np.array([0], np.uint32), np.array([5], np.uint64), np.array([1e-5]),
                          np.ones(1))
    ctx.step(1.0, "golovin", 1, 0)
    xi, r = ctx.state_numpy()
    assert xi.tolist() == [5] and r.tolist() == [1e-5] and ctx.stats() == (0, 0)
    ctx = sdm_mod.Context(np.array([0, 0, 1, 1], np.uint32), np.array([0, 0, 3, 4], np.uint64),
                          np.array([1e-5, 2e-5, 3e-5, 9e-5]), np.array([1e-9, 1e-9]))
    ctx.step(1.0, "geometric", 1, 0)
    assert ctx.stats()[0] == 1


def test_invalid_inputs_rejected(sdm_mod):
    with pytest.raises(sdm_mod.SdmError) as e:
        sdm_mod.Context(np.array([0, 2], np.uint32), np.ones(2, np.uint64), np.ones(2) * 1e-5,
                        np.ones(2))
    assert e.value.status == -1
    with pytest.raises(sdm_mod.SdmError):
        sdm_mod.Context(np.array([0, 1], np.uint32), np.ones(2, np.uint64),
                        np.array([1e-5, -1.0]), np.ones(2))
    with pytest.raises(sdm_mod.SdmError):
        sdm_mod.Context(np.array([0, 1], np.uint32), np.ones(2, np.uint64),
                        np.array([1e-5, np.nan]), np.ones(2))
    with pytest.raises(sdm_mod.SdmError):
        sdm_mod.Context(np.array([0, 1], np.uint32), np.ones(2, np.uint64), np.ones(2) * 1e-5,
                        np.array([1.0, 0.0]))
    ctx = sdm_mod.Context(np.array([0, 1], np.uint32), np.ones(2, np.uint64), np.ones(2) * 1e-5,
                          np.ones(2))
    for dt in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(sdm_mod.SdmError):
            ctx.step(dt, "geometric", 0, 0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.step(1.0, 7, 0, 0)
    with pytest.raises(sdm_mod.SdmError):
        ctx.step(1.0, "geometric", 0, 2 ** 32)


def test_domain_2d_full_run(sdm_mod, oracle_mod):
    pop = synth.domain_2d(seed=synth.SEEDS[1])
    ctx, ref = _run_pair(sdm_mod, oracle_mod, pop, pop.steps, pop.dt, pop.kernel, threads=16)
    _assert_same(ctx, ref, "domain_2d 600 steps")


def test_box_golovin(sdm_mod, oracle_mod):
    pop = synth.box_golovin(seed=synth.SEEDS[2])
    ctx, ref = _run_pair(sdm_mod, oracle_mod, pop, 400, pop.dt, pop.kernel, threads=1)
    _assert_same(ctx, ref, "box golovin 400 steps")
    assert ctx.plan()[1:] == (0, 1, 0)


def test_large_domain_reduced_full_parity(sdm_mod, oracle_mod):
    pop = synth.large_domain(seed=synth.SEEDS[3], nx=128, ny=128, shuffle=True)
    ctx, ref = _run_pair(sdm_mod, oracle_mod, pop, 6, pop.dt, pop.kernel, threads=16)
    _assert_same(ctx, ref, "large domain 128x128")


def test_large_domain_full_size_sampled_cells(sdm_mod, oracle_mod):
    """1024 x 1024 cells (~134M SDs) in the launch configuration the benchmark's
    autotuner selects on the state, as bench.py does, for 50 steps (a quarter of the
    set-up's 200: every step is the same kernel on the same layout, and 50 steps
    take the sampled cells through tens of collisions each); the oracle advances
    4096 sampled cells (plus every injected empty/single cell kind) one by one
    with their own RNG cell index."""
    pop = synth.large_domain(seed=synth.SEEDS[0])
    ctx = sdm_mod.Context(pop.cell, pop.xi, pop.r, pop.dV)
    ctx.autotune(pop.dt, pop.kernel, seed=pop.seed ^ 0x5A5A, reps=8)   # as bench.py selects it
    cnt = np.bincount(pop.cell, minlength=pop.n_cells)
    off = np.concatenate([[0], np.cumsum(cnt)])
    g = np.random.default_rng(5)
    sample = np.unique(np.concatenate([g.choice(pop.n_cells, 4096, replace=False),
                                       [0, 1, 997, 992, pop.n_cells - 1]]))
    steps = 50
    refs = {}
    for c in sample:
        sl = slice(off[c], off[c + 1])
        refs[c] = [pop.xi[sl].copy(), pop.r[sl].copy()]
    params = np.array(oracle_mod.DEFAULT_PARAMS, dtype=np.float64)
    stats = np.zeros(2, np.uint64)
    for t in range(steps):
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
        for c in sample:
            xi_c, r_c = refs[c]
            offs = np.array([0, xi_c.size], np.uint64)
            dv = np.ascontiguousarray(pop.dV[c:c + 1])
            oracle_mod.lib().oracle_step(1, offs.ctypes.data, dv.ctypes.data, xi_c.ctypes.data,
                                         r_c.ctypes.data, pop.dt, oracle_mod.GEOMETRIC,
                                         params.ctypes.data, pop.seed, t, int(c),
                                         stats.ctypes.data)
    xi_g, r_g = ctx.state_numpy()          # input order == storage order (cell-major input)
    for c in sample:
        sl = slice(off[c], off[c + 1])
        assert np.array_equal(xi_g[sl], refs[c][0]), c
        assert np.array_equal(r_g[sl].view(np.uint64), refs[c][1].view(np.uint64)), c
    # every cell: droplet volume conserved, number non-increasing
    torch.cuda.empty_cache()
    v0 = np.bincount(pop.cell, weights=pop.xi.astype(np.float64) * pop.r ** 3,
                     minlength=pop.n_cells)
    v1 = np.bincount(pop.cell, weights=xi_g.astype(np.float64) * r_g ** 3, minlength=pop.n_cells)
    nz = v0 > 0
    assert np.all(np.abs(v1[nz] - v0[nz]) <= 1e-12 * v0[nz])
    pairs, coll = ctx.stats()
    live = cnt[cnt > 0]
    assert pairs >= steps * int((live // 2).sum()) * 0.999
    assert coll > 0
