"""sdm_coalesce_sorted_static -- the step that allocates nothing (its launch plan,
counters and flags live in the library's static device scratch) -- against the
context path (sdm_init + sdm_coalesce_step) on the same SDs, bit for bit, on two
calls in a row, the second with a smaller input; and its error paths."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu


def _sorted_population(seed, n_cells, max_per_cell, xi_max):
    pop = synth.tiny_cells(seed=seed, n_cells=n_cells, max_per_cell=max_per_cell, xi_max=xi_max)
    o = np.argsort(pop.cell, kind="stable")
    cell, xi, r = pop.cell[o], pop.xi[o], pop.r[o]
    offsets = np.zeros(n_cells + 1, dtype=np.uint32)
    np.cumsum(np.bincount(cell, minlength=n_cells), out=offsets[1:])
    return cell, xi, r, pop.dV * 1e-4, offsets


def _device(xi, r, dV, offsets):
    return (torch.from_numpy(offsets.view(np.int32).copy()).cuda(),
            torch.from_numpy(xi.view(np.int64).copy()).cuda(),
            torch.from_numpy(r.copy()).cuda(),
            torch.from_numpy(dV.copy()).cuda())


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_step_matches_context(sdm_mod, oracle_mod, order):
    cases = [  # (seed, cells, max slots per cell, kernel, step): the first plans 512-slot groups
        (31, 3000, 300, "geometric", 5),
        (32, 500, 200, "golovin", 6),
    ]
    seed_rng = 0xC0FFEE
    for seed, n_cells, max_per_cell, kernel, step in cases:
        print(f"static step: seed {seed}, {n_cells} cells, <= {max_per_cell} slots, {kernel}",
              flush=True)
        cell, xi, r, dV, offsets = _sorted_population(seed, n_cells, max_per_cell, 60)
        ctx = sdm_mod.Context(cell, xi, r, dV)
        ctx.step(3.0, kernel, seed_rng, step)
        xi_c, r_c = ctx.state_numpy()
        off_t, xi_t, r_t, dv_t = _device(xi, r, dV, offsets)
        pairs, colls = sdm_mod.coalesce_sorted_static(off_t, xi_t, r_t, dv_t, 3.0, kernel,
                                                      seed_rng, step)
        torch.cuda.synchronize()
        xi_s = xi_t.cpu().numpy().view(np.uint64)
        r_s = r_t.cpu().numpy()
        assert np.array_equal(xi_s, xi_c), f"{n_cells} cells: multiplicities differ"
        assert np.array_equal(r_s.view(np.uint64), r_c.view(np.uint64)), \
            f"{n_cells} cells: radii differ"
        assert (pairs, colls) == ctx.stats()
        assert colls > 0
        # and the oracle agrees (one step)
        kind = oracle_mod.GOLOVIN if kernel == "golovin" else oracle_mod.GEOMETRIC
        ref = oracle_mod.SlotState(cell, xi, r, dV)
        ref.step(3.0, kind, seed_rng, step)
        xi_o, r_o = ref.input_order()
        assert np.array_equal(xi_s, xi_o)
        assert np.array_equal(r_s.view(np.uint64), r_o.view(np.uint64))
        ctx.close()


def test_static_step_rejects(sdm_mod):
    L = sdm_mod.lib()
    cell, xi, r, dV, offsets = _sorted_population(33, 50, 40, 60)
    # one cell of 600 slots: beyond the 512-slot groups
    big_xi = np.concatenate([xi, np.full(600, 5, dtype=np.uint64)])
    big_r = np.concatenate([r, np.full(600, 1e-5)])
    big_dV = np.concatenate([dV, [10.0]])
    big_off = np.concatenate([offsets, [offsets[-1] + 600]]).astype(np.uint32)
    off_t, xi_t, r_t, dv_t = _device(big_xi, big_r, big_dV, big_off)
    before = xi_t.clone()
    with pytest.raises(sdm_mod.SdmError) as e:
        sdm_mod.coalesce_sorted_static(off_t, xi_t, r_t, dv_t, 1.0, "geometric", 1, 0)
    assert e.value.status == -1 and b"512" in L.sdm_last_error()
    assert torch.equal(xi_t, before)
    # offsets that do not end at n_sd
    bad_off = offsets.copy()
    bad_off[-1] -= 1
    off_t, xi_t, r_t, dv_t = _device(xi, r, dV, bad_off)
    with pytest.raises(sdm_mod.SdmError):
        sdm_mod.coalesce_sorted_static(off_t, xi_t, r_t, dv_t, 1.0, "geometric", 1, 0)
    # a non-positive volume
    off_t, xi_t, r_t, dv_t = _device(xi, r, np.where(np.arange(dV.size) == 3, 0.0, dV), offsets)
    with pytest.raises(sdm_mod.SdmError):
        sdm_mod.coalesce_sorted_static(off_t, xi_t, r_t, dv_t, 1.0, "geometric", 1, 0)
    # more cells than the static plan holds: rejected on the host
    st = L.sdm_coalesce_sorted_static(None, 0, (1 << 20) + 1, ctypes.c_void_p(8),
                                      None, None, ctypes.c_void_p(8), 1.0, 1, None, 0, 0,
                                      None, None)
    assert st == -1 and b"cells" in L.sdm_last_error()
    assert L.sdm_static_scratch_bytes() == 16 << 20
