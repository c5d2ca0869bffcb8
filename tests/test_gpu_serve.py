"""The continuous-batching request loop (paper_1310_1905_amd.serve.Engine) on a
small Poisson stream whose requests cannot all fit at once: every request's final
state is bit-identical to the same request served alone with plain launches, and
to the oracle; admission waited for retirements and requests overlapped on the
device.
"""
import numpy as np
import pytest

from paper_1310_1905_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_results_equal_alone(sdm_mod, oracle_mod, use_graph):
    from paper_1310_1905_amd import serve
    reqs = synth.request_stream(seed=synth.SEEDS[7], n_requests=14, rate=200.0, log2_lo=8,
                                log2_hi=13, steps_lo=3, steps_hi=30, max_cells=12)
    biggest = max(q.pop.n_sd for q in reqs)
    # room for about three of the largest requests at a time
    budget = int(sdm_mod.lib().sdm_batch_workspace_bytes(3 * biggest, 1024, 64))
    eng = serve.Engine(budget_bytes=budget, max_instances=64, keep_state=True,
                       use_graph=use_graph)
    assert eng.capacity[0] < sum(q.pop.n_sd for q in reqs)
    res = eng.run(reqs, time_scale=0.0)
    iterations = eng.iterations
    eng.close()
    alone = serve.run_sequential(reqs, time_scale=0.0, keep_state=True)
    by_alone = {r.index: r for r in alone}
    assert sorted(r.index for r in res) == list(range(len(reqs)))
    for r in res:
        a = by_alone[r.index]
        assert r.steps == reqs[r.index].pop.steps
        assert np.array_equal(r.xi, a.xi), r.index
        assert np.array_equal(r.r.view(np.uint64), a.r.view(np.uint64)), r.index
        assert r.pair_tests == a.pair_tests
    # the work overlapped (fewer batch iterations than steps in total) and was throttled
    assert iterations < sum(q.pop.steps for q in reqs)
    assert iterations >= max(q.pop.steps for q in reqs)
    # two requests against the oracle
    for i in (0, len(reqs) - 1):
        p = reqs[i].pop
        kind = oracle_mod.GOLOVIN if p.kernel == "golovin" else oracle_mod.GEOMETRIC
        st = oracle_mod.SlotState(p.cell, p.xi, p.r, p.dV)
        for t in range(p.steps):
            st.step(p.dt, kind, p.seed, t)
        xi_o, r_o = st.input_order()
        r_res = next(x for x in res if x.index == i)
        assert np.array_equal(r_res.xi, xi_o)
        assert np.array_equal(r_res.r.view(np.uint64), r_o.view(np.uint64))


def test_served_stream_with_a_2e20_request(sdm_mod, oracle_mod):
    """A request of 2^20 SDs (one cell: the grid tier) arrives among small ones:
    every result equals the request served alone, and the big one equals the
    oracle."""
    from paper_1310_1905_amd import serve
    reqs = synth.request_stream(seed=synth.SEEDS[8], n_requests=12, rate=500.0, log2_lo=8,
                                log2_hi=12, steps_lo=3, steps_hi=12, max_cells=8)
    big = synth.box_golovin(seed=synth.SEEDS[9], n_sd=1 << 20, dV=1e6)
    big.steps = 4
    reqs.insert(5, synth.Request(reqs[4].arrival, big))
    budget = int(sdm_mod.lib().sdm_batch_workspace_bytes(3 << 20, 4096, 64))
    eng = serve.Engine(budget_bytes=budget, max_instances=64, keep_state=True, use_graph=True)
    res = eng.run(reqs, time_scale=0.0)
    eng.close()
    alone = {r.index: r for r in serve.run_sequential(reqs, time_scale=0.0, keep_state=True)}
    assert sorted(r.index for r in res) == list(range(len(reqs)))
    for r in res:
        a = alone[r.index]
        assert np.array_equal(r.xi, a.xi), r.index
        assert np.array_equal(r.r.view(np.uint64), a.r.view(np.uint64)), r.index
        assert r.pair_tests == a.pair_tests
    st = oracle_mod.SlotState(big.cell, big.xi, big.r, big.dV)
    for t in range(big.steps):
        st.step(big.dt, oracle_mod.GOLOVIN, big.seed, t)
    xi_o, r_o = st.input_order()
    r_big = next(x for x in res if x.index == 5)
    assert np.array_equal(r_big.xi, xi_o)
    assert np.array_equal(r_big.r.view(np.uint64), r_o.view(np.uint64))
