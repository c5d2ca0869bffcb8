"""The HIP step against the analytic solution of the coalescence equation for
Golovin's kernel and an exponential initial spectrum, over the full run of the
box set-up (one 1e6 m^3 cell, 2^13 super-droplets, N0 = 2^23 m^-3, radius of mean
volume 30.531 um, b = 1500 s^-1, dt = 1 s, 3600 steps), eight seeds advanced
together as one batch with the captured step graph.

Checks at 1200, 2400 and 3600 s: mean N(t) / (N0 exp(-b N0 v0 t)) within 5 %,
the seed-averaged mass spectrum within L1 0.12 of the analytic one with its peak
bin within one bin, total volume conserved to 1e-12, and the first seed's final
state bit for bit equal to the oracle's 3600-step run.
"""
import numpy as np
import pytest

from paper_1310_1905_amd import synth
from test_oracle_golovin import _analytic_mass_fraction

pytestmark = pytest.mark.gpu

CHECK_TIMES = (1200, 2400, 3600)


def test_golovin_analytic_on_device(sdm_mod, oracle_mod):
    pops = [synth.box_golovin(seed=s) for s in synth.SEEDS[:8]]
    b = sdm_mod.Batch(max_sd=sum(p.n_sd for p in pops), max_cells=len(pops),
                      max_instances=len(pops))
    handles = [b.add(p.cell, p.xi, p.r, p.dV, p.kernel, p.dt, p.seed) for p in pops]
    snaps = {}
    t = 0
    for t_check in CHECK_TIMES:
        while t < t_check:
            b.step(use_graph=True)
            t += 1
        snaps[t_check] = []
        for h in handles:
            xi, r, cnt = b.get(h)
            assert cnt.steps_done == t_check
            snaps[t_check].append((xi.cpu().numpy().view(np.uint64).copy(), r.cpu().numpy().copy()))
    p0 = pops[0]
    N0, v0, bb = p0.meta["N0"], p0.meta["v0"], p0.meta["b"]
    dV = float(p0.dV[0])
    B = bb * N0 * v0
    edges = np.exp(np.linspace(np.log(1e-6), np.log(5e-3), 65))
    for t_check in CHECK_TIMES:
        ratios = [xi.astype(np.float64).sum() / dV / (N0 * np.exp(-B * t_check))
                  for xi, _ in snaps[t_check]]
        assert abs(float(np.mean(ratios)) - 1.0) < 0.05, (t_check, ratios)
        hist = np.zeros(64)
        for (xi, r), p in zip(snaps[t_check], pops):
            w = xi.astype(np.float64) * r ** 3
            v_init = float(np.sum(p.xi.astype(np.float64) * p.r ** 3))
            assert abs(float(w.sum()) - v_init) <= 1e-12 * v_init
            h, _ = np.histogram(r, bins=edges, weights=w)
            hist += h / w.sum()
        hist /= len(pops)
        ref = _analytic_mass_fraction(edges, t_check, N0, v0, bb)
        assert float(np.abs(hist - ref).sum()) < 0.12, t_check
        assert abs(int(np.argmax(hist)) - int(np.argmax(ref))) <= 1, t_check
    # the first seed's whole run, bit for bit against the oracle
    st = oracle_mod.SlotState(p0.cell, p0.xi, p0.r, p0.dV)
    for step in range(CHECK_TIMES[-1]):
        st.step(p0.dt, oracle_mod.GOLOVIN, p0.seed, step)
    xi_o, r_o = st.input_order()
    xi_g, r_g = snaps[CHECK_TIMES[-1]][0]
    assert np.array_equal(xi_g, xi_o)
    assert np.array_equal(r_g.view(np.uint64), r_o.view(np.uint64))
