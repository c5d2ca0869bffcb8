"""Shapes and value ranges of the synthetic workloads (inputs only)."""
import numpy as np

from paper_1310_1905_amd import synth


def test_box_golovin_shape():
    p = synth.box_golovin(seed=1)
    assert p.n_sd == 8192 and p.n_cells == 1
    assert np.all(p.xi == 1_024_000_000)
    v0 = p.meta["v0"]
    v = 4 / 3 * np.pi * p.r ** 3
    assert abs(v.mean() / v0 - 1) < 0.05           # exponential in volume, mean v0


def test_domain_2d_shape():
    p = synth.domain_2d(seed=1, nx=10, ny=8)
    assert p.n_cells == 80 and p.n_sd == 80 * 64
    assert np.all(p.xi == 625_000_000)
    assert abs(np.median(p.r) / 10e-6 - 1) < 0.05
    assert np.all(np.bincount(p.cell, minlength=80) == 64)


def test_large_domain_injected_cells():
    p = synth.large_domain(seed=1, nx=64, ny=64)
    cnt = np.bincount(p.cell, minlength=p.n_cells)
    c = np.arange(p.n_cells)
    assert np.all(cnt[c % 997 == 0] == 0)
    assert np.all(cnt[(c % 991 == 1) & (c % 997 != 0)] == 1)
    assert abs(cnt.mean() - 128) < 5
    live = cnt > 0
    xi_cell = np.zeros(p.n_cells)
    np.maximum.at(xi_cell, p.cell, p.xi.astype(float))
    assert np.all(xi_cell[live] == np.floor(4e10 / cnt[live]))


def test_ensemble_and_stream_ranges():
    ens = synth.ensemble(seed=2, n_instances=64)
    sizes = np.array([e.n_sd for e in ens])
    assert sizes.min() >= 2 ** 8 and sizes.max() <= 2 ** 16
    assert {e.kernel for e in ens} == {"golovin", "geometric"}
    reqs = synth.request_stream(seed=3, n_requests=40)
    t = np.array([q.arrival for q in reqs])
    assert np.all(np.diff(t) > 0)
    for q in reqs:
        assert 1 <= q.pop.n_cells <= 256
        assert 2 ** 10 - 1 <= q.pop.n_sd <= 2 ** 20 + 1
        assert np.all(q.pop.cell < q.pop.n_cells)
