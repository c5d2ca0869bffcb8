"""Element-wise parity of the device arithmetic with the oracle, bit for bit:
Philox4x32-10, the correctly rounded cube root, and one collision test (kernel
K, probability p, collision count gamma, updated multiplicities and radii)
over random and edge-case inputs.  Called through the C ABI."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_device_vs_oracle(sdm_mod, oracle_mod):
    g = np.random.default_rng(11)
    n = 20000
    ctr = g.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)
    key = g.integers(0, 2 ** 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    # add the published known-answer vectors
    kat = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                kat.append([int(x, 16) for x in line.split()])
    kat = np.array(kat, dtype=np.uint64)
    ctr = np.vstack([ctr, kat[:, 0:4].astype(np.uint32)])
    key = np.vstack([key, kat[:, 4:6].astype(np.uint32)])
    out = sdm_mod.debug_philox(torch.from_numpy(ctr.view(np.int32).ravel()).cuda(),
                               torch.from_numpy(key.view(np.int32).ravel()).cuda())
    got = out.cpu().numpy().view(np.uint32).reshape(-1, 4)
    assert np.array_equal(got[n:], kat[:, 6:10].astype(np.uint32))
    for i in range(0, n, 7):
        assert tuple(int(x) for x in got[i]) == oracle_mod.philox4x32_10(ctr[i], key[i])


def _hard_cbrt_inputs(g, count):
    xs = []
    for _ in range(count):
        Y = int(g.integers(2 ** 52, 2 ** 53))
        e = int(g.integers(-80, 20))
        x = float((Fraction(2 * Y + 1) * Fraction(2) ** (e - 1)) ** 3)
        if x > 0 and math.isfinite(x):
            xs.append(x)
    return xs


def test_cbrt_device_vs_oracle(sdm_mod, oracle_mod):
    g = np.random.default_rng(12)
    xs = list(np.exp(g.uniform(np.log(1e-300), np.log(1e300), 20000)))
    xs += list(np.exp(g.uniform(np.log(1e-18), np.log(1e-6), 20000)))   # r^3 of droplets
    xs += _hard_cbrt_inputs(g, 5000)
    xs += [float(k) ** 3 for k in range(1, 2000)] + [5e-324, 2.2250738585072014e-308]
    x = np.array(xs, dtype=np.float64)
    y = sdm_mod.debug_cbrt(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = np.array([oracle_mod.cbrt_rn(float(v)) for v in x])
    bad = np.nonzero(y.view(np.uint64) != ref.view(np.uint64))[0]
    assert bad.size == 0, [(x[i], y[i], ref[i]) for i in bad[:5]]


def _collide_cases(g, n, kernel):
    xi_a = np.empty(n, np.uint64)
    xi_b = np.empty(n, np.uint64)
    big = g.integers(1, 10 ** 10, n).astype(np.uint64)
    small = g.integers(1, 1000, n).astype(np.uint64)
    kind = g.integers(0, 5, n)
    for i in range(n):
        if kind[i] == 0:        # equal multiplicities
            xi_a[i] = xi_b[i] = small[i]
        elif kind[i] == 1:      # exact multiple: the equal-split case when gamma hits the cap
            xi_a[i] = small[i] * int(g.integers(1, 6))
            xi_b[i] = small[i]
        elif kind[i] == 2:      # one droplet each
            xi_a[i] = xi_b[i] = 1
        else:
            xi_a[i], xi_b[i] = big[i], small[i]
    swap = g.random(n) < 0.5
    xi_a[swap], xi_b[swap] = xi_b[swap].copy(), xi_a[swap].copy()
    r_a = np.exp(g.uniform(np.log(1e-6), np.log(3e-3), n))
    r_b = np.exp(g.uniform(np.log(1e-6), np.log(3e-3), n))
    edges = [40e-6, math.nextafter(40e-6, 0), math.nextafter(40e-6, 1), 600e-6,
             math.nextafter(600e-6, 0), math.nextafter(600e-6, 1)]
    pick = g.random(n) < 0.1
    r_a[pick] = g.choice(edges, int(pick.sum()))
    n_live = g.integers(2, 300, n).astype(np.uint32)
    dt = 1.0
    # volumes chosen for log-uniform target probabilities in [1e-3, 1e3]
    target = np.exp(g.uniform(np.log(1e-3), np.log(1e3), n))
    return xi_a, xi_b, r_a, r_b, n_live, target, dt


@pytest.mark.parametrize("kernel", ["geometric", "golovin"])
def test_collide_device_vs_oracle(sdm_mod, oracle_mod, kernel):
    g = np.random.default_rng(13 if kernel == "geometric" else 14)
    n = 30000
    kind = oracle_mod.GEOMETRIC if kernel == "geometric" else oracle_mod.GOLOVIN
    xi_a, xi_b, r_a, r_b, n_live, target, dt = _collide_cases(g, n, kernel)
    dV = np.empty(n)
    for i in range(n):
        K = oracle_mod.kernel(kind, float(r_a[i]), float(r_b[i]))
        m = max(int(xi_a[i]), int(xi_b[i]))
        raw = m * K * dt * oracle_mod.upscale(int(n_live[i]))
        dV[i] = raw / target[i] if raw > 0 else 1.0
    u = np.array([oracle_mod.pair_uniform(5, i, 0, 0) for i in range(n)])
    t = {k: torch.from_numpy(v.copy()).cuda() for k, v in
         dict(n_live=n_live.view(np.int32), dV=dV, u=u, xi_a=xi_a.view(np.int64),
              r_a=r_a, xi_b=xi_b.view(np.int64), r_b=r_b).items()}
    K, p, gam = sdm_mod.debug_collide(kernel, dt, t["n_live"], t["dV"], t["u"], t["xi_a"],
                                      t["r_a"], t["xi_b"], t["r_b"])
    K, p, gam = K.cpu().numpy(), p.cpu().numpy(), gam.cpu().numpy().view(np.uint64)
    xa2 = t["xi_a"].cpu().numpy().view(np.uint64)
    xb2 = t["xi_b"].cpu().numpy().view(np.uint64)
    ra2, rb2 = t["r_a"].cpu().numpy(), t["r_b"].cpu().numpy()
    n_events = 0
    for i in range(n):
        Ko = oracle_mod.kernel(kind, float(r_a[i]), float(r_b[i]))
        a_is_j = int(xi_a[i]) >= int(xi_b[i])
        xj, xk = (int(xi_a[i]), int(xi_b[i])) if a_is_j else (int(xi_b[i]), int(xi_a[i]))
        rj, rk = (float(r_a[i]), float(r_b[i])) if a_is_j else (float(r_b[i]), float(r_a[i]))
        po = oracle_mod.probability(xj, Ko, dt, float(dV[i]), oracle_mod.upscale(int(n_live[i])))
        go = oracle_mod.gamma(po, float(u[i]), xj, xk)
        xj2, rj2, xk2, rk2 = oracle_mod.collide_pair(go, xj, rj, xk, rk)
        exp_a = (xj2, rj2) if a_is_j else (xk2, rk2)
        exp_b = (xk2, rk2) if a_is_j else (xj2, rj2)
        assert np.float64(Ko).view(np.uint64) == K[i:i + 1].view(np.uint64)[0], i
        assert np.float64(po).view(np.uint64) == p[i:i + 1].view(np.uint64)[0], i
        assert int(gam[i]) == go, i
        assert (int(xa2[i]), float(ra2[i])) == exp_a, i
        assert (int(xb2[i]), float(rb2[i])) == exp_b, i
        n_events += go > 0
    assert n_events > n // 4
