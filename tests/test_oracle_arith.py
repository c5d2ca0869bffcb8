"""Pins of the oracle's per-pair arithmetic against exact mathematics:
correctly rounded cube root (exact rational midpoint test), collection kernels
(closed forms and special cases), the upscaling factor of eq. (P_ij), the
collision count with the gamma cap, and hand-worked collision outcomes."""
import math
from fractions import Fraction

import numpy as np
import pytest


def _is_correctly_rounded_cbrt(x: float, y: float) -> bool:
    up = math.nextafter(y, math.inf)
    dn = math.nextafter(y, 0.0)
    mid_up = (Fraction(y) + Fraction(up)) / 2
    mid_dn = (Fraction(y) + Fraction(dn)) / 2
    fx = Fraction(x)
    return mid_dn ** 3 < fx < mid_up ** 3


def test_cbrt_rn_random(oracle_mod):
    g = np.random.default_rng(3)
    xs = np.exp(g.uniform(np.log(1e-300), np.log(1e300), 4000))
    for x in xs:
        y = oracle_mod.cbrt_rn(float(x))
        assert _is_correctly_rounded_cbrt(float(x), y), x


def test_cbrt_rn_near_midpoints(oracle_mod):
    # x rounded from the exact cube of a midpoint between two doubles: the
    # hardest inputs for rounding (the true cube root is within ~1e-16 ulp of
    # the midpoint)
    g = np.random.default_rng(4)
    for _ in range(3000):
        Y = int(g.integers(2 ** 52, 2 ** 53))
        e = int(g.integers(-80, 20))
        mid = Fraction(2 * Y + 1) * Fraction(2) ** (e - 1)
        x = float(mid ** 3)
        if x == 0.0 or math.isinf(x):
            continue
        y = oracle_mod.cbrt_rn(x)
        assert _is_correctly_rounded_cbrt(x, y), (Y, e)


def test_cbrt_rn_exact_cubes_and_specials(oracle_mod):
    for k in [1, 2, 3, 7, 10, 123, 1000, 99991]:
        for e in [-60, -20, 0, 10]:
            y = math.ldexp(k, e)
            assert oracle_mod.cbrt_rn(y * y * y) == y
    assert oracle_mod.cbrt_rn(0.0) == 0.0
    assert oracle_mod.cbrt_rn(-8.0) == -2.0
    assert math.isinf(oracle_mod.cbrt_rn(math.inf))
    sub = 5e-324
    assert _is_correctly_rounded_cbrt(sub, oracle_mod.cbrt_rn(sub))


def test_golovin_kernel_closed_form(oracle_mod):
    b = 1500.0
    for ra, rb in [(10e-6, 10e-6), (5e-6, 30e-6), (1e-3, 2e-6)]:
        K = oracle_mod.kernel(oracle_mod.GOLOVIN, ra, rb)
        exact = b * 4.0 / 3.0 * math.pi * (ra ** 3 + rb ** 3)
        assert K == pytest.approx(exact, rel=4e-16)
        assert K == oracle_mod.kernel(oracle_mod.GOLOVIN, rb, ra)


def test_terminal_velocity_branches(oracle_mod):
    k1, k2, k3 = 1.19e8, 8.0e3, 201.0
    r1, r2 = 40e-6, 600e-6
    below = math.nextafter(r1, 0.0)
    assert oracle_mod.terminal_velocity(below) == pytest.approx(k1 * below ** 2, rel=1e-15)
    assert oracle_mod.terminal_velocity(r1) == pytest.approx(k2 * r1, rel=1e-15)           # 40 um is in the linear branch
    assert oracle_mod.terminal_velocity(r2) == pytest.approx(k2 * r2, rel=1e-15)           # 600 um is still linear
    above = math.nextafter(r2, 1.0)
    assert oracle_mod.terminal_velocity(above) == pytest.approx(k3 * math.sqrt(above), rel=1e-15)
    # Stokes regime: v = k1 r^2 (10 um -> 1.19 cm/s)
    assert oracle_mod.terminal_velocity(10e-6) == pytest.approx(0.0119, rel=1e-12)


def test_geometric_kernel_special_cases(oracle_mod):
    G = oracle_mod.GEOMETRIC
    # equal radii fall at equal speed: no geometric collisions
    for r in [3e-6, 50e-6, 1e-3]:
        assert oracle_mod.kernel(G, r, r) == 0.0
    # symmetric, and the closed form pi (ra+rb)^2 |va - vb| in the Stokes regime
    ra, rb = 10e-6, 20e-6
    K = oracle_mod.kernel(G, ra, rb)
    assert K == oracle_mod.kernel(G, rb, ra)
    exact = math.pi * (ra + rb) ** 2 * 1.19e8 * (rb ** 2 - ra ** 2)
    assert K == pytest.approx(exact, rel=1e-14)
    # collection efficiency multiplies the kernel
    K_half = oracle_mod.kernel(G, ra, rb, params=(1500.0, 1.19e8, 8.0e3, 201.0, 40e-6, 600e-6, 0.5))
    assert K_half == K * 0.5


@pytest.mark.parametrize("n", range(2, 40))
def test_upscale_factor(oracle_mod, n):
    # n(n-1)/2 pairs over floor(n/2) examined: n-1 for even n, n for odd n
    assert oracle_mod.upscale(n) == (n - 1 if n % 2 == 0 else n)


def test_probability_order_of_operations(oracle_mod):
    p = oracle_mod.probability(625_000_000, 2.5e-10, 1.0, 400.0, 63.0)
    assert p == ((625_000_000 * 2.5e-10) * 1.0) / 400.0 * 63.0
    assert p == pytest.approx(625e6 * 2.5e-10 / 400.0 * 63.0, rel=1e-15)


def test_gamma_rule(oracle_mod):
    gam = oracle_mod.gamma
    # p < 1: the paper's rule "collide iff p > u"
    assert gam(0.3, 0.29, 10, 3) == 1
    assert gam(0.3, 0.31, 10, 3) == 0
    assert gam(0.3, 0.3, 10, 3) == 0               # strict: u must be below frac(p)
    # multiple coalescence: floor(p) + [u < frac(p)]
    assert gam(2.7, 0.5, 100, 2) == 3
    assert gam(2.7, 0.8, 100, 2) == 2
    # capped at floor(xi_j / xi_k)
    assert gam(2.7, 0.5, 5, 2) == 2
    assert gam(9.1, 0.01, 7, 3) == 2
    assert gam(1e30, 0.5, 12, 5) == 2
    assert gam(0.0, 1e-300, 3, 3) == 0


def test_collision_outcomes_hand_worked(oracle_mod):
    c = oracle_mod.collide_pair
    # gamma*xi_k droplets of j merge with the xi_k droplets of k: k keeps xi_k and
    # takes (gamma r_j^3 + r_k^3)^(1/3); j keeps r_j and loses gamma*xi_k
    assert c(2, 5, 1.0, 2, 2.0) == (1, 1.0, 2, oracle_mod.cbrt_rn(10.0))        # 2*1 + 8 = 10
    assert c(1, 9, 1.0, 2, 1.0) == (7, 1.0, 2, oracle_mod.cbrt_rn(2.0))
    assert c(7, 100, 1.0, 3, 1.0) == (79, 1.0, 3, 2.0)                 # 7*1 + 1 = 8
    assert c(37, 1000, 1.0, 10, 3.0) == (630, 1.0, 10, 4.0)            # 37 + 27 = 64
    # j emptied: the xi_k merged droplets are shared floor/ceil
    assert c(1, 4, 1.0, 4, 1.0) == (2, oracle_mod.cbrt_rn(2.0), 2, oracle_mod.cbrt_rn(2.0))
    assert c(2, 6, 1.0, 3, 2.0) == (1, oracle_mod.cbrt_rn(10.0), 2, oracle_mod.cbrt_rn(10.0))
    assert c(19, 19, 1.0, 1, 2.0) == (0, 3.0, 1, 3.0)                  # 19 + 8 = 27; j dies
    assert c(1, 1, 1.0, 1, 1.0) == (0, oracle_mod.cbrt_rn(2.0), 1, oracle_mod.cbrt_rn(2.0))
    # no event: nothing changes
    assert c(0, 5, 1.5, 2, 2.5) == (5, 1.5, 2, 2.5)


def test_collision_conserves_number_of_droplet_volume(oracle_mod):
    g = np.random.default_rng(5)
    for _ in range(2000):
        xk = int(g.integers(1, 1000))
        gam = int(g.integers(1, 20))
        xj = gam * xk + int(g.integers(0, 1000))
        rj, rk = float(g.uniform(1e-6, 1e-3)), float(g.uniform(1e-6, 1e-3))
        xj2, rj2, xk2, rk2 = oracle_mod.collide_pair(gam, xj, rj, xk, rk)
        # number of droplets drops by gamma*xi_k - (new droplets counted once)
        assert xj2 + xk2 == xj + xk - gam * xk
        before = Fraction(xj) * Fraction(rj) ** 3 + Fraction(xk) * Fraction(rk) ** 3
        after = Fraction(xj2) * Fraction(rj2) ** 3 + Fraction(xk2) * Fraction(rk2) ** 3
        assert abs(float((after - before) / before)) < 4e-15
