"""Seeded synthetic super-droplet populations shaped like the paper's set-ups.

Inputs only: this module draws cell indices, multiplicities, radii and cell volumes
with numpy ``Generator(PCG64(seed))``; it holds none of the coalescence arithmetic and
is shared by the HIP path's tests/bench and the oracle's tests.  Kernel choices are
returned as the labels ``"golovin"`` / ``"geometric"``.

Workloads (sizes are keyword arguments so tests can shrink them):
  box_golovin     -- one cell of dV = 1e6 m^3, 2^13 SDs, exponential-in-volume spectrum
                     (radius of mean volume 30.531 um, N0 = 2^23 m^-3), Golovin kernel.
  domain_2d       -- 75 x 75 cells of 20 m x 20 m x 1 m, 64 SDs per cell, lognormal
                     radii (median 10 um, sigma_g 1.4), 100 cm^-3, geometric kernel
                     (the paper's 2D kinematic grid and SD density).
  large_domain    -- 1024 x 1024 cells, Poisson(128) SDs per cell with empty and
                     single-SD cells injected, bimodal lognormal radii, geometric kernel.
  ensemble        -- many independent single-cell boxes of log-uniform size.
  request_stream  -- Poisson arrivals of box / column runs for the serving loop.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEEDS = [20250101 + i for i in range(16)]

R_MEAN_VOLUME_BOX = 30.531e-6      # m, radius of the mean droplet volume (box set-up)
N0_BOX = 2.0 ** 23                 # m^-3
CONC_LOGNORMAL = 1e8               # 100 cm^-3 in m^-3


@dataclass
class Population:
    """One run's input: SD arrays (input order) and per-cell volumes."""
    name: str
    cell: np.ndarray                 # uint32
    xi: np.ndarray                   # uint64
    r: np.ndarray                    # float64, metres
    dV: np.ndarray                   # float64, m^3
    kernel: str                      # "golovin" | "geometric"
    dt: float
    steps: int
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n_sd(self) -> int:
        return int(self.cell.size)

    @property
    def n_cells(self) -> int:
        return int(self.dV.size)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _exponential_volume_radii(g, n, r_mean_volume):
    v0 = 4.0 / 3.0 * np.pi * r_mean_volume ** 3
    v = -v0 * np.log1p(-g.random(n))
    return np.cbrt(3.0 * v / (4.0 * np.pi))


def _lognormal_radii(g, n, median, sigma_g):
    return np.exp(g.normal(np.log(median), np.log(sigma_g), n))


def box_golovin(seed: int = SEEDS[0], n_sd: int = 2 ** 13, dV: float = 1e6,
                steps: int = 3600) -> Population:
    g = _rng(seed)
    r = _exponential_volume_radii(g, n_sd, R_MEAN_VOLUME_BOX)
    xi = np.full(n_sd, int(round(N0_BOX * dV / n_sd)), dtype=np.uint64)
    return Population("box_golovin", np.zeros(n_sd, np.uint32), xi, r,
                      np.array([dV]), "golovin", 1.0, steps, seed,
                      {"v0": 4.0 / 3.0 * np.pi * R_MEAN_VOLUME_BOX ** 3, "N0": N0_BOX,
                       "b": 1500.0})


def domain_2d(seed: int = SEEDS[0], nx: int = 75, ny: int = 75, per_cell: int = 64,
              steps: int = 600) -> Population:
    g = _rng(seed)
    n_cells = nx * ny
    n = n_cells * per_cell
    dV = 20.0 * 20.0 * 1.0
    cell = np.repeat(np.arange(n_cells, dtype=np.uint32), per_cell)
    r = _lognormal_radii(g, n, 10e-6, 1.4)
    xi = np.full(n, int(round(CONC_LOGNORMAL * dV / per_cell)), dtype=np.uint64)
    return Population("domain_2d", cell, xi, r, np.full(n_cells, dV), "geometric", 1.0,
                      steps, seed, {"nx": nx, "ny": ny, "per_cell": per_cell})


def _bimodal_radii(g, n):
    first = g.random(n) < 0.9
    r = np.empty(n)
    k = int(first.sum())
    r[first] = _lognormal_radii(g, k, 8e-6, 1.3)
    r[~first] = _lognormal_radii(g, n - k, 25e-6, 1.5)
    return r


def large_domain(seed: int = SEEDS[0], nx: int = 1024, ny: int = 1024, mean: float = 128.0,
                 dV: float = 400.0, steps: int = 200, shuffle: bool = False) -> Population:
    """Poisson(mean) SDs per cell; cells c = 0 (mod 997) are emptied and cells
    c = 1 (mod 991) hold one SD, since Poisson(128) almost never gives either.
    Multiplicity floor(4e10 / n_c) (100 cm^-3 in 400 m^3).  SDs come cell-major
    unless ``shuffle``."""
    g = _rng(seed)
    n_cells = nx * ny
    counts = g.poisson(mean, n_cells).astype(np.int64)
    c = np.arange(n_cells)
    counts[c % 997 == 0] = 0
    counts[(c % 991 == 1) & (c % 997 != 0)] = 1
    n = int(counts.sum())
    cell = np.repeat(np.arange(n_cells, dtype=np.uint32), counts)
    r = _bimodal_radii(g, n)
    per_cell_xi = np.where(counts > 0, np.floor(CONC_LOGNORMAL * dV / np.maximum(counts, 1)), 0)
    xi = np.repeat(per_cell_xi.astype(np.uint64), counts)
    if shuffle:
        p = g.permutation(n)
        cell, r, xi = cell[p], r[p], xi[p]
    return Population("large_domain", cell, xi, r, np.full(n_cells, dV), "geometric", 0.5,
                      steps, seed, {"nx": nx, "ny": ny, "mean": mean})


def _box_instance(g, n_sd, dV, kernel, spectrum, steps, seed, name):
    if spectrum == "exponential":
        r = _exponential_volume_radii(g, n_sd, R_MEAN_VOLUME_BOX)
        conc = N0_BOX
    else:
        r = _lognormal_radii(g, n_sd, 10e-6, 1.4)
        conc = CONC_LOGNORMAL
    xi_val = max(1, int(round(conc * dV / n_sd)))
    return Population(name, np.zeros(n_sd, np.uint32), np.full(n_sd, xi_val, np.uint64), r,
                      np.array([dV]), kernel, 1.0, steps, seed, {"spectrum": spectrum})


def ensemble(seed: int = SEEDS[0], n_instances: int = 4096, log2_lo: float = 8,
             log2_hi: float = 16, steps: int = 1000) -> list:
    """Independent single-cell boxes: N_sd log-uniform in [2^lo, 2^hi], dV uniform
    in [1, 1e6] m^3, half Golovin / half geometric (shuffled), exponential or
    lognormal spectrum per instance."""
    g = _rng(seed)
    kernels = np.array(["golovin"] * (n_instances // 2) +
                       ["geometric"] * (n_instances - n_instances // 2))
    g.shuffle(kernels)
    out = []
    for i in range(n_instances):
        n_sd = int(round(2.0 ** g.uniform(log2_lo, log2_hi)))
        dV = float(g.uniform(1.0, 1e6))
        spectrum = "exponential" if g.random() < 0.5 else "lognormal"
        inst_seed = int(g.integers(0, 2 ** 63))
        out.append(_box_instance(g, n_sd, dV, str(kernels[i]), spectrum, steps, inst_seed,
                                 f"ensemble[{i}]"))
    return out


@dataclass
class Request:
    arrival: float                   # seconds after the stream starts
    pop: Population


def request_stream(seed: int = SEEDS[0], n_requests: int = 2000, rate: float = 10.0,
                   log2_lo: float = 10, log2_hi: float = 20, steps_lo: int = 100,
                   steps_hi: int = 3600, max_cells: int = 256) -> list:
    """Poisson arrivals at ``rate`` per second; each request is a box (one cell) or a
    1D column of U{1..max_cells} cells with N_sd log-uniform in [2^lo, 2^hi] split
    evenly over its cells; run length U{steps_lo..steps_hi}; kernel, spectrum and
    dV drawn as for the ensemble."""
    g = _rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(g.exponential(1.0 / rate))
        n_sd = int(round(2.0 ** g.uniform(log2_lo, log2_hi)))
        n_cells = 1 if g.random() < 0.5 else int(g.integers(1, max_cells + 1))
        n_cells = min(n_cells, n_sd)
        dV = float(g.uniform(1.0, 1e6))
        kernel = "golovin" if g.random() < 0.5 else "geometric"
        spectrum = "exponential" if g.random() < 0.5 else "lognormal"
        steps = int(g.integers(steps_lo, steps_hi + 1))
        inst_seed = int(g.integers(0, 2 ** 63))
        if spectrum == "exponential":
            r = _exponential_volume_radii(g, n_sd, R_MEAN_VOLUME_BOX)
            conc = N0_BOX
        else:
            r = _lognormal_radii(g, n_sd, 10e-6, 1.4)
            conc = CONC_LOGNORMAL
        cell = (np.arange(n_sd, dtype=np.int64) * n_cells // n_sd).astype(np.uint32)
        per_cell = n_sd / n_cells
        xi_val = max(1, int(round(conc * dV / per_cell)))
        pop = Population(f"request[{i}]", cell, np.full(n_sd, xi_val, np.uint64), r,
                         np.full(n_cells, dV), kernel, 1.0, steps, inst_seed,
                         {"spectrum": spectrum})
        out.append(Request(t, pop))
    return out


def tiny_cells(seed: int, n_cells: int, max_per_cell: int, xi_max: int = 1000,
               dead_fraction: float = 0.1, r_lo: float = 5e-6, r_hi: float = 2e-3) -> Population:
    """Edge-case population for parity tests: ragged cells (0..max_per_cell SDs,
    including empty and single-SD cells), small integer multiplicities (many ties
    and equal pairs), some dead SDs, radii log-uniform over [r_lo, r_hi] (all three
    branches of the terminal velocity), SDs in shuffled input order."""
    g = _rng(seed)
    counts = g.integers(0, max_per_cell + 1, n_cells)
    n = int(counts.sum())
    cell = np.repeat(np.arange(n_cells, dtype=np.uint32), counts)
    p = g.permutation(n)
    cell = cell[p]
    xi = g.integers(1, xi_max + 1, n).astype(np.uint64)
    xi[g.random(n) < dead_fraction] = 0
    r = np.exp(g.uniform(np.log(r_lo), np.log(r_hi), n))
    dV = g.uniform(1.0, 100.0, n_cells)
    return Population("tiny_cells", cell, xi, r, dV, "geometric", 1.0, 1, seed)


# ---------------------------------------------------------------- transport inputs
def positions_in_cells(pop: Population, nx: int, nz: int, dx: float, dz: float,
                       seed: int) -> tuple:
    """Positions uniform within each SD's cell (cell = i + nx k), input order."""
    g = _rng(seed ^ 0x5EED)
    i = (pop.cell % nx).astype(np.float64)
    k = (pop.cell // nx).astype(np.float64)
    x = (i + g.random(pop.n_sd)) * dx
    z = (k + g.random(pop.n_sd)) * dz
    # keep every position strictly inside its cell
    x = np.minimum(x, np.nextafter((i + 1.0) * dx, 0.0))
    z = np.minimum(z, np.nextafter((k + 1.0) * dz, 0.0))
    return x, z


def eddy_courant(nx: int, nz: int, dx: float, dz: float, dt: float,
                 w_max: float = 0.6) -> tuple:
    """Courant numbers of the single-eddy kinematic flow on an Arakawa-C grid.

    Stream function psi = -w_max X/pi sin(pi z/Z) cos(2 pi x/X) (X = nx dx,
    Z = nz dz) at the cell corners, constant dry-air density; u = -d psi/dz on the
    x-edges and w = d psi/dx on the z-edges by differences of corner values, so the
    discrete divergence vanishes to round-off.  Returns (cx, cz): cx[k nx + i] on the
    left edge of cell (i, k), cz[k nx + i] on its bottom edge (k = 0..nz)."""
    X, Z = nx * dx, nz * dz
    xc = np.arange(nx + 1) * dx
    zc = np.arange(nz + 1) * dz
    psi = -w_max * X / np.pi * np.sin(np.pi * zc[:, None] / Z) * np.cos(2 * np.pi * xc[None, :] / X)
    u = -(psi[1:, :nx] - psi[:-1, :nx]) / dz           # (nz, nx) on x-edges
    w = (psi[:, 1:] - psi[:, :-1]) / dx                 # (nz + 1, nx) on z-edges
    return (np.ascontiguousarray((u * dt / dx).ravel()),
            np.ascontiguousarray((w * dt / dz).ravel()))
