"""FP64 CPU oracle for the super-droplet coalescence step -- TEST INFRASTRUCTURE ONLY.

Loads ``sdm_oracle.c`` (built with gcc, ``-O2 -ffp-contract=off``) through ctypes and
offers the whole-run helpers the tests use.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package; the HIP library
never does, and this package imports nothing from it.

The method follows the Coalescence subsection (Sect. 5.1.4) of the libcloudph++ 0.2
paper: random non-overlapping pairs per cell and sub-step, the collision probability of
eq. (P_ij), comparison against a uniform deviate on (0,1), and the multiplicity / radius
bookkeeping of a collision event, extended by multiple coalescence with the gamma cap.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdm_oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD_DIR, "libsdm_oracle.so")

GOLOVIN = 0
GEOMETRIC = 1

# Outcome rules (bit flags): the paper's release rule (one event when u < P_ij,
# equal multiplicities leave a zero-multiplicity particle) and recycling of
# zero-multiplicity particles at the start of each step.
RULE_FIDELITY = 1
RULE_RECYCLE = 2
# Recycling over the whole domain: donors are the highest-multiplicity particles
# of the domain and a recycled particle takes all of a donor's properties,
# location included (so it joins the donor's cell); see SlotState.recycle_domain.
RULE_RECYCLE_DOMAIN = 4

# Default kernel parameters: Golovin b = 1500 s^-1; terminal velocity after
# Rogers & Yau (1989) in SI units (k1 r^2 below 40 um, k2 r up to 600 um,
# k3 sqrt(r) above); collection efficiency E = 1.
DEFAULT_PARAMS = (1500.0, 1.19e8, 8.0e3, 201.0, 40e-6, 600e-6, 1.0)

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (no fast-math, no FP contraction)."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    if (not force and os.path.exists(_LIB_PATH)
            and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC)):
        return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    path = build()
    L = ctypes.CDLL(path)
    u32, u64, dbl, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    P = ctypes.c_void_p
    L.oracle_philox4x32_10.argtypes = [P, P, P]
    L.oracle_philox4x32_10.restype = None
    L.oracle_philox_range.argtypes = [u64, u64, P, P, P]
    L.oracle_philox_range.restype = None
    L.oracle_shuffle_key.argtypes = [u64, u32, u32, u32]
    L.oracle_shuffle_key.restype = u32
    L.oracle_pair_uniform.argtypes = [u64, u32, u32, u32]
    L.oracle_pair_uniform.restype = dbl
    L.oracle_cbrt_rn.argtypes = [dbl]
    L.oracle_cbrt_rn.restype = dbl
    L.oracle_terminal_velocity.argtypes = [P, dbl]
    L.oracle_terminal_velocity.restype = dbl
    L.oracle_kernel.argtypes = [i32, P, dbl, dbl]
    L.oracle_kernel.restype = dbl
    L.oracle_upscale.argtypes = [u32]
    L.oracle_upscale.restype = dbl
    L.oracle_probability.argtypes = [u64, dbl, dbl, dbl, dbl]
    L.oracle_probability.restype = dbl
    L.oracle_gamma.argtypes = [dbl, dbl, u64, u64]
    L.oracle_gamma.restype = u64
    L.oracle_collide_pair.argtypes = [u64, P, P, P, P]
    L.oracle_collide_pair.restype = None
    L.oracle_cell_order.argtypes = [u32, P, u64, u32, u32, P]
    L.oracle_cell_order.restype = u32
    L.oracle_step.argtypes = [u32, P, P, P, P, dbl, i32, P, u64, u32, u32, P]
    L.oracle_step.restype = i32
    L.oracle_step_rules.argtypes = [u32, P, P, P, P, dbl, i32, P, u64, u32, u32, P, u32]
    L.oracle_step_rules.restype = i32
    L.oracle_gamma_fidelity.argtypes = [dbl, dbl]
    L.oracle_gamma_fidelity.restype = u64
    L.oracle_collide_pair_fidelity.argtypes = [u64, P, P, P, P]
    L.oracle_collide_pair_fidelity.restype = None
    L.oracle_recycle_cell.argtypes = [u32, P, P]
    L.oracle_recycle_cell.restype = u32
    L.oracle_recycle_cell_dry.argtypes = [u32, P, P, P, P]
    L.oracle_recycle_cell_dry.restype = u32
    L.oracle_recycle_domain.argtypes = [u32, P, P, P, P, P, P]
    L.oracle_recycle_domain.restype = u32
    L.oracle_step_dry.argtypes = [u32, P, P, P, P, dbl, i32, P, u64, u32, u32, P, u32, P, P]
    L.oracle_step_dry.restype = i32
    L.oracle_dry_merge.argtypes = [u64, dbl, dbl, dbl, dbl, P, P]
    L.oracle_dry_merge.restype = None
    L.oracle_dry_radii.argtypes = [u64, P, P]
    L.oracle_dry_radii.restype = None
    L.oracle_sort_by_cell.argtypes = [u64, P, u32, P, P]
    L.oracle_sort_by_cell.restype = i32
    L.oracle_moments.argtypes = [u32, P, P, P, P, i32, dbl, dbl, P, P]
    L.oracle_moments.restype = None
    L.oracle_moment_cell.argtypes = [u32, P, P, i32, dbl, dbl, dbl, dbl]
    L.oracle_moment_cell.restype = dbl
    L.oracle_sd_conc.argtypes = [u32, P, P, P]
    L.oracle_sd_conc.restype = None
    L.oracle_max_probability.argtypes = [u32, P, P, P, P, dbl, i32, P, u64, u32, u32, P]
    L.oracle_max_probability.restype = dbl
    L.oracle_advect_1d.argtypes = [dbl, dbl, u32, dbl, dbl]
    L.oracle_advect_1d.restype = dbl
    L.oracle_transport.argtypes = [u64, u32, u32, dbl, dbl, P, P, dbl, i32, P, P, P, P, P, P]
    L.oracle_transport.restype = None
    L.oracle_resort.argtypes = [u64, P, u32, P, P]
    L.oracle_resort.restype = None
    _lib = L
    return L


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _params(params) -> np.ndarray:
    p = np.asarray(DEFAULT_PARAMS if params is None else params, dtype=np.float64)
    assert p.shape == (7,)
    return np.ascontiguousarray(p)


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key) -> tuple:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(v) for v in out)


def philox_range(n: int, ctr, key, threads: int = 8) -> np.ndarray:
    """uint32 [n, 4]: Philox of the counters (c0 + lo32(i), c1 + hi32(i), c2, c3),
    i < n, under key (k0, k1); ranges of i run in separate threads."""
    c = np.asarray([int(v) & 0xFFFFFFFF for v in ctr], dtype=np.uint32)
    k = np.asarray([int(v) & 0xFFFFFFFF for v in key], dtype=np.uint32)
    out = np.empty((n, 4), dtype=np.uint32)
    bounds = np.linspace(0, n, max(1, threads) + 1).astype(np.int64)

    def part(t):
        lo, hi = int(bounds[t]), int(bounds[t + 1])
        if hi > lo:
            lib().oracle_philox_range(lo, hi - lo, _ptr(c), _ptr(k), out[lo:].ctypes.data)

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(part, range(len(bounds) - 1)))
    return out


def shuffle_key(seed: int, cell: int, step: int, slot: int) -> int:
    return int(lib().oracle_shuffle_key(seed, cell, step, slot))


def pair_uniform(seed: int, cell: int, step: int, m: int) -> float:
    return float(lib().oracle_pair_uniform(seed, cell, step, m))


def cbrt_rn(x: float) -> float:
    return float(lib().oracle_cbrt_rn(x))


def terminal_velocity(r: float, params=None) -> float:
    p = _params(params)
    return float(lib().oracle_terminal_velocity(_ptr(p), r))


def kernel(kind: int, ra: float, rb: float, params=None) -> float:
    p = _params(params)
    return float(lib().oracle_kernel(kind, _ptr(p), ra, rb))


def upscale(n: int) -> float:
    return float(lib().oracle_upscale(n))


def probability(xi_max: int, K: float, dt: float, dV: float, scale: float) -> float:
    return float(lib().oracle_probability(xi_max, K, dt, dV, scale))


def gamma(p: float, u: float, xi_j: int, xi_k: int) -> int:
    return int(lib().oracle_gamma(p, u, xi_j, xi_k))


def collide_pair(g: int, xi_j: int, r_j: float, xi_k: int, r_k: float):
    a = np.array([xi_j, xi_k], dtype=np.uint64)
    r = np.array([r_j, r_k], dtype=np.float64)
    lib().oracle_collide_pair(g, a.ctypes.data, r.ctypes.data, a.ctypes.data + 8,
                              r.ctypes.data + 8)
    return int(a[0]), float(r[0]), int(a[1]), float(r[1])


def gamma_fidelity(p: float, u: float) -> int:
    return int(lib().oracle_gamma_fidelity(p, u))


def collide_pair_fidelity(g: int, xi_j: int, r_j: float, xi_k: int, r_k: float):
    a = np.array([xi_j, xi_k], dtype=np.uint64)
    r = np.array([r_j, r_k], dtype=np.float64)
    lib().oracle_collide_pair_fidelity(g, a.ctypes.data, r.ctypes.data, a.ctypes.data + 8,
                                       r.ctypes.data + 8)
    return int(a[0]), float(r[0]), int(a[1]), float(r[1])


def recycle_cell(xi_cell, r_cell, rd3_cell=None, kappa_cell=None):
    """Recycle one cell in place on copies; returns (xi, r, number recycled), or
    (xi, r, rd3, kappa, number recycled) with the dry attributes."""
    xi = np.array(xi_cell, dtype=np.uint64)
    r = np.array(r_cell, dtype=np.float64)
    if rd3_cell is None:
        n = lib().oracle_recycle_cell(xi.size, _ptr(xi), _ptr(r))
        return xi, r, int(n)
    rd3 = np.array(rd3_cell, dtype=np.float64)
    kappa = np.array(kappa_cell, dtype=np.float64)
    n = lib().oracle_recycle_cell_dry(xi.size, _ptr(xi), _ptr(r), _ptr(rd3), _ptr(kappa))
    return xi, r, rd3, kappa, int(n)


def dry_merge(g: int, rd3_j: float, kappa_j: float, rd3_k: float, kappa_k: float):
    """(r_d^3, kappa) of the droplets formed by g events between j and k."""
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().oracle_dry_merge(g, rd3_j, kappa_j, rd3_k, kappa_k, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def _column(v: float, d: float, n: int) -> int:
    """floor(v / d) clamped to [0, n - 1], as the oracle's transport computes it."""
    f = np.floor(v / d)
    return 0 if f < 0 else (n - 1 if f >= n else int(f))


def advect_1d(x: float, d: float, i: int, c_l: float, c_r: float) -> float:
    return float(lib().oracle_advect_1d(x, d, i, c_l, c_r))


def cell_order(xi_cell: np.ndarray, seed: int, cell: int, step: int) -> np.ndarray:
    xi_cell = np.ascontiguousarray(xi_cell, dtype=np.uint64)
    order = np.zeros(max(1, xi_cell.size), dtype=np.uint32)
    n = lib().oracle_cell_order(xi_cell.size, _ptr(xi_cell), seed, cell, step, _ptr(order))
    return order[:n].copy()


# ---------------------------------------------------------------- whole runs
class SlotState:
    """Super-droplets in canonical storage order: stable-sorted by cell."""

    def __init__(self, cell, xi, r, dV):
        cell = np.ascontiguousarray(cell, dtype=np.uint32)
        self.n_cells = int(len(dV))
        self.dV = np.ascontiguousarray(dV, dtype=np.float64)
        self.offsets = np.zeros(self.n_cells + 1, dtype=np.uint64)
        self.id = np.zeros(cell.size, dtype=np.uint64)
        rc = lib().oracle_sort_by_cell(cell.size, _ptr(cell), self.n_cells,
                                       _ptr(self.offsets), _ptr(self.id))
        if rc != 0:
            raise ValueError("cell index out of range")
        idx = self.id.astype(np.int64)
        self.xi = np.ascontiguousarray(np.asarray(xi, dtype=np.uint64)[idx])
        self.r = np.ascontiguousarray(np.asarray(r, dtype=np.float64)[idx])
        self.stats = np.zeros(2, dtype=np.uint64)
        self.rd3 = None
        self.kappa = None

    def set_dry(self, rd3, kappa):
        """Attach the optional dry attributes (input order): r_d^3 and kappa."""
        idx = self.id.astype(np.int64)
        self.rd3 = np.ascontiguousarray(np.asarray(rd3, dtype=np.float64)[idx])
        self.kappa = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64)[idx])

    def _dry_ptrs(self, base: int):
        if self.rd3 is None:
            return None, None
        return self.rd3[base:].ctypes.data, self.kappa[base:].ctypes.data

    def recycle_domain(self) -> int:
        """Recycling over the whole domain (the procedure of Sect. 5.1.4 with no
        restriction to a cell): each recycled slot takes its donor's properties,
        location included.  With positions attached the storage is then re-sorted
        by the cells of the positions (stable in the old storage order); a state of
        one cell needs no positions.  Returns the number of recycled slots."""
        has_pos = hasattr(self, "x")
        if self.n_cells > 1 and not has_pos:
            raise ValueError("domain-wide recycling of several cells needs positions")
        rd3_p = None if self.rd3 is None else _ptr(self.rd3)
        kappa_p = None if self.rd3 is None else _ptr(self.kappa)
        n = int(lib().oracle_recycle_domain(self.xi.size, _ptr(self.xi), _ptr(self.r), rd3_p,
                                            kappa_p, _ptr(self.x) if has_pos else None,
                                            _ptr(self.z) if has_pos else None))
        self.recycled = getattr(self, "recycled", 0) + n
        if has_pos and n > 0:
            nx, nz, dx, dz = self.grid
            i = np.clip(np.floor(self.x / dx), 0, nx - 1).astype(np.uint32)
            k = np.clip(np.floor(self.z / dz), 0, nz - 1).astype(np.uint32)
            self._resort(i + np.uint32(nx) * k)
        return n

    def step(self, dt: float, kind: int, seed: int, step: int, params=None,
             cells: tuple | None = None, cell_index_base: int = 0, rules: int = 0):
        """One coalescence step over all cells, or over the cell range ``cells``.
        With RULE_RECYCLE_DOMAIN the domain-wide recycling runs first."""
        if rules & RULE_RECYCLE_DOMAIN:
            assert cells is None, "domain-wide recycling steps the whole domain"
            self.recycle_domain()
            rules &= ~RULE_RECYCLE_DOMAIN
        p = _params(params)
        c0, c1 = (0, self.n_cells) if cells is None else cells
        off = np.ascontiguousarray(self.offsets[c0:c1 + 1])
        dv = np.ascontiguousarray(self.dV[c0:c1])
        base = int(off[0]) if off.size else 0
        # slices of xi / r starting at the first slot of cell c0, offsets rebased
        rel = np.ascontiguousarray(off - np.uint64(base))
        xi_view = self.xi[base:]
        r_view = self.r[base:]
        st = np.zeros(2, dtype=np.uint64)
        rd3_p, kappa_p = self._dry_ptrs(base)
        lib().oracle_step_dry(c1 - c0, _ptr(rel), _ptr(dv), xi_view.ctypes.data,
                              r_view.ctypes.data, dt, kind, _ptr(p), seed, step,
                              cell_index_base + c0, _ptr(st), rules, rd3_p, kappa_p)
        self.stats += st
        return st

    def step_parallel(self, dt, kind, seed, step, params=None, threads: int = 8, rules: int = 0):
        """Same result as ``step``: cells are independent, so ranges of cells run
        in separate threads (ctypes releases the GIL)."""
        if rules & RULE_RECYCLE_DOMAIN:
            self.recycle_domain()
            rules &= ~RULE_RECYCLE_DOMAIN
        n = self.n_cells
        if threads <= 1 or n < 2 * threads:
            return self.step(dt, kind, seed, step, params, rules=rules)
        bounds = np.linspace(0, n, threads + 1).astype(int)
        parts = [(int(bounds[i]), int(bounds[i + 1])) for i in range(threads)]
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(lambda cr: self._step_range(dt, kind, seed, step, params, cr, rules),
                              parts))
        st = np.sum(res, axis=0).astype(np.uint64)
        self.stats += st
        return st

    def _step_range(self, dt, kind, seed, step, params, cr, rules=0):
        p = _params(params)
        c0, c1 = cr
        off = np.ascontiguousarray(self.offsets[c0:c1 + 1])
        dv = np.ascontiguousarray(self.dV[c0:c1])
        base = int(off[0])
        rel = np.ascontiguousarray(off - np.uint64(base))
        st = np.zeros(2, dtype=np.uint64)
        rd3_p, kappa_p = self._dry_ptrs(base)
        lib().oracle_step_dry(c1 - c0, _ptr(rel), _ptr(dv), self.xi[base:].ctypes.data,
                              self.r[base:].ctypes.data, dt, kind, _ptr(p), seed, step, c0,
                              _ptr(st), rules, rd3_p, kappa_p)
        return st

    def moments(self, k: int, r_min: float = 0.0, r_max: float = float("inf"), rho_d=None):
        """Per-cell k-th moment of the radius distribution, (rho_d dV)^-1 sum N r^k."""
        out = np.zeros(self.n_cells)
        rho = None if rho_d is None else np.ascontiguousarray(rho_d, dtype=np.float64)
        lib().oracle_moments(self.n_cells, _ptr(self.offsets), _ptr(self.dV), _ptr(self.xi),
                             _ptr(self.r), k, r_min, r_max,
                             None if rho is None else _ptr(rho), _ptr(out))
        return out

    def dry_moments(self, k: int, rd_min: float = 0.0, rd_max: float = float("inf"),
                    rho_d=None):
        """Per-cell k-th moment of the dry-radius distribution, r_d the correctly
        rounded cube root of r_d^3; same selection and summation as ``moments``."""
        rd = np.zeros(max(1, self.rd3.size))
        lib().oracle_dry_radii(self.rd3.size, _ptr(self.rd3), _ptr(rd))
        rd = np.ascontiguousarray(rd[:self.rd3.size])
        out = np.zeros(self.n_cells)
        rho = None if rho_d is None else np.ascontiguousarray(rho_d, dtype=np.float64)
        lib().oracle_moments(self.n_cells, _ptr(self.offsets), _ptr(self.dV), _ptr(self.xi),
                             _ptr(rd), k, rd_min, rd_max,
                             None if rho is None else _ptr(rho), _ptr(out))
        return out

    def sd_conc(self):
        out = np.zeros(self.n_cells, dtype=np.uint32)
        lib().oracle_sd_conc(self.n_cells, _ptr(self.offsets), _ptr(self.xi), _ptr(out))
        return out

    def max_probability(self, dt, kind, seed, step, params=None, per_cell: bool = False):
        """Largest P_ij over the pairs ``step`` would test; with ``per_cell`` also
        the per-cell maxima.  The state is not changed."""
        p = _params(params)
        cm = np.zeros(max(1, self.n_cells))
        g = float(lib().oracle_max_probability(self.n_cells, _ptr(self.offsets), _ptr(self.dV),
                                               _ptr(self.xi), _ptr(self.r), dt, kind, _ptr(p),
                                               seed, step, 0, _ptr(cm)))
        return (g, cm[:self.n_cells].copy()) if per_cell else g

    def set_positions(self, x, z, nx: int, nz: int, dx: float, dz: float):
        """Attach positions (input order) on an nx x nz grid; the cells are taken from
        the positions and the storage is re-sorted by them (stable)."""
        assert nx * nz == self.n_cells
        self.grid = (int(nx), int(nz), float(dx), float(dz))
        idx = self.id.astype(np.int64)
        self.x = np.ascontiguousarray(np.asarray(x, dtype=np.float64)[idx])
        self.z = np.ascontiguousarray(np.asarray(z, dtype=np.float64)[idx])
        i = np.clip(np.floor(self.x / dx), 0, nx - 1).astype(np.uint32)
        k = np.clip(np.floor(self.z / dz), 0, nz - 1).astype(np.uint32)
        self._resort(i + np.uint32(nx) * k)

    def _resort(self, cell):
        order = np.zeros(max(1, cell.size), dtype=np.uint64)
        off = np.zeros(self.n_cells + 1, dtype=np.uint64)
        cell = np.ascontiguousarray(cell, dtype=np.uint32)
        lib().oracle_resort(cell.size, _ptr(cell), self.n_cells, _ptr(off), _ptr(order))
        o = order[:cell.size].astype(np.int64)
        self.offsets = off
        self.xi = np.ascontiguousarray(self.xi[o])
        self.r = np.ascontiguousarray(self.r[o])
        self.id = np.ascontiguousarray(self.id[o])
        self.x = np.ascontiguousarray(self.x[o])
        self.z = np.ascontiguousarray(self.z[o])
        if self.rd3 is not None:
            self.rd3 = np.ascontiguousarray(self.rd3[o])
            self.kappa = np.ascontiguousarray(self.kappa[o])

    def transport(self, cx, cz, dt: float, sediment: bool = True, params=None):
        """Advect (Courant fields cx: nz*nx, cz: (nz+1)*nx, either None), sediment,
        drop leavers, re-sort by cell."""
        nx, nz, dx, dz = self.grid
        p = _params(params)
        cxa = None if cx is None else np.ascontiguousarray(cx, dtype=np.float64)
        cza = None if cz is None else np.ascontiguousarray(cz, dtype=np.float64)
        cell = np.zeros(max(1, self.xi.size), dtype=np.uint32)
        lib().oracle_transport(self.xi.size, nx, nz, dx, dz,
                               None if cxa is None else _ptr(cxa),
                               None if cza is None else _ptr(cza), dt, 1 if sediment else 0,
                               _ptr(p), _ptr(self.x), _ptr(self.z), _ptr(self.xi),
                               _ptr(self.r), _ptr(cell))
        self._resort(cell[:self.xi.size])

    def positions_input_order(self):
        x = np.empty_like(self.x)
        z = np.empty_like(self.z)
        x[self.id.astype(np.int64)] = self.x
        z[self.id.astype(np.int64)] = self.z
        return x, z

    def dry_input_order(self):
        """(r_d^3, kappa) scattered back to input order."""
        rd3 = np.empty_like(self.rd3)
        kappa = np.empty_like(self.kappa)
        idx = self.id.astype(np.int64)
        rd3[idx] = self.rd3
        kappa[idx] = self.kappa
        return rd3, kappa

    def input_order(self):
        """(xi, r) scattered back to input order."""
        xi = np.empty_like(self.xi)
        r = np.empty_like(self.r)
        idx = self.id.astype(np.int64)
        xi[idx] = self.xi
        r[idx] = self.r
        return xi, r


def run(cell, xi, r, dV, steps: int, dt: float, kind: int, seed: int,
        first_step: int = 0, params=None, threads: int = 1):
    """Run ``steps`` coalescence steps (step numbers first_step, first_step+1, ...)
    and return (xi, r, stats) in input order."""
    st = SlotState(cell, xi, r, dV)
    for t in range(first_step, first_step + steps):
        if threads > 1:
            st.step_parallel(dt, kind, seed, t, params, threads)
        else:
            st.step(dt, kind, seed, t, params)
    xo, ro = st.input_order()
    return xo, ro, st.stats.copy()
