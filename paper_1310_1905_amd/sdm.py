"""Python binding of the C ABI in ``include/sdm.h`` (ctypes).

Argument marshalling only: PyTorch provides device memory (the workspace and the
SD arrays) and streams; every step of the method runs in the HIP kernels of
``libsdm.so``.  There is no CPU fallback -- loading fails loudly when the library
is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdm.so")

GOLOVIN = 0
GEOMETRIC = 1
KERNELS = {"golovin": GOLOVIN, "geometric": GEOMETRIC}
RULE_RELEASE = 1   # one event when u < P_ij; equal multiplicities leave a zero
RULE_RECYCLE = 2   # recycle zero-multiplicity particles at the start of each step, per cell
RULE_RECYCLE_DOMAIN = 4   # the same over the whole domain (positions needed for several cells)

_P = ctypes.c_void_p
_u32, _u64, _i32, _dbl, _sz = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_size_t)


class KernelParams(ctypes.Structure):
    _fields_ = [("golovin_b", _dbl), ("vt_k1", _dbl), ("vt_k2", _dbl), ("vt_k3", _dbl),
                ("vt_r1", _dbl), ("vt_r2", _dbl), ("efficiency", _dbl)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("group_slots", _u32), ("groups_per_wave", _u32), ("waves_per_block", _u32),
                ("xcd_remap", _u32), ("block_slots", _u32), ("block_split", _u32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class InstanceDesc(ctypes.Structure):
    _fields_ = [("n_sd", _u64), ("n_cells", _u32), ("cell", _P), ("xi", _P), ("r", _P),
                ("dV", _P), ("kernel", ctypes.c_int), ("params", KernelParams), ("dt", _dbl),
                ("seed", _u64), ("first_step", _u64)]


class SdmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsdm.so (build it with ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing; build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "sdm_default_params": (None, [_P]),
        "sdm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sdm_last_error": (ctypes.c_char_p, []),
        "sdm_workspace_bytes": (_sz, [_u64, _u32]),
        "sdm_init": (ctypes.c_int, [_P, _P, _P, _sz, _u64, _P, _P, _P, _u32, _P, _P]),
        "sdm_coalesce_step": (ctypes.c_int, [_P, _dbl, ctypes.c_int, _u64, _u64]),
        "sdm_get_state": (ctypes.c_int, [_P, _P, _P]),
        "sdm_get_stats": (ctypes.c_int, [_P, _P, _P]),
        "sdm_get_layout": (ctypes.c_int, [_P, _P, _P]),
        "sdm_debug_permutation": (ctypes.c_int, [_P, _u64, _u64, _P, _P]),
        "sdm_debug_split_wait": (ctypes.c_int, [_P, _u32, _u32]),
        "sdm_get_plan": (ctypes.c_int, [_P, _P, _P, _P, _P]),
        "sdm_set_rules": (ctypes.c_int, [_P, _u32]),
        "sdm_get_rules": (ctypes.c_int, [_P, _P]),
        "sdm_recycle": (ctypes.c_int, [_P]),
        "sdm_recycle_domain": (ctypes.c_int, [_P]),
        "sdm_get_recycled": (ctypes.c_int, [_P, _P]),
        "sdm_transport_workspace_bytes": (_sz, [_u64, _u32]),
        "sdm_transport_attach": (ctypes.c_int, [_P, _P, _sz, _u32, _u32, _dbl, _dbl, _P, _P]),
        "sdm_transport_step": (ctypes.c_int, [_P, _P, _P, _dbl, ctypes.c_int]),
        "sdm_transport_get_positions": (ctypes.c_int, [_P, _P, _P]),
        "sdm_dry_workspace_bytes": (_sz, [_u64]),
        "sdm_dry_attach": (ctypes.c_int, [_P, _P, _sz, _P, _P]),
        "sdm_dry_get": (ctypes.c_int, [_P, _P, _P]),
        "sdm_diag_dry_moments": (ctypes.c_int, [_P, _u32, _dbl, _dbl, _P, _P]),
        "sdm_diag_sd_conc": (ctypes.c_int, [_P, _P]),
        "sdm_diag_moments": (ctypes.c_int, [_P, _u32, _dbl, _dbl, _P, _P]),
        "sdm_probe_probability": (ctypes.c_int, [_P, _dbl, ctypes.c_int, _u64, _u64, _P, _P]),
        "sdm_coalesce_substeps": (ctypes.c_int, [_P, _dbl, _u32, ctypes.c_int, _u64, _u64]),
        "sdm_coalesce_adaptive": (ctypes.c_int, [_P, _dbl, _dbl, _u32, ctypes.c_int, _u64, _u64,
                                                 _P]),
        "sdm_get_launch_config": (ctypes.c_int, [_P, _P]),
        "sdm_set_launch_config": (ctypes.c_int, [_P, _P]),
        "sdm_autotune_workspace_bytes": (_sz, [_P]),
        "sdm_autotune": (ctypes.c_int, [_P, _P, _sz, _dbl, ctypes.c_int, _u64, _u32, _P]),
        "sdm_destroy": (None, [_P]),
        "sdm_batch_workspace_bytes": (_sz, [_u64, _u32, _u32]),
        "sdm_batch_create": (ctypes.c_int, [_P, _P, _P, _sz, _u64, _u32, _u32]),
        "sdm_batch_add": (ctypes.c_int, [_P, _P, _P]),
        "sdm_batch_step": (ctypes.c_int, [_P, ctypes.c_int]),
        "sdm_batch_get": (ctypes.c_int, [_P, _i32, _P, _P, _P, _P, _P]),
        "sdm_batch_remove": (ctypes.c_int, [_P, _i32, _P, _P]),
        "sdm_batch_info": (ctypes.c_int, [_P, _P, _P, _P]),
        "sdm_batch_destroy": (None, [_P]),
        "sdm_batch_get_launch_config": (ctypes.c_int, [_P, _P]),
        "sdm_batch_set_launch_config": (ctypes.c_int, [_P, _P]),
        "sdm_batch_autotune_workspace_bytes": (_sz, [_P]),
        "sdm_batch_autotune": (ctypes.c_int, [_P, _P, _sz, _u32, _P]),
        "sdm_static_scratch_bytes": (_sz, []),
        "sdm_coalesce_sorted_static": (ctypes.c_int, [_P, _u64, _u32, _P, _P, _P, _P, _dbl,
                                                      ctypes.c_int, _P, _u64, _u64, _P, _P]),
        "sdm_debug_philox": (ctypes.c_int, [_P, _u64, _P, _P, _P]),
        "sdm_debug_cbrt": (ctypes.c_int, [_P, _u64, _P, _P]),
        "sdm_debug_philox_range": (ctypes.c_int, [_P, _u64, _P, _P, _P]),
        "sdm_debug_sqrt_div": (ctypes.c_int, [_P, _u64, _P, _P, _P, _P]),
        "sdm_debug_collide": (ctypes.c_int, [_P, _u64, ctypes.c_int, _P, _dbl, _P, _P, _P,
                                             _P, _P, _P, _P, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols() -> list:
    return [n for n in dir(lib()) if n.startswith("sdm_")]


def _check(status: int, where: str):
    if status != 0:
        L = lib()
        raise SdmError(status, where, f"{L.sdm_strerror(status).decode()}: "
                                      f"{L.sdm_last_error().decode()}")


def _dptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


def _stream_ptr(stream: torch.cuda.Stream | None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def default_params() -> KernelParams:
    p = KernelParams()
    lib().sdm_default_params(ctypes.byref(p))
    return p


def make_params(**kw) -> KernelParams:
    p = default_params()
    for k, v in kw.items():
        setattr(p, k, float(v))
    return p


def _u64_tensor(xi, device) -> torch.Tensor:
    """uint64 multiplicities as an int64 tensor of the same bits."""
    import numpy as np
    if isinstance(xi, torch.Tensor):
        return xi.to(device=device).contiguous()
    a = np.ascontiguousarray(np.asarray(xi, dtype=np.uint64)).view(np.int64)
    return torch.from_numpy(a).to(device)


class Context:
    """One run: SDs in cells, advanced by ``step``.  Owns its workspace tensor."""

    def __init__(self, cell, xi, r, dV, params: KernelParams | None = None,
                 stream: torch.cuda.Stream | None = None, device="cuda"):
        L = lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cell_t = torch.as_tensor(cell, dtype=torch.int32).to(self.device).contiguous()
        xi_t = _u64_tensor(xi, self.device)
        r_t = torch.as_tensor(r, dtype=torch.float64).to(self.device).contiguous()
        dv_t = torch.as_tensor(dV, dtype=torch.float64).to(self.device).contiguous()
        self.n_sd = int(cell_t.numel())
        self.n_cells = int(dv_t.numel())
        ws_bytes = int(L.sdm_workspace_bytes(self.n_sd, self.n_cells))
        self.workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._ctx = _P()
        torch.cuda.synchronize(self.device)
        st = L.sdm_init(ctypes.byref(self._ctx), _stream_ptr(self.stream), aligned,
                        ws_bytes + 256 - (aligned - base), self.n_sd, _dptr(cell_t),
                        _dptr(xi_t), _dptr(r_t), self.n_cells, _dptr(dv_t),
                        ctypes.byref(params) if params is not None else None)
        _check(st, "sdm_init")

    def step(self, dt: float, kernel: int | str, seed: int, step: int):
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        _check(lib().sdm_coalesce_step(self._ctx, float(dt), k, int(seed), int(step)),
               "sdm_coalesce_step")

    def attach_transport(self, x, z, nx: int, nz: int, dx: float, dz: float):
        """Positions (input order) on an nx x nz grid; re-sorts the storage by them."""
        L = lib()
        x_t = torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous()
        z_t = torch.as_tensor(z, dtype=torch.float64).to(self.device).contiguous()
        ws_bytes = int(L.sdm_transport_workspace_bytes(self.n_sd, self.n_cells))
        self.transport_workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8,
                                               device=self.device)
        base = self.transport_workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        torch.cuda.synchronize(self.device)
        _check(L.sdm_transport_attach(self._ctx, aligned, ws_bytes + 256 - (aligned - base),
                                      int(nx), int(nz), float(dx), float(dz), _dptr(x_t),
                                      _dptr(z_t)), "sdm_transport_attach")

    def transport(self, cx, cz, dt: float, sediment: bool = True):
        """Advect by the Courant fields (device tensors or arrays, either None), sediment,
        flag leavers, re-sort by cell."""
        cx_t = None if cx is None else torch.as_tensor(cx, dtype=torch.float64).to(self.device).contiguous()
        cz_t = None if cz is None else torch.as_tensor(cz, dtype=torch.float64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_transport_step(self._ctx, _dptr(cx_t), _dptr(cz_t), float(dt),
                                        1 if sediment else 0), "sdm_transport_step")

    def positions(self):
        """(x, z) float64 tensors in input order."""
        x = torch.empty(max(1, self.n_sd), dtype=torch.float64, device=self.device)
        z = torch.empty(max(1, self.n_sd), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_transport_get_positions(self._ctx, _dptr(x), _dptr(z)),
               "sdm_transport_get_positions")
        return x[: self.n_sd], z[: self.n_sd]

    def attach_dry(self, rd3, kappa):
        """Optional dry attributes (input order): r_d^3 (m^3) and kappa."""
        L = lib()
        rd3_t = torch.as_tensor(rd3, dtype=torch.float64).to(self.device).contiguous()
        kappa_t = torch.as_tensor(kappa, dtype=torch.float64).to(self.device).contiguous()
        ws_bytes = int(L.sdm_dry_workspace_bytes(self.n_sd))
        self.dry_workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.dry_workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        torch.cuda.synchronize(self.device)
        _check(L.sdm_dry_attach(self._ctx, aligned, ws_bytes + 256 - (aligned - base),
                                _dptr(rd3_t), _dptr(kappa_t)), "sdm_dry_attach")

    def dry(self):
        """(r_d^3, kappa) float64 tensors in input order."""
        rd3 = torch.empty(max(1, self.n_sd), dtype=torch.float64, device=self.device)
        kappa = torch.empty(max(1, self.n_sd), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_dry_get(self._ctx, _dptr(rd3), _dptr(kappa)), "sdm_dry_get")
        return rd3[: self.n_sd], kappa[: self.n_sd]

    def dry_moments(self, k: int, rd_min: float = 0.0, rd_max: float = float("inf"),
                    rho_d=None):
        """Per-cell k-th dry-radius moment over r_d in [rd_min, rd_max]."""
        out = torch.empty(max(1, self.n_cells), dtype=torch.float64, device=self.device)
        rho = None
        if rho_d is not None:
            rho = torch.as_tensor(rho_d, dtype=torch.float64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_diag_dry_moments(self._ctx, int(k), float(rd_min), float(rd_max),
                                          _dptr(rho), _dptr(out)), "sdm_diag_dry_moments")
        torch.cuda.synchronize(self.device)
        return out[: self.n_cells]

    def set_rules(self, rules: int):
        """SDM rule flags (RULE_RELEASE | RULE_RECYCLE) for every later step."""
        _check(lib().sdm_set_rules(self._ctx, int(rules)), "sdm_set_rules")

    def rules(self) -> int:
        v = _u32()
        _check(lib().sdm_get_rules(self._ctx, ctypes.byref(v)), "sdm_get_rules")
        return int(v.value)

    def recycle(self):
        _check(lib().sdm_recycle(self._ctx), "sdm_recycle")

    def recycle_domain(self):
        _check(lib().sdm_recycle_domain(self._ctx), "sdm_recycle_domain")

    def recycled(self) -> int:
        v = _u64()
        _check(lib().sdm_get_recycled(self._ctx, ctypes.byref(v)), "sdm_get_recycled")
        return int(v.value)

    def substeps(self, dt: float, n_substeps: int, kernel: int | str, seed: int, first_step: int):
        """n_substeps steps of dt / n_substeps with counters first_step, first_step + 1, ..."""
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        _check(lib().sdm_coalesce_substeps(self._ctx, float(dt), int(n_substeps), k, int(seed),
                                           int(first_step)), "sdm_coalesce_substeps")

    def adaptive(self, dt: float, p_limit: float, max_substeps: int, kernel: int | str, seed: int,
                 first_step: int) -> int:
        """Probe, then ceil(pmax / p_limit) sub-steps; returns the number taken."""
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        n = _u32()
        _check(lib().sdm_coalesce_adaptive(self._ctx, float(dt), float(p_limit), int(max_substeps),
                                           k, int(seed), int(first_step), ctypes.byref(n)),
               "sdm_coalesce_adaptive")
        return int(n.value)

    def probe(self, dt: float, kernel: int | str, seed: int, step: int, per_cell: bool = False):
        """Largest P_ij of step ``step`` (and, with ``per_cell``, a float64 tensor of the
        per-cell maxima); the state is not changed."""
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        cm = torch.empty(max(1, self.n_cells), dtype=torch.float64, device=self.device) \
            if per_cell else None
        g = _dbl()
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_probe_probability(self._ctx, float(dt), k, int(seed), int(step),
                                           _dptr(cm), ctypes.byref(g)), "sdm_probe_probability")
        return (float(g.value), cm[: self.n_cells]) if per_cell else float(g.value)

    def sd_conc(self):
        """Live super-droplets per cell (int32 tensor holding uint32 values)."""
        out = torch.empty(max(1, self.n_cells), dtype=torch.int32, device=self.device)
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_diag_sd_conc(self._ctx, _dptr(out)), "sdm_diag_sd_conc")
        torch.cuda.synchronize(self.device)
        return out[: self.n_cells]

    def moments(self, k: int, r_min: float = 0.0, r_max: float = float("inf"), rho_d=None):
        """Per-cell k-th radius moment, (rho_d dV)^-1 sum xi r^k over r in [r_min, r_max]."""
        out = torch.empty(max(1, self.n_cells), dtype=torch.float64, device=self.device)
        rho = None
        if rho_d is not None:
            rho = torch.as_tensor(rho_d, dtype=torch.float64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_diag_moments(self._ctx, int(k), float(r_min), float(r_max), _dptr(rho),
                                      _dptr(out)), "sdm_diag_moments")
        torch.cuda.synchronize(self.device)
        return out[: self.n_cells]

    def state(self):
        """(xi int64-bits-of-uint64 tensor, r float64 tensor) in input order."""
        xi = torch.empty(self.n_sd, dtype=torch.int64, device=self.device)
        r = torch.empty(self.n_sd, dtype=torch.float64, device=self.device)
        _check(lib().sdm_get_state(self._ctx, _dptr(xi), _dptr(r)), "sdm_get_state")
        return xi, r

    def state_numpy(self):
        import numpy as np
        xi, r = self.state()
        return xi.cpu().numpy().view(np.uint64), r.cpu().numpy()

    def stats(self):
        p, c = _u64(), _u64()
        _check(lib().sdm_get_stats(self._ctx, ctypes.byref(p), ctypes.byref(c)), "sdm_get_stats")
        return int(p.value), int(c.value)

    def layout(self):
        """(offsets int32[n_cells+1], input index int32[n_sd]) device tensors (copies)."""
        off, idx = _P(), _P()
        _check(lib().sdm_get_layout(self._ctx, ctypes.byref(off), ctypes.byref(idx)),
               "sdm_get_layout")
        o = torch.empty(self.n_cells + 1, dtype=torch.int32, device=self.device)
        i = torch.empty(max(1, self.n_sd), dtype=torch.int32, device=self.device)
        nbytes_o = 4 * (self.n_cells + 1)
        nbytes_i = 4 * self.n_sd
        _memcpy_d2d(o.data_ptr(), off.value, nbytes_o, self.stream)
        if nbytes_i:
            _memcpy_d2d(i.data_ptr(), idx.value, nbytes_i, self.stream)
        torch.cuda.synchronize(self.device)
        return o, i[: self.n_sd]

    def permutation(self, seed: int, step: int):
        """(order int32[n_sd] storage-indexed, n_live int32[n_cells]) device tensors."""
        order = torch.full((max(1, self.n_sd),), -1, dtype=torch.int32, device=self.device)
        nlive = torch.zeros(max(1, self.n_cells), dtype=torch.int32, device=self.device)
        torch.cuda.synchronize(self.device)
        _check(lib().sdm_debug_permutation(self._ctx, int(seed), int(step), _dptr(order),
                                           _dptr(nlive)), "sdm_debug_permutation")
        return order[: self.n_sd], nlive[: self.n_cells]

    def debug_split_wait(self, spin_limit: int, epoch_skew: int = 0):
        """Test hook of the split tier's bounded wait (see sdm_debug_split_wait)."""
        _check(lib().sdm_debug_split_wait(self._ctx, int(spin_limit), int(epoch_skew)),
               "sdm_debug_split_wait")

    def plan(self):
        """(wave-tier groups, cells in them, workgroup-tier cells, grid-tier cells)."""
        g, w, b, d = _u32(), _u32(), _u32(), _u32()
        _check(lib().sdm_get_plan(self._ctx, ctypes.byref(g), ctypes.byref(w), ctypes.byref(b),
                                  ctypes.byref(d)), "sdm_get_plan")
        return int(g.value), int(w.value), int(b.value), int(d.value)

    def launch_config(self) -> LaunchConfig:
        c = LaunchConfig()
        _check(lib().sdm_get_launch_config(self._ctx, ctypes.byref(c)), "sdm_get_launch_config")
        return c

    def set_launch_config(self, **kw):
        c = self.launch_config()
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(lib().sdm_set_launch_config(self._ctx, ctypes.byref(c)), "sdm_set_launch_config")

    def autotune(self, dt: float, kernel, seed: int = 0, reps: int = 3) -> LaunchConfig:
        L = lib()
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        nbytes = int(L.sdm_autotune_workspace_bytes(self._ctx))
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = scratch.data_ptr()
        aligned = (base + 255) // 256 * 256
        best = LaunchConfig()
        _check(L.sdm_autotune(self._ctx, aligned, nbytes + 256 - (aligned - base), float(dt), k,
                              int(seed), int(reps), ctypes.byref(best)), "sdm_autotune")
        del scratch
        return best

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().sdm_destroy(self._ctx)
            self._ctx = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _memcpy_d2d(dst: int, src: int, nbytes: int, stream):
    hip = _hip()
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes),
                            ctypes.c_int(3), ctypes.c_void_p(_stream_ptr(stream)))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed: {rc}")


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpyAsync.argtypes = [_P, _P, _sz, ctypes.c_int, _P]
        _hip_lib.hipMemcpyAsync.restype = ctypes.c_int
    return _hip_lib


@dataclass
class InstanceCounters:
    steps_done: int
    pair_tests: int
    collisions: int


class Batch:
    """Many independent instances advanced together (``sdm_batch_*``)."""

    def __init__(self, max_sd: int, max_cells: int, max_instances: int,
                 stream: torch.cuda.Stream | None = None, device="cuda"):
        L = lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        nbytes = int(L.sdm_batch_workspace_bytes(int(max_sd), int(max_cells), int(max_instances)))
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._b = _P()
        torch.cuda.synchronize(self.device)
        _check(L.sdm_batch_create(ctypes.byref(self._b), _stream_ptr(self.stream), aligned,
                                  nbytes + 256 - (aligned - base), int(max_sd), int(max_cells),
                                  int(max_instances)), "sdm_batch_create")
        self.n_sd = {}

    def add(self, cell, xi, r, dV, kernel, dt: float, seed: int, first_step: int = 0,
            params: KernelParams | None = None) -> int:
        """Admit an instance; returns its handle.  Raises SdmError (status -5) when full."""
        cell_t = torch.as_tensor(cell, dtype=torch.int32).to(self.device).contiguous()
        xi_t = _u64_tensor(xi, self.device)
        r_t = torch.as_tensor(r, dtype=torch.float64).to(self.device).contiguous()
        dv_t = torch.as_tensor(dV, dtype=torch.float64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        d = InstanceDesc()
        d.n_sd = int(cell_t.numel())
        d.n_cells = int(dv_t.numel())
        d.cell, d.xi, d.r, d.dV = _dptr(cell_t), _dptr(xi_t), _dptr(r_t), _dptr(dv_t)
        d.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        d.params = params if params is not None else default_params()
        d.dt = float(dt)
        d.seed = int(seed)
        d.first_step = int(first_step)
        h = _i32()
        _check(lib().sdm_batch_add(self._b, ctypes.byref(d), ctypes.byref(h)), "sdm_batch_add")
        self.n_sd[int(h.value)] = d.n_sd
        return int(h.value)

    def step(self, use_graph: bool = True):
        _check(lib().sdm_batch_step(self._b, 1 if use_graph else 0), "sdm_batch_step")

    def get(self, handle: int, with_state: bool = True):
        n = self.n_sd[handle]
        xi = torch.empty(max(1, n), dtype=torch.int64, device=self.device) if with_state else None
        r = torch.empty(max(1, n), dtype=torch.float64, device=self.device) if with_state else None
        sd, pt, co = _u64(), _u64(), _u64()
        _check(lib().sdm_batch_get(self._b, int(handle), _dptr(xi), _dptr(r), ctypes.byref(sd),
                                   ctypes.byref(pt), ctypes.byref(co)), "sdm_batch_get")
        cnt = InstanceCounters(int(sd.value), int(pt.value), int(co.value))
        if with_state:
            return xi[:n], r[:n], cnt
        return None, None, cnt

    def remove(self, handle: int, with_state: bool = True):
        n = self.n_sd[handle]
        xi = torch.empty(max(1, n), dtype=torch.int64, device=self.device) if with_state else None
        r = torch.empty(max(1, n), dtype=torch.float64, device=self.device) if with_state else None
        _check(lib().sdm_batch_remove(self._b, int(handle), _dptr(xi), _dptr(r)),
               "sdm_batch_remove")
        del self.n_sd[handle]
        if with_state:
            return xi[:n], r[:n]
        return None, None

    def launch_config(self) -> LaunchConfig:
        c = LaunchConfig()
        _check(lib().sdm_batch_get_launch_config(self._b, ctypes.byref(c)),
               "sdm_batch_get_launch_config")
        return c

    def set_launch_config(self, **kw):
        c = self.launch_config()
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(lib().sdm_batch_set_launch_config(self._b, ctypes.byref(c)),
               "sdm_batch_set_launch_config")

    def autotune(self, reps: int = 3) -> LaunchConfig:
        """Pick the fastest launch shape for the admitted instances (state unchanged)."""
        L = lib()
        nbytes = int(L.sdm_batch_autotune_workspace_bytes(self._b))
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = scratch.data_ptr()
        aligned = (base + 255) // 256 * 256
        best = LaunchConfig()
        torch.cuda.synchronize(self.device)
        _check(L.sdm_batch_autotune(self._b, aligned, nbytes + 256 - (aligned - base), int(reps),
                                    ctypes.byref(best)), "sdm_batch_autotune")
        return best

    def info(self):
        n, fsd, fc = _u32(), _u64(), _u32()
        _check(lib().sdm_batch_info(self._b, ctypes.byref(n), ctypes.byref(fsd), ctypes.byref(fc)),
               "sdm_batch_info")
        return int(n.value), int(fsd.value), int(fc.value)

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().sdm_batch_destroy(self._b)
            self._b = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ element-wise checks
def coalesce_sorted_static(offsets: torch.Tensor, xi: torch.Tensor, r: torch.Tensor,
                           dV: torch.Tensor, dt: float, kernel, seed: int, step: int,
                           params: KernelParams | None = None, stream=None):
    """sdm_coalesce_sorted_static: one step, in place, of SDs kept sorted by cell
    (offsets uint32[n_cells + 1] as int32 or uint32 storage, xi int64 viewed as
    uint64, r and dV float64, all on the device).  Returns (pair tests,
    collisions) of the step."""
    L = lib()
    n_cells = int(dV.numel())
    assert offsets.numel() == n_cells + 1
    assert offsets.element_size() == 4 and xi.element_size() == 8
    pt, co = ctypes.c_uint64(0), ctypes.c_uint64(0)
    st = L.sdm_coalesce_sorted_static(
        _stream_ptr(stream), int(xi.numel()), n_cells, _dptr(offsets), _dptr(xi), _dptr(r),
        _dptr(dV), float(dt), KERNELS.get(kernel, kernel),
        ctypes.byref(params) if params is not None else None, int(seed), int(step),
        ctypes.byref(pt), ctypes.byref(co))
    _check(st, "sdm_coalesce_sorted_static")
    return int(pt.value), int(co.value)


def debug_philox(ctr: torch.Tensor, key: torch.Tensor) -> torch.Tensor:
    n = ctr.numel() // 4
    out = torch.empty(4 * n, dtype=torch.int32, device=ctr.device)
    _check(lib().sdm_debug_philox(_stream_ptr(None), n, _dptr(ctr), _dptr(key), _dptr(out)),
           "sdm_debug_philox")
    return out


def debug_philox_range(n: int, counter, key, out: torch.Tensor | None = None) -> torch.Tensor:
    """uint32 (as int32) tensor [n, 4]: Philox of counters (c0 + lo32(i), c1 + hi32(i),
    c2, c3) under key (k0, k1)."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in counter])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    _check(lib().sdm_debug_philox_range(_stream_ptr(None), n, c, k, _dptr(out)),
           "sdm_debug_philox_range")
    return out


def debug_sqrt_div(a: torch.Tensor, b: torch.Tensor):
    """(sqrt(a), a / b) float64 tensors, with the step's own arithmetic."""
    sq = torch.empty_like(a)
    q = torch.empty_like(a)
    _check(lib().sdm_debug_sqrt_div(_stream_ptr(None), a.numel(), _dptr(a), _dptr(b), _dptr(sq),
                                    _dptr(q)), "sdm_debug_sqrt_div")
    return sq, q


def debug_cbrt(x: torch.Tensor) -> torch.Tensor:
    y = torch.empty_like(x)
    _check(lib().sdm_debug_cbrt(_stream_ptr(None), x.numel(), _dptr(x), _dptr(y)),
           "sdm_debug_cbrt")
    return y


def debug_collide(kernel, dt, n_live, dV, u, xi_a, r_a, xi_b, r_b, params=None):
    """Runs one collision test per element; updates xi/r tensors in place and returns (K, p, gamma)."""
    n = xi_a.numel()
    K = torch.empty(n, dtype=torch.float64, device=xi_a.device)
    p = torch.empty_like(K)
    g = torch.empty(n, dtype=torch.int64, device=xi_a.device)
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    _check(lib().sdm_debug_collide(_stream_ptr(None), n, k,
                                   ctypes.byref(params) if params is not None else None,
                                   float(dt), _dptr(n_live), _dptr(dV), _dptr(u), _dptr(xi_a),
                                   _dptr(r_a), _dptr(xi_b), _dptr(r_b), _dptr(K), _dptr(p),
                                   _dptr(g)), "sdm_debug_collide")
    return K, p, g
