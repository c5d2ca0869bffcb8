"""The C-ABI library loads on the CPU host and exports every function that
include/sdm.h declares; host-only calls (sizes, defaults, error paths that fail
before any device work) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "sdm.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1310_1905_amd import sdm
    if not os.path.exists(sdm.LIB_PATH):
        from paper_1310_1905_amd import build
        build.build()
    return sdm.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["sdm_init", "sdm_coalesce_step", "sdm_get_state", "sdm_get_stats",
                     "sdm_debug_permutation", "sdm_destroy", "sdm_workspace_bytes",
                     "sdm_batch_create", "sdm_batch_add", "sdm_batch_step", "sdm_batch_remove"]:
        assert required in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_calls(L):
    from paper_1310_1905_amd import sdm
    p = sdm.default_params()
    assert (p.golovin_b, p.vt_k1, p.vt_k2, p.vt_k3, p.vt_r1, p.vt_r2, p.efficiency) == \
        (1500.0, 1.19e8, 8.0e3, 201.0, 40e-6, 600e-6, 1.0)
    small = L.sdm_workspace_bytes(1000, 10)
    big = L.sdm_workspace_bytes(2000, 10)
    assert 16 * 1000 < small < big
    assert L.sdm_batch_workspace_bytes(1000, 10, 4) > 16 * 1000
    assert L.sdm_strerror(0) == b"ok"
    assert L.sdm_strerror(-1) == b"invalid argument"


def test_error_paths_before_device_work(L):
    # NULL out pointer / NULL context / bad workspace are rejected on the host
    assert L.sdm_init(None, None, None, 0, 0, None, None, None, 0, None, None) == -1
    assert L.sdm_coalesce_step(None, 1.0, 0, 0, 0) == -1
    assert b"NULL" in L.sdm_last_error()
    out = ctypes.c_void_p()
    # misaligned workspace
    assert L.sdm_init(ctypes.byref(out), None, 8, 1 << 20, 0, None, None, None, 0, None, None) == -1
    # n_sd >= 2^32
    assert L.sdm_init(ctypes.byref(out), None, 256, 1 << 20, 1 << 32, 256, 256, 256, 1, 256,
                      None) == -1
    assert out.value is None
    assert L.sdm_batch_create(ctypes.byref(out), None, 256, 1 << 20, 100, 0, 1) == -1


def test_null_context_rejected_by_every_context_call(L):
    """Every entry point that takes a context reports SDM_EINVAL for NULL, on the host."""
    calls = [
        lambda: L.sdm_get_state(None, None, None),
        lambda: L.sdm_get_stats(None, None, None),
        lambda: L.sdm_debug_permutation(None, 0, 0, None, None),
        lambda: L.sdm_set_rules(None, 0),
        lambda: L.sdm_get_rules(None, None),
        lambda: L.sdm_recycle(None),
        lambda: L.sdm_get_recycled(None, None),
        lambda: L.sdm_diag_sd_conc(None, None),
        lambda: L.sdm_diag_moments(None, 0, 0.0, 1.0, None, None),
        lambda: L.sdm_probe_probability(None, 1.0, 0, 0, 0, None, None),
        lambda: L.sdm_coalesce_substeps(None, 1.0, 1, 0, 0, 0),
        lambda: L.sdm_coalesce_adaptive(None, 1.0, 0.5, 4, 0, 0, 0, None),
        lambda: L.sdm_transport_attach(None, None, 0, 1, 1, 1.0, 1.0, None, None),
        lambda: L.sdm_transport_step(None, None, None, 1.0, 0),
        lambda: L.sdm_transport_get_positions(None, None, None),
    ]
    for call in calls:
        assert call() == -1
        assert b"NULL" in L.sdm_last_error()


def test_transport_workspace_grows_with_size(L):
    a = L.sdm_transport_workspace_bytes(1000, 16)
    b = L.sdm_transport_workspace_bytes(2000, 16)
    c = L.sdm_transport_workspace_bytes(2000, 4096)
    assert 56 * 1000 < a < b < c
