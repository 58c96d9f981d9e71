"""The C-ABI library loads, exports every declared entry point and reports
argument errors through codes and pepsgo_last_error (no device compute)."""
import os
import re

import pytest

from paper_1611_09467_amd import binding as bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pepsgo.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(pepsgo_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(bd.DEFAULT_LIB):
        pytest.fail("libpepsgo.so is not built (python -m paper_1611_09467_amd.build)")
    return bd.load_library()


def test_exports_every_declared_symbol(L):
    decl = declared_functions()
    assert len(decl) >= 12
    assert set(decl) == set(bd.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name


def test_version(L):
    assert bd.pepsgo_version(L) == (0, 1)


def test_null_arguments_are_einval(L):
    import ctypes
    assert L.pepsgo_create(0, None) == bd.PEPSGO_EINVAL
    assert b"NULL" in L.pepsgo_last_error()
    assert L.pepsgo_destroy(None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_peps_free(None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_evaluate(None, None, 0, None, None, None, None, None, None, None, 0,
                             None) == bd.PEPSGO_EINVAL
    n = ctypes.c_size_t()
    assert L.pepsgo_workspace_bytes(None, None, 1, ctypes.byref(n)) == bd.PEPSGO_EINVAL
    assert L.pepsgo_profile(None, 1) == bd.PEPSGO_EINVAL
    h = ctypes.c_void_p()
    assert L.pepsgo_serve_create(None, None, ctypes.byref(h)) == bd.PEPSGO_EINVAL
    rid = ctypes.c_uint64()
    assert L.pepsgo_serve_submit(None, None, None, 1, None, None, None, None, None, None,
                                 ctypes.byref(rid)) == bd.PEPSGO_EINVAL
    assert L.pepsgo_serve_poll(None, None, 0, 0) == bd.PEPSGO_EINVAL
    k = ctypes.c_int()
    assert L.pepsgo_serve_pending(None, ctypes.byref(k)) == bd.PEPSGO_EINVAL
    assert L.pepsgo_serve_destroy(None) == bd.PEPSGO_EINVAL
    t = bd.Tuning()
    assert L.pepsgo_tune_get(None, 6, 12, 0, ctypes.byref(t)) == bd.PEPSGO_EINVAL
    assert L.pepsgo_tune_set(None, 6, 12, 0, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_autotune(None, None, 1, None, None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_tune_save(None, b"x") == bd.PEPSGO_EINVAL
    assert L.pepsgo_tune_load(None, b"x") == bd.PEPSGO_EINVAL
    assert L.pepsgo_graph_create(None, None, 1, None, None, None, None, None, None, None, 0,
                                 ctypes.byref(h)) == bd.PEPSGO_EINVAL
    assert L.pepsgo_graph_launch(None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_graph_free(None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_metropolis_step(None, None, 1, None, None, None, None, None, None, None,
                                    None, None, None, 0, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_peps_read(None, None, 0, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_go_accumulate(None, 1, None, None, None, None, None, None, None,
                                  None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_go_update(None, None, None, None, 0.1, None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_su_workspace_bytes(None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_su_evolve(None, None, None, 1.0, 0.01, 1, None, 0, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_su_to_peps(None, None, None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_su_pad(None, None, None, None, None, None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_sz_counts(4, 4, 0, 0, 4, 4, 1, None, None, None, None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_sz_counts(4, 4, 1, 1, 4, 4, 0, None, None, None, None, None) == bd.PEPSGO_EINVAL
    assert L.pepsgo_structure_factor(4, 4, None, None, 0.0, 0.0, 3.0, None, None) == bd.PEPSGO_EINVAL


def test_create_reports_missing_device_as_error_code(L):
    import ctypes
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    rc = L.pepsgo_create(0, ctypes.byref(h))
    assert rc in (bd.PEPSGO_EDEVICE, bd.PEPSGO_EINVAL)
    assert L.pepsgo_last_error()
