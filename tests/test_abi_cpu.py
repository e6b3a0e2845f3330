"""Host-side checks of the C ABI that need no GPU: the library loads, every
function declared in include/*.h is exported, and argument errors are
reported before anything touches a device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(fe_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    import paper_1609_05722_amd as fe
    return fe.library()


def test_header_declares_the_abi():
    names = _declared()
    for n in ("fe_create", "fe_denoise", "fe_energy_grad", "fe_destroy",
              "fe_workspace_size", "fe_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in sorted(_declared()):
        assert hasattr(lib, name), name


def test_binding_lists_every_export():
    import paper_1609_05722_amd as fe
    assert set(fe.EXPORTS) == _declared()


def _prior_struct(fe, m, nf):
    f = np.zeros((nf, m, m), np.float32)
    w = np.ones(nf, np.float32)
    pr = fe._Prior(m, nf, f.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                   w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return pr, (f, w)


def test_create_rejects_bad_priors(lib):
    import paper_1609_05722_amd as fe
    h = ctypes.c_void_p()
    for m, nf, status in ((4, 8, fe.FE_ERR_UNSUPPORTED), (9, 8, fe.FE_ERR_UNSUPPORTED),
                          (7, 0, fe.FE_ERR_UNSUPPORTED), (7, 65, fe.FE_ERR_UNSUPPORTED)):
        pr, keep = _prior_struct(fe, m, nf)
        assert lib.fe_create(ctypes.byref(pr), 0, ctypes.byref(h)) == status
        assert h.value is None
        assert len(lib.fe_last_error()) > 0
    assert lib.fe_create(None, 0, ctypes.byref(h)) == fe.FE_ERR_INVALID
    pr, keep = _prior_struct(fe, 7, 48)
    keep[1][3] = -1.0
    assert lib.fe_create(ctypes.byref(pr), 0, ctypes.byref(h)) == fe.FE_ERR_INVALID
    keep[1][3] = 1.0
    keep[0][2, 1, 1] = np.nan
    assert lib.fe_create(ctypes.byref(pr), 0, ctypes.byref(h)) == fe.FE_ERR_INVALID


def test_create_rejects_missing_device(lib):
    import paper_1609_05722_amd as fe
    pr, keep = _prior_struct(fe, 7, 48)
    h = ctypes.c_void_p()
    assert lib.fe_create(ctypes.byref(pr), 1 << 20, ctypes.byref(h)) == fe.FE_ERR_INVALID


def test_null_context_is_rejected(lib):
    import paper_1609_05722_amd as fe
    sz = ctypes.c_size_t()
    assert lib.fe_workspace_size(None, None, 0, ctypes.byref(sz)) == fe.FE_ERR_INVALID
    assert lib.fe_denoise(None, None, 0, None, 0, None) == fe.FE_ERR_INVALID
    assert lib.fe_energy_grad_workspace_size(None, 8, 8, ctypes.byref(sz)) == fe.FE_ERR_INVALID
    assert lib.fe_energy_grad_batch_workspace_size(None, None, 0,
                                                   ctypes.byref(sz)) == fe.FE_ERR_INVALID
    assert lib.fe_energy_grad_batch(None, None, 0, 0, None, None, 0, None) == fe.FE_ERR_INVALID
    assert lib.fe_energy_grad(None, 8, 8, None, None, 1.0, 1, 0, None, None, None, 0,
                              None) == fe.FE_ERR_INVALID
    lib.fe_destroy(None)  # NULL-safe


def test_stepping_calls_validate_before_device_work(lib):
    import paper_1609_05722_amd as fe
    sz = ctypes.c_size_t()
    assert lib.fe_state_bytes(None, 8, 8, ctypes.byref(sz)) == fe.FE_ERR_INVALID
    assert lib.fe_advance_workspace_size(None, 4, ctypes.byref(sz)) == fe.FE_ERR_INVALID
    assert lib.fe_begin(None, None, None, 0, None) == fe.FE_ERR_INVALID
    assert lib.fe_advance(None, None, None, None, None, 0, None, 0, None) == fe.FE_ERR_INVALID
    assert lib.fe_end(None, None, None, None, 0, None) == fe.FE_ERR_INVALID
    assert lib.fe_advance_noalloc(None, None, None, None, None, 0, None) == fe.FE_ERR_INVALID


def test_server_calls_validate_before_device_work(lib):
    import paper_1609_05722_amd as fe
    from paper_1609_05722_amd import serving
    serving._bind()
    h = ctypes.c_void_p()
    cfg = serving._Cfg(1 << 20, 10, 4, 2)
    assert lib.fe_server_create(None, ctypes.byref(cfg), None, ctypes.byref(h)) == fe.FE_ERR_INVALID
    assert lib.fe_server_submit(None, None, 0) == fe.FE_ERR_INVALID
    n = ctypes.c_int32()
    assert lib.fe_server_poll(None, None, 0, ctypes.byref(n), 0) == fe.FE_ERR_INVALID
    lib.fe_server_destroy(None)


def test_tuning_and_graph_calls_validate_before_device_work(lib):
    import paper_1609_05722_amd as fe
    assert lib.fe_autotune(None, None, 0, 4, None) == fe.FE_ERR_INVALID
    assert lib.fe_tuning_save(None, b"/tmp/x") == fe.FE_ERR_INVALID
    assert lib.fe_tuning_load(None, b"/tmp/x") == fe.FE_ERR_INVALID
    h = ctypes.c_void_p()
    assert lib.fe_advance_graph_create(None, None, None, None, None, 0, None, 0,
                                       ctypes.byref(h)) == fe.FE_ERR_INVALID
    assert h.value is None
    assert lib.fe_graph_launch(None, None) == fe.FE_ERR_INVALID
    lib.fe_graph_destroy(None)  # NULL-safe


def test_binding_rejects_host_or_malformed_tensors():
    """The binding marshals device tensors only: host, non-contiguous,
    non-float32 or non-2-D inputs are refused before the library is called."""
    import torch
    import paper_1609_05722_amd as fe
    for bad in (torch.zeros(8, 8), torch.zeros(8, 8, dtype=torch.float64), torch.zeros(8),
                torch.zeros(8, 16)[:, ::2]):
        with pytest.raises(ValueError):
            fe.make_jobs([fe.JobSpec(bad, 1.0, 1, 0.1, 0.5)])


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libfe.so every entry point raises: there is no other path."""
    import paper_1609_05722_amd as fe
    monkeypatch.setattr(fe, "_lib", None)
    monkeypatch.setattr(fe, "LIB_PATH", str(tmp_path / "libfe.so"))
    with pytest.raises(ImportError, match="not built"):
        fe.library()
    k = np.zeros((8, 3, 3), np.float32)
    k[:, 1, 1] = 1.0
    with pytest.raises(ImportError, match="not built"):
        fe.Prior(k, np.ones(8, np.float32))
