"""The C ABI library loads and exports every function include/lq.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lq_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("lq_create", "lq_destroy", "lq_upload_gauge", "lq_dslash",
                     "lq_clover_apply", "lq_solve"):
        assert required in names


def test_library_exports_all_declared_symbols():
    from paper_1103_1363_amd import lq
    if not os.path.exists(lq.LIB_PATH):
        pytest.fail("liblq.so is not built (run python -m paper_1103_1363_amd.build)")
    lib = ctypes.CDLL(lq.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1103_1363_amd import lq
    monkeypatch.setattr(lq, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lq, "_lib", None)
    with pytest.raises(ImportError):
        lq.lib()


def _lib():
    from paper_1103_1363_amd import lq
    if not os.path.exists(lq.LIB_PATH):
        pytest.fail("liblq.so is not built (run python -m paper_1103_1363_amd.build)")
    lib = ctypes.CDLL(lq.LIB_PATH)
    lib.lq_create.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_void_p)]
    lib.lq_create.restype = ctypes.c_int
    lib.lq_last_error.argtypes = [ctypes.c_void_p]
    lib.lq_last_error.restype = ctypes.c_char_p
    lib.lq_ensemble_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_void_p)]
    lib.lq_ensemble_create.restype = ctypes.c_int
    lib.lq_ensemble_last_error.argtypes = [ctypes.c_void_p]
    lib.lq_ensemble_last_error.restype = ctypes.c_char_p
    return lib


@pytest.mark.parametrize("dims,msg", [((3, 4, 4, 4), b"even"), ((4, 4, 4, 0), b"even"),
                                      ((4, 1, 4, 4), b"even"),
                                      ((64, 64, 64, 256), b"too large")])
def test_create_rejects_bad_lattices_before_any_device_call(dims, msg):
    """Odd or vanishing extents and lattices beyond the reduction scratch
    (more than 65536 x 256 sites of one parity) are refused on the host."""
    lib = _lib()
    out = ctypes.c_void_p(123)
    rc = lib.lq_create((ctypes.c_int * 4)(*dims), 1, None, ctypes.byref(out))
    assert rc == -1  # LQ_EINVAL
    assert msg in lib.lq_last_error(None)


def test_ensemble_create_rejects_bad_arguments_on_the_host():
    lib = _lib()
    out = ctypes.c_void_p(123)
    assert lib.lq_ensemble_create(None, 0, ctypes.byref(out)) == -1
    assert out.value is None
    assert b"member" in lib.lq_ensemble_last_error(None)
    members = (ctypes.c_void_p * 2)(None, None)
    assert lib.lq_ensemble_create(members, 2, ctypes.byref(out)) == -1
    assert lib.lq_ensemble_create(members, 65, ctypes.byref(out)) == -1
    assert lib.lq_ensemble_create(members, 2, None) == -1


def test_sap_calls_reject_missing_context():
    """The SAP entry points refuse a null context before any device work."""
    lib = _lib()
    vp = ctypes.c_void_p
    lib.lq_sap_apply.argtypes = [vp, vp, vp, vp]
    lib.lq_solve_sap.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 vp, vp]
    params = (ctypes.c_int * 11)(4, 4, 4, 4, 0, 0, 0, 0, 0, 0, 0)  # lq_sap_params: block[4] + 7 ints
    buf = ctypes.create_string_buffer(64)
    assert lib.lq_sap_apply(None, buf, buf, params) == -1
    assert lib.lq_solve_sap(None, buf, buf, 0.13, 1.0, 1e-10, params, None) == -1


def test_tune_tiles_rejects_bad_arguments_on_the_host():
    """The tile tuner checks its precision and right-hand-side count before
    touching the device."""
    lib = _lib()
    lib.lq_tune_tiles.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_char_p, ctypes.c_void_p]
    lib.lq_tune_tiles.restype = ctypes.c_int
    lib.lq_tune_last_error.restype = ctypes.c_char_p
    dims = (ctypes.c_int * 4)(8, 8, 8, 8)
    assert lib.lq_tune_tiles(dims, 1, 7, 1, None, None) == -1
    assert b"nrhs" in lib.lq_tune_last_error()
    assert lib.lq_tune_tiles(dims, 1, 2, 2, None, None) == -1
    assert lib.lq_tune_tiles(None, 1, 2, 1, None, None) == -1
