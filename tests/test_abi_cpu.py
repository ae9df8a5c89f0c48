"""CPU-side checks of the C-ABI library: it loads and exports every symbol
that include/hgp.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hgp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hgp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2604_14411_amd import hgp

    if not os.path.exists(hgp.LIB_PATH):
        pytest.skip("libhgp.so not built")
    lib = hgp.load()
    names = _declared()
    assert "hgp_partition" in names and "hgp_partition_device" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hgp.EXPORTS)


def test_strerror_and_defaults_without_gpu():
    from paper_2604_14411_amd import hgp

    if not os.path.exists(hgp.LIB_PATH):
        pytest.skip("libhgp.so not built")
    lib = hgp.load()
    assert lib.hgp_strerror(hgp.EBADCSR) == b"malformed CSR hypergraph"
    assert lib.hgp_strerror(12345) == b"unknown error"
    o, _ = hgp.options()
    assert o.k == 0 and o.max_refine_rounds == 8 and o.proposal == hgp.PLAIN
    assert lib.hgp_ctx_create(None, 0) == hgp.EINVAL
    assert lib.hgp_partition(None, None, 1, 1, None, None, None) == hgp.EINVAL
    assert lib.hgp_last_error() != b""


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2604_14411_amd import hgp

    monkeypatch.setattr(hgp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hgp, "_lib", None)
    with pytest.raises(RuntimeError):
        hgp.load()


def test_probe_library_exports_its_entry_and_checks_arguments():
    """The LDS-atomic micro-benchmark (bench.py --lds-probe) is a library of
    its own; argument errors return -1 before any HIP call."""
    path = os.path.join(ROOT, "paper_2604_14411_amd", "libhgp_probe.so")
    if not os.path.exists(path):
        pytest.skip("libhgp_probe.so not built")
    lib = ctypes.CDLL(path)
    f = lib.hgp_probe_lds_atomics
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_float)]
    f.restype = ctypes.c_int
    ms = ctypes.c_float(0.0)
    assert f(0, 0, 1, ctypes.c_void_p(1), None, ctypes.byref(ms)) == -1
    assert f(0, 1, 0, ctypes.c_void_p(1), None, ctypes.byref(ms)) == -1
    assert f(1, 1, 1, None, None, ctypes.byref(ms)) == -1
    assert f(1, 1, 1, ctypes.c_void_p(1), None, None) == -1
