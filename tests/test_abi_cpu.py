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
