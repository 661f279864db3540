"""The C-ABI library loads and exports every entry point include/mcg.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcg.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_method_calls():
    names = declared_symbols()
    for n in ("mcg_smear", "mcg_fix", "mcg_apply_gauge", "mcg_center_project", "mcg_count_vortices",
              "mcg_fix_batch", "mcg_smear_mcg_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0807_0264_amd import _abi
    if not os.path.exists(_abi.LIBPATH):
        pytest.skip("libmcg.so not built")
    lib = ctypes.CDLL(_abi.LIBPATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    # and the Python binding declares exactly those
    assert sorted(_abi.SIGNATURES) == declared_symbols()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_0807_0264_amd import _abi
    with pytest.raises(RuntimeError, match="not built"):
        _abi._lib = None
        try:
            _abi.load(str(tmp_path / "absent.so"))
        finally:
            _abi._lib = None


def test_buffer_sizes():
    """A link field holds 4 links x 9 complex entries per site, a gauge field
    9 complex entries per site (host-only calls, no device needed)."""
    from paper_0807_0264_amd import _abi
    if not os.path.exists(_abi.LIBPATH):
        pytest.skip("libmcg.so not built")
    lib = _abi.load()
    d = _abi.Dims()
    for k, v in enumerate((6, 4, 2, 8)):
        d.L[k] = v
    V = 6 * 4 * 2 * 8
    assert lib.mcg_field_bytes(d, _abi.MCG_F64) == V * 4 * 9 * 2 * 8
    assert lib.mcg_field_bytes(d, _abi.MCG_F32) == V * 4 * 9 * 2 * 4
    assert lib.mcg_gauge_bytes(d) == V * 9 * 2 * 8
    d.L[1] = 5
    assert lib.mcg_field_bytes(d, _abi.MCG_F64) == 0 and lib.mcg_gauge_bytes(d) == 0
    # the largest lattices: 80 V < 2^32 (32-bit byte offsets of FP64 elements)
    for k, v in enumerate((64, 64, 64, 204)):
        d.L[k] = v
    assert lib.mcg_gauge_bytes(d) == 64 ** 3 * 204 * 9 * 16
    d.L[3] = 206
    assert lib.mcg_field_bytes(d, _abi.MCG_F32) == 0 and lib.mcg_gauge_bytes(d) == 0
