"""The C ABI without a GPU: the library loads, exports every symbol that
include/nnp.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2207_14276_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "nnp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nnp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("nnp_create", "nnp_energy_forces", "nnp_destroy", "nnp_status"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = nat.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert sorted(nat.EXPORTS) == declared_symbols()


def test_null_model_is_rejected_without_a_device():
    lib = nat.load()
    offs = (C.c_int64 * 2)(0, 3)
    box = (C.c_float * 3)(0, 0, 0)
    rc = lib.nnp_energy_forces(None, 1, offs, None, None, box, None, None, None, None, None)
    assert rc == nat.NNP_EINVAL
    assert "null model" in nat.last_error()


def test_null_descriptor_is_rejected():
    lib = nat.load()
    h = C.c_void_p()
    assert lib.nnp_create(None, -1, C.byref(h)) == nat.NNP_EINVAL
    assert lib.nnp_create_dp(None, 0, C.byref(h)) == nat.NNP_EINVAL
    assert nat.last_error() != ""


def test_status_and_reserve_reject_null_model():
    lib = nat.load()
    assert lib.nnp_status(None, None, None) == nat.NNP_EINVAL
    assert lib.nnp_reserve(None, 10, 1, 0) == nat.NNP_EINVAL
    assert lib.nnp_aev_dim(None) == nat.NNP_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(nat, "_lib", None)
    monkeypatch.setattr(nat, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        nat.load()
