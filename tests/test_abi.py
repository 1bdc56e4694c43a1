"""The C-ABI library loads and exports every function include/qimax.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_2505_03307_amd import qimax as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qimax.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qimax_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("qimax_create", "qimax_apply_layer", "qimax_get_generators", "qimax_expect",
                     "qimax_apply_circuit", "qimax_destroy", "qimax_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(Q.LIB_PATH):
        pytest.fail("libqimax.so is not built")
    lib = ctypes.CDLL(Q.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(Q.EXPORTS) <= set(declared_functions())


def test_default_opts_without_gpu():
    lib = Q.load()
    o = Q.Opts()
    lib.qimax_default_opts(ctypes.byref(o))
    assert o.precision == 64 and o.validate == 1 and o.prune_eps == 0.0 and o.device == -1


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(Q, "_lib", None)
    monkeypatch.setattr(Q, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        Q.load()
