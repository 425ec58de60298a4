"""CPU checks of the C ABI library: it builds, loads, exports every function that
include/mgcd.h declares, and the product package never reaches for the oracle."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgcd.h")
PKG = os.path.join(ROOT, "paper_2411_02268_amd")


@pytest.fixture(scope="module")
def libpath():
    import paper_2411_02268_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2411_02268_amd import build
        build.build()
    return m.LIB_PATH


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("lpa_run", "louvain_run", "leiden_run", "modularity", "mgcd_workspace_bytes",
              "mgcd_default_params", "mgcd_last_error", "mgcd_move_sweep", "mgcd_refine",
              "mgcd_aggregate"):
        assert f in names


def test_every_declared_symbol_is_exported(libpath):
    L = ct.CDLL(libpath)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_host_only_calls(libpath):
    import paper_2411_02268_amd as m
    p = m.params(m.ALGO_LEIDEN)
    assert (p.k, p.chunk_len, p.max_iterations, p.max_passes) == (16, 128, 20, 10)
    n = m.lib().mgcd_workspace_bytes(m.ALGO_LOUVAIN, 1 << 20, 31_000_000, ct.byref(p))
    assert n > (1 << 20) * 16
    assert m.lib().mgcd_last_error() == b""


def test_product_never_imports_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", src, flags=re.M), f
                assert "oracle.h" not in src and "liboracle" not in src, f


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2411_02268_amd as m
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(m, "_lib", None)
    with pytest.raises(RuntimeError):
        m.lib()
