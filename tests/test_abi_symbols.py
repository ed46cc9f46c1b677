"""The C ABI library loads on the host and exports every function include/*.h declares
(no compute calls: there may be no GPU here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2403_08220_amd", "libdino.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(dino_[A-Za-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2403_08220_amd.build import build
        build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["dino_ctx_create", "dino_load_prior", "dino_load_network", "dino_problem_create",
                 "dino_chains_init", "dino_step", "dino_read_states", "dino_read_diagnostics"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_strings(lib):
    lib.dino_version.restype = ctypes.c_char_p
    lib.dino_last_error.restype = ctypes.c_char_p
    assert b"gfx950" in lib.dino_version()
    assert lib.dino_last_error() == b""


def test_argument_errors_without_gpu(lib):
    """Null arguments are rejected before any device call."""
    lib.dino_last_error.restype = ctypes.c_char_p
    assert lib.dino_load_prior(None, 33, ctypes.c_double(0.1), ctypes.c_double(1.0), 32) == -1
    assert b"null" in lib.dino_last_error()
    assert lib.dino_step(None, 1, None) == -1
    size = ctypes.c_size_t()
    assert lib.dino_problem_workspace_bytes(None, None, ctypes.byref(size)) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2403_08220_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
