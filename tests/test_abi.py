"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srgrav.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2606_17145_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tree_build", "shortrange_accel", "shortrange_accel_adjoint", "tree_free",
              "srgrav_last_error", "tree_export", "tree_node_count"):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(declared_functions()) <= exported


def test_binding_names_match_header(libpath):
    from paper_2606_17145_amd import _lib
    assert set(_lib.EXPORTED) == set(declared_functions())
    L = _lib.lib()
    assert L.srgrav_last_error() == b""


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2606_17145_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        _lib.lib()


def test_host_side_argument_errors(libpath):
    """Argument checks that return before any device work."""
    from paper_2606_17145_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p(None)
    dummy = ctypes.c_void_p(16)
    # n out of range
    assert L.tree_build(dummy, dummy, None, 1e-3, 0, 1.0, 1, None, ctypes.byref(h)) == -1
    # box not positive
    assert L.tree_build(dummy, dummy, None, 1e-3, 10, 0.0, 1, None, ctypes.byref(h)) == -1
    # leaf size
    assert L.tree_build(dummy, dummy, None, 1e-3, 10, 1.0, 2, None, ctypes.byref(h)) == -5
    # softening
    assert L.tree_build(dummy, dummy, None, 0.0, 10, 1.0, 1, None, ctypes.byref(h)) == -1
    assert b"eps" in L.srgrav_last_error()
    # calls on a handle that was never built
    p = _lib.make_params(dict(r_s=0.01, r_cut=0.045))
    tok = ctypes.c_int64(7)
    assert L.shortrange_accel(None, ctypes.byref(p), None, 1, None, dummy, None, ctypes.byref(tok), None) == -4
    assert tok.value == 0
    # adjoint: a negative token, and a token on a handle that was never built
    assert L.shortrange_accel_adjoint(None, ctypes.byref(p), None, 1, None, dummy, dummy, dummy, -1, None) == -1
    assert L.shortrange_accel_adjoint(None, ctypes.byref(p), None, 1, None, dummy, dummy, dummy, 3, None) == -4
    n = ctypes.c_int64(0)
    assert L.tree_node_count(None, ctypes.byref(n)) == -4
    L.tree_free(None)


def test_pm_and_sph_argument_errors(libpath):
    """The PM and SPH entry points reject bad arguments before any device work."""
    from paper_2606_17145_amd import _lib
    L = _lib.lib()
    dummy = ctypes.c_void_p(16)
    h = ctypes.c_void_p(None)
    # an odd or out-of-range mesh, and no output slot
    assert L.pm_create(7, ctypes.byref(h)) == -1 and not h.value
    assert b"n_mesh" in L.srgrav_last_error()
    assert L.pm_create(4096, ctypes.byref(h)) == -1
    assert L.pm_create(64, None) == -1
    assert b"out is NULL" in L.srgrav_last_error()
    # calls on a NULL handle
    assert L.pm_accel(None, dummy, dummy, 4, 1.0, 0.1, 1.0, dummy, None) == -4
    assert L.pm_accel_adjoint(None, dummy, dummy, 4, 1.0, 0.1, 1.0, dummy, dummy, dummy, None) == -4
    L.pm_free(None)
    bad = ctypes.c_int64(-1)
    assert L.sph_density(None, 64.0, dummy, dummy, ctypes.byref(bad), None) == -4
