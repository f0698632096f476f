"""Host-side checks of the C ABI that need no GPU: the library builds and
exports every entry point include/adg.h declares, and descriptors are
validated on the host before any device work."""
import os
import re
import subprocess

import pytest

import paper_1806_07984_amd as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "adg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adg_[a-z_]+)\s*\(", text)))


def test_library_exports_header_symbols():
    assert os.path.exists(A.LIB_PATH), "libadg.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(adg_\w+)", out))
    missing = [f for f in header_functions() if f not in exported]
    assert not missing, missing
    lib = A.load()
    for f in header_functions():
        assert hasattr(lib, f)
    assert sorted(A.EXPORTS) == header_functions()


def expect(code, **kw):
    with pytest.raises(A.AdgError) as e:
        A.Mesh(A.instance(**kw))
    assert e.value.code == code, str(e.value)


def test_rejects_unsupported_order():
    expect(2, order=8, n=(3, 3, 3))
    expect(2, order=-1, n=(3, 3, 3))


def test_rejects_bad_levels_and_refinement():
    expect(2, order=2, n=(3, 3, 3), max_level=4)
    expect(1, order=2, n=(3, 3, 3), max_level=1, refine=[[0, 3, 0, 0]])       # outside the grid
    expect(1, order=2, n=(3, 3, 3), max_level=1, refine=[[1, 0, 0, 0]])       # level not below max_level
    expect(1, order=2, n=(3, 3, 3), max_level=2, refine=[[1, 0, 0, 0]])       # not a leaf
    expect(1, order=2, n=(3, 3, 3), max_level=1, refine=[[0, 1, 1, 1], [0, 1, 1, 1]])  # duplicate


def test_rejects_bad_box_and_physics():
    expect(1, order=2, n=(0, 3, 3))
    expect(1, order=2, n=(3, 3, 3), lo=(0, 0, 0), hi=(1, 0, 1))
    expect(1, order=2, n=(3, 3, 3), gamma=1.0)
    expect(1, order=2, n=(3, 3, 3), cfl=0.0)


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(A, "_lib", None)
    monkeypatch.setattr(A, "LIB_PATH", "/nonexistent/libadg.so")
    with pytest.raises(ImportError):
        A.load()
