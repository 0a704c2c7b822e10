"""The C-ABI libraries load on a machine without a GPU and export exactly what the
headers declare (no compute calls: those need a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2004_09350_amd", "libmorphgpu.so")
HEADER = os.path.join(ROOT, "include", "morphgpu.h")


def declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(ms_[a-z0-9_]+)\s*\(", text))


def exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if re.search(r" T ms_", line)}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared(HEADER)
    assert len(names) >= 39
    missing = sorted(n for n in names if not hasattr(lib, n))
    assert not missing, missing


def test_no_undeclared_exports():
    extra = sorted(exported(LIB) - declared(HEADER))
    assert not extra, extra


def test_binding_fails_loudly_without_library(tmp_path):
    # a copy of the binding next to no library must refuse to import
    src = open(os.path.join(ROOT, "paper_2004_09350_amd", "morphgpu.py")).read()
    pkg = tmp_path / "pkg"
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    (pkg / "morphgpu.py").write_text(src)
    r = subprocess.run(["python", "-c", "import pkg.morphgpu"], cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0 and "is not built" in r.stderr
