"""The C-ABI library is built for gfx950, loads, and exports every function include/rpd.h declares (CPU only: no
compute calls)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpd.h")
LIB = os.path.join(ROOT, "paper_2403_18761_amd", "librpd.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rpd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2403_18761_amd import build

        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("rpd_build", "rpd_euler", "rpd_components", "rpd_mesh_create", "rpd_free", "rpd_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rpd_[a-z_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_reports_version(lib_path):
    from paper_2403_18761_amd import rpd

    assert "gfx950" in rpd.version()
    assert rpd.load().rpd_last_error() == b""


def test_library_contains_gfx950_code(lib_path):
    data = open(lib_path, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_binding_constants_match_the_header():
    """Every RPD_ constant of the header has the same value in the Python binding."""
    from paper_2403_18761_amd import rpd

    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    seen = 0
    for name, expr in re.findall(r"^#define (RPD_[A-Z0-9_]+)[ \t]+(.+?)\s*$", src, flags=re.M):
        value = eval(expr.replace("u <<", " <<"), {})  # integer literals and shifts only
        assert getattr(rpd, name) == value, name
        seen += 1
    assert seen >= 20
