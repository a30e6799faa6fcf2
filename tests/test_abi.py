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


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the header's fields, in its order, at the offsets and sizes a
    C compiler gives them (gcc on the header itself)."""
    import ctypes as C

    from paper_2403_18761_amd import rpd

    pairs = [(rpd._MeshDesc, "rpd_mesh_desc"), (rpd._MeshInfo, "rpd_mesh_info"), (rpd._Sites, "rpd_sites"),
             (rpd._Opts, "rpd_opts"), (rpd._Stats, "rpd_stats"), (rpd._SessionOpts, "rpd_session_opts"),
             (rpd._SessionInfo, "rpd_session_info")]
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "rpd.h"', "int main(void) {"]
    for cls, name in pairs:
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, flags=re.S).group(1)
        declared = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):  # "const float *sx, *sy" declares several fields
                declared.append(re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*$", part.strip())[0])
        assert declared == [f for f, _ in cls._fields_], (name, declared)
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.splitlines() if line)
    for cls, name in pairs:
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
