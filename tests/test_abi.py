"""CPU checks of the C boundary: the library loads, exports every function
include/te.h declares, and the ctypes structures match the C layouts (a tiny
gcc-compiled probe prints sizeof/offsetof).  No GPU call is made."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "te.h")


def _lib():
    from paper_1804_10060_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1804_10060_amd import build
        build.build()
    return L


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


def test_header_declares_the_exports_list():
    L = _lib()
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = C.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(rf"\sT {name}$", out, flags=re.M), name


STRUCTS = {"te_mesh": "TeMesh", "te_material": "TeMaterial", "te_material_tables": "TeMaterialTables",
           "te_pressure": "TePressure", "te_bsr": "TeBsr", "amg_options": "AmgOptions",
           "amg_info": "AmgInfo", "pcg_options": "PcgOptions", "pcg_report": "PcgReport", "te_csr": "TeCsr",
           "te_thermal_tables": "TeThermalTables", "te_robin": "TeRobin", "camg_options": "CamgOptions",
           "camg_info": "CamgInfo", "newton_options": "NewtonOptions", "newton_report": "NewtonReport"}


@pytest.fixture(scope="module")
def c_layout():
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "te.h"', "int main(void) {"]
    L = _lib()
    for cname, pyname in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(L, pyname)._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        r = subprocess.run(["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                            "-I", "/opt/rocm/include", src, "-o", exe], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("cannot compile the layout probe: " + r.stderr[-400:])
        out = subprocess.run([exe], capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        a, b, v = line.split()
        res[(a, b)] = int(v)
    return res


def test_struct_layouts_match(c_layout):
    L = _lib()
    for cname, pyname in STRUCTS.items():
        cls = getattr(L, pyname)
        assert C.sizeof(cls) == c_layout[(cname, "size")], cname
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == c_layout[(cname, fname)], (cname, fname)


def test_constants_match_header():
    L = _lib()
    text = open(HEADER).read()
    for name in ["TE_OK", "TE_ENOTCONV", "TE_EINVAL", "TE_ENOMEM", "TE_EHIP", "TE_EINDEF", "TE_ENAN", "TE_ERANK",
                 "TE_ECHOL", "TE_PREC_FP64", "TE_PREC_MIXED", "TE_OP_A", "TE_OP_P", "TE_OP_R", "TE_OP_SMOOTH",
                 "TE_OP_VCYCLE"]:
        m = re.search(rf"#define\s+{name}\s+\(?(-?\d+)\)?", text)
        assert m and int(m.group(1)) == getattr(L, name), name
    m = re.search(r"#define\s+TE_K_COUNT\s+(\d+)", text)
    assert int(m.group(1)) == len(L.KERNEL_CLASSES)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    L = _lib()
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.load()
