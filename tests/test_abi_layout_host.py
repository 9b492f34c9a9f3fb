"""The ctypes binding agrees with the C header (no GPU): struct sizes and
field offsets and the enum values as a C compiler lays them out from
include/gfem.h, and every declared prototype's argument and return types
against the binding's signature table.  A mismatch here would pass every
call silently with shifted or truncated arguments."""
import ctypes as C
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2103_14870_amd import gfem  # noqa: E402

HEADER = os.path.join(ROOT, "include", "gfem.h")
STRUCTS = {"gf_params": gfem.GfParams, "gf_step_stats": gfem.GfStepStats, "gf_qs_stats": gfem.GfQsStats}
ENUMS = {
    "GF_OK": gfem.GF_OK, "GF_EINVAL": gfem.GF_EINVAL, "GF_EDEGENERATE": gfem.GF_EDEGENERATE,
    "GF_ENOMEM": gfem.GF_ENOMEM, "GF_EDEVICE": gfem.GF_EDEVICE, "GF_ENOTCONVERGED": gfem.GF_ENOTCONVERGED,
    "GF_ESTATE": gfem.GF_ESTATE,
    "GF_PREC_FP64": gfem.PREC["fp64"], "GF_PREC_SPLIT": gfem.PREC["split"],
    "GF_PC_BLOCK_JACOBI": gfem.PRECOND["block_jacobi"], "GF_PC_LEARNED": gfem.PRECOND["learned"],
    "GF_ENERGY_STABLE_NEO_HOOKEAN": gfem.ENERGY["stable_neo_hookean"], "GF_ENERGY_STVK": gfem.ENERGY["stvk"],
    "GF_REORDER_NONE": gfem.REORDER["none"], "GF_REORDER_RCM": gfem.REORDER["rcm"],
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    """Sizes, offsets and enum values printed by a C program built against the header."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gfem.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("size {cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("off {cname}.{f} %zu %zu\\n", offsetof({cname}, {f}), '
                         f"sizeof((({cname}*)0)->{f}));")
    for e in ENUMS:
        lines.append(f'  printf("enum {e} %d\\n", (int){e});')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    res = {}
    for ln in out:
        parts = ln.split()
        if parts:
            res[parts[1]] = tuple(int(v) for v in parts[2:])
    return res


def test_struct_layouts_match_the_header(c_layout):
    for cname, py in STRUCTS.items():
        assert c_layout[cname] == (C.sizeof(py),), cname
        for f, t in py._fields_:
            assert c_layout[f"{cname}.{f}"] == (getattr(py, f).offset, C.sizeof(t)), (cname, f)


def test_enum_values_match_the_header(c_layout):
    for e, v in ENUMS.items():
        assert c_layout[e] == (v,), e


# C parameter type (const dropped, spaces normalised) -> ctypes type in the binding
_CTYPES = {
    "double*": C.POINTER(C.c_double), "double": C.c_double, "float*": C.POINTER(C.c_float),
    "int32_t": C.c_int32, "int32_t*": C.POINTER(C.c_int32), "uint8_t*": C.POINTER(C.c_uint8),
    "uint64_t": C.c_uint64, "size_t": C.c_size_t, "size_t*": C.POINTER(C.c_size_t),
    "void*": C.c_void_p, "gf_mesh*": C.c_void_p, "gf_net*": C.c_void_p,
    "gf_mesh**": C.POINTER(C.c_void_p), "gf_net**": C.POINTER(C.c_void_p),
    "gf_params*": C.POINTER(gfem.GfParams), "gf_step_stats*": C.POINTER(gfem.GfStepStats),
    "gf_qs_stats*": C.POINTER(gfem.GfQsStats),
}
_RET = {"gf_status": C.c_int, "char*": C.c_char_p}


def _norm(t):
    t = re.sub(r"\bconst\b", "", t)
    t = re.sub(r"\s*\*\s*", "*", t)
    return " ".join(t.split())


def header_prototypes():
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    protos = {}
    for ret, name, args in re.findall(r"^\s*((?:const\s+)?\w+\s*\**)\s*(gf_\w+)\s*\(([^)]*)\)\s*;", text, re.M):
        params = []
        if args.strip() not in ("", "void"):
            for a in args.split(","):
                m = re.match(r"(.*?)(\w+)\s*$", a.strip())
                params.append(_norm(m.group(1)))
        protos[name] = (_norm(ret), params)
    return protos


def test_every_prototype_matches_the_binding_signature():
    protos = header_prototypes()
    assert len(protos) >= 30
    assert set(protos) == set(gfem._SIGS), set(protos) ^ set(gfem._SIGS)
    for name, (ret, params) in protos.items():
        args, res = gfem._SIGS[name]
        assert res == _RET[ret], (name, ret)
        assert len(args) == len(params), (name, params)
        for k, (p, a) in enumerate(zip(params, args)):
            assert a == _CTYPES[p], (name, k, p, a)
