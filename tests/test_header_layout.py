"""The Python binding's ctypes structures against the C header (include/pmg.h).

A C program compiled from the header prints the size of every structure and
the offset of every field; the binding's structures must agree field by field
(name, order, offset) and in size, so that arguments cross the C ABI intact.
Host only: nothing here touches a device.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

import paper_1901_01685_amd as pmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmg.h")

PAIRS = [("pmg_problem", pmg.Problem), ("pmg_options", pmg.Options), ("pmg_result", pmg.Result),
         ("pmg_info", pmg.Info), ("pmg_server_options", pmg.ServerOptions),
         ("pmg_request_info", pmg.RequestInfo), ("pmg_server_stats", pmg.ServerStats)]


def _fields_in_header(name):
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    out = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):  # several declarators of one type
            field = re.search(r"(\w+)\s*(\[\s*\d+\s*\])?\s*$", part.strip())
            out.append(field.group(1))
    return out


@pytest.fixture(scope="module")
def c_layout():
    src = ["#include <stddef.h>", "#include <stdio.h>", f'#include "{HEADER}"', "int main(void) {"]
    for name, _ in PAIRS:
        src.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in _fields_in_header(name):
            src.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    src += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write("\n".join(src) + "\n")
        subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-o", exe, c], check=True)
        lines = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    lay = {}
    for ln in lines:
        if ln:
            s, f, v = ln.split()
            lay[(s, f)] = int(v)
    return lay


@pytest.mark.parametrize("name,cls", PAIRS, ids=[p[0] for p in PAIRS])
def test_ctypes_structure_matches_header(name, cls, c_layout):
    names = [f for f, _ in cls._fields_]
    assert names == _fields_in_header(name), name
    for f in names:
        assert getattr(cls, f).offset == c_layout[(name, f)], (name, f)
    assert C.sizeof(cls) == c_layout[(name, "size")], name
