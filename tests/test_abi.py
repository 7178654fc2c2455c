"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad host arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2211_14438_amd import bernnn as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bernnn.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bern_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = _declared()
    assert "bern_bounds" in names and "bern_net_create" in names
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in B.EXPORTED:
        assert n in names, f"binding uses {n} which the header does not declare"


def test_status_strings():
    assert B.status_str(0) == "BERN_OK"
    assert B.status_str(-7) == "BERN_E_WORKSPACE"
    assert B.status_str(12345) == "BERN_UNKNOWN"


def test_create_rejects_bad_networks_on_host():
    L = B.lib()
    h = ctypes.c_void_p()
    W = np.zeros(4)
    b = np.zeros(2)
    pd = ctypes.POINTER(ctypes.c_double)
    widths = (ctypes.c_int32 * 2)(2, 2)
    # H = 0
    assert L.bern_net_create(0, widths, W.ctypes.data_as(pd), b.ctypes.data_as(pd), ctypes.byref(h)) == -1
    # input dimension 0
    w0 = (ctypes.c_int32 * 2)(0, 2)
    assert L.bern_net_create(1, w0, W.ctypes.data_as(pd), b.ctypes.data_as(pd), ctypes.byref(h)) == -1
    # non-finite weight
    Wn = np.array([0.0, np.inf, 0.0, 0.0])
    assert L.bern_net_create(1, widths, Wn.ctypes.data_as(pd), b.ctypes.data_as(pd), ctypes.byref(h)) == -9
    assert b"non-finite" in L.bern_last_error()
    # null output handle
    assert L.bern_net_create(1, widths, W.ctypes.data_as(pd), b.ctypes.data_as(pd), None) == -1


def test_null_arguments_rejected():
    L = B.lib()
    o = B.make_opts()
    sz = ctypes.c_size_t()
    assert L.bern_workspace_size(None, ctypes.byref(o), 1, ctypes.byref(sz), None) == -1
    assert L.bern_bounds(None, ctypes.byref(o), 1, None, None, None, None, None, None, None, None, None, 0, None,
                         None) == -1
    assert L.bern_poly_mul(0, 1, 1, 1, None, None, None, 1, None) == -1
    assert L.bern_relu_poly(1, 9, None, None, None, None, None) == -1
    assert L.bern_basis_minmax(2, 2, 0, None, 1, None, None, None, None, None, 0, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """Every option and result struct the binding marshals has the header's
    size and field offsets (a C program built against the header prints them)."""
    structs = {"bern_opts": B.bern_opts, "bern_stats": B.bern_stats, "bern_verify_result": B.bern_verify_result,
               "bern_train_opts": B.bern_train_opts}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bernnn.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = {}
    for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        parts = l.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
