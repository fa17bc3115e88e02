"""The C-ABI boundary without a GPU: the shared library loads, exports every
function include/rfmls.h declares, and the ctypes mirrors of the header's
structs have the C compiler's sizes and offsets."""

import ctypes as C
import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "rfmls.h"


def _declared_functions():
    text = re.sub(r"/\*.*?\*/", " ", HEADER.read_text(), flags=re.S)
    names = re.findall(r"(?:void|rfmls_status|int64_t|const\s+char\s*\*)\s*\*?\s*(rfmls_\w+)\s*\(", text)
    assert names, "no declarations found in the header"
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2409_15818_amd import _lib

    if not _lib.LIB_PATH.exists():
        from paper_2409_15818_amd.build import build_library

        build_library()
    return C.CDLL(str(_lib.LIB_PATH))


def test_every_declared_function_is_exported(lib):
    from paper_2409_15818_amd import _lib

    declared = _declared_functions()
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing
    assert sorted(_lib.EXPORTED) == declared


def test_default_opts_without_device(lib):
    from paper_2409_15818_amd import _lib

    o = _lib.rfmls_opts()
    lib.rfmls_default_opts(C.byref(o))
    assert o.atol == 1e-10 and o.btol == 1e-10 and o.itmax == 0 and o.refine >= 0
    assert o.check_every >= 1 and o.lockstep == 1 and o.graph == 1 and o.reserved == 0


def test_struct_layout_matches_header(tmp_path):
    from paper_2409_15818_amd import _lib

    structs = {"rfmls_csr": _lib.rfmls_csr, "rfmls_opts": _lib.rfmls_opts,
               "rfmls_info": _lib.rfmls_info, "rfmls_trace_entry": _lib.rfmls_trace_entry,
               "rfmls_tune_entry": _lib.rfmls_tune_entry}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            sname, key, val = ln.split()
            got[(sname, key)] = int(val)
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
