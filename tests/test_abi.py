"""The C-ABI library loads, exports every entry point the header declares, and
rejects bad arguments before touching a GPU (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2309_09609_amd as sw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "swsearch.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = sw.load()
    names = header_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(sw.EXPORTS)


def test_status_strings():
    lib = sw.load()
    for code, name in sw.STATUS.items():
        assert lib.sw_status_str(code).decode() == name


def test_argument_errors_without_gpu():
    lib = sw.load()
    h = ctypes.c_void_p()
    offs = np.array([0, 3], dtype=np.int64)
    # negative n and NULL output
    assert lib.sw_db_pack(None, offs.ctypes.data, -1, None, None, ctypes.byref(h)) == -1
    assert lib.sw_db_pack(None, offs.ctypes.data, 1, None, None, None) == -1
    assert b"out" in lib.sw_last_error()
    # NULL handle
    sm = np.zeros(400, dtype=np.int8)
    q = np.zeros(3, dtype=np.int8)
    assert lib.sw_search(q.ctypes.data, 3, None, None, 0, sm.ctypes.data, 10, 2, None, None) == -1
    # k outside 1..1024
    assert lib.sw_topk(None, 0, 0, None, None, None) == -5
    assert lib.sw_topk(None, 0, 2000, None, None, None) == -5
    # batch: NULL handle
    assert lib.sw_search_batch(None, None, 0, None, sm.ctypes.data, 1, 1, 0, None, None, None, None) == -1
    # alignments: NULL handle, negative gap
    assert lib.sw_align(q.ctypes.data, 3, None, None, 0, sm.ctypes.data, 10, 2, None, None, 0, None) == -1
    assert lib.sw_align(q.ctypes.data, 3, None, None, 0, sm.ctypes.data, -1, 2, None, None, 0, None) == -1
    qo = np.array([0, 3], dtype=np.int64)
    assert lib.sw_align_batch(q.ctypes.data, qo.ctypes.data, 1, None, None, qo.ctypes.data, sm.ctypes.data, 10, 2,
                              None, None, 0, None) == -1


def test_alignment_record_layout():
    assert ctypes.sizeof(sw.Alignment) == 48
    assert sw.Alignment.subject.offset == 16 and sw.Alignment.n_ops.offset == 40


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, from a C program compiled with gcc."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "swsearch.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("struct,mirror", [("sw_pack_opts", "PackOpts"), ("sw_alignment", "Alignment")])
def test_struct_mirrors_match_the_header(tmp_path, struct, mirror):
    cls = getattr(sw, mirror)
    fields = [f[0] for f in cls._fields_]
    size, offs = _c_layout(struct, fields, tmp_path)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs
