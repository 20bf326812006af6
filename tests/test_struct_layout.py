"""The binding's ctypes structures have the layout of the C header's structs.

A small C program, compiled with the host C compiler against include/bkd.h, prints every
public struct's size and each field's offset; the ctypes mirrors in the Python binding must
agree field by field (name, order, offset) and in size.  A field added to one side only, or
a type that changes alignment, fails here instead of corrupting memory across the boundary.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1512_02831_amd as bkd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [
    ("bkd_options", bkd.Options),
    ("bkd_tree_info", bkd.TreeInfo),
    ("bkd_stats", bkd.Stats),
    ("bkd_instance", bkd.Instance),
    ("bkd_tuning", bkd.Tuning),
    ("bkd_batch_stats", bkd.BatchStats),
    ("bkd_server_opts", bkd.ServerOpts),
    ("bkd_server_stats", bkd.ServerStats),
]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bkd.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    table = {}
    for line in out.splitlines():
        cname, key, val = line.split()
        table[(cname, key)] = int(val)
    return table


@pytest.mark.parametrize("cname,cls", PAIRS, ids=[p[0] for p in PAIRS])
def test_ctypes_mirror_matches_header(c_layout, cname, cls):
    assert ctypes.sizeof(cls) == c_layout[(cname, "size")]
    for fname, _ in cls._fields_:
        assert getattr(cls, fname).offset == c_layout[(cname, fname)], fname
