"""The binding's ctypes structures match include/sphidx.h byte for byte.

A small C program compiled against the header prints sizeof and offsetof of
every field of every struct the ABI passes by pointer; the test compares
them with the ctypes layout the binding uses.  A field added to one side
only, or reordered, fails here on the CPU instead of corrupting a launch."""
import os
import subprocess

import pytest

from paper_cs_0608108_amd import sphidx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "sphidx_lattice_desc": sphidx.LatticeDesc,
    "sphidx_lattice_view": sphidx.LatticeView,
    "sphidx_tables_info": sphidx.TablesInfo,
    "sphidx_queries": sphidx.Queries,
    "sphidx_csr": sphidx.CSRDesc,
    "sphidx_launch": sphidx.LaunchDesc,
    "sphidx_batch": sphidx.BatchDesc,
    "sphidx_batch_result": sphidx.BatchResult,
}


def _c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sphidx.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu %zu\\n", offsetof({cname}, {fname}), '
                         f'sizeof((({cname}*)0)->{fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    sizes, fields = {}, {}
    for line in out.splitlines():
        parts = line.split()
        if parts[1] == "size":
            sizes[parts[0]] = int(parts[2])
        else:
            fields[(parts[0], parts[1])] = (int(parts[2]), int(parts[3]))
    return sizes, fields


def test_ctypes_structs_match_the_header(tmp_path):
    sizes, fields = _c_layout(tmp_path)
    for cname, cls in STRUCTS.items():
        assert sizes[cname] == __import__("ctypes").sizeof(cls), cname
        for fname, _ in cls._fields_:
            desc = getattr(cls, fname)
            assert fields[(cname, fname)] == (desc.offset, desc.size), (cname, fname)


def test_header_declares_no_field_the_binding_lacks(tmp_path):
    """Every member named in a header struct appears in the ctypes mirror."""
    import re
    text = open(os.path.join(ROOT, "include", "sphidx.h")).read()
    for cname, cls in STRUCTS.items():
        end = re.search(r"\}\s*" + cname + ";", text)
        assert end, cname
        start = text.rindex("typedef struct {", 0, end.start())
        body = re.sub(r"/\*.*?\*/", "", text[start + len("typedef struct {"):end.start()], flags=re.S)
        names = set()
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                nm = re.findall(r"([A-Za-z_]\w*)\s*(?:\[\d+\])?\s*$", part.strip())
                if nm:
                    names.add(nm[-1])
        assert names == {f for f, _ in cls._fields_}, (cname, names ^ {f for f, _ in cls._fields_})


def test_stash_bytes_grow_with_pairs():
    lib = sphidx.load()
    a = lib.sphidx_query_stash_bytes(0, 0)
    b = lib.sphidx_query_stash_bytes(1_000_000, 0)
    c = lib.sphidx_query_stash_bytes(1_000_000, 1)
    assert a < b < c
    assert b >= 4 * 1_000_000 and c >= 12 * 1_000_000
