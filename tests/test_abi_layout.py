"""The Python binding's ctypes structures against include/mp.h (host only):
a small C program built with gcc from the header prints the size of every
structure of the ABI and the offset of every field, and the ctypes
declarations in paper_2409_10774_amd/mp.py must agree field by field."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def c_layout(tmp_path, structs):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mp.h"', "int main(void) {"]
    for name, fields in structs.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    return got


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_ctypes_structures_match_the_header(tmp_path):
    from paper_2409_10774_amd import mp
    # the C field names where the binding uses other ones
    rename = {"mp_phase": {"lam": "lambda"}, "mp_request": {}, "mp_problem": {}, "mp_aniso": {},
              "mp_batch_config": {}}
    classes = {"mp_phase": mp.mp_phase, "mp_aniso": mp.mp_aniso, "mp_problem": mp.mp_problem,
               "mp_batch_config": mp.mp_batch_config, "mp_request": mp.mp_request}
    structs = {name: [rename[name].get(f[0], f[0]) for f in cls._fields_] for name, cls in classes.items()}
    got = c_layout(tmp_path, structs)
    for name, cls in classes.items():
        assert got[(name, "sizeof")] == mp.C.sizeof(cls), name
        for f in cls._fields_:
            cf = rename[name].get(f[0], f[0])
            assert got[(name, cf)] == getattr(cls, f[0]).offset, (name, f[0])
