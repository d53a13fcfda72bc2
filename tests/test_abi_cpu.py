"""CPU checks of the C ABI: the library loads, exports every declared symbol, and the
ctypes structure layouts match the C compiler's (no compute calls: no GPU here)."""

import ctypes
import os
import re
import subprocess

import pytest

from paper_2411_03002_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apx.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(apx_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.PROTOTYPES), set(names) ^ set(binding.PROTOTYPES)


def test_basis_size_without_device():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    assert lib.apx_ace_num_basis(10, 4) == 7895
    assert lib.apx_ace_num_basis(8, 3) == 2344
    assert lib.apx_ace_num_basis(8, 5) == -1


def test_struct_layouts_match_c(tmp_path):
    structs = {"apx_atoms": binding.Atoms, "apx_nlist": binding.NList, "apx_prec_params": binding.PrecParams,
               "apx_eam_params": binding.EamParams, "apx_ace_desc": binding.AceDesc,
               "apx_md_params": binding.MdParams, "apx_md_stats": binding.MdStats,
               "apx_avg_state": binding.AvgState, "apx_thermo_params": binding.ThermoParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "apx.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
