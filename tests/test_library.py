"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports every
entry point that include/hz.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hz.h")).read()
    return sorted(set(re.findall(r"\b(hz_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hz_mesh", "hz_assemble", "hz_setup_ddm", "hz_solve", "hz_serve_start", "hz_serve_submit"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2004_07930_amd import hz

    if not os.path.exists(hz.LIB_PATH):
        from paper_2004_07930_amd import build

        build.build(verbose=False)
    lib = hz.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(hz.EXPORTS) == _declared()


def test_binding_refuses_missing_library(tmp_path):
    from paper_2004_07930_amd import hz

    with pytest.raises(ImportError):
        hz.load(str(tmp_path / "nope.so"))


STRUCTS = {  # header type -> binding class name
    "hz_init_opts": "InitOpts", "hz_coarse_mesh": "CoarseMesh", "hz_col_info": "ColInfo",
    "hz_solve_opts": "SolveOpts", "hz_ddm_opts": "DdmOpts", "hz_ddm_stats": "DdmStats", "hz_ddm_level": "DdmLevel",
    "hz_kernel_stat": "KernelStat", "hz_request": "Request", "hz_serve_stats": "ServeStats",
}


def test_binding_struct_layouts_match_header(tmp_path):
    """Every struct the binding passes through the ABI has the header's size and field offsets
    (a C program compiled against include/hz.h prints them)."""
    import ctypes
    import shutil
    import subprocess

    from paper_2004_07930_amd import hz

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hz.h"', "int main(void) {"]
    for ctype, cls in STRUCTS.items():
        lines.append(f'  printf("{ctype} size %zu\\n", sizeof({ctype}));')
        for fname, _ in getattr(hz, cls)._fields_:
            lines.append(f'  printf("{ctype} {fname} %zu\\n", offsetof({ctype}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_side = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for ctype, cls in STRUCTS.items():
        k = getattr(hz, cls)
        assert c_side[(ctype, "size")] == ctypes.sizeof(k), ctype
        for fname, _ in k._fields_:
            assert c_side[(ctype, fname)] == getattr(k, fname).offset, (ctype, fname)
