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
