"""The C-ABI library loads and exports every entry point include/janc.h declares
(no compute calls: no GPU here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "janc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(janc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["janc_create", "janc_destroy", "janc_step", "janc_step_blocks", "janc_adjoint",
              "janc_plan_create", "janc_init_state", "janc_sync_status"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2504_13750_amd as janc
    lib = janc.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    from paper_2504_13750_amd import _lib as L
    assert ctypes.sizeof(L.janc_block) == 40
    assert ctypes.sizeof(L.janc_physics) == 40
    assert ctypes.sizeof(L.janc_time) == 32
    assert ctypes.sizeof(L.janc_grid) == 8 + 16 + 16 + 4 * 16 * 8
    assert ctypes.sizeof(L.janc_mech) == 8 + 12 * 8


def test_struct_layouts_match_c_compiler(tmp_path):
    """sizeof and field offsets of the binding's structs equal those the C compiler
    gives the header's declarations."""
    import shutil
    import subprocess
    from paper_2504_13750_amd import _lib as L
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"janc_block": L.janc_block, "janc_physics": L.janc_physics,
               "janc_time": L.janc_time, "janc_grid": L.janc_grid, "janc_mech": L.janc_mech,
               "janc_domain": L.janc_domain, "janc_regrid_params": L.janc_regrid_params}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "janc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])


def test_block_dtype_matches_cases():
    import numpy as np
    import paper_2504_13750_amd as janc
    from cases.common import BLOCK_DTYPE
    assert janc.BLOCK_DTYPE == BLOCK_DTYPE
    assert janc.BLOCK_DTYPE.itemsize == 40


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2504_13750_amd import _lib as L
    monkeypatch.setattr(L, "_LIB", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(L.LibraryMissing):
        L.lib()


def test_plan_flags_match_header(tmp_path):
    """The binding's PLAN_* constants equal the header's JANC_PLAN_* values."""
    import shutil
    import subprocess
    import paper_2504_13750_amd as janc
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    names = [n for n in dir(janc) if n.startswith("PLAN_")]
    assert "PLAN_RESOLVE_HALOS" in names
    lines = ["#include <stdio.h>", '#include "janc.h"', "int main(void) {"]
    lines += [f'printf("{n} %d\\n", (int)JANC_{n});' for n in names]
    lines += ["return 0; }"]
    src = tmp_path / "flags.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "flags"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {ln.split()[0]: int(ln.split()[1]) for ln in out.splitlines()}
    assert got == {n: getattr(janc, n) for n in names}
