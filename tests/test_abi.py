"""The C-ABI library (CPU-side checks; no kernel is launched)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlcc.h")
LIB = os.path.join(ROOT, "paper_2506_02121_amd", "libmlcc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlcc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmlcc.so is not built (python -m paper_2506_02121_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["mlcc_set_lenses", "mlcc_find_critical_curves", "mlcc_map_caustics",
                 "mlcc_caustic_crossings", "mlcc_caustic_distances"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mlcc_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        getattr(lib, name)


def test_binding_names_match_header():
    from paper_2506_02121_amd import mlcc
    assert sorted(mlcc.EXPORTED) == sorted(n for n in declared_functions())


def test_params_default_is_the_papers_setting(lib):
    from paper_2506_02121_amd import mlcc
    p = mlcc.CCParams()
    lib.mlcc_cc_params_default(ctypes.byref(p), ctypes.c_int64(1000))
    assert p.m_steps == 1000 and p.tol_step == 1e-9 and p.tol_inv_mu == 1e-9
    assert p.max_iter_cold > 0 and p.max_iter_warm > 0 and p.precision == 0


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the header structs have the sizes and field offsets a
    C compiler gives the header."""
    from paper_2506_02121_amd import mlcc
    mirrors = {"mlcc_cc_params": mlcc.CCParams, "mlcc_cc_stats": mlcc.CCStats,
               "mlcc_grid": mlcc.GridC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mlcc.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_errors_without_context(lib):
    from paper_2506_02121_amd import mlcc
    lib.mlcc_set_lenses.restype = ctypes.c_int
    rc = lib.mlcc_set_lenses(None, ctypes.c_int64(1), None, None, None, ctypes.c_double(0.0),
                             ctypes.c_double(0.3))
    assert rc == mlcc.MLCC_ERR_INVALID
    assert "ctx" in mlcc.last_error()
