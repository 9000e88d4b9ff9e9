"""The C-ABI library loads and exports every entry point that include/ddps.h
declares, and the Python binding's structs match the C layout.  No GPU
work is done here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddps.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ddps_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1008_1700_amd import ddps
    if not os.path.exists(ddps.LIB_PATH):
        from paper_1008_1700_amd import build
        build.build()
    return ddps.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(lib, nm), nm


def test_binding_covers_the_header():
    from paper_1008_1700_amd import ddps
    assert sorted(ddps.exported_symbols()) == _declared()


def test_struct_layouts_match_c(tmp_path):
    from paper_1008_1700_amd import ddps
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ddps.h"\nint main(void){'
                    'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ddps_options), sizeof(ddps_info),'
                    'offsetof(ddps_options, mem_budget), offsetof(ddps_options, stream),'
                    'offsetof(ddps_info, bad_block), offsetof(ddps_info, bad_row)); return 0;}')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    exp = [ctypes.sizeof(ddps.ddps_options), ctypes.sizeof(ddps.ddps_info),
           ddps.ddps_options.mem_budget.offset, ddps.ddps_options.stream.offset,
           ddps.ddps_info.bad_block.offset, ddps.ddps_info.bad_row.offset]
    assert got == exp


def test_defaults_and_status_strings(lib):
    from paper_1008_1700_amd import ddps
    o = ddps.ddps_default_options()
    assert o.struct_size == ctypes.sizeof(ddps.ddps_options)
    assert o.factor_dtype == ddps.F64 and o.inner_tol == 1e-12 and o.outer_maxit == 1000
    for code in ddps.STATUS:
        assert ddps.ddps_status_string(code).startswith(ddps.STATUS[code])


def test_null_arguments_are_rejected_without_a_gpu(lib):
    h = ctypes.c_void_p()
    assert lib.ddps_setup(ctypes.byref(h), 0, 1, None, None, None, None, 0, None) == -1
    assert lib.ddps_factor(None) == -1
    assert lib.ddps_solve(None, None, None, 1e-10, None) == -1
