"""The C-ABI library loads, exports every symbol include/mgmlmc.h declares,
and the binding's ctypes structures match the C layout (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mgmlmc.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mgm_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("mgm_set_gauge", "mgm_setup_mg", "mgm_solve_batch", "mgm_apply_D",
                 "mgm_trace_estimate"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2303_11512_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmgmlmc.so not built: run python -m paper_2303_11512_amd.build")
    lib = C.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_missing_library_fails_loudly(tmp_path):
    from paper_2303_11512_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.load_library(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def _c_layout(struct, fields):
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    src.append(f'printf("%zu\\n", sizeof({struct}));')
    for f in fields:
        src.append(f'printf("%zu\\n", offsetof({struct}, {f}));')
    src.append("return 0;}")
    return "\n".join(src)


@pytest.mark.parametrize("cname,pyname", [
    ("mgm_mg_params", "MGParams"), ("mgm_solve_params", "SolveParams"),
    ("mgm_solve_stats", "SolveStats"), ("mgm_trace_params", "TraceParams"),
    ("mgm_trace_result", "TraceResult"), ("mgm_adam_params", "AdamParams"),
    ("mgm_cnn_train_params", "CnnTrainParams"), ("mgm_job", "Job")])
def test_struct_layout_matches_header(cname, pyname, tmp_path):
    from paper_2303_11512_amd import _lib
    py = getattr(_lib, pyname)
    fields = [f for f, _ in py._fields_]
    c_src = tmp_path / "probe.c"
    c_src.write_text(_c_layout(cname, fields))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-o", str(exe), str(c_src)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == C.sizeof(py)
    for f, off in zip(fields, out[1:]):
        assert getattr(py, f).offset == off, f
