"""The C-ABI library builds for gfx950, loads, and exports every entry point
include/lgdm.h declares; the binding's struct layouts match the header.
CPU only: no compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lgdm.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lgdm_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_expected_api():
    from paper_2301_06503_amd import binding
    assert header_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2301_06503_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load_library()
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (lgdm_[a-z_0-9]+)\b", out))
    assert set(header_functions()) <= exported


def test_struct_layouts_match_header():
    """Compile a tiny C program against the header that prints sizeof/offsetof
    and compare with the ctypes mirrors."""
    from paper_2301_06503_amd import binding
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "lgdm.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(lgdm_material), offsetof(lgdm_material, plane), offsetof(lgdm_material, thickness));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(lgdm_solver_opts), offsetof(lgdm_solver_opts, max_restarts), offsetof(lgdm_solver_opts, idr_s), offsetof(lgdm_solver_opts, precond), offsetof(lgdm_solver_opts, max_increment_krylov), offsetof(lgdm_solver_opts, max_increment_seconds));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(lgdm_increment_report), offsetof(lgdm_increment_report, reaction), offsetof(lgdm_increment_report, restarts), offsetof(lgdm_increment_report, krylov_rel_e), offsetof(lgdm_increment_report, krylov_spmv), offsetof(lgdm_increment_report, precond_fallbacks));
  printf("%zu %zu\n", sizeof(lgdm_csr_view), offsetof(lgdm_csr_view, vals32));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    m = [int(v) for v in lines[0].split()]
    assert m == [ctypes.sizeof(binding.Material), binding.Material.plane.offset,
                 binding.Material.thickness.offset]
    o = [int(v) for v in lines[1].split()]
    assert o == [ctypes.sizeof(binding.SolverOpts), binding.SolverOpts.max_restarts.offset,
                 binding.SolverOpts.idr_s.offset, binding.SolverOpts.precond.offset,
                 binding.SolverOpts.max_increment_krylov.offset, binding.SolverOpts.max_increment_seconds.offset]
    r = [int(v) for v in lines[2].split()]
    assert r == [ctypes.sizeof(binding.IncrementReport), binding.IncrementReport.reaction.offset,
                 binding.IncrementReport.restarts.offset, binding.IncrementReport.krylov_rel_e.offset,
                 binding.IncrementReport.krylov_spmv.offset, binding.IncrementReport.precond_fallbacks.offset]
    v = [int(v) for v in lines[3].split()]
    assert v == [ctypes.sizeof(binding.CsrView), binding.CsrView.vals32.offset]


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2301_06503_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
