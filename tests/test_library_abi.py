"""The C-ABI library loads without a GPU and exports what its header declares.

No compute entry point is called here: the checks are symbol presence, the binding's list of
names, the host-only option defaults, and the layout of the structs shared through ctypes
(compared with what a C compiler reports for the header).
"""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1709_06350_amd import build, mr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(mr_\w+)\s*\(", text, flags=re.M)))


def _lib():
    if not os.path.exists(build.LIB):
        pytest.skip("libmr.so not built")
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("mr_create", "mr_destroy", "mr_deposit_cic", "mr_residual", "mr_solve",
                     "mr_adjoint_solve", "mr_solve_batched"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_exactly_the_declared_symbols():
    assert sorted(mr.EXPORTED) == _declared()


def test_no_undeclared_exports():
    nm = shutil.which("nm")
    if nm is None or not os.path.exists(build.LIB):
        pytest.skip("nm or libmr.so missing")
    out = subprocess.run([nm, "-D", "--defined-only", build.LIB], capture_output=True, text=True, check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if re.search(r" T mr_\w+$", ln)})
    assert exported == _declared()


def test_default_options_are_host_only():
    _lib()
    o = mr.default_opts()
    assert o.tol == 1e-10 and o.max_cycles == 100 and o.npre == 2 and o.npost == 2
    assert o.precision == mr.PREC_FP64 and o.flags == 0


C_LAYOUT = r"""
#include <stddef.h>
#include <stdio.h>
#include "mr.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(mr_opts), offsetof(mr_opts, flags), sizeof(mr_info), offsetof(mr_info, history));
  printf("%zu %zu\n", sizeof(mr_timing), offsetof(mr_timing, finest_cells));
  return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(C_LAYOUT)
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:2]
    so, of, si, oh = map(int, a.split())
    st, ofc = map(int, b.split())
    assert so == ctypes.sizeof(mr.mr_opts) and of == mr.mr_opts.flags.offset
    assert si == ctypes.sizeof(mr.mr_info) and oh == mr.mr_info.history.offset
    assert st == ctypes.sizeof(mr.mr_timing) and ofc == mr.mr_timing.finest_cells.offset


def test_binding_constants_match_the_header_enums():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    enums = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", text, flags=re.S):
        for name, val in re.findall(r"(MR_\w+)\s*=\s*(-?\d+)", body):
            enums[name] = int(val)
    assert enums, "no enum constants found in the header"
    for name, val in enums.items():
        py = name if hasattr(mr, name) else name[len("MR_"):]
        assert getattr(mr, py) == val, name
