"""The C-ABI library loads without a GPU and exports every entry point its
header declares (no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgrid.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*((?:grid|batch)_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("grid_build", "grid_trace", "grid_locate", "grid_import", "grid_export",
                 "grid_free", "grid_strerror", "grid_last_hip_error"):
        assert want in names, want


def test_library_exports_every_declared_symbol():
    import __graft_entry__  # noqa: F401  (puts the repo root on sys.path)
    import paper_1311_0705_amd as hg
    if not os.path.exists(hg.LIB_PATH):
        from paper_1311_0705_amd import _build
        _build.build()
    lib = ctypes.CDLL(hg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # host-only calls are safe without a device
    lib.grid_strerror.restype = ctypes.c_char_p
    assert lib.grid_strerror(0) == b"success"
    assert b"capacity" in lib.grid_strerror(-4)


def test_binding_signatures_match_header():
    import paper_1311_0705_amd as hg
    bound = {name for name, _, _ in hg._SIGS}
    assert bound == set(declared_functions())


def test_struct_layouts_match_header():
    # sizes of the ABI structs as the C compiler lays them out
    import subprocess
    import tempfile
    import paper_1311_0705_amd as hg
    prog = r'''
#include <stdio.h>
#include "hgrid.h"
int main(void){printf("%zu %zu %zu %zu %zu\n", sizeof(hg_density), sizeof(hg_criteria),
 sizeof(hg_trace_opts), sizeof(hg_trace_out), sizeof(hg_grid_arrays));return 0;}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(t) for t in (hg.Density, hg.Criteria, hg.TraceOpts, hg.TraceOut,
                                       hg.GridArrays)]
    assert got == want
