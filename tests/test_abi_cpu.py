"""Host-side checks of the C-ABI library (no GPU calls).

The library must load and export every function that include/*.h declares,
and the ctypes binding must declare exactly those.  Nothing here launches
device work.
"""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cgd_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib_path():
    from paper_1409_0001_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1409_0001_amd import build
        build.build()
    return _abi.LIB_PATH


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("cgd_deposit", "cgd_diffuse", "cgd_coarse_grain", "cgd_mesh_create_hex",
                 "cgd_mesh_create_tet", "cgd_mesh_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = declared_functions() - exported
    assert not missing, missing


def test_library_loads_and_binding_matches(lib_path):
    from paper_1409_0001_amd import _abi
    lib = _abi.load(lib_path)
    assert set(_abi.SIGNATURES) == declared_functions()
    assert lib.cgd_version() >= 100
    assert lib.cgd_status_string(-1) == b"CGD_E_INVALID"
    assert lib.cgd_status_string(0) == b"CGD_OK"


def test_struct_layouts_match_header():
    """Sizes of the option / statistics structs as the C compiler lays them out."""
    from paper_1409_0001_amd import _abi
    src = os.path.join(ROOT, "include", "cgd.h")
    prog = ("#include <stdio.h>\n#include \"%s\"\nint main(){printf(\"%%zu %%zu\\n\","
            "sizeof(cgd_solver_opts), sizeof(cgd_solve_stats));return 0;}\n" % src)
    exe = os.path.join("/tmp", f"cgd_sizes_{os.getpid()}")
    subprocess.run(["gcc", "-x", "c", "-", "-o", exe], input=prog, text=True, check=True)
    a, b = map(int, subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split())
    os.unlink(exe)
    assert a == ctypes.sizeof(_abi.SolverOpts)
    assert b == ctypes.sizeof(_abi.SolveStats)


def test_binding_refuses_without_gpu():
    """No silent CPU fallback: the product path raises when no GPU is visible."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_1409_0001_amd as cgd
    with pytest.raises(RuntimeError):
        cgd.HexMesh((4, 4, 4))
