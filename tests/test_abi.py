"""CPU checks of the C ABI: the library loads and exports every function the header declares,
and the host-only entry points behave (no GPU compute is called here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwfmm.h")


@pytest.fixture(scope="module")
def dwlib():
    import paper_2402_09531_amd as dw
    if not os.path.exists(dw.LIB_PATH):
        from paper_2402_09531_amd import build as B
        B.build(verbose=False)
    return dw


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dwfmm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dwfmm_build_tree", "dwfmm_fmm_create", "dwfmm_fmm_matvec", "dwfmm_fmm_solve"):
        assert required in names


def test_library_exports_every_declared_symbol(dwlib):
    L = C.CDLL(dwlib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", dwlib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dwfmm_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(dwlib.EXPORTS) == set(declared_functions())


def test_library_has_gfx950_code(dwlib):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", dwlib.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_host_only_entry_points(dwlib):
    L = dwlib.lib()
    # argument errors are reported before any device work
    h = C.c_void_p()
    st = L.dwfmm_build_tree(None, 10, 3, None, 16, 0.8, None, C.byref(h))
    assert st == dwlib.E_INVALID
    assert b"NULL" in L.dwfmm_last_error()
    assert L.dwfmm_fmm_matvec(None, None, None, 1, None) == dwlib.E_INVALID
    assert dwlib.estimate_bytes(1_000_000, 20, 128, 15, 1) > 1_000_000 * 20 * 8
    assert dwlib.estimate_bytes(0, 20, 128, 15, 1) == 0
    L.dwfmm_op_destroy(None)
    L.dwfmm_tree_destroy(None)
