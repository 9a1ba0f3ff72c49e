"""CPU checks of the C ABI library: it loads and exports every entry point
include/prrtc.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_06757_amd", "libprrtc.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "prrtc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prrtc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("prrtc_create", "prrtc_destroy", "prrtc_last_error", "prrtc_load_robot",
              "prrtc_load_scene", "prrtc_check_edges", "prrtc_plan"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches():
    lib = ctypes.CDLL(LIB)
    from paper_2503_06757_amd import prrtc as P
    for n in declared_functions():
        assert hasattr(lib, n)
        assert n in P.EXPORTED
    # without a device, creating a context fails cleanly (status, null handle)
    h = ctypes.c_void_p()
    lib.prrtc_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    lib.prrtc_destroy.argtypes = [ctypes.c_void_p]
    st = lib.prrtc_create(ctypes.byref(h), 0)
    if st == 0:
        lib.prrtc_destroy(h)
    else:
        assert not h.value
    assert lib.prrtc_create(ctypes.byref(h), 1 << 20) != 0     # no such device
    lib.prrtc_destroy(None)
