"""The C-ABI library loads on the CPU and exports every entry point the header declares."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nystrom_schur.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nystrom_schur_\w+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared_functions()
    for req in ("nystrom_schur_setup", "nystrom_schur_apply", "nystrom_schur_pcg_solve", "nystrom_schur_destroy",
                "nystrom_schur_last_error"):
        assert req in names


def test_library_exports_all_declared_symbols():
    from paper_2101_12164_amd import EXPORTED, library_path

    path = library_path()
    if not os.path.exists(path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(EXPORTED) == declared_functions()
    # exported with C linkage (no mangling)
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(r"\bT " + name + r"$", out, flags=re.M), name


def test_last_error_without_handle():
    from paper_2101_12164_amd import library_path

    path = library_path()
    if not os.path.exists(path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(path)
    lib.nystrom_schur_last_error.restype = ctypes.c_char_p
    lib.nystrom_schur_last_error.argtypes = [ctypes.c_void_p]
    assert lib.nystrom_schur_last_error(None) is not None


def test_setup_rejects_bad_arguments_without_touching_the_gpu():
    """NULL options / bad sizes are rejected on the host before any device call."""
    from paper_2101_12164_amd import library_path
    from paper_2101_12164_amd.nystrom_schur import NsOptions

    path = library_path()
    if not os.path.exists(path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(path)
    lib.nystrom_schur_setup.restype = ctypes.c_int32
    h = ctypes.c_void_p(1)
    st = lib.nystrom_schur_setup(ctypes.c_int64(0), ctypes.c_int64(0), None, None, None, None, None, ctypes.byref(h),
                                 None)
    assert st == 1 and h.value is None
    opt = NsOptions()
    opt.k = -1
    st = lib.nystrom_schur_setup(ctypes.c_int64(4), ctypes.c_int64(4), ctypes.c_void_p(8), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.byref(opt), ctypes.byref(h), None)
    assert st == 1


def test_package_exposes_every_entry_point():
    import paper_2101_12164_amd as ns

    for name in ns.EXPORTED:
        assert callable(getattr(ns, name, None)), name


def test_kernel_family_names_match_the_library():
    """Every timing family the binding names is one the library knows (statistics of an untimed run: zeros)."""
    from paper_2101_12164_amd import library_path
    from paper_2101_12164_amd.nystrom_schur import KERNEL_FAMILIES, nystrom_schur_kernel_stats

    if not os.path.exists(library_path()):
        pytest.skip("library not built")
    assert len(KERNEL_FAMILIES) == len(set(KERNEL_FAMILIES)) <= 32
    for f in KERNEL_FAMILIES:
        st = nystrom_schur_kernel_stats(f)
        assert st["launches"] == 0 and st["ms"] == 0.0
    with pytest.raises(Exception):
        nystrom_schur_kernel_stats("no_such_family")
