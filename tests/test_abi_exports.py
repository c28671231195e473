"""The C ABI library loads without a GPU and exports every function that
include/*.h declares, and the Python binding names exactly those functions.
No compute call is made."""
import ctypes
import glob
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(ccfr_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def _lib_path():
    from paper_2607_26901_amd import ccfr
    if not os.path.exists(ccfr.LIB_PATH):
        subprocess.run([sys.executable, os.path.join(ROOT, "paper_2607_26901_amd", "build.py")], check=True)
    return ccfr.LIB_PATH


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("ccfr_build_candidates", "ccfr_build_regions", "ccfr_project_displacements", "ccfr_xpbd_step",
              "ccfr_batch_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2607_26901_amd import ccfr
    assert set(ccfr.EXPORTS) == _declared()


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(_lib_path())
    lib.ccfr_status_string.restype = ctypes.c_char_p
    assert lib.ccfr_status_string(0)
    for code in range(-7, 0):
        assert lib.ccfr_status_string(code) != lib.ccfr_status_string(0)
    lib.ccfr_batch_footprint.restype = ctypes.c_int64
    lib.ccfr_batch_footprint.argtypes = [ctypes.c_int32] * 3
    assert lib.ccfr_batch_footprint(-1, 0, 0) == -1
    small = lib.ccfr_batch_footprint(256, 450, 705)
    big = lib.ccfr_batch_footprint(65536, 130050, 195585)
    assert 0 < small < big
