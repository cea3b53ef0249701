"""The C-ABI library builds, loads and exports every entry point declared in
include/*.h (no compute calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(swf_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_render_boundary():
    names = declared_symbols()
    for n in ("swf_create", "swf_destroy", "swf_scene_upload", "swf_render", "swf_render_backward",
              "swf_radix_sort", "swf_exclusive_scan"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2506_12787_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libswiftwrf.so is not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    from paper_2506_12787_amd import binding
    L = binding.lib()
    assert L.swf_status_string(0) == b"ok"
    assert L.swf_status_string(-1) == b"invalid argument"
