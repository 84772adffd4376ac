"""The C ABI library loads and exports every entry point declared in include/*.h
(no compute calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2208_14567_amd import links

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(links_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for fn in ("links_solve_order", "links_simulate", "links_normalize_paths", "links_create", "links_destroy"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(links.LIB_PATH):
        pytest.skip("liblinks.so not built")
    lib = ctypes.CDLL(links.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(links.EXPORTS) <= _declared()


def test_create_fails_cleanly_without_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = links.load()
    h = ctypes.c_void_p()
    rc = L.links_create(0, ctypes.byref(h))
    assert rc != 0 and not h.value
    assert L.links_last_error().decode()
    assert L.links_version().decode().startswith("links")
