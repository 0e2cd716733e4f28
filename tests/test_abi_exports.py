"""The C-ABI library loads and exports every function include/aiwc.h
declares (no GPU calls)."""
import ctypes
import os
import re

import paper_1805_04207_amd as aiwc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "aiwc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aiwc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("aiwc_trace_create", "aiwc_characterize", "aiwc_characterize_batch",
                 "aiwc_metrics_read"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(aiwc.aiwc.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_export():
    assert set(declared()) == set(aiwc.aiwc.EXPORTS)
    aiwc.load_library()
