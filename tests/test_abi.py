"""The C-ABI library loads and exports every entry point include/libfsmi.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libfsmi.h")
LIB = os.path.join(ROOT, "paper_1905_02238_amd", "libfsmi.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fsmi_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("fsmi_raycast", "fsmi_eval_beams", "fsmi_rle_eval_beams", "fsmi_eval_poses",
              "fsmi_create", "fsmi_destroy", "fsmi_sync", "fsmi_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsmi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsmi.so not built")
def test_status_strings_and_defaults_without_device():
    from paper_1905_02238_amd import fsmi as F
    L = F.load()
    assert L.fsmi_status_string(0) == b"ok"
    p = F.fsmi_params()
    L.fsmi_default_params(ctypes.byref(p))
    assert p.delta_occ == 1.5 and p.variant == F.FSMI_EXACT and p.precision == F.FSMI_FP32
    assert p.flags == 0 and p.sigma_slope == 0.0
    # double, 5 x int32, uint32, double: the C layout, no padding before the last double
    assert ctypes.sizeof(F.fsmi_params) == 40


def test_binding_names_match_header():
    from paper_1905_02238_amd import fsmi as F
    assert sorted(F.EXPORTS) == declared()
