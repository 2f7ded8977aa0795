"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects invalid descriptors and arguments before making any HIP call."""

import ctypes
import os
import re

import pytest

from paper_2510_10070_amd import _lib
from paper_2510_10070_amd._lib import SbpBox, SbpShear

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbp.h")


def lib():
    return _lib.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib(), n), n
    assert set(names) == set(_lib.EXPORTS)


def test_status_strings():
    for code in range(7):
        s = lib().sbp_status_str(code)
        assert s and s.decode() != "unknown status"
    assert lib().sbp_status_str(99).decode() == "unknown status"


def _create(boxes, prec=1, flags=0, nbox=None):
    arr = (SbpBox * len(boxes))(*boxes)
    h = ctypes.c_void_p(1234)
    st = lib().sbp_plan_create(arr, len(boxes) if nbox is None else nbox, prec, 0, flags, ctypes.byref(h))
    return st, h


def good():
    return SbpBox(32, 32, 32, 1.0, 1.0, 1.0, 2, 0.0, 0)


@pytest.mark.parametrize(
    "mutate,expect",
    [
        (lambda b: setattr(b, "nx", 0), 1),
        (lambda b: setattr(b, "nx", 40), 2),
        (lambda b: setattr(b, "ny", 2048), 2),
        (lambda b: setattr(b, "nz", 7), 2),
        (lambda b: setattr(b, "nz", 2), 2),
        (lambda b: setattr(b, "nz", 1024), 2),
        (lambda b: setattr(b, "pad", 3), 1),
        (lambda b: setattr(b, "lx", 0.0), 1),
        (lambda b: setattr(b, "lz", float("nan")), 1),
        (lambda b: setattr(b, "ly", float("inf")), 1),
        (lambda b: setattr(b, "alpha", 1.1), 1),  # P = 2 with alpha = 1.1: images overlap
        (lambda b: setattr(b, "alpha", 0.5), 1),
        (lambda b: setattr(b, "method", 7), 1),
    ],
)
def test_invalid_descriptor_rejected_before_hip(mutate, expect):
    b = good()
    mutate(b)
    st, h = _create([b])
    assert st == expect, (st, lib().sbp_last_error())
    assert h.value is None  # *out cleared
    assert lib().sbp_last_error().decode()


def test_paper_padding_accepted_by_validation():
    # P = 4 with alpha = 1.1 (the paper's VGF setting) passes validation; whatever status comes
    # back is from the device layer, never an argument error
    b = good()
    b.pad, b.alpha = 4, 1.1
    st, h = _create([b])
    assert st in (0, 5)
    if st == 0:
        lib().sbp_plan_destroy(h)


def test_bad_plan_arguments():
    st, _ = _create([good()], prec=5)
    assert st == 1
    st, _ = _create([good()], flags=0x80)
    assert st == 1
    st, _ = _create([good()], prec=1, flags=_lib.SBP_FLAG_PLAIN)  # plain path is FP64 only
    assert st == 1
    st, _ = _create([good()], prec=0, flags=_lib.SBP_FLAG_PLAIN | _lib.SBP_FLAG_FUSED)
    assert st == 1
    st, _ = _create([good()], flags=_lib.SBP_FLAG_FUSED | _lib.SBP_FLAG_FIVE_PASS)  # exclusive schedules
    assert st == 1
    lin = good()
    lin.remap = _lib.SBP_REMAP_LINEAR
    st, _ = _create([lin], prec=0, flags=_lib.SBP_FLAG_PLAIN)  # the plain path is spectral only
    assert st == 1
    bad = good()
    bad.remap = 2
    st, _ = _create([bad])
    assert st == 1
    st, _ = _create([good()], nbox=0)
    assert st == 1
    h = ctypes.c_void_p()
    assert lib().sbp_plan_create(None, 1, 0, 0, 0, ctypes.byref(h)) == 1
    arr = (SbpBox * 1)(good())
    assert lib().sbp_plan_create(arr, 1, 0, -1, 0, ctypes.byref(h)) == 1
    assert lib().sbp_plan_create(arr, 1, 0, 0, 0, None) == 1


def test_null_plan_calls():
    n = ctypes.c_size_t()
    assert lib().sbp_workspace_size(None, ctypes.byref(n)) == 1
    assert lib().sbp_set_workspace(None, None, 0) == 1
    assert lib().sbp_solve(None, None, None, None, None) == 1
    assert lib().sbp_plan_destroy(None) == 0
    assert lib().sbp_profile_enable(None, 1) == 1
    cnt = ctypes.c_int32()
    assert lib().sbp_profile_read(None, None, None, None, 0, ctypes.byref(cnt)) == 1
    assert lib().sbp_plan_describe(None, ctypes.create_string_buffer(8), 8) == 1


def test_no_device_reports_hip_error():
    try:
        import torch

        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    st, h = _create([good()])
    assert st == 5 and h.value is None
