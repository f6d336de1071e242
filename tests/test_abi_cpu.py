"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0901_1913_amd import fchi2 as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fchi2.h")).read()
    return sorted(set(re.findall(r"\b(fchi2_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    L = F.lib()
    names = _declared()
    assert set(names) == set(F.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = F.lib()
    for s in range(6):
        assert L.fchi2_status_string(s)
    assert L.fchi2_status_string(99) == b"unknown status"


def _plan(**kw):
    off = np.array(kw.pop("offsets", [0, 100]), dtype=np.int64)
    d = dict(n_curves=off.shape[0] - 1, f_max=1.0, H=3, n_freq=2 ** 12,
             precision=F.MIXED, flags=0, kernel_width=0, curves_per_wave=0)
    d.update(kw)
    desc = F.PlanDesc(offsets=off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), **d)
    h = ctypes.c_void_p()
    st = F.lib().fchi2_plan(ctypes.byref(desc), None, ctypes.byref(h))
    return st, F.lib().fchi2_last_error().decode()


@pytest.mark.parametrize("kw,code,frag", [
    (dict(H=0), F.ERR_ARG, "H must be"),
    (dict(H=F.H_MAX + 1), F.ERR_ARG, "H must be"),
    (dict(n_freq=3000), F.ERR_ARG, "power of two"),
    (dict(n_freq=2 ** 9), F.ERR_UNSUPPORTED, "2^10"),
    (dict(n_freq=2 ** 25), F.ERR_UNSUPPORTED, "2^10"),
    (dict(f_max=0.0), F.ERR_ARG, "f_max"),
    (dict(f_max=float("nan")), F.ERR_ARG, "f_max"),
    (dict(precision=7), F.ERR_ARG, "precision"),
    (dict(flags=64), F.ERR_ARG, "flag"),
    (dict(kernel_width=3), F.ERR_ARG, "kernel_width"),
    (dict(kernel_width=2), F.ERR_ARG, "kernel_width"),
    (dict(offsets=[1, 5]), F.ERR_ARG, "offsets[0]"),
    (dict(offsets=[0, 5, 3]), F.ERR_ARG, "nondecreasing"),
    (dict(curves_per_wave=-1), F.ERR_ARG, "curves_per_wave"),
    (dict(first_bin=-1), F.ERR_ARG, "first_bin"),
    (dict(first_bin=2 ** 41), F.ERR_UNSUPPORTED, "first_bin"),
    (dict(first_bin=4096, flags=F.KEEP_FOR_BACKWARD), F.ERR_UNSUPPORTED, "no backward"),
    (dict(first_bin=4096, kernel_width=1), F.ERR_UNSUPPORTED, "no floor gridding"),
])
def test_plan_argument_errors(kw, code, frag):
    st, msg = _plan(**kw)
    assert st == code, (st, msg)
    assert frag in msg


def test_null_arguments():
    L = F.lib()
    h = ctypes.c_void_p()
    assert L.fchi2_plan(None, None, ctypes.byref(h)) == F.ERR_ARG
    assert L.fchi2_search(None, None, None, None, None, 0, None, None, None, None) == F.ERR_ARG
    assert L.fchi2_backward(None, None, None, None, None, None, 0, None, None, None) == F.ERR_ARG
    assert L.fchi2_top_peaks(None, None, 0, 1, 1, None, 0, None, None) == F.ERR_ARG
    assert L.fchi2_search_curves(None, 0, 1, None, None, None, None, 0, None, None, None,
                                 None) == F.ERR_ARG
    assert L.fchi2_autotune(None, None, None, None, None, 0, None, None, None) == F.ERR_ARG
    assert L.fchi2_plan_info(None, None, 8) == F.ERR_ARG
    assert L.fchi2_profile(None, 1) == F.ERR_ARG
    assert L.fchi2_profile_read(None, None, None) == F.ERR_ARG
    assert L.fchi2_workspace_bytes(None) == 0
    assert L.fchi2_top_peaks_scratch_bytes(None, 4) == 0
    assert L.fchi2_search_top(None, None, None, None, None, 0, 0, 1, 4, None, None,
                              None) == F.ERR_ARG
    assert L.fchi2_search_top_workspace_bytes(None, 4) == 0
    assert L.fchi2_fine_search(None, None, None, None, None, 4, 8, 0.1, 0, None, 0, None,
                               None) == F.ERR_ARG
    assert L.fchi2_fine_scratch_bytes(None, 4, 8) == 0
    assert L.fchi2_search_multi(None, None, None, None, None, 4, None, 0, None, None, None,
                                None) == F.ERR_ARG
    assert L.fchi2_search_multi_workspace_bytes(None, 4) == 0
    assert L.fchi2_detrend(None, None, None, None, 1, None, None, None) == F.ERR_ARG
    assert L.fchi2_autotune_multi(None, None, None, None, None, 4, None, 0, None, None) == F.ERR_ARG
    L.fchi2_destroy(None)
