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
    (dict(kernel_width=3), F.ERR_ARG, "kernel_width"),
    (dict(kernel_width=2), F.ERR_ARG, "kernel_width"),
    (dict(offsets=[1, 5]), F.ERR_ARG, "offsets[0]"),
    (dict(offsets=[0, 5, 3]), F.ERR_ARG, "nondecreasing"),
    (dict(curves_per_wave=-1), F.ERR_ARG, "curves_per_wave"),
    (dict(first_bin=-1), F.ERR_ARG, "first_bin"),
    (dict(first_bin=2 ** 41), F.ERR_UNSUPPORTED, "first_bin"),
    (dict(first_bin=4096, flags=F.KEEP_FOR_BACKWARD), F.ERR_UNSUPPORTED, "no backward"),
    (dict(first_bin=4096, kernel_width=1), F.ERR_UNSUPPORTED, "no floor gridding"),
    (dict(H=9, flags=F.KEEP_FOR_BACKWARD), F.ERR_UNSUPPORTED, "backward needs H <= 8"),
    (dict(H=3, flags=F.KEEP_FOR_BACKWARD | F.WIDE_SOLVE), F.ERR_UNSUPPORTED, "backward needs"),
    (dict(H=12, first_bin=4096), F.ERR_UNSUPPORTED, "band plans need H <= 8"),
    (dict(flags=64), F.ERR_ARG, "flag"),
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
    assert L.fchi2_backward_at(None, 0, None, None, None, None, None, 0, None, None,
                               None) == F.ERR_ARG
    assert L.fchi2_search_generation(None) == 0
    assert L.fchi2_top_peaks(None, None, 0, 1, 1, None, 0, None, None) == F.ERR_ARG
    assert L.fchi2_search_curves(None, 0, 1, None, None, None, None, 0, None, None, None,
                                 None) == F.ERR_ARG
    assert L.fchi2_autotune(None, None, None, None, None, 0, None, None, None) == F.ERR_ARG
    assert L.fchi2_plan_info(None, None, 8) == F.ERR_ARG
    arr = (ctypes.c_int32 * 14)()
    assert L.fchi2_plan_set_schedule(None, arr, 14) == F.ERR_ARG
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


def test_auto_n_freq_rule():
    """n_freq = 0: next power of two >= ceil(os H span f_max), at least 2^10."""
    # The plain and long-curve workloads' grids follow from os = 5.
    assert F.auto_n_freq(3, 10.0, 5.0, 100.0) == 2 ** 14
    assert F.auto_n_freq(5, 50.0, 5.0, 3000.0) == 2 ** 22
    # The paper's own density (os = 2, spacing 1/(2 H span)).
    assert F.auto_n_freq(3, 12.0, 2.0, 1000.0) == 2 ** 17
    rng = np.random.default_rng(3)
    for _ in range(200):
        H = int(rng.integers(1, F.H_MAX + 1))
        fm, os_, sp = 10 ** rng.uniform(-1, 2), rng.uniform(0.5, 8), 10 ** rng.uniform(0, 3.5)
        want = max(2 ** 10, 1 << int(np.ceil(np.log2(np.ceil(os_ * H * sp * fm)))))
        got = F.auto_n_freq(H, fm, os_, sp)
        assert got == (want if want <= 2 ** 24 else 0), (H, fm, os_, sp, got, want)
        if got:
            assert got >= os_ * H * sp * fm and (got == 2 ** 10 or got / 2 < np.ceil(os_ * H * sp * fm))
    for bad in ((0, 1.0, 5.0, 1.0), (3, 0.0, 5.0, 1.0), (3, 1.0, -1.0, 1.0),
                (3, 1.0, 5.0, float("inf")), (3, 1e6, 5.0, 1e6)):
        assert F.auto_n_freq(*bad) == 0


def test_plan_auto_n_freq_argument_errors():
    off = np.array([0, 100, 250], dtype=np.int64)
    for spans, os_, frag in ((None, 5.0, "t_span"), ([10.0, float("nan")], 5.0, "t_span[1]"),
                             ([0.0, 0.0], 5.0, "span > 0"), ([10.0, 20.0], -2.0, "oversampling"),
                             ([1e5, 1e5], 50.0, "exceeds")):
        d = dict(n_curves=2, f_max=10.0, H=3, n_freq=0, precision=F.MIXED, flags=0,
                 kernel_width=0, curves_per_wave=0, oversampling=os_)
        desc = F.PlanDesc(offsets=off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), **d)
        if spans is not None:
            arr = np.asarray(spans, dtype=np.float64)
            desc.t_span = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        st = F.lib().fchi2_plan(ctypes.byref(desc), None, ctypes.byref(h))
        msg = F.lib().fchi2_last_error().decode()
        assert st in (F.ERR_ARG, F.ERR_UNSUPPORTED) and frag in msg, (spans, st, msg)
