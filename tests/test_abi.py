"""The C-ABI library loads, exports every function declared in
include/sncc.h, and rejects bad arguments without a GPU (no compute calls)."""

import ctypes as C

import numpy as np
import pytest

import paper_2502_01286_amd as S


def test_every_declared_function_is_exported():
    names = S.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(S.lib, n), n
        assert callable(getattr(S, n, None)), f"binding lacks {n}"


def test_status_strings_and_version():
    for code in [0, -1, -2, -3, -4, -5, -6]:
        assert S.sncc_status_string(code) not in ("", "unknown status")
    assert S.sncc_status_string(-99) == "unknown status"
    assert S.sncc_version() >= 10000


def test_sat_pitch():
    assert S.sncc_sat_pitch(1) == 64
    assert S.sncc_sat_pitch(63) == 64
    assert S.sncc_sat_pitch(64) == 128
    assert S.sncc_sat_pitch(1920) == 1984
    with pytest.raises(S.SnccError):
        S.sncc_sat_pitch(0)


def test_null_handles_are_rejected():
    L = S.lib
    assert L.sncc_sync(None) == S.SNCC_EINVAL
    assert L.sncc_build_sats(None, None, 1, 1, 1, 1, None, None, 64) == S.SNCC_EINVAL
    assert L.sncc_score(None, None, 0, None, None, 1, 1, 64, 0, None, 1, None) == S.SNCC_EINVAL
    assert L.sncc_batch_run(None) == S.SNCC_EINVAL
    assert L.sncc_tmpl_info(None, 0, None, None, None, None) == S.SNCC_EINVAL
    assert L.sncc_ctx_destroy(None) == S.SNCC_OK
    assert L.sncc_tmpl_destroy(None) == S.SNCC_OK
    assert L.sncc_batch_destroy(None) == S.SNCC_OK
    assert "NULL" in S.sncc_last_error() or S.sncc_last_error() == ""


def test_ctx_create_bad_device_reports_error():
    h = C.c_void_p()
    rc = S.lib.sncc_ctx_create(10_000, 0, C.byref(h))
    assert rc in (S.SNCC_EINVAL, S.SNCC_EDEVICE)
    assert not h.value


def test_segment_dtype_layout():
    assert S.SEGMENT_DTYPE.itemsize == 32
    a = np.zeros(2, S.SEGMENT_DTYPE)
    assert a.strides == (32,)


def test_header_constants_match_binding():
    """Every numeric macro of the header has the same value in the binding."""
    import os
    import re
    import paper_2502_01286_amd._native as nat
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "include", "sncc.h")) as fh:
        text = fh.read()
    macros = re.findall(r"^#define (SNCC_\w+) \(?(-?\d+)(?:LL)?\)?", text, re.M)
    assert len(macros) >= 10
    for name, val in macros:
        assert getattr(nat, name) == int(val), name
