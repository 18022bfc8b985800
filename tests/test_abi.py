"""The C-ABI library on the CPU: it loads, exports every symbol include/sse.h
declares, and its host-side validation returns the documented statuses
(no compute calls; nothing here touches a GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sse():
    from paper_1912_08810_amd import sse
    return sse


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sse.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sse_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    sse = _sse()
    out = subprocess.run(["nm", "-D", "--defined-only", sse.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)", out))
    declared = declared_functions()
    assert declared, "no declarations parsed"
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert sorted(sse.EXPORTS) == declared


def plan_status(**kw):
    sse = _sse()
    base = dict(NA=16, NB=4, Norb=4, Nkz=3, Nqz=3, NE=64, Nw=4, ncomp=1, prec=0)
    shift = kw.pop("shift", None)
    base.update(kw)
    d = sse.make_desc(**base)
    if shift is None:
        shift = np.arange(1, base["Nw"] + 1)
    s = np.ascontiguousarray(shift, dtype=np.int32)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = sse.lib.sse_plan(ctypes.byref(d), s.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h),
                          ctypes.byref(ws))
    if st == 0:
        sse.lib.sse_plan_destroy(h)
    return st, ws.value


def test_valid_plan_and_workspace():
    st, ws = plan_status()
    assert st == 0 and ws >= 4


@pytest.mark.parametrize("kw", [dict(NA=0), dict(NB=0), dict(NB=51), dict(Norb=0), dict(Norb=31),
                                dict(Nqz=4), dict(Nw=0), dict(Nw=129), dict(NE=0),
                                dict(ncomp=3), dict(shift=[1, 2, 3, 64]),
                                dict(shift=[1, 2, -64, 3])])
def test_shape_errors(kw):
    sse = _sse()
    st, _ = plan_status(**kw)
    assert st == sse.ERR_SHAPE
    assert sse.last_error()


def test_argument_errors():
    sse = _sse()
    assert plan_status(prec=7)[0] == sse.ERR_ARG
    h = ctypes.c_void_p()
    assert sse.lib.sse_plan(None, None, ctypes.byref(h), None) == sse.ERR_ARG
    assert sse.lib.sse_poll(123456789) == sse.ERR_ARG
    assert "ticket" in sse.last_error()


def test_submit_rejects_small_workspace_before_any_device_call():
    sse = _sse()
    p = sse.sse_plan(sse.make_desc(16, 4, 4, 3, 3, 64, 4), np.arange(1, 5))
    args = sse._args([(1, 1, 1, 1, 1)])
    t = ctypes.c_uint64()
    st = sse.lib.sse_submit(p.handle, args, ctypes.c_void_p(8), 0, None, ctypes.byref(t))
    assert st == sse.ERR_ARG and "workspace" in sse.last_error()


def test_batch_plan_validation():
    sse = _sse()
    d1 = sse.make_desc(16, 4, 4, 3, 3, 64, 4)
    d2 = sse.make_desc(30, 4, 5, 3, 3, 40, 6)  # different Norb
    with pytest.raises(sse.SSEError) as ei:
        sse.sse_plan_batch([d1, d2], [np.arange(1, 5), np.arange(1, 7)])
    assert ei.value.status == sse.ERR_ARG
    p = sse.sse_plan_batch([d1, sse.make_desc(30, 4, 4, 3, 3, 40, 6)],
                           [np.arange(1, 5), np.arange(1, 7)])
    assert p.workspace_bytes >= 512
    many = [d1] * 65
    with pytest.raises(sse.SSEError):
        sse.sse_plan_batch(many, [np.arange(1, 5)] * 65)


def test_tile_e_and_chunk_taps_fields():
    sse = _sse()
    assert plan_status(tile_e=3)[0] == 0
    assert plan_status(tile_e=-1)[0] == sse.ERR_ARG
    assert plan_status(chunk_taps=2)[0] == 0
    assert plan_status(chunk_taps=3, prec=2)[0] == 0
    d = sse.make_desc(16, 4, 4, 3, 3, 64, 4)
    d.chunk_taps = -1
    with pytest.raises(sse.SSEError):
        sse.sse_plan(d, np.arange(1, 5))
