"""GPU: a caller workspace smaller than bz_workspace_bytes is refused with BZ_ENOMEM.

bz_min_distance and bz_min_distance_batch take an optional device workspace
(o->workspace, o->workspace_bytes). One byte short of what bz_workspace_bytes
reports must return BZ_ENOMEM before any device work, with a message, and
leave nothing behind: the same call with the full size then succeeds and
matches the search that lets the library allocate.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_1911_08963_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1911_08963_amd import bz as _bz
    _bz.lib()
    torch.cuda.init()
    return _bz


def _result(bz):
    r = bz.Result()
    wit = np.zeros(4, dtype=np.uint64)
    r.witness = wit.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    r.stats = None
    r.stats_cap = 0
    return r, wit


def test_single_search_short_workspace(bz):
    import torch
    c = inputs.plain_code("plain40")
    code = bz.Code(c.G, c.n)
    need = bz.workspace_bytes()
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    o = bz._opts(0, 0, stream, ws, None, 0, 0)
    o.workspace_bytes = need - 1
    r, _ = _result(bz)
    st = bz.lib().bz_min_distance(code.handle, ctypes.byref(o), ctypes.byref(r))
    assert st == bz.BZ_ENOMEM
    assert "workspace" in bz.lib().bz_last_error().decode()
    # the full size works and gives the library-allocated search's answer
    o.workspace_bytes = need
    r, wit = _result(bz)
    assert bz.lib().bz_min_distance(code.handle, ctypes.byref(o), ctypes.byref(r)) == bz.BZ_OK
    ref = bz.min_distance(code)
    assert r.d == ref.d == 4
    assert int(np.bitwise_count(wit).sum()) == r.d
    code.close()


def test_batch_short_workspace(bz):
    import torch
    objs = [bz.Code(c.G, c.n) for c in (inputs.batch_code(i) for i in range(3, 7))]
    cnt = len(objs)
    handles = (ctypes.c_void_p * cnt)(*[o.handle.value for o in objs])
    stream = torch.cuda.current_stream().cuda_stream
    o = bz._opts(0, 0, stream, None, None, 0, 0)
    need = ctypes.c_size_t()
    assert bz.lib().bz_workspace_bytes(handles, cnt, ctypes.byref(o), ctypes.byref(need)) == bz.BZ_OK
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    o = bz._opts(0, 0, stream, ws, None, 0, 0)
    o.workspace_bytes = need.value - 1
    res = (bz.Result * cnt)()
    wits = np.zeros((cnt, 4), dtype=np.uint64)
    for i in range(cnt):
        res[i].witness = ctypes.cast(wits.ctypes.data + 32 * i, ctypes.POINTER(ctypes.c_uint64))
        res[i].stats = None
        res[i].stats_cap = 0
    per = (ctypes.c_int * cnt)()
    st = bz.lib().bz_min_distance_batch(handles, cnt, ctypes.byref(o), res, per)
    assert st == bz.BZ_ENOMEM
    assert "workspace" in bz.lib().bz_last_error().decode()
    o.workspace_bytes = need.value
    assert bz.lib().bz_min_distance_batch(handles, cnt, ctypes.byref(o), res, per) == bz.BZ_OK
    for i, c in enumerate(objs):
        assert per[i] == bz.BZ_OK
        assert res[i].d == bz.min_distance(c).d
        assert int(np.bitwise_count(wits[i]).sum()) == res[i].d
        c.close()
