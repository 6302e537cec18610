"""GPU checks of the boundary's error paths: a workspace limit below what the
plan needs returns JP_ENOMEM and leaves nothing behind (the next plan of the
same query succeeds and equals the oracle); calls out of order return
JP_ESTATE; peak_bytes stays within a limit that is enough."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu


def test_workspace_limit_enomem_then_success():
    import paper_2206_04995_amd as P

    inst = synth.config1()
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    want = oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
    for limit in (1 << 16, 1 << 20):
        with pytest.raises(P.JpError) as e:
            P.jp_plan_create(*cols, opt=P.make_options(workspace_limit_bytes=limit))
        assert e.value.status == 2 and "workspace limit" in str(e.value)
    with pytest.raises(P.JpError) as e:
        P.jp_batch_create([tuple(cols)] * 3, opt=P.make_options(workspace_limit_bytes=1 << 20))
    assert e.value.status == 2
    with P.Plan(*cols) as p:
        p.execute()
        assert p.count()[0] == want
        peak = p.stats()["peak_bytes"]
    assert peak > 0
    # a limit at the plan's own peak is enough
    with P.Plan(*cols, opt=P.make_options(workspace_limit_bytes=peak)) as p:
        p.execute()
        assert p.count()[0] == want
        assert p.stats()["peak_bytes"] <= peak


def test_calls_out_of_order_estate():
    import paper_2206_04995_amd as P
    from paper_2206_04995_amd import binding as B

    inst = synth.small_random(5, 500, 400)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    h = P.jp_plan_create(*cols)
    try:
        t = ctypes.c_int64()
        assert B.lib.jp_count(h, ctypes.byref(t), None, None, None) == B.JP_ESTATE
        n = ctypes.c_int64()
        out = dev(np.zeros(4, np.int32))
        assert B.lib.jp_materialize(h, 0, 0, 4, out.data_ptr(), out.data_ptr(), ctypes.byref(n), None) == B.JP_ESTATE
        off = np.zeros(P.jp_plan_stats(h)["n_x"] + 1, np.int64)
        assert B.lib.jp_row_info(h, 0, None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None) == B.JP_ESTATE
        tm = B.jp_timings()
        assert B.lib.jp_plan_work(h, ctypes.byref(tm), None) == B.JP_ESTATE
        P.jp_execute(h)
        assert P.jp_count(h)[0] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
    finally:
        P.jp_plan_destroy(h)
    b = P.jp_batch_create([tuple(cols)] * 2)
    try:
        tot = np.zeros(2, np.int64)
        assert B.lib.jp_batch_counts(b, tot.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None) == B.JP_ESTATE
    finally:
        P.jp_batch_destroy(b)
