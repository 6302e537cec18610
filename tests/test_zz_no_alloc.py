"""jp_count_static: the Join-Project count computed inside the library's static
device scratch, with no device allocation.  Checked through the C ABI against
the allocating entry points (jp_plan_create + jp_execute + jp_count) on the same
inputs, on two calls in a row (the second smaller, so stale scratch contents of
the first call would show), and against the oracle's count; oversized inputs and
the flags it does not take are refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu


def _alloc_path(cols, opt=None):
    import paper_2206_04995_amd as P

    h = P.jp_plan_create(*cols, opt=opt)
    try:
        P.jp_execute(h)
        return P.jp_count(h)
    finally:
        P.jp_plan_destroy(h)


def _case(inst):
    import torch
    import paper_2206_04995_amd as P

    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    got = P.jp_count_static(*cols)
    torch.cuda.synchronize()
    want = _alloc_path(cols)
    assert got == want, (got, want)
    assert got[0] == oracle.row_counts(inst.rx, inst.ry, inst.sz, inst.sy)[3]
    assert got[0] == got[1] + got[2]
    return got


def test_static_count_matches_allocating_path_twice():
    # a Zipf(1.2) batched-style instance (dense and sparse parts), then a smaller uniform one
    big = synth.config4_instance(5, lo=300_000, hi=400_000)
    small = synth.small_random(3, 20_000, 15_000, dom_x=2_000, dom_y=300, dom_z=1_500, offset=-700, zipf_y=1.1)
    print(f"[case] static big n_r={big.n_r} n_s={big.n_s}", flush=True)
    a = _case(big)
    print(f"[case] static small n_r={small.n_r} n_s={small.n_s}", flush=True)
    b = _case(small)
    assert a[0] > b[0] > 0


def test_static_count_options_and_edges():
    import paper_2206_04995_amd as P

    inst = synth.small_random(8, 5_000, 6_000, dom_x=400, dom_y=90, dom_z=500, zipf_y=1.0)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    want = oracle.row_counts(inst.rx, inst.ry, inst.sz, inst.sy)[3]
    for opt in (P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=-1),
                P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=P.INT64_MAX),
                P.make_options(dense_kernel=P.JP_DENSE_MFMA)):
        got = P.jp_count_static(*cols, opt=opt)
        assert got == _alloc_path(cols, opt) and got[0] == want
    e = dev(np.zeros(0, np.int32))
    assert P.jp_count_static(e, e, cols[2], cols[3]) == (0, 0, 0)
    assert P.jp_count_static(cols[0], cols[1], e, e) == (0, 0, 0)


def test_static_count_refusals():
    import paper_2206_04995_amd as P
    from paper_2206_04995_amd import binding as B

    one = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    t = ctypes.c_int64()
    half = B.lib.jp_count_static
    assert half(one, one, (1 << 19) + 1, one, one, 1 << 19, None, None, ctypes.byref(t), None, None) == B.JP_EINVAL
    assert "at most" in P.last_error()
    for flag in (P.JP_FLAG_TIMING, P.JP_FLAG_GRAPH):
        o = P.make_options(flags=flag)
        assert half(one, one, 1, one, one, 1, ctypes.byref(o), None, ctypes.byref(t), None, None) == B.JP_EINVAL
