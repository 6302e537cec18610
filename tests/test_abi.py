"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "jp.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(jp_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    import paper_2206_04995_amd as P

    assert sorted(P.EXPORTS) == _declared()


def test_library_exports_every_symbol():
    import paper_2206_04995_amd as P

    for name in _declared():
        assert hasattr(P.lib, name), name


def test_invalid_arguments_rejected_before_device_work():
    import paper_2206_04995_amd as P
    from paper_2206_04995_amd import binding as B

    lib = P.lib
    h = ctypes.c_void_p()
    one = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    # null output handle
    assert lib.jp_plan_create(None, None, 0, None, None, 0, None, None, None) == B.JP_EINVAL
    # negative count
    assert lib.jp_plan_create(None, None, -1, None, None, 0, None, None, ctypes.byref(h)) == B.JP_EINVAL
    assert "negative" in P.last_error()
    # null column with n > 0
    assert lib.jp_plan_create(None, None, 5, None, None, 0, None, None, ctypes.byref(h)) == B.JP_EINVAL
    # more than 2^31 - 1 tuples
    assert lib.jp_plan_create(one, one, 2 ** 31, one, one, 1, None, None, ctypes.byref(h)) == B.JP_EINVAL
    # bad options
    for kw in ({"tau_mode": 7}, {"dense_kernel": 9}, {"k_hot_max": 5000}, {"workspace_limit_bytes": -1},
               {"window_group": 65}, {"window_group": -1}, {"strategy": 3}, {"strategy": -1},
                   {"sparse_light_max": 2000}, {"sparse_med_max": 100}, {"sparse_med_max": 9000}, {"mfma_tile": 3},
                   {"reserved": 1},
               {"tau_mode": 1, "dense_threshold": -2}):
        o = P.make_options()
        for k, v in kw.items():
            setattr(o, k, v)
        assert lib.jp_plan_create(one, one, 1, one, one, 1, ctypes.byref(o), None, ctypes.byref(h)) == B.JP_EINVAL
    o = P.make_options()
    o.flags = 8  # not a defined JP_FLAG_* bit
    assert lib.jp_plan_create(one, one, 1, one, one, 1, ctypes.byref(o), None, ctypes.byref(h)) == B.JP_EINVAL
    # null plan everywhere
    n = ctypes.c_int64()
    assert lib.jp_execute(None, None) == B.JP_EINVAL
    assert lib.jp_count(None, None, None, None, None) == B.JP_EINVAL
    assert lib.jp_materialize(None, 0, 0, 0, None, None, ctypes.byref(n), None) == B.JP_EINVAL
    assert lib.jp_plan_stats(None, None) == B.JP_EINVAL
    lib.jp_plan_destroy(None)
    # batches
    assert lib.jp_batch_create(None, 0, None, None, ctypes.byref(h)) == B.JP_EINVAL
    arr = (B.jp_instance * 1)()
    arr[0].n_r = -3
    assert lib.jp_batch_create(arr, 1, None, None, ctypes.byref(h)) == B.JP_EINVAL
    assert lib.jp_batch_execute(None, None) == B.JP_EINVAL
    lib.jp_batch_destroy(None)
    # the tuner
    r = B.jp_tune_result()
    assert lib.jp_tune(one, one, 1, one, one, 1, None, None, None) == B.JP_EINVAL
    assert lib.jp_tune(one, one, -1, one, one, 1, None, None, ctypes.byref(r)) == B.JP_EINVAL
    assert lib.jp_tune(None, None, 3, one, one, 1, None, None, ctypes.byref(r)) == B.JP_EINVAL
    o = P.make_options(window_group=99)
    assert lib.jp_tune(one, one, 1, one, one, 1, ctypes.byref(o), None, ctypes.byref(r)) == B.JP_EINVAL
    assert lib.jp_tune_clear() == B.JP_OK


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2206_04995_amd as P

    t = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(TypeError):
        P.jp_plan_create(t, t, t, t)
