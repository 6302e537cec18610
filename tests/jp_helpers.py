"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int32))).to("cuda")


_SHOWN = []


def hip_runtimes():
    return sorted({l.split()[-1] for l in open("/proc/self/maps") if "amdhip64" in l})


def run_plan(inst, opt=None, chunk=None):
    """(counts, dense z values, stats, full sorted ALL/DENSE/SPARSE lists) via the C ABI."""
    import torch
    import paper_2206_04995_amd as P

    if not _SHOWN:
        _SHOWN.append(1)
        print("[hip runtimes]", hip_runtimes(), flush=True)

    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols, opt=opt) as p:
        p.execute()
        cnt = p.count()
        dz = p.dense_z()
        st = p.stats()
        lists = {}
        for part in (P.JP_PART_ALL, P.JP_PART_DENSE, P.JP_PART_SPARSE):
            total = cnt[part]
            xs, zs = [], []
            step = chunk or max(total, 1)
            first = 0
            while first < total:
                ox, oz = p.materialize(part, first, min(step, total - first))
                xs.append(ox.cpu().numpy())
                zs.append(oz.cpu().numpy())
                first += step
            lists[part] = (np.concatenate(xs) if xs else np.zeros(0, np.int32),
                           np.concatenate(zs) if zs else np.zeros(0, np.int32))
        torch.cuda.synchronize()
    return cnt, dz, st, lists


def assert_parity(inst, opt=None, chunk=None):
    """Bit-exact comparison of every part with the oracle; returns the plan stats."""
    import paper_2206_04995_amd as P

    cnt, dz, st, lists = run_plan(inst, opt, chunk)
    ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    ax, az = lists[P.JP_PART_ALL]
    assert cnt[0] == ox.size, (cnt, ox.size)
    assert np.array_equal(ax, ox) and np.array_equal(az, oz)
    (dx, dzz), (sx, szz) = oracle.split_by_z(ox, oz, dz)
    assert cnt[1] == dx.size and cnt[2] == sx.size
    assert np.array_equal(lists[P.JP_PART_DENSE][0], dx) and np.array_equal(lists[P.JP_PART_DENSE][1], dzz)
    assert np.array_equal(lists[P.JP_PART_SPARSE][0], sx) and np.array_equal(lists[P.JP_PART_SPARSE][1], szz)
    return st, dz
