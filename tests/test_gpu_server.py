"""GPU tests of the query server: every result in the mix equals the result of
the same query alone (and the oracle), admission respects the HBM budget, and
a query that can never fit fails cleanly."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu


def _alone(cols):
    import paper_2206_04995_amd as P

    with P.Plan(*cols) as p:
        p.execute()
        return p.count()


def test_server_results_equal_alone_and_oracle():
    import paper_2206_04995_amd as P

    insts = [synth.small_random(300 + i, 200 + 50 * i, 150 + 40 * i, dom_x=20 + i, dom_y=15 + i, dom_z=25 + i,
                                offset=-7 * i, zipf_y=1.1 if i % 3 == 0 else 0.0) for i in range(24)]
    insts += [synth.config4_instance(i, hi=30_000) for i in range(8)]
    insts.append(synth.Instance(np.zeros(0, np.int32), np.zeros(0, np.int32), np.array([3], np.int32),
                                np.array([4], np.int32), "empty-r"))
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    alone = [_alone(c) for c in cols]
    print("[case] server mix", flush=True)
    with P.Server(max_batch=8) as srv:
        tickets = [srv.submit(*c) for c in cols]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    for a, inst, r, ref in zip(range(len(insts)), insts, res, alone):
        assert r["status"] == 0
        assert (r["total"], r["dense"], r["sparse"]) == ref
        if inst.n_r * inst.n_s < 5e7:
            assert r["total"] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
        assert r["submit_us"] <= r["admit_us"] <= r["done_us"]
    assert st["completed"] == len(insts) and st["failed"] == 0
    assert st["batches"] >= (len(insts) + 7) // 8
    assert max(r["batch_size"] for r in res) <= 8
    assert 0 < st["p50_us"] <= st["p99_us"]


def test_server_budget_admission_and_rejection():
    import paper_2206_04995_amd as P

    insts = [synth.small_random(400 + i, 60_000, 60_000, dom_x=3000, dom_y=2000, dom_z=3000) for i in range(6)]
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    est = 96 * 120_000 + (1 << 20)
    budget = 2 * est + est // 2  # two queries fit, three do not
    big = synth.small_random(499, 400_000, 400_000, dom_x=3000, dom_y=2000, dom_z=3000)
    big_cols = tuple(dev(c) for c in (big.rx, big.ry, big.sz, big.sy))
    print("[case] server budget", flush=True)
    with P.Server(hbm_budget_bytes=budget) as srv:
        tickets = [srv.submit(*c) for c in cols]
        tb = srv.submit(*big_cols)
        res = [srv.wait(t) for t in tickets]
        rb = srv.wait(tb)
        st = srv.stats()
    for inst, r in zip(insts, res):
        assert r["status"] == 0
        assert r["batch_size"] <= 2
        assert r["total"] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
    assert rb["status"] == 2  # JP_ENOMEM: its estimate exceeds the whole budget
    assert st["failed"] == 1 and st["completed"] == len(insts)
