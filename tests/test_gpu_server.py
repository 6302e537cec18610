"""GPU tests of the query server: every result in the mix equals the result of
the same query alone (counts, device digest and the materialised pairs) and
the oracle's; a failing group is split so a failure stays with its query;
admission keeps the live batches within the HBM budget; a query that can
never fit fails cleanly."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu

I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1


def _alone(cols):
    """Counts and the full sorted list of one query on its own plan."""
    import paper_2206_04995_amd as P

    with P.Plan(*cols) as p:
        p.execute()
        cnt = p.count()
        x, z = p.materialize()
        return cnt, x.cpu().numpy(), z.cpu().numpy()


def _mix():
    insts = [synth.small_random(300 + i, 200 + 50 * i, 150 + 40 * i, dom_x=20 + i, dom_y=15 + i, dom_z=25 + i,
                                offset=-7 * i, zipf_y=1.1 if i % 3 == 0 else 0.0) for i in range(24)]
    insts += [synth.config4_instance(i, hi=30_000) for i in range(8)]
    insts.append(synth.Instance(np.zeros(0, np.int32), np.zeros(0, np.int32), np.array([3], np.int32),
                                np.array([4], np.int32), "empty-r"))
    return insts


def test_server_results_equal_alone_and_oracle():
    import paper_2206_04995_amd as P

    insts = _mix()
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    alone = [_alone(c) for c in cols]
    print("[case] server mix (digest, keep)", flush=True)
    with P.Server(max_batch=8, flags=P.JP_SERVER_DIGEST | P.JP_SERVER_KEEP, chunk_pairs=1 << 12) as srv:
        tickets = [srv.submit(*c) for c in cols]
        res = [srv.wait(t) for t in tickets]
        for inst, t, r, (cnt, ax, az) in zip(insts, tickets, res, alone):
            assert r["status"] == 0 and r["kept"] == 1 and r["has_digest"] == 1
            assert (r["total"], r["dense"], r["sparse"]) == cnt
            assert r["digest"] == oracle.digest_pairs(ax, az)  # alone and in the mix: the same pairs
            _, _, _, total, digest = oracle.row_counts(inst.rx, inst.ry, inst.sz, inst.sy)
            assert r["total"] == total and r["digest"] == digest
            mx, mz = srv.materialize(t, r["total"])
            assert np.array_equal(mx.cpu().numpy(), ax) and np.array_equal(mz.cpu().numpy(), az)
            assert r["submit_us"] <= r["admit_us"] <= r["done_us"]
        # parts and chunks of a kept result, then release
        t, r = tickets[-2], res[-2]
        dx, _ = srv.materialize(t, r["dense"], part=P.JP_PART_DENSE)
        sx, _ = srv.materialize(t, r["sparse"], part=P.JP_PART_SPARSE)
        assert dx.numel() + sx.numel() == r["total"]
        half = r["total"] // 2
        a, _ = srv.materialize(t, r["total"], first=0, max_pairs=half)
        b, _ = srv.materialize(t, r["total"], first=half)
        assert np.array_equal(np.concatenate([a.cpu().numpy(), b.cpu().numpy()]), alone[-2][1])
        for t in tickets:
            srv.release(t)
        with pytest.raises(P.JpError):
            srv.materialize(tickets[0], res[0]["total"])
        st = srv.stats()
        assert st["charged_bytes"] == 0  # every kept batch released
    assert st["completed"] == len(insts) and st["failed"] == 0
    assert st["batches"] >= (len(insts) + 7) // 8
    assert max(r["batch_size"] for r in res) <= 8
    assert 0 < st["p50_us"] <= st["p99_us"]
    assert 0 < st["peak_bytes"] <= st["budget_bytes"]


def test_server_counts_only_mode():
    import paper_2206_04995_amd as P

    insts = _mix()[:12]
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    with P.Server(max_batch=5) as srv:
        res = [srv.wait(srv.submit(*c)) for c in cols]
    for inst, r in zip(insts, res):
        assert r["status"] == 0 and r["has_digest"] == 0 and r["kept"] == 0
        assert r["total"] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]


def _full_range(seed):
    """A query whose y and z values span the whole int32 range."""
    rng = np.random.default_rng(seed)
    rx = rng.integers(0, 50, 400).astype(np.int32)
    ry = rng.choice(np.array([I32_MIN, I32_MAX, -5, 0, 7, 12345], np.int64), 400).astype(np.int32)
    sz = rng.choice(np.array([I32_MIN, I32_MAX, 1, -1, 99], np.int64), 300).astype(np.int32)
    sy = rng.choice(np.array([I32_MIN, I32_MAX, 0, 7, 3], np.int64), 300).astype(np.int32)
    return synth.Instance(rx, ry, sz, sy, f"full-range-{seed}")


def test_server_full_range_queries_in_one_mix():
    # two full-range queries cannot share one batch's stacked key space; the
    # server splits the group and both succeed with the results they have alone
    import paper_2206_04995_amd as P

    insts = [_full_range(1), synth.small_random(7, 300, 300), _full_range(2), synth.small_random(8, 200, 250)]
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    alone = [_alone(c) for c in cols]
    print("[case] server full-range mix", flush=True)
    with P.Server(max_batch=8, flags=P.JP_SERVER_DIGEST) as srv:
        tickets = [srv.submit(*c) for c in cols]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    for inst, r, (cnt, ax, az) in zip(insts, res, alone):
        assert r["status"] == 0, r
        assert (r["total"], r["dense"], r["sparse"]) == cnt
        assert r["digest"] == oracle.digest_pairs(ax, az)
        assert r["total"] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
    assert st["splits"] >= 1 and st["failed"] == 0


def test_server_budget_admission_and_rejection():
    import paper_2206_04995_amd as P

    insts = [synth.small_random(400 + i, 60_000, 60_000, dom_x=3000, dom_y=2000, dom_z=3000) for i in range(6)]
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    est = 160 * 120_000 + (2 << 20)  # the server's estimate per query (counts only)
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
    assert 0 < st["peak_bytes"] <= budget and st["budget_bytes"] == budget
    print("[server] peak bytes", st["peak_bytes"], "budget", budget, flush=True)


def test_digest_pairs_matches_oracle():
    import torch
    import paper_2206_04995_amd as P

    rng = np.random.default_rng(3)
    x = rng.integers(I32_MIN, I32_MAX, 100_003, dtype=np.int64, endpoint=True).astype(np.int32)
    z = rng.integers(I32_MIN, I32_MAX, 100_003, dtype=np.int64, endpoint=True).astype(np.int32)
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    dx, dz = dev(x), dev(z)
    P.jp_digest_pairs(dx, dz, 60_000, acc)
    P.jp_digest_pairs(dx[60_000:], dz[60_000:], x.size - 60_000, acc)
    got = int(acc.cpu().numpy().view(np.uint64)[0])
    assert got == oracle.digest_pairs(x, z)
