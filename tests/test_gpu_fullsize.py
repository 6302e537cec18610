"""Parity at the full workload sizes the benchmark times, through the same
entry points and launch configuration (one plan or one batch, execute, count,
then chunked materialisation), against goldens the oracle wrote
(tests/golden/make_fullsize.py):

* skewed query, 1e7 tuples per side: sampled rows (random and the heaviest)
  equal the oracle's rows; the union equals dense + sparse; the count is the
  same with the pivot split off, with the bit path forced and with another
  hot-key cap (the paths compute it differently);
* graph self-join, 2e7 edges: count and order-independent digest of all pairs,
  streamed in 64M-pair chunks, equal the oracle's (stored by
  tests/golden/make_fullsize.py);
* dense uniform query, 1e7 tuples over a 1e4 domain: the INT8-MFMA count
  equals the bit path's and |X| * |Z|, and sampled rows equal the oracle's;
* skewed query: total count and OUT_J, and every 1000th distinct x of R plus
  the 100 heaviest rows in count and digest;
* the 4096-instance batch: per-instance counts and OUT_J, and digests of the
  instances with at most 5e7 pairs.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fullsize.json")


def _sample_rows(p, inst, xs, offs, n_random, n_heavy, seed):
    import paper_2206_04995_amd as P

    rng = np.random.default_rng(seed)
    lens = np.diff(offs)
    pick = np.unique(np.concatenate([rng.choice(xs.size, n_random, replace=False), np.argsort(lens)[-n_heavy:]]))
    want = oracle.rows(inst.rx, inst.ry, inst.sz, inst.sy, xs[pick])
    for k, i in enumerate(pick):
        assert want[k].size == lens[i], (int(xs[i]), want[k].size, int(lens[i]))
        if lens[i] == 0:
            continue
        mx, mz = p.materialize(P.JP_PART_ALL, int(offs[i]), int(lens[i]))
        assert np.all(mx.cpu().numpy() == xs[i])
        assert np.array_equal(mz.cpu().numpy(), want[k]), int(xs[i])


def test_skewed_1e7_sampled_rows_and_paths(monkeypatch):
    import paper_2206_04995_amd as P

    print("[case] skewed 1e7", flush=True)
    inst = synth.config2()
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols) as p:
        p.execute()
        total, dense, sparse = p.count()
        st = p.stats()
        assert total == dense + sparse and st["out_j"] == oracle.out_j(inst.rx, inst.ry, inst.sz, inst.sy)
        xs, offs = p.row_info(P.JP_PART_ALL)
        assert offs[-1] == total and xs.size == st["n_x"]
        _sample_rows(p, inst, xs, offs, 24, 6, 11)
    variants = [({"JP_PIVOT": "0"}, None),
                ({}, P.make_options(dense_kernel=P.JP_DENSE_BITS, k_hot_max=512)),
                ({}, P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=12))]
    for env, opt in variants:
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        with P.Plan(*cols, opt=opt) as q:
            q.execute()
            got = q.count()
        for k in env:
            monkeypatch.delenv(k)
        print("[case] skewed variant", env, got, flush=True)
        assert got[0] == total


def test_graph_2e7_count_and_digest():
    import paper_2206_04995_amd as P

    with open(GOLD) as f:
        want = json.load(f)["graph_2e6_2e7"]
    print("[case] graph 2e7", flush=True)
    g = synth.config3()
    cols = [dev(c) for c in (g.rx, g.ry, g.sz, g.sy)]
    with P.Plan(*cols) as p:
        p.execute()
        total, dense, sparse = p.count()
        assert total == want["pairs"] == dense + sparse
        assert p.stats()["out_j"] == want["out_j"]
        chunk = 1 << 26
        digest = 0
        first = 0
        prev = None
        while first < total:
            n = min(chunk, total - first)
            mx, mz = p.materialize(P.JP_PART_ALL, first, n)
            x, z = mx.cpu().numpy(), mz.cpu().numpy()
            key = (x.astype(np.int64) << 32) | (z.astype(np.int64) & 0xFFFFFFFF)
            assert np.all(np.diff(key) > 0) and (prev is None or key[0] > prev)  # sorted, distinct, across chunks
            prev = key[-1]
            digest = (digest + oracle.digest_pairs(x, z)) % (1 << 64)
            first += n
        assert str(digest) == want["digest"]


def test_dense_1e7_mfma_equals_bits_and_rows():
    import paper_2206_04995_amd as P

    print("[case] dense 1e7", flush=True)
    inst = synth.uniform_paper_default(n_tuples=10_000_000, n_domain=10_000)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols) as p:
        p.execute()
        total = p.count()
        st = p.stats()
        assert st["dense_mfma"] == 1
        assert total[0] == st["n_x"] * st["n_z"]  # every pair: each x reaches every z through ~1000 keys
        xs, offs = p.row_info(P.JP_PART_ALL)
        _sample_rows(p, inst, xs, offs, 12, 2, 5)
    with P.Plan(*cols, opt=P.make_options(dense_kernel=P.JP_DENSE_BITS)) as q:
        q.execute()
        assert q.stats()["dense_mfma"] == 0
        assert q.count() == total


SKEWED_GOLD = os.path.join(os.path.dirname(__file__), "golden", "skewed_1e7.json")
BATCHED_GOLD = os.path.join(os.path.dirname(__file__), "golden", "batched_4096.json")


def _device_digest(ox, oz, n):
    import torch
    import paper_2206_04995_amd as P

    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    if n:
        P.jp_digest_pairs(ox, oz, n, acc)
    return int(acc.cpu().numpy().view(np.uint64)[0])


def test_skewed_1e7_total_and_golden_rows():
    """The skewed query's total count and OUT_J equal the oracle's, and every
    1000th distinct x of R plus the 100 heaviest rows equal the oracle's rows in
    count and digest (stored by tests/golden/make_fullsize.py)."""
    import paper_2206_04995_amd as P

    with open(SKEWED_GOLD) as f:
        want = json.load(f)
    print("[case] skewed 1e7 golden", flush=True)
    inst = synth.config2()
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols) as p:
        p.execute()
        total, dense, sparse = p.count()
        assert total == want["pairs"] == dense + sparse
        assert p.stats()["out_j"] == want["out_j"]
        xs, offs = p.row_info(P.JP_PART_ALL)
        for key in ("every_1000th_x", "heaviest_100"):
            rows = want[key]
            for x, cnt, dig in zip(rows["x"], rows["count"], rows["digest"]):
                i = int(np.searchsorted(xs, x))
                if i == xs.size or xs[i] != x:  # no R tuple of x survives the semi-join
                    assert cnt == 0, x
                    continue
                lo, hi = int(offs[i]), int(offs[i + 1])
                assert hi - lo == cnt, (x, hi - lo, cnt)
                mx, mz = p.materialize(P.JP_PART_ALL, lo, hi - lo)
                assert _device_digest(mx, mz, hi - lo) == int(dig), x
        print(f"[case] skewed 1e7: {total} pairs, {len(want['every_1000th_x']['x'])} + 100 rows", flush=True)


def test_batched_4096_per_instance_counts_and_digests():
    """The 4096-instance batch in one batched plan: every instance's pair count
    and OUT_J equal the oracle's; the 3521 instances with at most 5e7 pairs
    (1.4e10 pairs together) are materialised in chunks and their digests equal
    the oracle's."""
    import torch
    import paper_2206_04995_amd as P

    with open(BATCHED_GOLD) as f:
        want = json.load(f)["instances"]
    print("[case] batched 4096 golden", flush=True)
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(8) as ex:
        insts = list(ex.map(synth.config4_instance, range(4096)))
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    for a, w in zip(insts, want):
        assert (a.n_r, a.n_s) == (w["n_r"], w["n_s"])
    with P.Batch(cols) as b:
        b.execute()
        counts = b.counts()
        assert np.array_equal(counts, np.array([w["pairs"] for w in want], dtype=np.int64))
        cap = 1 << 26
        ox = torch.empty(cap, dtype=torch.int32, device="cuda")
        oz = torch.empty(cap, dtype=torch.int32, device="cuda")
        n_dig = 0
        for i, w in enumerate(want):
            assert b.stats(i)["out_j"] == w["out_j"], i
            if w["pairs"] > 50_000_000 or w["pairs"] == 0:
                continue
            acc = torch.zeros(1, dtype=torch.int64, device="cuda")
            first = 0
            while first < w["pairs"]:
                n = P.jp_batch_materialize(b.h, i, P.JP_PART_ALL, first, cap, ox, oz)
                P.jp_digest_pairs(ox, oz, n, acc)
                first += n
            assert int(acc.cpu().numpy().view(np.uint64)[0]) == int(w["digest"]), i
            n_dig += 1
        print(f"[case] batched: {n_dig} instance digests", flush=True)
