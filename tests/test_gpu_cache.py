"""GPU tests of partial result caching (paper Sec. 3): the cached pairs are
exactly the oracle's pairs with a cached z, a plan over the remaining S tuples
gives exactly the rest, and the cached z are the greedy CacheScore choice
under the budget (recomputed here from the oracle's result)."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu


def _zipf_z_instance(seed, n=60_000, dom=3_000):
    rng = np.random.default_rng(seed)
    rx = rng.integers(0, dom, n).astype(np.int32)
    ry = rng.integers(0, dom // 4, n).astype(np.int32)
    sz = synth.zipf_sample(rng, dom, 1.1, n)
    sy = rng.integers(0, dom // 4, n).astype(np.int32)
    return synth.Instance(rx, ry, sz, sy, f"zipf-z-{seed}")


def _expected_choice(inst, n_x, dense_z, budget, c_de=0.05):
    ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    zv, k = np.unique(oz, return_counts=True)
    # OUT_{J,z}: every S tuple adds the number of R tuples with its y
    ys, dr = np.unique(inst.ry, return_counts=True)
    d = np.zeros(inst.n_s, np.int64)
    pos = np.searchsorted(ys, inst.sy)
    ok = (pos < ys.size) & (ys[np.minimum(pos, ys.size - 1)] == inst.sy)
    d[ok] = dr[pos[ok]]
    uz, inv = np.unique(inst.sz, return_inverse=True)
    outj = np.zeros(uz.size, np.int64)
    np.add.at(outj, inv.reshape(-1), d)
    outj_of = dict(zip(uz.tolist(), outj.tolist()))
    dense = set(int(z) for z in dense_z)
    cand = []
    for z, kk in zip(zv.tolist(), k.tolist()):
        space = 2 + min(kk, n_x - kk)
        cost = c_de * n_x if z in dense else float(outj_of[z])
        cand.append((z, cost / space, space))
    cand.sort(key=lambda t: -t[1])  # stable: ties keep ascending z
    pick, used = [], 0
    for z, _, space in cand:
        if used + 4 * space <= budget:
            used += 4 * space
            pick.append(z)
    return sorted(pick), ox, oz


@pytest.mark.parametrize("seed,budget", [(1, 4_000), (2, 40_000), (3, 400_000), (4, 0)])
def test_cache_exact_and_greedy(seed, budget):
    import torch
    import paper_2206_04995_amd as P

    inst = _zipf_z_instance(seed)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    opt = P.make_options(strategy=P.JP_STRATEGY_HYBRID)
    print(f"[case] cache seed={seed} budget={budget}", flush=True)
    with P.Plan(*cols, opt=opt) as p:
        p.execute()
        total = p.count()[0]
        n_x = p.stats()["n_x"]
        dense_z = p.dense_z()
        c = P.jp_cache_build(p.h, budget)
    try:
        info = P.jp_cache_info(c)
        zc = P.jp_cache_z(c)
        want_z, ox, oz = _expected_choice(inst, n_x, dense_z, budget)
        assert zc.tolist() == want_z
        assert 4 * info["words"] <= budget
        # cached pairs: the oracle's pairs with a cached z, in (z, x) order
        m = np.isin(oz, zc)
        order = np.lexsort((ox[m], oz[m]))
        wx, wz = ox[m][order], oz[m][order]
        assert info["pairs"] == wx.size
        gx = torch.empty(max(wx.size, 1), dtype=torch.int32, device="cuda")
        gz = torch.empty(max(wx.size, 1), dtype=torch.int32, device="cuda")
        got_x, got_z, first = [], [], 0
        while first < wx.size:  # ragged chunks
            n = P.jp_cache_materialize(c, first, 777, gx, gz)
            got_x.append(gx[:n].cpu().numpy())
            got_z.append(gz[:n].cpu().numpy())
            first += n
        if wx.size:
            assert np.array_equal(np.concatenate(got_x), wx) and np.array_equal(np.concatenate(got_z), wz)
        # the rest: a plan over S without the cached z
        h = P.jp_plan_create_cached(*cols, c, opt=opt)
        try:
            P.jp_execute(h)
            rest = P.jp_count(h)[0]
            assert rest + info["pairs"] == total
            tx = torch.empty(max(rest, 1), dtype=torch.int32, device="cuda")
            tz = torch.empty(max(rest, 1), dtype=torch.int32, device="cuda")
            n = P.jp_materialize(h, P.JP_PART_ALL, 0, rest, tx, tz)
            assert np.array_equal(tx[:n].cpu().numpy(), ox[~m]) and np.array_equal(tz[:n].cpu().numpy(), oz[~m])
        finally:
            P.jp_plan_destroy(h)
    finally:
        P.jp_cache_destroy(c)


def test_cache_refusals():
    import paper_2206_04995_amd as P

    inst = _zipf_z_instance(9, n=2000, dom=300)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    print("[case] cache refusals", flush=True)
    with P.Plan(*cols, opt=P.make_options(strategy=P.JP_STRATEGY_HYBRID)) as p:
        with pytest.raises(P.JpError) as ei:
            P.jp_cache_build(p.h, 1000)
        assert ei.value.status == 4  # not executed
        p.execute()
        with pytest.raises(P.JpError):
            P.jp_cache_build(p.h, -1)
        c = P.jp_cache_build(p.h, 10_000)
    try:
        with pytest.raises(P.JpError):
            P.jp_plan_create_cached(cols[0][:10], cols[1][:10], cols[2], cols[3], c)  # other tables
        with pytest.raises(P.JpError) as ei:
            P.jp_cache_materialize(c, P.jp_cache_info(c)["pairs"] + 1, 1, cols[0], cols[1])
        assert ei.value.status == 5
    finally:
        P.jp_cache_destroy(c)
    with P.Plan(*cols, opt=P.make_options(strategy=P.JP_STRATEGY_CLASSICAL)) as q:
        q.execute()
        with pytest.raises(P.JpError):
            P.jp_cache_build(q.h, 1000)
