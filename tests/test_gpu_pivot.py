"""DenseEC pivot split: rows holding their instance's most shared hot key are
counted outside that key's S row and given its size as a base count.  The
counts must equal the oracle's, and the write pass (which does not use the
split) must produce lists of exactly those lengths."""
import os

import numpy as np
import pytest

import oracle
import synth
from jp_helpers import assert_parity, dev, run_plan

pytestmark = pytest.mark.gpu


@pytest.fixture
def pivot_env():
    old = os.environ.get("JP_PIVOT")
    yield lambda v: os.environ.__setitem__("JP_PIVOT", v)
    if old is None:
        os.environ.pop("JP_PIVOT", None)
    else:
        os.environ["JP_PIVOT"] = old


def _all_dense():
    # the bit path (these small panels are dense enough for the MFMA product otherwise)
    import paper_2206_04995_amd as P

    return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=-1, dense_kernel=P.JP_DENSE_BITS)


@pytest.mark.parametrize("seed", range(6))
def test_forced_pivot_small_random(pivot_env, seed):
    pivot_env("2")
    inst = synth.small_random(100 + seed, 4000 + 700 * seed, 3000 + 500 * seed, dom_x=300, dom_y=60, dom_z=500,
                              offset=-250 * seed, zipf_y=1.0)
    print("[case] forced pivot seed", seed, flush=True)
    st, _ = assert_parity(inst, _all_dense())
    assert st["pivot_cover"] > 0


def test_forced_pivot_many_windows(pivot_env):
    # dense z over several windows, rows longer than 64 keys
    pivot_env("2")
    inst = synth.small_random(7, 60_000, 70_000, dom_x=400, dom_y=300, dom_z=50_000, zipf_y=1.1)
    print("[case] forced pivot, windows", flush=True)
    st, _ = assert_parity(inst, _all_dense(), chunk=3_000_000)
    assert st["pivot_cover"] > 0


def test_forced_pivot_covers_everything(pivot_env):
    # one key joins every z: the space outside its row is empty for that instance
    pivot_env("2")
    z = np.arange(2000, dtype=np.int32)
    sz = np.concatenate([z, z[:300], z[500:900]])
    sy = np.concatenate([np.zeros(2000, np.int32), np.ones(300, np.int32), np.full(400, 2, np.int32)])
    rx = np.array([0, 0, 1, 2, 2, 3, 4, 4, 4], np.int32)
    ry = np.array([0, 1, 1, 2, 0, 2, 0, 1, 2], np.int32)
    st, _ = assert_parity(synth.Instance(rx, ry, sz, sy, "cover"), _all_dense())
    assert st["pivot_cover"] == 2000


def test_pivot_batch_matches_single(pivot_env):
    import paper_2206_04995_amd as P

    pivot_env("2")
    insts = [synth.small_random(200 + i, 3000, 2500, dom_x=200 + 50 * i, dom_y=40, dom_z=400, zipf_y=1.0)
             for i in range(5)]
    cols = [[dev(c) for c in (a.rx, a.ry, a.sz, a.sy)] for a in insts]
    with P.Batch([tuple(c) for c in cols], opt=_all_dense()) as b:
        b.execute()
        got = list(b.counts())
        for i, a in enumerate(insts):
            assert b.stats(i)["pivot_cover"] > 0
            assert got[i] == oracle.count(a.rx, a.ry, a.sz, a.sy)[0]
            ox, oz = oracle.join_project(a.rx, a.ry, a.sz, a.sy)
            mx, mz = b.materialize(i)
            assert np.array_equal(mx.cpu().numpy(), ox) and np.array_equal(mz.cpu().numpy(), oz)


def test_auto_pivot_medium_skewed(pivot_env, monkeypatch):
    """Skewed query that meets the automatic split's conditions (dense z > one
    window, the top key in a quarter of the rows and half of the z; the size
    gate is lowered to this query's cells): counts equal the oracle's and the
    run without the split; sampled rows are exact."""
    import paper_2206_04995_amd as P

    monkeypatch.setenv("JP_PIVOT_MIN_CELLS", "1e6")

    inst = synth.config2(3, n=150_000, dom_xz=20_000, dom_y=2_000)
    print("[case] auto pivot medium skewed", flush=True)
    o_cnt, o_dig = oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    res = {}
    for mode in ("1", "0"):
        pivot_env(mode)
        with P.Plan(*cols) as p:
            p.execute()
            res[mode] = (p.count(), p.stats())
            if mode == "1":
                xs, offs = p.row_info(P.JP_PART_ALL)
                rng = np.random.default_rng(5)
                pick = np.unique(np.concatenate([rng.choice(xs.size, 40, replace=False),
                                                 np.argsort(np.diff(offs))[-5:]]))
                want = oracle.rows(inst.rx, inst.ry, inst.sz, inst.sy, xs[pick])
                for k, i in enumerate(pick):
                    if offs[i + 1] == offs[i]:
                        assert want[k].size == 0
                        continue
                    mx, mz = p.materialize(P.JP_PART_ALL, int(offs[i]), int(offs[i + 1] - offs[i]))
                    assert np.all(mx.cpu().numpy() == xs[i])
                    assert np.array_equal(mz.cpu().numpy(), want[k]), int(xs[i])
    assert res["1"][1]["pivot_cover"] > 0, res["1"][1]
    assert res["0"][1]["pivot_cover"] == 0
    assert res["1"][0] == res["0"][0]
    assert res["1"][0][0] == o_cnt
