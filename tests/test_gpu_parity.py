"""GPU parity: the HIP path through the C ABI against the CPU oracle,
bit-exact as sorted (x, z) lists and counts, for the union and for both sides
of the partition by z."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from jp_helpers import assert_parity, dev, run_plan

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BIG = 2 ** 63 - 1


def _opts(kind):
    import paper_2206_04995_amd as P

    if kind == "auto":
        return None
    if kind == "all_dense":  # bit path
        return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=-1, dense_kernel=P.JP_DENSE_BITS)
    if kind == "all_dense_mfma":
        return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=-1, dense_kernel=P.JP_DENSE_MFMA)
    if kind == "all_sparse":
        return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=BIG)
    return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=int(kind))


def test_hand_examples():
    with open(os.path.join(GOLD, "hand_examples.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        r = np.array(case["R"], dtype=np.int64).reshape(-1, 2)
        s = np.array(case["S"], dtype=np.int64).reshape(-1, 2)
        inst = synth.Instance(r[:, 0].astype(np.int32), r[:, 1].astype(np.int32), s[:, 0].astype(np.int32),
                              s[:, 1].astype(np.int32), case["name"])
        for kind in ("auto", "all_dense", "all_dense_mfma", "all_sparse"):
            print(f"[case] hand {case['name']} {kind}", flush=True)
            st, _ = assert_parity(inst, _opts(kind))
            assert st["out_j"] == case["out_j"]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("kind", ["auto", "all_dense", "all_dense_mfma", "all_sparse", "3"])
def test_small_random(seed, kind):
    inst = synth.small_random(seed, 300 + 97 * seed, 250 + 61 * seed, dom_x=40 + 5 * seed, dom_y=30 + 3 * seed,
                              dom_z=50 + 7 * seed, offset=(-2 ** 31 if seed == 3 else -20 * seed),
                              zipf_y=1.0 if seed % 2 else 0.0)
    print(f"[case] small seed={seed} kind={kind}", flush=True)
    assert_parity(inst, _opts(kind))


def test_edge_cases():
    z = np.zeros(0, np.int32)
    cases = [
        synth.Instance(z, z, z, z, "both-empty"),
        synth.Instance(np.array([1], np.int32), np.array([2], np.int32), z, z, "s-empty"),
        synth.Instance(z, z, np.array([1], np.int32), np.array([2], np.int32), "r-empty"),
        synth.Instance(np.array([5], np.int32), np.array([7], np.int32), np.array([9], np.int32),
                       np.array([7], np.int32), "one-pair"),
        synth.Instance(np.full(1000, 3, np.int32), np.full(1000, 4, np.int32), np.full(800, -3, np.int32),
                       np.full(800, 4, np.int32), "all-equal"),
        synth.Instance(np.array([-2 ** 31, 2 ** 31 - 1, 0], np.int32), np.array([2 ** 31 - 1, 2 ** 31 - 1, -2 ** 31], np.int32),
                       np.array([2 ** 31 - 1, -2 ** 31, 0], np.int32), np.array([2 ** 31 - 1, -2 ** 31, -2 ** 31], np.int32),
                       "extremes"),
        synth.Instance(np.arange(100, dtype=np.int32), np.arange(100, dtype=np.int32) + 1000,
                       np.arange(100, dtype=np.int32), np.arange(100, dtype=np.int32) + 5000, "no-match"),
    ]
    for inst in cases:
        for kind in ("auto", "all_dense", "all_dense_mfma", "all_sparse"):
            print(f"[case] edge {inst.name} {kind}", flush=True)
            assert_parity(inst, _opts(kind))


def test_config1_exact():
    inst = synth.config1()
    for kind in ("auto", "all_dense", "all_dense_mfma", "all_sparse"):
        print(f"[case] config1 {kind}", flush=True)
        st, _ = assert_parity(inst, _opts(kind), chunk=700_001)
        assert st["n_x"] == np.unique(inst.rx[np.isin(inst.ry, inst.sy)]).size


def test_heavy_sparse_rows_many_windows():
    # rows with far more than 1024 join rows over a z range wider than one
    # 2^19-bit window: the workgroup/bitmap path of SparseBMM
    rng = np.random.default_rng(1)
    rx = np.repeat(np.arange(40, dtype=np.int32), 150)
    ry = rng.integers(0, 400, rx.size).astype(np.int32)
    sz = rng.integers(-1_500_000, 1_500_000, 400 * 60).astype(np.int32)
    sy = np.repeat(np.arange(400, dtype=np.int32), 60)
    inst = synth.Instance(rx, ry, sz, sy, "heavy")
    print("[case] heavy sparse", flush=True)
    assert_parity(inst, _opts("all_sparse"), chunk=50_000)


@pytest.mark.parametrize("bounds", [(256, 0), (512, 2048), (1024, 1024), (256, 4096)])
def test_sparse_class_bounds(bounds):
    """Every choice of the SparseBMM bounds (one wavefront, one workgroup or z
    windows per row) gives the oracle's result."""
    import paper_2206_04995_amd as P

    light, med = bounds
    inst = synth.config3(n_vertices=30_000, n_edges=300_000)
    rng = np.random.default_rng(2)
    rx = np.concatenate([inst.rx, np.repeat(np.arange(20, dtype=np.int32), 300)])
    ry = np.concatenate([inst.ry, rng.integers(0, 30_000, 6000).astype(np.int32)])
    inst = synth.Instance(rx, ry, inst.sz, inst.sy, "graph+heavy")
    opt = P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=2 ** 63 - 1, sparse_light_max=light,
                         sparse_med_max=med)
    print(f"[case] sparse bounds {bounds}", flush=True)
    assert_parity(inst, opt, chunk=1_000_000)


def test_dense_many_windows_and_long_rows():
    # > 65536 dense z (three DenseEC windows), hot keys, cold keys, and x rows
    # with more than 64 join keys (cursor chunk 0 plus binary-searched chunks)
    rng = np.random.default_rng(2)
    n = 200_000
    rx = rng.integers(0, 300, n).astype(np.int32)
    ry = synth.zipf_sample(rng, 3000, 1.1, n)
    sz = rng.integers(0, 90_000, n).astype(np.int32)
    sy = synth.zipf_sample(rng, 3000, 1.1, n)
    inst = synth.Instance(rx, ry, sz, sy, "dense-windows")
    print("[case] dense windows", flush=True)
    st, _ = assert_parity(inst, _opts("all_dense"), chunk=3_000_000)
    assert st["n_z_dense"] > 65536 and st["k_hot"] > 0


def test_tau_invariance():
    # the partition only decides which kernel produces a pair (Sec. 2.3)
    inst = synth.small_random(77, 20_000, 20_000, dom_x=2000, dom_y=500, dom_z=3000, zipf_y=0.9)
    ref = None
    for kind in ("auto", "all_dense", "all_sparse", "5", "10", "20", "40"):
        print(f"[case] tau {kind}", flush=True)
        cnt, dz, st, lists = run_plan(inst, _opts(kind))
        import paper_2206_04995_amd as P

        allx, allz = lists[P.JP_PART_ALL]
        if ref is None:
            ref = (allx, allz)
            ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
            assert np.array_equal(allx, ox) and np.array_equal(allz, oz)
        else:
            assert np.array_equal(allx, ref[0]) and np.array_equal(allz, ref[1])
        # dense z are exactly those with m_z > tau
        if kind not in ("auto",):
            tau = st["tau"]
            u, c = np.unique(inst.sz, return_counts=True)
            want = u[c > tau] if tau < BIG else u[:0]
            assert np.array_equal(np.sort(dz), want)


def test_stats_match_numpy():
    inst = synth.small_random(5, 30_000, 25_000, dom_x=3000, dom_y=700, dom_z=2000, offset=-1000, zipf_y=1.0)
    cnt, dz, st, _ = run_plan(inst)
    keep = np.isin(inst.ry, inst.sy)
    assert st["n_x"] == np.unique(inst.rx[keep]).size
    assert st["n_y"] == np.unique(inst.sy).size
    assert st["n_z"] == np.unique(inst.sz).size
    assert st["n_r_kept"] == int(keep.sum())
    assert st["out_j"] == oracle.out_j(inst.rx, inst.ry, inst.sz, inst.sy)


def test_row_info_and_chunks():
    import paper_2206_04995_amd as P

    inst = synth.small_random(8, 20_000, 20_000, dom_x=1500, dom_y=400, dom_z=2500, offset=-700)
    ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols) as p:
        p.execute()
        total = p.count()[0]
        xv, off = p.row_info(P.JP_PART_ALL)
        assert np.array_equal(xv, np.unique(inst.rx[np.isin(inst.ry, inst.sy)]))
        assert off[-1] == total
        # rows one at a time
        for i in (0, 1, len(xv) // 2, len(xv) - 1):
            rx_, rz_ = p.materialize(P.JP_PART_ALL, int(off[i]), int(off[i + 1] - off[i]))
            assert np.all(rx_.cpu().numpy() == xv[i])
            assert np.array_equal(rz_.cpu().numpy(), oz[ox == xv[i]])
        # ragged chunks concatenate to the whole list
        rng = np.random.default_rng(0)
        cuts = np.sort(rng.choice(np.arange(1, total), size=7, replace=False))
        bounds = [0] + cuts.tolist() + [total]
        xs, zs = [], []
        for a, b in zip(bounds[:-1], bounds[1:]):
            cx, cz = p.materialize(P.JP_PART_ALL, a, b - a)
            xs.append(cx.cpu().numpy())
            zs.append(cz.cpu().numpy())
        assert np.array_equal(np.concatenate(xs), ox) and np.array_equal(np.concatenate(zs), oz)
        # first == count writes nothing; first > count is an error
        cx, _ = p.materialize(P.JP_PART_ALL, total, 10)
        assert cx.numel() == 0
        with pytest.raises(P.JpError) as ei:
            p.materialize(P.JP_PART_ALL, total + 1, 10)
        assert ei.value.status == 5


def test_batch_matches_single_plans():
    import paper_2206_04995_amd as P

    insts = [synth.small_random(200 + i, 500 + 300 * i, 400 + 250 * i, dom_x=30 + 10 * i, dom_y=20 + 5 * i,
                                dom_z=40 + 9 * i, offset=-50 * i, zipf_y=1.2 if i % 2 else 0.0) for i in range(9)]
    insts.insert(3, synth.Instance(np.zeros(0, np.int32), np.zeros(0, np.int32), np.array([1], np.int32),
                                   np.array([1], np.int32), "empty-r"))
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    print("[case] batch", flush=True)
    with P.Batch(cols) as b:
        b.execute()
        counts = b.counts()
        for i, inst in enumerate(insts):
            ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
            assert counts[i] == ox.size
            if ox.size:
                bx, bz = b.materialize(i)
                assert np.array_equal(bx.cpu().numpy(), ox) and np.array_equal(bz.cpu().numpy(), oz)


def test_graph_selfjoin_small():
    inst = synth.config3(n_vertices=50_000, n_edges=500_000)
    print("[case] graph small", flush=True)
    assert_parity(inst, None, chunk=1_000_000)
    inst2 = synth.config3(n_vertices=50_000, n_edges=500_000, two_hop=True)
    print("[case] graph 2-hop small", flush=True)
    assert_parity(inst2, None, chunk=1_000_000)


def test_skewed_small_exact():
    inst = synth.config2(n=40_000, dom_xz=4_000, dom_y=400)
    for kind in ("auto", "all_dense", "all_sparse"):
        print(f"[case] skewed small {kind}", flush=True)
        assert_parity(inst, _opts(kind), chunk=5_000_000)


def _ids_opts(direct, kind="auto"):
    import paper_2206_04995_amd as P

    base = _opts(kind)
    o = base if base is not None else P.make_options()
    if direct:
        o.flags |= P.JP_FLAG_DIRECT_IDS
    return o


@pytest.mark.parametrize("seed", range(6))
def test_direct_and_sorted_ids_agree(seed):
    """Radix-sorted ids (default) and, with JP_FLAG_DIRECT_IDS, the direct-range
    mapping of dense value ranges (key histogram, scans, scatter): both must equal
    the oracle."""
    inst = synth.small_random(400 + seed, 2000 + 500 * seed, 1500 + 400 * seed, dom_x=60 + 30 * seed,
                              dom_y=40 + 10 * seed, dom_z=80 + 20 * seed, offset=-1000 * seed,
                              zipf_y=1.1 if seed % 2 else 0.0)
    for direct in (False, True):
        for kind in ("auto", "all_dense", "all_sparse"):
            print(f"[case] ids seed={seed} direct={direct} {kind}", flush=True)
            st, _ = assert_parity(inst, _ids_opts(direct, kind))
            assert st["map_direct"] == (3 if direct else 0), st


def test_sparse_value_range_takes_sorted_ids():
    """Values spread over the int32 range are too sparse for the direct mapping,
    which then falls back to sorted ids."""
    rng = np.random.default_rng(7)
    vals = rng.integers(-2 ** 31, 2 ** 31 - 1, 64, dtype=np.int64).astype(np.int32)
    rx = vals[rng.integers(0, 64, 3000)]
    ry = vals[rng.integers(0, 16, 3000)]
    sz = vals[rng.integers(0, 64, 2500)]
    sy = vals[rng.integers(0, 16, 2500)]
    inst = synth.Instance(rx, ry, sz, sy, "wide")
    print("[case] ids wide range", flush=True)
    st, _ = assert_parity(inst, _ids_opts(True))
    assert st["map_direct"] == 0, st


@pytest.mark.parametrize("direct", [False, True])
def test_batch_mapping_paths(direct):
    """A batch of dense-range instances with an empty one and one without a
    match, through both mapping paths; every instance must equal the oracle."""
    import paper_2206_04995_amd as P

    insts = [synth.small_random(600 + i, 800 + 200 * i, 700 + 150 * i, dom_x=50 + 10 * i, dom_y=25 + 5 * i,
                                dom_z=45 + 9 * i, offset=-300 * i, zipf_y=1.2 if i % 2 else 0.0) for i in range(6)]
    insts.insert(2, synth.Instance(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                                   np.zeros(0, np.int32), "empty"))
    insts.insert(4, synth.Instance(np.array([7, 7, 9], np.int32), np.array([1, 2, 3], np.int32),
                                   np.array([5], np.int32), np.array([4], np.int32), "no-match"))
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    opt = P.make_options(flags=P.JP_FLAG_DIRECT_IDS if direct else 0)
    print(f"[case] batch ids direct={direct}", flush=True)
    with P.Batch(cols, opt=opt) as b:
        b.execute()
        counts = b.counts()
        assert b.stats(0)["map_direct"] == (3 if direct else 0)
        for i, inst in enumerate(insts):
            ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
            assert counts[i] == ox.size
            st = b.stats(i)
            assert st["out_j"] == oracle.out_j(inst.rx, inst.ry, inst.sz, inst.sy)
            if ox.size:
                bx, bz = b.materialize(i)
                assert np.array_equal(bx.cpu().numpy(), ox) and np.array_equal(bz.cpu().numpy(), oz)


@pytest.mark.parametrize("direct", [False, True])
def test_batch_without_z_sort_pass(direct):
    """Batches whose z keys need no sort pass (every instance holds one S.z
    value; a batch with a single S tuple), so the key pass makes the keys from
    the instances' columns; both mapping paths, every instance equal to the oracle."""
    import paper_2206_04995_amd as P

    batches = [
        [synth.small_random(900 + i, 300 + 50 * i, 200 + 40 * i, dom_x=30, dom_y=15, dom_z=1, offset=17 * i)
         for i in range(5)],
        [synth.Instance(np.array([1, 2, 2], np.int32), np.array([3, 3, 4], np.int32), np.array([7], np.int32),
                        np.array([3], np.int32), "one-s"),
         synth.Instance(np.array([5], np.int32), np.array([3], np.int32), np.zeros(0, np.int32),
                        np.zeros(0, np.int32), "empty-s")],
    ]
    opt = P.make_options(flags=P.JP_FLAG_DIRECT_IDS if direct else 0)
    for k, insts in enumerate(batches):
        cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
        print(f"[case] batch without z sort pass {k} direct={direct}", flush=True)
        with P.Batch(cols, opt=opt) as b:
            b.execute()
            counts = b.counts()
            for i, inst in enumerate(insts):
                ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
                assert counts[i] == ox.size
                if ox.size:
                    bx, bz = b.materialize(i)
                    assert np.array_equal(bx.cpu().numpy(), ox) and np.array_equal(bz.cpu().numpy(), oz)
