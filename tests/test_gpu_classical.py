"""GPU parity of the classical path (paper Sec. 1.1: hash join, then
deduplication of the projected join rows in a device hash set) and of the
strategy choice f1 (Sec. 2.6) between it and the hybrid path: bit-exact sorted
lists, counts and statistics against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import assert_parity, dev

pytestmark = pytest.mark.gpu


def _classical():
    import paper_2206_04995_amd as P

    return P.make_options(strategy=P.JP_STRATEGY_CLASSICAL)


def _hybrid():
    import paper_2206_04995_amd as P

    return P.make_options(strategy=P.JP_STRATEGY_HYBRID)


@pytest.mark.parametrize("seed", range(6))
def test_classical_small_random(seed):
    inst = synth.small_random(700 + seed, 400 + 150 * seed, 300 + 120 * seed, dom_x=50 + 9 * seed,
                              dom_y=35 + 4 * seed, dom_z=45 + 6 * seed, offset=(-2 ** 31 if seed == 2 else -25 * seed),
                              zipf_y=1.0 if seed % 2 else 0.0)
    print(f"[case] classical small seed={seed}", flush=True)
    st, dz = assert_parity(inst, _classical(), chunk=997)
    assert st["strategy"] == 2 and dz.size == 0
    assert st["out_j"] == oracle.out_j(inst.rx, inst.ry, inst.sz, inst.sy)
    keep = np.isin(inst.ry, inst.sy)
    assert st["n_r_kept"] == int(keep.sum())
    assert st["n_x"] == np.unique(inst.rx[keep]).size
    assert st["n_y"] == np.unique(inst.sy).size and st["n_z"] == np.unique(inst.sz).size


def test_classical_edge_cases():
    z = np.zeros(0, np.int32)
    big = 2 ** 31 - 1
    cases = [
        synth.Instance(z, z, z, z, "both-empty"),
        synth.Instance(np.array([1], np.int32), np.array([2], np.int32), z, z, "s-empty"),
        synth.Instance(z, z, np.array([1], np.int32), np.array([2], np.int32), "r-empty"),
        synth.Instance(np.array([5], np.int32), np.array([7], np.int32), np.array([9], np.int32),
                       np.array([7], np.int32), "one-pair"),
        # the pair (INT32_MAX, INT32_MAX) is the dedup set's free marker and takes its own flag
        synth.Instance(np.array([-2 ** 31, big, 0, big], np.int32), np.array([big, big, -2 ** 31, big], np.int32),
                       np.array([big, -2 ** 31, 0, big], np.int32), np.array([big, -2 ** 31, -2 ** 31, big], np.int32),
                       "extremes"),
        synth.Instance(np.full(1000, 3, np.int32), np.full(1000, 4, np.int32), np.full(800, -3, np.int32),
                       np.full(800, 4, np.int32), "all-equal"),
        synth.Instance(np.arange(100, dtype=np.int32), np.arange(100, dtype=np.int32) + 1000,
                       np.arange(100, dtype=np.int32), np.arange(100, dtype=np.int32) + 5000, "no-match"),
    ]
    for inst in cases:
        print(f"[case] classical edge {inst.name}", flush=True)
        st, _ = assert_parity(inst, _classical(), chunk=3)
        assert st["strategy"] == 2


def test_classical_row_info_and_graph():
    import paper_2206_04995_amd as P

    inst = synth.config3(n_vertices=20_000, n_edges=60_000)
    print("[case] classical graph", flush=True)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    with P.Plan(*cols, opt=_classical()) as p:
        p.execute()
        assert p.count() == (ox.size, 0, ox.size)
        xs, offs = p.row_info(P.JP_PART_ALL)
        ux, first = np.unique(ox, return_index=True)
        assert np.array_equal(xs, ux) and np.array_equal(offs[:-1], first) and offs[-1] == ox.size
        _, doffs = p.row_info(P.JP_PART_DENSE)
        assert not doffs.any()
        p.execute()  # a second execute gives the same result
        assert p.count()[0] == ox.size


def test_f1_auto_choice():
    """AUTO takes the classical path for joins far sparser than their inputs and
    the hybrid path otherwise; both exact."""
    import paper_2206_04995_amd as P

    sparse = synth.uniform_paper_default(n_tuples=20_000, n_domain=2_000_000, seed_index=3)  # OUT_J ~ 200
    dense = synth.uniform_paper_default(n_tuples=20_000, n_domain=200, seed_index=4)  # OUT_J ~ 2e6
    print("[case] f1 auto", flush=True)
    st, _ = assert_parity(sparse, None)
    assert st["strategy"] == 2, st
    st, _ = assert_parity(dense, None)
    assert st["strategy"] == 1, st
    st, _ = assert_parity(sparse, _hybrid())
    assert st["strategy"] == 1
    # a fixed threshold asks for the hybrid path's partition
    st, _ = assert_parity(sparse, P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=1))
    assert st["strategy"] == 1


def test_classical_limits_and_refusals():
    import paper_2206_04995_amd as P

    n_r, n_s = 40_000, 30_000  # one shared key: 1.2e9 join rows > 2^30
    cols = [dev(np.arange(n_r, dtype=np.int32)), dev(np.zeros(n_r, np.int32)), dev(np.arange(n_s, dtype=np.int32)),
            dev(np.zeros(n_s, np.int32))]
    print("[case] classical refusals", flush=True)
    with pytest.raises(P.JpError) as ei:
        P.Plan(*cols, opt=_classical())
    assert ei.value.status == 1
    with pytest.raises(P.JpError):
        P.Plan(*cols, opt=P.make_options(strategy=P.JP_STRATEGY_CLASSICAL, flags=P.JP_FLAG_GRAPH))
    small = [dev(np.array([1, 2], np.int32))] * 4
    with pytest.raises(P.JpError):
        P.Batch([tuple(small)], opt=_classical())
    with pytest.raises(P.JpError) as ei:
        P.jp_count_static(*small, opt=_classical())
    assert ei.value.status == 1


def test_classical_timings_and_work():
    import paper_2206_04995_amd as P

    inst = synth.small_random(11, 5000, 4000, dom_x=3000, dom_y=20000, dom_z=3000)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    print("[case] classical timings", flush=True)
    with P.Plan(*cols, opt=P.make_options(strategy=P.JP_STRATEGY_CLASSICAL, flags=P.JP_FLAG_TIMING)) as p:
        with pytest.raises(P.JpError) as ei:
            p.count()
        assert ei.value.status == 4  # JP_ESTATE before execute
        p.execute()
        assert p.count()[0] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
        tm = P.jp_plan_timings(p.h)
        assert tm["map_ms"] > 0 and tm["execute_ms"] >= 0
        assert all(v == 0 for v in P.jp_plan_work(p.h).values())
