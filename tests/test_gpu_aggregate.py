"""GPU parity of the Join-Aggregate (paper Sec. 4.1): groups (x, z) with the
number of join rows and the sum of R.v * S.u, against the oracle's hash-map
aggregation, element by element, through chunked materialisation."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu


def _run(rx, ry, rv, sz, sy, su, chunk=None):
    import paper_2206_04995_amd as P

    with P.Aggregate(dev(rx), dev(ry), dev(rv), dev(sz), dev(sy), dev(su)) as a:
        with pytest.raises(P.JpError) as ei:
            a.count()
        assert ei.value.status == 4  # JP_ESTATE before execute
        a.execute()
        groups, out_j = a.count()
        parts = []
        step = chunk or max(groups, 1)
        first = 0
        while first < groups:
            parts.append([t.cpu().numpy() for t in a.materialize(first, min(step, groups - first))])
            first += step
        if groups:
            assert a.materialize(groups, 5)[0].numel() == 0
        with pytest.raises(P.JpError) as ei:
            a.materialize(groups + 1, 5)
        assert ei.value.status == 5
    cols = [np.concatenate([p[k] for p in parts]) if parts else np.zeros(0) for k in range(4)]
    return groups, out_j, cols


def _check(inst, rv, su, chunk=None):
    groups, out_j, (x, z, c, s) = _run(inst.rx, inst.ry, rv, inst.sz, inst.sy, su, chunk)
    ox, oz, oc, osum = oracle.aggregate(inst.rx, inst.ry, rv, inst.sz, inst.sy, su)
    assert groups == ox.size and out_j == oracle.out_j(inst.rx, inst.ry, inst.sz, inst.sy)
    assert np.array_equal(x, ox) and np.array_equal(z, oz)
    assert np.array_equal(c, oc) and np.array_equal(s, osum)


@pytest.mark.parametrize("seed", range(6))
def test_aggregate_small_random(seed):
    rng = np.random.default_rng(900 + seed)
    inst = synth.small_random(900 + seed, 800 + 300 * seed, 700 + 250 * seed, dom_x=60 + 10 * seed,
                              dom_y=30 + 5 * seed, dom_z=70 + 9 * seed, offset=(-2 ** 31 if seed == 4 else -30 * seed),
                              zipf_y=1.1 if seed % 2 else 0.0)
    rv = rng.integers(-2 ** 31, 2 ** 31 - 1, inst.n_r, dtype=np.int64).astype(np.int32)
    su = rng.integers(-2 ** 31, 2 ** 31 - 1, inst.n_s, dtype=np.int64).astype(np.int32)
    print(f"[case] aggregate small seed={seed}", flush=True)
    _check(inst, rv, su, chunk=331)


def test_aggregate_heavy_rows_many_windows():
    """Rows with thousands of join rows over a z range of several windows."""
    rng = np.random.default_rng(17)
    n_r, n_s = 3000, 200_000
    rx = rng.integers(0, 40, n_r).astype(np.int32)
    ry = rng.integers(0, 300, n_r).astype(np.int32)
    sz = rng.integers(-30_000, 30_000, n_s).astype(np.int32)
    sy = rng.integers(0, 300, n_s).astype(np.int32)
    rv = rng.integers(-50, 50, n_r).astype(np.int32)
    su = rng.integers(-50, 50, n_s).astype(np.int32)
    print("[case] aggregate heavy", flush=True)
    _check(synth.Instance(rx, ry, sz, sy), rv, su, chunk=100_000)


def test_aggregate_edges_and_unit_values():
    z = np.zeros(0, np.int32)
    print("[case] aggregate edges", flush=True)
    _check(synth.Instance(z, z, z, z), z, z)
    _check(synth.Instance(np.array([1], np.int32), np.array([2], np.int32), np.array([3], np.int32),
                          np.array([4], np.int32)), np.array([5], np.int32), np.array([6], np.int32))
    inst = synth.small_random(3, 5000, 4000, dom_x=100, dom_y=50, dom_z=80)
    ones_r, ones_s = np.ones(inst.n_r, np.int32), np.ones(inst.n_s, np.int32)
    groups, out_j, (x, zz, c, s) = _run(inst.rx, inst.ry, ones_r, inst.sz, inst.sy, ones_s)
    ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    assert np.array_equal(x, ox) and np.array_equal(zz, oz)  # the groups are the Join-Project result
    assert int(c.sum()) == out_j and np.array_equal(c, s)
