"""Pins for the CPU oracle: checks against things other than the oracle itself.

* hand-worked cases from the definition (tests/golden/hand_examples.json);
* the definition written as nested loops (brute force) on random tiny inputs;
* the matrix form of the paper (Sec. 1.1): (x, z) is in the result iff
  (R S)[x, z] > 0, with numpy's integer matrix product as the library step;
* closed forms and invariants (full matrices, one shared key, disjoint keys,
  transposition, self-join symmetry, repeats, value relabelling);
* OUT_J = sum over y of d_R(y) d_S(y), counted with numpy bincount;
* the SplitMix64 published test vector for the digest finaliser.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _cols(case):
    r = np.array(case["R"], dtype=np.int64).reshape(-1, 2)
    s = np.array(case["S"], dtype=np.int64).reshape(-1, 2)
    return (r[:, 0].astype(np.int32), r[:, 1].astype(np.int32), s[:, 0].astype(np.int32),
            s[:, 1].astype(np.int32))


@pytest.mark.parametrize("case", _load("hand_examples.json")["cases"], ids=lambda c: c["name"])
def test_hand_examples(oracle_mod, case):
    rx, ry, sz, sy = _cols(case)
    expect = [tuple(p) for p in case["expect"]]
    assert oracle_mod.brute_force(rx, ry, sz, sy) == expect
    ox, oz = oracle_mod.join_project(rx, ry, sz, sy)
    assert list(zip(ox.tolist(), oz.tolist())) == expect
    c, d = oracle_mod.count(rx, ry, sz, sy)
    assert c == len(expect)
    assert oracle_mod.out_j(rx, ry, sz, sy) == case["out_j"]
    assert d == oracle_mod.digest_pairs(ox, oz)
    _check_row_counts(oracle_mod, rx, ry, sz, sy, expect)


def _check_row_counts(oracle_mod, rx, ry, sz, sy, expect, threads=None):
    """row_counts against an explicit pair list: one row per distinct x of R
    (ascending), its count and digest, and the totals."""
    xs, cnt, dig, total, digest = oracle_mod.row_counts(rx, ry, sz, sy, threads=threads)
    assert xs.tolist() == sorted(set(np.asarray(rx).tolist()))
    by_x = {}
    for x, z in expect:
        by_x.setdefault(x, []).append(z)
    for x, c, d in zip(xs.tolist(), cnt.tolist(), dig.tolist()):
        zs = by_x.get(x, [])
        assert c == len(zs)
        assert d == oracle_mod.digest_pairs(np.full(len(zs), x, np.int32), np.array(zs, np.int32))
    assert total == len(expect)
    ex = np.array([p[0] for p in expect], np.int32)
    ez = np.array([p[1] for p in expect], np.int32)
    assert digest == oracle_mod.digest_pairs(ex, ez)


def test_splitmix64_vector(oracle_mod):
    g = _load("splitmix64.json")
    gamma = int(g["gamma"], 16)
    state = 0
    for want in g["outputs"]:
        state = (state + gamma) & (2 ** 64 - 1)
        hi, lo = state >> 32, state & 0xFFFFFFFF
        x = np.array([hi ^ 0x80000000], dtype=np.uint32).view(np.int32)
        z = np.array([lo ^ 0x80000000], dtype=np.uint32).view(np.int32)
        assert oracle_mod.digest_pairs(x, z) == int(want, 16)


small_ints = st.integers(min_value=-3, max_value=6)
extreme = st.sampled_from([-(2 ** 31), 2 ** 31 - 1, -1, 0, 1])
vals = st.one_of(small_ints, small_ints, extreme)
table = st.lists(st.tuples(vals, vals), min_size=0, max_size=60)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(r=table, s=table, self_join=st.booleans())
def test_oracle_equals_brute_force(oracle_mod, r, s, self_join):
    if self_join:
        s = list(r)
    rx = np.array([a for a, _ in r], dtype=np.int32)
    ry = np.array([b for _, b in r], dtype=np.int32)
    sz = np.array([a for a, _ in s], dtype=np.int32)
    sy = np.array([b for _, b in s], dtype=np.int32)
    expect = oracle_mod.brute_force(rx, ry, sz, sy)
    ox, oz = oracle_mod.join_project(rx, ry, sz, sy, threads=3)
    assert list(zip(ox.tolist(), oz.tolist())) == expect
    c, d = oracle_mod.count(rx, ry, sz, sy, threads=2)
    assert c == len(expect)
    _check_row_counts(oracle_mod, rx, ry, sz, sy, expect, threads=3)
    bag = sum(1 for _, y in r for _, y2 in s if y == y2)
    assert oracle_mod.out_j(rx, ry, sz, sy) == bag


def _matrix_form(rx, ry, sz, sy):
    """Sec. 1.1 matrix form: 0/1 matrices over the distinct values, C = R S,
    result = nonzero entries of C (numpy integer matmul as the library step)."""
    xs = np.unique(rx)
    ys = np.unique(np.concatenate([ry, sy]))
    zs = np.unique(sz)
    R = np.zeros((xs.size, ys.size), dtype=np.int64)
    S = np.zeros((ys.size, zs.size), dtype=np.int64)
    R[np.searchsorted(xs, rx), np.searchsorted(ys, ry)] = 1
    S[np.searchsorted(ys, sy), np.searchsorted(zs, sz)] = 1
    C = R @ S
    i, j = np.nonzero(C > 0)
    return xs[i], zs[j]


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_matrix_form(oracle_mod, seed):
    inst = synth.small_random(seed, 400 + 37 * seed, 350 + 11 * seed, dom_x=60, dom_y=40, dom_z=70,
                              offset=-30 + 7 * seed, zipf_y=0.8 if seed % 2 else 0.0)
    mx, mz = _matrix_form(inst.rx, inst.ry, inst.sz, inst.sy)
    ox, oz = oracle_mod.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    assert np.array_equal(ox, mx) and np.array_equal(oz, mz)
    xs, cnt, _, total, digest = oracle_mod.row_counts(inst.rx, inst.ry, inst.sz, inst.sy, threads=4)
    assert total == mx.size and digest == oracle_mod.digest_pairs(mx, mz)
    u, c = np.unique(mx, return_counts=True)
    assert np.array_equal(cnt[np.isin(xs, u)], c) and not cnt[~np.isin(xs, u)].any()


def test_closed_forms(oracle_mod):
    rng = np.random.default_rng(5)
    # full matrices: every (x, z) pair
    X = np.arange(-5, 12, dtype=np.int32)
    Y = np.arange(100, 109, dtype=np.int32)
    Z = np.arange(1000, 1013, dtype=np.int32)
    rx, ry = [a.ravel() for a in np.meshgrid(X, Y, indexing="ij")]
    sz, sy = [a.ravel() for a in np.meshgrid(Z, Y, indexing="ij")]
    c, _ = oracle_mod.count(rx, ry, sz, sy)
    assert c == X.size * Z.size
    assert oracle_mod.out_j(rx, ry, sz, sy) == X.size * Y.size * Z.size
    xs, cnt, _, total, _ = oracle_mod.row_counts(rx, ry, sz, sy)
    assert np.array_equal(xs, X) and (cnt == Z.size).all() and total == X.size * Z.size
    # one shared key: |X_y| * |Z_y|
    rx = rng.integers(0, 50, 300).astype(np.int32)
    ry = np.where(rng.random(300) < 0.3, 7, rng.integers(10, 20, 300)).astype(np.int32)
    sz = rng.integers(0, 80, 200).astype(np.int32)
    sy = np.where(rng.random(200) < 0.4, 7, rng.integers(30, 40, 200)).astype(np.int32)
    c, _ = oracle_mod.count(rx, ry, sz, sy)
    assert c == np.unique(rx[ry == 7]).size * np.unique(sz[sy == 7]).size
    assert oracle_mod.row_counts(rx, ry, sz, sy)[3] == c
    # disjoint key domains: empty
    c, _ = oracle_mod.count(rx, ry + 1000, sz, sy)
    assert c == 0
    xs, cnt, dig, total, digest = oracle_mod.row_counts(rx, ry + 1000, sz, sy)
    assert total == 0 and digest == 0 and not cnt.any() and not dig.any()
    # empty sides
    e = np.zeros(0, np.int32)
    assert oracle_mod.row_counts(e, e, sz, sy)[0].size == 0
    xs, cnt, _, total, _ = oracle_mod.row_counts(rx, ry, e, e)
    assert total == 0 and xs.size == np.unique(rx).size


@pytest.mark.parametrize("seed", range(3))
def test_invariants(oracle_mod, seed):
    inst = synth.small_random(100 + seed, 3000, 2500, dom_x=300, dom_y=200, dom_z=250, offset=-100)
    rx, ry, sz, sy = inst.rx, inst.ry, inst.sz, inst.sy
    ox, oz = oracle_mod.join_project(rx, ry, sz, sy)
    # transposition: JP(S, R) is the transpose of JP(R, S)
    tx, tz = oracle_mod.join_project(sz, sy, rx, ry)
    a = sorted(zip(ox.tolist(), oz.tolist()))
    b = sorted(zip(tz.tolist(), tx.tolist()))
    assert a == b
    # repeats do not change the set
    dx, dz = oracle_mod.join_project(np.concatenate([rx, rx[::3]]), np.concatenate([ry, ry[::3]]),
                                     np.concatenate([sz[::2], sz]), np.concatenate([sy[::2], sy]))
    assert np.array_equal(dx, ox) and np.array_equal(dz, oz)
    # relabelling values by a bijection permutes the output identically
    perm = np.random.default_rng(seed).permutation(1000).astype(np.int32) * 7 - 3000

    def f(v):
        return perm[v.astype(np.int64) + 100]

    px, pz = oracle_mod.join_project(f(rx), ry * 3 + 1, f(sz), sy * 3 + 1)
    assert sorted(zip(px.tolist(), pz.tolist())) == sorted(zip(f(ox).tolist(), f(oz).tolist()))
    # witness: every output pair has a shared y; bound OUT_P <= min(OUT_J, |X||Z|)
    ys_of_x = {}
    for x, y in zip(rx.tolist(), ry.tolist()):
        ys_of_x.setdefault(x, set()).add(y)
    ys_of_z = {}
    for z, y in zip(sz.tolist(), sy.tolist()):
        ys_of_z.setdefault(z, set()).add(y)
    for x, z in zip(ox[::17].tolist(), oz[::17].tolist()):
        assert ys_of_x[x] & ys_of_z[z]
    outj = oracle_mod.out_j(rx, ry, sz, sy)
    assert ox.size <= min(outj, np.unique(rx).size * np.unique(sz).size)
    # strictly increasing (x, z): no pair twice
    key = (ox.astype(np.int64) << 32) + oz.astype(np.int64)
    assert np.all(np.diff(key) > 0)
    # self join: symmetric and contains (x, x) for every x with a y
    sx, sz2 = oracle_mod.join_project(rx, ry, rx, ry)
    st_ = set(zip(sx.tolist(), sz2.tolist()))
    assert all((z, x) in st_ for x, z in st_)
    assert all((x, x) in st_ for x in np.unique(rx).tolist())


def test_out_j_is_sum_of_degree_products(oracle_mod):
    inst = synth.small_random(7, 20000, 15000, dom_x=500, dom_y=800, dom_z=400, zipf_y=1.1)
    dr = np.bincount(inst.ry, minlength=800).astype(np.int64)
    ds = np.bincount(inst.sy, minlength=800).astype(np.int64)
    assert oracle_mod.out_j(inst.rx, inst.ry, inst.sz, inst.sy) == int((dr * ds).sum())


def test_rows_match_list(oracle_mod):
    inst = synth.small_random(9, 5000, 4000, dom_x=200, dom_y=100, dom_z=300, offset=-50)
    ox, oz = oracle_mod.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    xs = np.array([-50, -49, 10, 149, 999], dtype=np.int32)
    rows = oracle_mod.rows(inst.rx, inst.ry, inst.sz, inst.sy, xs)
    for x, row in zip(xs.tolist(), rows):
        assert np.array_equal(row, oz[ox == x])


def test_split_by_z_is_a_partition(oracle_mod):
    inst = synth.small_random(11, 3000, 3000, dom_x=100, dom_y=60, dom_z=90)
    ox, oz = oracle_mod.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    dense = np.unique(inst.sz)[::3]
    (dx, dz), (sx, sz_) = oracle_mod.split_by_z(ox, oz, dense)
    assert np.isin(dz, dense).all() and not np.isin(sz_, dense).any()
    assert dx.size + sx.size == ox.size
    a = set(zip(dx.tolist(), dz.tolist()))
    b = set(zip(sx.tolist(), sz_.tolist()))
    assert not (a & b)
    assert a | b == set(zip(ox.tolist(), oz.tolist()))


# ------------------------------------------------------- composite keys


def _composite_case(seed, n_r, n_s, kx, ky, kz, dom, offset=0):
    rng = np.random.default_rng(seed)

    def cols(k, n):
        return [(rng.integers(0, dom, n) + offset).astype(np.int32) for _ in range(k)]

    return cols(kx, n_r), cols(ky, n_r), cols(kz, n_s), cols(ky, n_s)


@pytest.mark.parametrize("seed", range(12))
def test_composite_oracle_equals_brute_force(oracle_mod, seed):
    """The rank-encoded composite oracle equals nested loops over tuples."""
    kx, ky, kz = 1 + seed % 3, 1 + (seed // 3) % 3, 1 + (seed // 2) % 2
    r_x, r_y, s_z, s_y = _composite_case(seed, 40 + seed, 35 + 2 * seed, kx, ky, kz, 3 + seed % 3,
                                         offset=-(seed % 2) * 2 ** 31)
    gx, gz = oracle_mod.join_project_composite(r_x, r_y, s_z, s_y)
    got = [(tuple(int(c[i]) for c in gx), tuple(int(c[i]) for c in gz)) for i in range(gx[0].size)]
    assert got == oracle_mod.brute_force_composite(r_x, r_y, s_z, s_y)


def test_composite_single_columns_reduce_to_plain_oracle(oracle_mod):
    """One column per key kind is the plain Join-Project."""
    r_x, r_y, s_z, s_y = _composite_case(99, 3000, 2500, 1, 1, 1, 60, offset=-30)
    gx, gz = oracle_mod.join_project_composite(r_x, r_y, s_z, s_y)
    ox, oz = oracle_mod.join_project(r_x[0], r_y[0], s_z[0], s_y[0])
    assert np.array_equal(gx[0], ox) and np.array_equal(gz[0], oz)


def test_composite_join_key_is_the_whole_tuple(oracle_mod):
    """Tuples that agree on one join column but not the other do not join."""
    r_x = [np.array([1, 2], np.int32)]
    r_y = [np.array([5, 5], np.int32), np.array([0, 1], np.int32)]
    s_z = [np.array([7, 8], np.int32), np.array([-1, -2], np.int32)]
    s_y = [np.array([5, 5], np.int32), np.array([1, 2], np.int32)]
    gx, gz = oracle_mod.join_project_composite(r_x, r_y, s_z, s_y)
    assert gx[0].tolist() == [2] and gz[0].tolist() == [7] and gz[1].tolist() == [-1]


# ------------------------------------------------------- Join-Aggregate


@pytest.mark.parametrize("seed", range(10))
def test_aggregate_oracle_equals_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(50 + seed)
    n_r, n_s, dom = 30 + 7 * seed, 25 + 5 * seed, 4 + seed % 4
    off = -(seed % 3) * 2 ** 30
    rx, ry = (rng.integers(0, dom, n_r) + off).astype(np.int32), rng.integers(0, dom, n_r).astype(np.int32)
    sz, sy = (rng.integers(0, dom, n_s) - off).astype(np.int32), rng.integers(0, dom, n_s).astype(np.int32)
    rv = rng.integers(-1000, 1000, n_r).astype(np.int32)
    su = rng.integers(-1000, 1000, n_s).astype(np.int32)
    got = oracle_mod.aggregate(rx, ry, rv, sz, sy, su)
    want = oracle_mod.brute_force_aggregate(rx, ry, rv, sz, sy, su)
    assert list(zip(*(a.tolist() for a in got))) == want


def test_aggregate_invariants(oracle_mod):
    """Groups are the Join-Project result; counts add up to OUT_J; with unit
    values the sum is the count; one shared key gives sum = (sum of v)(sum of u)
    for distinct x and z."""
    inst = synth.small_random(77, 4000, 3000, dom_x=200, dom_y=90, dom_z=150)
    ones_r, ones_s = np.ones(inst.n_r, np.int32), np.ones(inst.n_s, np.int32)
    x, z, c, s = oracle_mod.aggregate(inst.rx, inst.ry, ones_r, inst.sz, inst.sy, ones_s)
    ox, oz = oracle_mod.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    assert np.array_equal(x, ox) and np.array_equal(z, oz)
    assert int(c.sum()) == oracle_mod.out_j(inst.rx, inst.ry, inst.sz, inst.sy)
    assert np.array_equal(c, s)
    rv = np.arange(1, 51, dtype=np.int32)
    su = np.arange(-20, 0, dtype=np.int32)
    x, z, c, s = oracle_mod.aggregate(np.zeros(50, np.int32), np.full(50, 9, np.int32), rv,
                                      np.zeros(20, np.int32), np.full(20, 9, np.int32), su)
    assert x.tolist() == [0] and z.tolist() == [0] and c.tolist() == [1000]
    assert s.tolist() == [int(rv.sum()) * int(su.sum())]
