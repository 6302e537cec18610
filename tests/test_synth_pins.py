"""Pins that tie the seeded generators (and the oracle's counts on them) to the
sizes the paper prints for its synthetic tables (Sec. 5, sensitivity analysis
with synthetic data sets, defaults |R| = |S| = 1e6 and n = 1e4), and checks the
shape of every workload generator."""
import math

import numpy as np
import pytest

import synth


def _out_j_bincount(inst, n):
    dr = np.bincount(inst.ry, minlength=n).astype(np.int64)
    ds = np.bincount(inst.sy, minlength=n).astype(np.int64)
    return int((dr * ds).sum())


@pytest.mark.slow
def test_paper_uniform_default(oracle_mod):
    # Sec. 5 (2): uniform tables give OUT_J about 1e8 and OUT_P about 6e7.
    inst = synth.uniform_paper_default()
    outj = _out_j_bincount(inst, 10_000)
    assert abs(outj - 1e8) / 1e8 < 0.01
    c, _ = oracle_mod.count(inst.rx, inst.ry, inst.sz, inst.sy)
    assert abs(c - 6e7) / 6e7 < 0.06
    # closed form for i.i.d. uniform draws: P((x,y) in R) = q = 1 - (1 - 1/n^2)^N,
    # P((x,z) in OUT) = 1 - (1 - q^2)^n
    n, N = 10_000, 1_000_000
    q = 1 - (1 - 1 / n ** 2) ** N
    expect = n * n * (1 - (1 - q * q) ** n)
    assert abs(c - expect) / expect < 0.005


def test_paper_vary_n_out_j():
    # Sec. 5 (1): with |R| = |S| = 1e6 fixed, OUT_J falls from 1e9 to 1e6 as n
    # grows from 1e3 to 1e6; for uniform data OUT_J = N^2 / n in expectation.
    for n, want in ((1_000, 1e9), (1_000_000, 1e6)):
        inst = synth.uniform_paper_default(n_domain=n)
        outj = _out_j_bincount(inst, n)
        assert abs(outj - want) / want < 0.01


@pytest.mark.slow
def test_paper_zipf_xz(oracle_mod):
    # Sec. 5 (2): Zipf(1) on R.x and S.z keeps OUT_J near 1e8 and brings OUT_P
    # down to about 1.4e7 (i.i.d. draws with repeats).
    inst = synth.zipf_xz_paper(s=1.0)
    outj = _out_j_bincount(inst, 10_000)
    assert abs(outj - 1e8) / 1e8 < 0.02
    c, _ = oracle_mod.count(inst.rx, inst.ry, inst.sz, inst.sy)
    assert abs(c - 1.4e7) / 1.4e7 < 0.05


def test_config1_shape():
    inst = synth.config1()
    for a, b, da, db in ((inst.rx, inst.ry, 10_000, 5_000), (inst.sz, inst.sy, 10_000, 5_000)):
        assert a.shape == (100_000,) and a.dtype == np.int32
        assert a.min() >= 0 and a.max() < da and b.min() >= 0 and b.max() < db
        key = a.astype(np.int64) * 2 ** 32 + b
        assert np.unique(key).size == 100_000
    # about 2e6 join rows (20 tuples per y per side)
    outj = _out_j_bincount(inst, 5_000)
    assert 1.9e6 < outj < 2.1e6


def test_zipf_sampler_frequencies():
    rng = np.random.default_rng(0)
    v = synth.zipf_sample(rng, 1000, 1.0, 2_000_000)
    h = np.bincount(v, minlength=1000)
    w = 1.0 / np.arange(1, 1001)
    p = w / w.sum()
    # rank-0 and rank-9 frequencies within 2% of (k+1)^-1 / H
    for k in (0, 9):
        assert abs(h[k] / v.size - p[k]) / p[k] < 0.02


def test_distinct_skewed_small():
    inst = synth.config2(n=200_000, dom_xz=20_000, dom_y=2_000)
    key = inst.rx.astype(np.int64) * 2 ** 32 + inst.ry
    assert np.unique(key).size == 200_000
    h = np.bincount(inst.ry, minlength=2000)
    assert h[0] > h[1] > h[10] > h[1000]


def test_graph_shape_small():
    inst = synth.config3(n_vertices=20_000, n_edges=200_000)
    assert inst.rx.size == 200_000
    assert np.array_equal(inst.rx, inst.sz) and np.array_equal(inst.ry, inst.sy)
    key = inst.rx.astype(np.int64) * 20_000 + inst.ry
    assert np.unique(key).size == 200_000
    deg = np.bincount(inst.rx, minlength=20_000)
    assert abs(deg.mean() - 10) < 1e-9
    assert deg.max() > 100  # heavy tail


def test_config4_instance_shape():
    for i in (0, 1, 2, 3):
        inst = synth.config4_instance(i)
        assert 1_000 <= inst.n_r <= 1_000_000 and 1_000 <= inst.n_s <= 1_000_000
        dr = math.ceil(0.1 * inst.n_r)
        ds = math.ceil(0.1 * inst.n_s)
        assert inst.rx.max() < dr and inst.ry.max() < dr
        assert inst.sz.max() < ds and inst.sy.max() < ds
    # reproducible alone
    a = synth.config4_instance(3)
    b = synth.config4_instance(3)
    assert np.array_equal(a.ry, b.ry)


def test_trace_shape():
    tr = synth.config5_trace(n_queries=2000, rate_per_s=100.0)
    t = np.array([a for a, _, _ in tr])
    assert np.all(np.diff(t) >= 0)
    kinds = np.array([k for _, k, _ in tr])
    assert 0 < kinds.sum() < 100
