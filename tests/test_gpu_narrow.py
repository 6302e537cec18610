"""DenseEC count of narrow instances (at most 8192 dense z): a quarter wave per
row up to 512 dense z, a whole wave per row up to 2048 (one word per lane) and
8192 (four words per lane), the window kernel above.  Counts and the lists
written by the window kernel (whose row offsets come from these counts) must
equal the oracle's, at the boundaries of the four widths, for rows longer than
one group of keys, and in a batch that mixes the widths with a pivot split."""
import os

import numpy as np
import pytest

import oracle
import synth
from jp_helpers import assert_parity, dev

pytestmark = pytest.mark.gpu


def _all_dense_bits():
    import paper_2206_04995_amd as P

    return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=-1, dense_kernel=P.JP_DENSE_BITS)


@pytest.mark.parametrize("dom_z,zipf_y,n_s", [(37, 0.0, 1_500), (512, 0.0, 18_432), (513, 0.5, 20_000),
                                               (1_500, 0.0, 100_000), (2_048, 0.3, 80_000), (2_049, 0.0, 100_000),
                                               (4_096, 0.0, 250_000), (8_192, 0.0, 500_000), (8_193, 0.2, 500_000)])
def test_narrow_widths_single_query(dom_z, zipf_y, n_s):
    # every z value occurs, so the dense range is exactly dom_z; a row holds
    # about 100 join keys (several groups of 16 and of 64) and reaches 50-80%
    # of the dense z, from hot and from cold keys
    inst = synth.small_random(900 + dom_z, 10_000, n_s, dom_x=100, dom_y=5_000, dom_z=dom_z, offset=-7, zipf_y=zipf_y)
    print(f"[case] narrow dom_z={dom_z}", flush=True)
    st, _ = assert_parity(inst, _all_dense_bits(), chunk=2_000_000)
    assert st["n_z_dense"] == np.unique(inst.sz).size == dom_z
    assert 0 < st["k_hot"]


def test_narrow_cold_and_hot_keys():
    # uniform y: many keys below the hot threshold (cold scatter) beside hot ones
    inst = synth.small_random(77, 20_000, 60_000, dom_x=500, dom_y=3_000, dom_z=1_000, zipf_y=0.0)
    print("[case] narrow cold", flush=True)
    assert_parity(inst, _all_dense_bits(), chunk=2_000_000)


def test_narrow_batch_mixed_widths_with_pivot(monkeypatch):
    import paper_2206_04995_amd as P

    # the large instance gets an automatic pivot split, so its rows and the
    # narrow instances' rows are counted from row lists
    monkeypatch.setenv("JP_PIVOT_MIN_CELLS", "1e6")
    specs = [(60, 0.0), (512, 1.0), (513, 0.0), (1_800, 1.2), (2_049, 1.0), (100, 1.2), (6_000, 0.0), (20_000, 1.3)]
    insts = [synth.small_random(300 + i, 8_000 + 1_000 * i, 60_000 if dz == 20_000 else max(3_000, 12 * dz),
                                dom_x=150 + 40 * i, dom_y=1_500 + 100 * i, dom_z=dz, offset=-11 * i, zipf_y=zy)
             for i, (dz, zy) in enumerate(specs)]
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    print("[case] narrow batch", flush=True)
    with P.Batch(cols, opt=_all_dense_bits()) as b:
        b.execute()
        got = list(b.counts())
        assert b.stats(len(insts) - 1)["pivot_cover"] > 0
        for i, a in enumerate(insts):
            ox, oz = oracle.join_project(a.rx, a.ry, a.sz, a.sy)
            assert got[i] == ox.size, (i, got[i], ox.size)
            mx, mz = b.materialize(i)
            assert np.array_equal(mx.cpu().numpy(), ox) and np.array_equal(mz.cpu().numpy(), oz)
