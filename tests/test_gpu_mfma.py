"""DenseEC count on the INT8 matrix cores: the 0/1 product thresholded at > 0
must give the oracle's counts, and the bit-path write pass lists of exactly
those lengths.  Shapes are ragged against the 128 x 128 x 64 tiles."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import assert_parity, dev

pytestmark = pytest.mark.gpu


def _opt(kernel, tau=-1):
    import paper_2206_04995_amd as P

    if tau is None:
        return P.make_options(dense_kernel=kernel)
    return P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=tau, dense_kernel=kernel)


@pytest.mark.parametrize("case", range(6))
def test_mfma_forced_ragged(case):
    import paper_2206_04995_amd as P

    dims = [(130, 70, 129), (1, 1, 1), (300, 64, 128), (257, 200, 500), (77, 1000, 63), (1000, 30, 2000)][case]
    nx, ny, nz = dims
    n = max(200, min(60_000, nx * ny // 3))
    inst = synth.small_random(300 + case, n, max(150, min(60_000, ny * nz // 3)), dom_x=nx, dom_y=ny, dom_z=nz,
                              offset=(case - 3) * 1_000_000)
    print("[case] mfma forced", dims, flush=True)
    st, _ = assert_parity(inst, _opt(P.JP_DENSE_MFMA))
    assert st["dense_mfma"] == 1


def test_mfma_mixed_partition():
    # dense and sparse z both present: the MFMA counts only the dense part
    import paper_2206_04995_amd as P

    inst = synth.small_random(41, 40_000, 40_000, dom_x=900, dom_y=400, dom_z=3000, zipf_y=0.8)
    print("[case] mfma mixed", flush=True)
    for tau in (5, 12, 30):
        st, _ = assert_parity(inst, _opt(P.JP_DENSE_MFMA, tau))
        assert st["dense_mfma"] == (1 if st["n_z_dense"] > 0 else 0)


def test_mfma_auto_on_dense_uniform():
    """Uniform keys over small domains (the paper's dense regime): the automatic
    choice takes the product, and it agrees with the bit path and the oracle."""
    import paper_2206_04995_amd as P

    inst = synth.uniform_paper_default(n_tuples=400_000, n_domain=2_000, seed_index=4)
    print("[case] mfma auto dense uniform", flush=True)
    st, _ = assert_parity(inst, None)
    assert st["dense_mfma"] == 1, st
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols, opt=_opt(P.JP_DENSE_BITS, None)) as p:
        p.execute()
        assert p.stats()["dense_mfma"] == 0
        bits = p.count()
    with P.Plan(*cols) as p:
        p.execute()
        assert p.count() == bits


def test_mfma_not_used_for_batches_or_sparse_panels():
    import paper_2206_04995_amd as P

    inst = synth.config2(0, n=60_000, dom_xz=6_000, dom_y=3_000)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols, opt=_opt(P.JP_DENSE_AUTO, -1)) as p:
        assert p.stats()["dense_mfma"] == 0  # skewed: the panel is sparse
    with P.Batch([tuple(cols), tuple(cols)], opt=_opt(P.JP_DENSE_MFMA)) as b:
        b.execute()
        assert b.stats(0)["dense_mfma"] == 0
        o = oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
        assert list(b.counts()) == [o, o]


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("case", [0, 3, 5])
def test_mfma_tiles(tile, case):
    """The 128 x 256 and 256 x 128 tiles against the oracle (ragged shapes, early
    checks on dense panels)."""
    import paper_2206_04995_amd as P

    dims = [(130, 70, 129), (1, 1, 1), (300, 64, 128), (257, 200, 500), (77, 1000, 63), (1000, 30, 2000)][case]
    nx, ny, nz = dims
    n = max(200, min(60_000, nx * ny // 3))
    inst = synth.small_random(300 + case, n, max(150, min(60_000, ny * nz // 3)), dom_x=nx, dom_y=ny, dom_z=nz,
                              offset=(case - 3) * 1_000_000)
    print("[case] mfma tile", tile, dims, flush=True)
    opt = P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=-1, dense_kernel=P.JP_DENSE_MFMA, mfma_tile=tile)
    st, _ = assert_parity(inst, opt)
    assert st["dense_mfma"] == 1


def test_mfma_early_check_issued_work():
    """A dense panel: the early check stops tiles before the last key, so fewer
    ops are issued than the full product holds, with an exact count."""
    import paper_2206_04995_amd as P

    inst = synth.uniform_paper_default(n_tuples=400_000, n_domain=2_000, seed_index=4)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    print("[case] mfma early check", flush=True)
    with P.Plan(*cols, opt=_opt(P.JP_DENSE_MFMA)) as p:
        p.execute()
        assert p.count()[0] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
        wk = P.jp_plan_work(p.h)
        assert 0 < wk["dense_mfma_issued_ops"] < wk["dense_mfma_ops"], wk
