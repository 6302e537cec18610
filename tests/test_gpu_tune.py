"""Autotuner of the dense/sparse threshold: every candidate threshold must give
the same counts (the tuner checks this itself), the stored cost ratio must
reproduce the chosen threshold for a plan of the same query, and the result
stays exact."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import assert_parity, dev

pytestmark = pytest.mark.gpu


def test_tune_stores_ratio_and_plan_uses_it():
    import paper_2206_04995_amd as P

    P.jp_tune_clear()
    inst = synth.config2(1, n=120_000, dom_xz=12_000, dom_y=1_200)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols) as p:
        tau_model = p.stats()["tau"]
    r = P.jp_tune(*cols)
    print("[tune]", r, flush=True)
    assert r["model_tau"] == tau_model
    assert r["candidates"] >= 3
    assert r["best_ms"] <= r["model_ms"]
    with P.Plan(*cols) as p:
        st = p.stats()
        want = r["tau"] if r["tau"] != 2 ** 63 - 1 else st["tau"]
        assert st["tau"] == want or (r["tau"] < 0 and st["tau"] == 0)
        assert st["dense_mfma"] == (1 if r["dense_kernel"] == P.JP_DENSE_MFMA and st["n_z_dense"] > 0 else 0)
    assert r["k_hot_max"] in (0, 64, 128, 256, 512, 1024) and r["window_group"] in (0, 1, 2, 4, 8)
    st, _ = assert_parity(inst, None, chunk=4_000_000)
    P.jp_tune_clear()
    with P.Plan(*cols) as p:
        assert p.stats()["tau"] == tau_model


def test_tune_on_graph_and_uniform():
    import paper_2206_04995_amd as P

    for inst in (synth.config3(n_vertices=20_000, n_edges=200_000),
                 synth.uniform_paper_default(n_tuples=200_000, n_domain=3_000, seed_index=2)):
        P.jp_tune_clear()
        cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
        r = P.jp_tune(*cols)
        print("[tune]", inst.name, r, flush=True)
        assert r["sparse_light_max"] in (0, 256, 512) and r["sparse_med_max"] in (0, 2048, 4096)
        assert r["mfma_tile"] in (0, 1, 2)
        with P.Plan(*cols) as p:
            p.execute()
            assert p.count()[0] == oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
    P.jp_tune_clear()


def test_tune_choices_reach_plans_and_stay_exact():
    """A second tune of the same query replaces the stored choices; plans with
    every option automatic follow them and stay exact, including batches."""
    import paper_2206_04995_amd as P

    P.jp_tune_clear()
    inst = synth.uniform_paper_default(n_tuples=300_000, n_domain=2_500, seed_index=6)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    r1 = P.jp_tune(*cols)
    r2 = P.jp_tune(*cols)
    print("[tune]", r1, r2, flush=True)
    assert r2["model_tau"] == r1["model_tau"]  # the model's tau ignores stored choices
    o = oracle.count(inst.rx, inst.ry, inst.sz, inst.sy)[0]
    with P.Plan(*cols) as p:
        p.execute()
        assert p.count()[0] == o
    with P.Batch([tuple(cols), tuple(cols)]) as b:
        b.execute()
        assert list(b.counts()) == [o, o]
    P.jp_tune_clear()
