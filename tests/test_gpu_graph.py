"""JP_FLAG_GRAPH: the count pass recorded into a HIP graph on the second
execute and replayed afterwards must give the oracle's result on every call,
with unrelated eager work (another plan, torch ops, synchronisations) run
between the replays."""
import numpy as np
import pytest

import oracle
import synth
from jp_helpers import dev

pytestmark = pytest.mark.gpu


def _all_pairs(p, total):
    import paper_2206_04995_amd as P

    ox, oz = p.materialize(P.JP_PART_ALL)
    assert ox.numel() == total
    return ox.cpu().numpy(), oz.cpu().numpy()


@pytest.mark.parametrize("kind", ["mixed", "heavy_sparse"])
def test_graph_replays_match_oracle(kind):
    import torch
    import paper_2206_04995_amd as P

    if kind == "mixed":
        inst = synth.config2(0, n=200_000, dom_xz=20_000, dom_y=2_000)
        opt = P.make_options(flags=P.JP_FLAG_GRAPH)
    else:
        inst = synth.small_random(7, 60_000, 60_000, 300, 40, 50_000, zipf_y=1.0)
        opt = P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=2 ** 63 - 1, flags=P.JP_FLAG_GRAPH)
    print("[case]", kind, inst.rx.size, inst.sz.size, flush=True)
    ox, oz = oracle.join_project(inst.rx, inst.ry, inst.sz, inst.sy)
    other = synth.small_random(11, 5_000, 5_000, 400, 300, 400)
    o_cnt = oracle.count(other.rx, other.ry, other.sz, other.sy)[0]

    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    ocols = [dev(c) for c in (other.rx, other.ry, other.sz, other.sy)]
    with P.Plan(*cols, opt=opt) as p:
        for rep in range(5):
            p.execute()
            cnt = p.count()
            assert cnt[0] == ox.size, (rep, cnt, ox.size)
            assert cnt[1] + cnt[2] == cnt[0]
            ax, az = _all_pairs(p, cnt[0])
            assert np.array_equal(ax, ox) and np.array_equal(az, oz), rep
            # eager work between replays: another plan on the same stream, torch kernels, a sync
            with P.Plan(*ocols) as q:
                q.execute()
                assert q.count()[0] == o_cnt
            junk = torch.arange(1 << 20, device="cuda", dtype=torch.int32) * 3
            assert int(junk[-1].item()) == 3 * ((1 << 20) - 1)
            torch.cuda.synchronize()


def test_graph_and_eager_plans_agree_on_same_input():
    import paper_2206_04995_amd as P

    inst = synth.small_random(3, 30_000, 30_000, 2_000, 500, 2_000, zipf_y=1.0)
    cols = [dev(c) for c in (inst.rx, inst.ry, inst.sz, inst.sy)]
    with P.Plan(*cols) as e, P.Plan(*cols, opt=P.make_options(flags=P.JP_FLAG_GRAPH)) as g:
        e.execute()
        ref = e.count()
        ex = _all_pairs(e, ref[0])
        for _ in range(3):
            g.execute()
            assert g.count() == ref
            gx = _all_pairs(g, ref[0])
            assert np.array_equal(gx[0], ex[0]) and np.array_equal(gx[1], ex[1])
