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


def test_graph_replays_batch_of_every_width():
    """A batch whose count pass holds every kernel class, recorded once and
    replayed, each replay checked against the oracle with eager work between
    the replays.  With tau = 4 (z dense iff m_z > 4) the instances cover the
    quarter-wave, whole-wave and four-word narrow DenseEC kernels and the
    window kernel (300, 1500, 4040 and 9474 dense z), and SparseBMM rows of
    every work class (w <= 256, <= 1024, <= 8192 and heavier)."""
    import torch
    import paper_2206_04995_amd as P

    specs = [  # (seed, n_r, n_s, dom_x, dom_y, dom_z, zipf_y)
        (500, 20_000, 30_000, 200, 1_000, 300, 0.0),
        (501, 23_000, 32_000, 250, 1_200, 1_500, 1.0),
        (502, 26_000, 34_000, 300, 1_400, 6_000, 0.0),
        (503, 29_000, 80_000, 350, 1_600, 12_000, 0.0),
        (504, 32_000, 38_000, 400, 1_800, 40_000, 1.2),
        (600, 20_000, 40_000, 200, 2_000, 50_000, 0.0),
        (601, 6_000, 30_000, 600, 3_000, 50_000, 0.0),
    ]
    insts = [synth.small_random(sd, nr, ns, dom_x=dx, dom_y=dy, dom_z=dz, offset=-3 * k, zipf_y=zy)
             for k, (sd, nr, ns, dx, dy, dz, zy) in enumerate(specs)]
    want = [oracle.count(a.rx, a.ry, a.sz, a.sy)[0] for a in insts]
    cols = [tuple(dev(c) for c in (a.rx, a.ry, a.sz, a.sy)) for a in insts]
    opt = P.make_options(tau_mode=P.JP_TAU_FIXED, dense_threshold=4, dense_kernel=P.JP_DENSE_BITS,
                         flags=P.JP_FLAG_GRAPH)
    print("[case] graph batch", flush=True)
    with P.Batch(cols, opt=opt) as b:
        for rep in range(4):
            b.execute()
            got = [int(v) for v in b.counts()]
            assert got == want, (rep, got, want)
            junk = torch.arange(1 << 20, device="cuda", dtype=torch.int32) + rep
            assert int(junk[0].item()) == rep
            torch.cuda.synchronize()
        # the lists stay exact after the replays (sampled instances)
        for i in (0, 2, 5):
            a = insts[i]
            ox, oz = oracle.join_project(a.rx, a.ry, a.sz, a.sy)
            mx, mz = b.materialize(i)
            assert np.array_equal(mx.cpu().numpy(), ox) and np.array_equal(mz.cpu().numpy(), oz)
