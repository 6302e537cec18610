"""Writes the full-size goldens, calling only the oracle and the seeded
generators.  Run from the repository root:

    python tests/golden/make_fullsize.py [graph] [skewed] [batched] [--threads N]

* fullsize.json, key graph_2e6_2e7: count, digest and OUT_J of the graph
  self-join (2e6 vertices, 2e7 edges, Pareto(2.1) out-degrees; R = S = edges),
  from the hash-join oracle.
* skewed_1e7.json: the skewed query (1e7 distinct tuples per side, x and z
  uniform in [0, 1e6), y Zipf(1.0) over [0, 1e5)): total count and digest,
  OUT_J, and the count and digest of every 1000th distinct x of R (ascending)
  and of the 100 heaviest rows, from the oracle's row-by-row matrix form.
* batched_4096.json: for each of the 4096 batched instances (tuples
  log-uniform in [1e3, 1e6] per side, domains 10% of the tuples, y uniform or
  Zipf(1.2)), its tuple counts, pair count, digest and OUT_J, from the same
  row-by-row form.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _write(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1)


def graph(threads):
    g = synth.config3()
    count, digest = oracle.count(g.rx, g.ry, g.sz, g.sy, threads=threads)
    out = {"graph_2e6_2e7": {"generator": "synth.config3()", "pairs": int(count), "digest": str(int(digest)),
                             "out_j": int(oracle.out_j(g.rx, g.ry, g.sz, g.sy))}}
    _write("fullsize.json", out)
    print(out, flush=True)


def skewed(threads):
    inst = synth.config2()
    t0 = time.time()
    xs, cnt, dig, total, digest = oracle.row_counts(inst.rx, inst.ry, inst.sz, inst.sy, threads=threads)
    print(f"skewed: {total} pairs over {xs.size} rows in {time.time() - t0:.0f} s", flush=True)
    every = np.arange(0, xs.size, 1000)
    heavy = np.argsort(-cnt, kind="stable")[:100]

    def rows(idx):
        return {"x": xs[idx].tolist(), "count": cnt[idx].tolist(), "digest": [str(int(d)) for d in dig[idx]]}

    out = {"generator": "synth.config2()", "pairs": int(total), "digest": str(int(digest)),
           "out_j": int(oracle.out_j(inst.rx, inst.ry, inst.sz, inst.sy)), "n_x_of_r": int(xs.size),
           "every_1000th_x": rows(every), "heaviest_100": rows(heavy)}
    _write("skewed_1e7.json", out)


def batched(threads):
    out = {"generator": "synth.config4_instance(i) for i in range(4096)", "instances": []}
    t0 = time.time()
    for i in range(4096):
        a = synth.config4_instance(i)
        _, _, _, total, digest = oracle.row_counts(a.rx, a.ry, a.sz, a.sy, threads=threads)
        out["instances"].append({"n_r": a.n_r, "n_s": a.n_s, "pairs": int(total), "digest": str(int(digest)),
                                 "out_j": int(oracle.out_j(a.rx, a.ry, a.sz, a.sy))})
        if i % 256 == 255:
            print(f"batched: {i + 1} instances in {time.time() - t0:.0f} s", flush=True)
    _write("batched_4096.json", out)


def main():
    args = sys.argv[1:]
    threads = None
    if "--threads" in args:
        k = args.index("--threads")
        threads = int(args[k + 1])
        del args[k:k + 2]
    oracle.build(force=False)
    for name in args or ["graph", "skewed", "batched"]:
        {"graph": graph, "skewed": skewed, "batched": batched}[name](threads)


if __name__ == "__main__":
    main()
