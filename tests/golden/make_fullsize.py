"""Writes fullsize.json: the oracle's count and digest of the full-size graph
self-join (2e6 vertices, 2e7 edges, Pareto(2.1) out-degrees; R = S = edges).
Calls only the oracle and the seeded generators.  Run from the repository
root: python tests/golden/make_fullsize.py"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    oracle.build(force=False)
    g = synth.config3()
    count, digest = oracle.count(g.rx, g.ry, g.sz, g.sy)
    out = {"graph_2e6_2e7": {"generator": "synth.config3()", "pairs": int(count), "digest": str(int(digest)),
                             "out_j": int(oracle.out_j(g.rx, g.ry, g.sz, g.sy))}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
