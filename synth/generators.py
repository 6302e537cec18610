"""Seeded generators for Join-Project tables R(x, y) and S(z, y).

Every generator returns plain int32 numpy columns.  Nothing here computes any
part of the Join-Project itself.

Readings of the workload descriptions (stated once, used everywhere):

* "distinct tuples": draw i.i.d., drop repeats keeping first-seen order, and
  refill until exactly N distinct tuples exist.
* Zipf(s) over a domain [0, n): P(value = k) is proportional to (k + 1)^-s,
  so value 0 is the most frequent; columns are drawn independently.
* The paper's own synthetic tables (its sensitivity study, Sec. 5 "Sensitivity
  Analysis with Synthetic Data Sets") are i.i.d. draws with repeats allowed.
* Power-law graph: out-degrees follow a continuous Pareto(alpha, x_m) with
  x_m = 10 (alpha - 1) / alpha (mean 10), scaled to the exact edge count with
  largest-remainder rounding; destinations are uniform, never repeated for a
  source; self-loops are allowed.  R and S are the same (src, dst) arrays.
* Batched instances: per-side tuple counts log-uniform in [1e3, 1e6]; key
  domains are ceil(0.1 * n) for that side; even instances draw y uniformly,
  odd ones Zipf(1.2) over the side's y domain; i.i.d. with repeats.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Tuple

import numpy as np

SEED_ROOT = 2206_04995


@dataclasses.dataclass
class Instance:
    """One Join-Project input: R(x, y) and S(z, y) as int32 columns."""

    rx: np.ndarray
    ry: np.ndarray
    sz: np.ndarray
    sy: np.ndarray
    name: str = ""

    @property
    def n_r(self) -> int:
        return int(self.rx.shape[0])

    @property
    def n_s(self) -> int:
        return int(self.sz.shape[0])


def _child_rng(*path: int) -> np.random.Generator:
    """Generator for a fixed path below the root seed (config, instance, ...)."""
    ss = np.random.SeedSequence(SEED_ROOT)
    for p in path:
        ss = ss.spawn(p + 1)[p]
    return np.random.default_rng(ss)


def zipf_sample(rng: np.random.Generator, n_domain: int, s: float, size: int) -> np.ndarray:
    """Draw `size` values in [0, n_domain) with P(k) proportional to (k+1)^-s."""
    if s == 0.0:
        return rng.integers(0, n_domain, size=size, dtype=np.int64).astype(np.int32)
    w = np.arange(1, n_domain + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    k = np.searchsorted(cdf, u, side="right")
    np.minimum(k, n_domain - 1, out=k)
    return k.astype(np.int32)


def distinct_pairs(
    rng: np.random.Generator,
    draw: Callable[[np.random.Generator, int], Tuple[np.ndarray, np.ndarray]],
    n: int,
) -> Tuple[np.ndarray, np.ndarray]:
    """Exactly n distinct (a, b) pairs, first-seen order, refilled as needed.

    Both columns must hold values in [0, 2^31).
    """
    keys = np.empty(0, dtype=np.int64)
    rounds = 0
    while keys.shape[0] < n:
        need = n - keys.shape[0]
        m = need + need // 8 + 64
        a, b = draw(rng, m)
        k = (a.astype(np.int64) << 32) | b.astype(np.int64)
        cat = np.concatenate([keys, k])
        _, first = np.unique(cat, return_index=True)
        first.sort()
        keys = cat[first[:n]]
        rounds += 1
        if rounds > 200:
            raise RuntimeError("distinct_pairs: domain too small for the requested count")
    a = (keys >> 32).astype(np.int32)
    b = (keys & 0xFFFFFFFF).astype(np.int32)
    return a, b


def uniform_table(rng, n, dom_a, dom_b, distinct=False):
    def draw(g, m):
        return (g.integers(0, dom_a, m, dtype=np.int64), g.integers(0, dom_b, m, dtype=np.int64))

    if distinct:
        return distinct_pairs(rng, draw, n)
    a, b = draw(rng, n)
    return a.astype(np.int32), b.astype(np.int32)


# ---------------------------------------------------------------- configs


def config1(seed_index: int = 0) -> Instance:
    """Plain single query: 1e5 distinct tuples per side; x, z in [0, 1e4), y in [0, 5e3)."""
    rr = _child_rng(0, seed_index, 0)
    rs = _child_rng(0, seed_index, 1)
    rx, ry = uniform_table(rr, 100_000, 10_000, 5_000, distinct=True)
    sz, sy = uniform_table(rs, 100_000, 10_000, 5_000, distinct=True)
    return Instance(rx, ry, sz, sy, name="uniform-1e5")


def _zipf_y_table(rng, n, dom_a, dom_y, s, distinct):
    def draw(g, m):
        return (g.integers(0, dom_a, m, dtype=np.int64), zipf_sample(g, dom_y, s, m).astype(np.int64))

    if distinct:
        return distinct_pairs(rng, draw, n)
    a, b = draw(rng, n)
    return a.astype(np.int32), b.astype(np.int32)


def config2(seed_index: int = 0, n: int = 10_000_000, dom_xz: int = 1_000_000,
            dom_y: int = 100_000, s: float = 1.0) -> Instance:
    """Skewed single query: n distinct tuples per side; x, z uniform in [0, dom_xz);
    y Zipf(s) over [0, dom_y).  Defaults are the 1e7-tuple workload."""
    rr = _child_rng(1, seed_index, 0)
    rs = _child_rng(1, seed_index, 1)
    rx, ry = _zipf_y_table(rr, n, dom_xz, dom_y, s, True)
    sz, sy = _zipf_y_table(rs, n, dom_xz, dom_y, s, True)
    return Instance(rx, ry, sz, sy, name=f"zipf-y{s}-{n}")


def pareto_graph(rng, n_vertices: int, n_edges: int, alpha: float = 2.1):
    """Directed power-law graph as (src, dst) int32 arrays (see module notes)."""
    x_m = 10.0 * (alpha - 1.0) / alpha
    u = rng.random(n_vertices)
    d = x_m * (1.0 - u) ** (-1.0 / alpha)
    d = np.minimum(d, float(n_vertices))
    scaled = d * (n_edges / d.sum())
    base = np.floor(scaled).astype(np.int64)
    np.minimum(base, n_vertices, out=base)
    rem = n_edges - int(base.sum())
    if rem > 0:
        frac = scaled - base
        frac[base >= n_vertices] = -1.0
        order = np.argsort(-frac, kind="stable")[:rem]
        base[order] += 1
    deg = base
    src = np.repeat(np.arange(n_vertices, dtype=np.int64), deg)
    dst = rng.integers(0, n_vertices, size=src.shape[0], dtype=np.int64)
    # redraw repeated (src, dst) until every source has distinct destinations
    for _ in range(100):
        key = src * n_vertices + dst
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.shape[0], dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        pos = order[dup]
        dst[pos] = rng.integers(0, n_vertices, size=pos.shape[0], dtype=np.int64)
    else:
        raise RuntimeError("pareto_graph: could not make destinations distinct")
    perm = rng.permutation(src.shape[0])
    return src[perm].astype(np.int32), dst[perm].astype(np.int32)


def config3(seed_index: int = 0, n_vertices: int = 2_000_000, n_edges: int = 20_000_000,
            two_hop: bool = False) -> Instance:
    """Self-join on a power-law graph.  Default reading: R = S = (src, dst), so the
    output is every pair of sources sharing a destination.  two_hop=True swaps S's
    columns (S.z = dst, S.y = src), which gives x -> y -> z paths."""
    rng = _child_rng(2, seed_index)
    src, dst = pareto_graph(rng, n_vertices, n_edges)
    if two_hop:
        return Instance(src, dst, dst.copy(), src.copy(), name=f"graph2hop-{n_edges}")
    return Instance(src, dst, src.copy(), dst.copy(), name=f"graph-{n_edges}")


def config4_instance(i: int, lo: int = 1_000, hi: int = 1_000_000, batch_seed: int = 0) -> Instance:
    """Instance i of the batched workload (its own seed path, reproducible alone)."""
    rng = _child_rng(3, batch_seed, i)
    n_r = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    n_s = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    dr = max(1, math.ceil(0.1 * n_r))
    ds = max(1, math.ceil(0.1 * n_s))
    rx = rng.integers(0, dr, n_r, dtype=np.int64).astype(np.int32)
    sz = rng.integers(0, ds, n_s, dtype=np.int64).astype(np.int32)
    if i % 2 == 0:
        ry = rng.integers(0, dr, n_r, dtype=np.int64).astype(np.int32)
        sy = rng.integers(0, ds, n_s, dtype=np.int64).astype(np.int32)
    else:
        ry = zipf_sample(rng, dr, 1.2, n_r)
        sy = zipf_sample(rng, ds, 1.2, n_s)
    return Instance(rx, ry, sz, sy, name=f"batch{batch_seed}-{i}")


def config4(n_instances: int = 4096, lo: int = 1_000, hi: int = 1_000_000,
            batch_seed: int = 0) -> List[Instance]:
    return [config4_instance(i, lo, hi, batch_seed) for i in range(n_instances)]


def config5_trace(n_queries: int = 50_000, rate_per_s: float = 1000.0, p_large: float = 0.01,
                  trace_seed: int = 0):
    """Arrival trace: list of (arrival_s, kind, seed_index).  kind 0 = a fresh
    batched-mix instance (drawn with config4_instance(seed_index, batch_seed=1000+trace_seed)),
    kind 1 = a fresh 1e7-tuple skewed instance (config2(seed_index))."""
    rng = _child_rng(4, trace_seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_queries)
    t = np.cumsum(gaps)
    kind = (rng.random(n_queries) < p_large).astype(np.int32)
    out = []
    n_small = 0
    n_large = 0
    for q in range(n_queries):
        if kind[q] == 0:
            out.append((float(t[q]), 0, n_small))
            n_small += 1
        else:
            out.append((float(t[q]), 1, 1 + n_large))
            n_large += 1
    return out


# ------------------------------------------------------ paper's own tables


def uniform_paper_default(n_tuples: int = 1_000_000, n_domain: int = 10_000, seed_index: int = 0) -> Instance:
    """The paper's sensitivity default: |R| = |S| = N, x, y, z uniform over n values,
    i.i.d. with repeats (Sec. 5, sensitivity analysis)."""
    rng = _child_rng(5, seed_index)
    rx, ry = uniform_table(rng, n_tuples, n_domain, n_domain)
    sz, sy = uniform_table(rng, n_tuples, n_domain, n_domain)
    return Instance(rx, ry, sz, sy, name=f"paper-uniform-{n_tuples}-{n_domain}")


def zipf_xz_paper(n_tuples: int = 1_000_000, n_domain: int = 10_000, s: float = 1.0,
                  seed_index: int = 0) -> Instance:
    """Zipf(s) on R.x and S.z, y uniform, i.i.d. with repeats (Sec. 5, skew study)."""
    rng = _child_rng(6, seed_index)
    rx = zipf_sample(rng, n_domain, s, n_tuples)
    ry = rng.integers(0, n_domain, n_tuples, dtype=np.int64).astype(np.int32)
    sz = zipf_sample(rng, n_domain, s, n_tuples)
    sy = rng.integers(0, n_domain, n_tuples, dtype=np.int64).astype(np.int32)
    return Instance(rx, ry, sz, sy, name=f"paper-zipfxz{s}")


def small_random(seed: int, n_r: int, n_s: int, dom_x: int = 20, dom_y: int = 20, dom_z: int = 20,
                 offset: int = 0, zipf_y: float = 0.0) -> Instance:
    """Small i.i.d. tables (repeats allowed) for parity tests; `offset` shifts every
    value so negative and extreme int32 values are exercised."""
    rng = _child_rng(7, seed)
    rx = rng.integers(0, dom_x, n_r, dtype=np.int64)
    sz = rng.integers(0, dom_z, n_s, dtype=np.int64)
    if zipf_y > 0:
        ry = zipf_sample(rng, dom_y, zipf_y, n_r).astype(np.int64)
        sy = zipf_sample(rng, dom_y, zipf_y, n_s).astype(np.int64)
    else:
        ry = rng.integers(0, dom_y, n_r, dtype=np.int64)
        sy = rng.integers(0, dom_y, n_s, dtype=np.int64)

    def cast(v):
        v = v + offset
        return np.clip(v, -(2 ** 31), 2 ** 31 - 1).astype(np.int32)

    return Instance(cast(rx), cast(ry), cast(sz), cast(sy), name=f"small-{seed}")
