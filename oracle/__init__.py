"""CPU oracle for the Join-Project PI_{x,z}(R(x,y) JOIN_y S(z,y)).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package never imports the product.

Contents
* ``join_project`` / ``count`` / ``rows`` / ``out_j``: the C++ hash-join plus
  hash-set deduplication in ``jp_oracle.cpp`` (the paper's classical solution,
  Sec. 1.1, which reaches the plain definition of Eq. 1).
* ``row_counts``: per-row counts and digests from the matrix form of Sec. 1.1
  (row x of the Boolean product as a bit vector over z, one x at a time), for
  results too large to hold as a set or a list.
* ``brute_force``: nested loops over R x S for tiny inputs (definition of
  Eq. 1 written out directly), used to pin the C++ oracle.
* ``split_by_z``: the intersection-free partition of a result by the dense z
  set (Sec. 2.3): a pair belongs to the dense part iff its z is dense.
* ``digest_pairs``: order-independent digest (wrapping sum of SplitMix64
  finalised keys), used where a result is too large to list.
* ``aggregate`` / ``brute_force_aggregate``: Join-Aggregate (Sec. 4.1), per
  group (x, z) the number of join rows and the sum of R.v * S.u.
* ``join_project_composite`` / ``brute_force_composite``: multi-attribute
  keys (Sec. 2.2, wider range of operations).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jp_oracle.cpp")
_LIB = os.path.join(_HERE, "libjp_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (host code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        base = [i32p, i32p, ctypes.c_int64, i32p, i32p, ctypes.c_int64]
        lib.jpo_out_j.argtypes = base
        lib.jpo_out_j.restype = ctypes.c_int64
        lib.jpo_count.argtypes = base + [ctypes.c_int, u64p]
        lib.jpo_count.restype = ctypes.c_int64
        lib.jpo_list.argtypes = base + [ctypes.c_int, i32p, i32p, ctypes.c_int64]
        lib.jpo_list.restype = ctypes.c_int64
        lib.jpo_rows.argtypes = base + [i32p, ctypes.c_int64, ctypes.c_int, i64p, i32p, ctypes.c_int64]
        lib.jpo_rows.restype = ctypes.c_int64
        lib.jpo_row_counts.argtypes = base + [ctypes.c_int, i32p, i64p, u64p, i64p, u64p]
        lib.jpo_row_counts.restype = ctypes.c_int64
        lib.jpo_aggregate.argtypes = [i32p, i32p, i32p, ctypes.c_int64, i32p, i32p, i32p, ctypes.c_int64, ctypes.c_int,
                                      i32p, i32p, i64p, i64p, ctypes.c_int64]
        lib.jpo_aggregate.restype = ctypes.c_int64
        lib.jpo_digest_pairs.argtypes = [i32p, i32p, ctypes.c_int64]
        lib.jpo_digest_pairs.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _cols(rx, ry, sz, sy):
    cols = [np.ascontiguousarray(np.asarray(c, dtype=np.int32)) for c in (rx, ry, sz, sy)]
    if cols[0].shape != cols[1].shape or cols[2].shape != cols[3].shape:
        raise ValueError("column length mismatch")
    return cols


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def out_j(rx, ry, sz, sy) -> int:
    rx, ry, sz, sy = _cols(rx, ry, sz, sy)
    return int(_load().jpo_out_j(_p32(rx), _p32(ry), rx.size, _p32(sz), _p32(sy), sz.size))


def count(rx, ry, sz, sy, threads: Optional[int] = None) -> Tuple[int, int]:
    """(number of distinct pairs, digest) of the whole result."""
    rx, ry, sz, sy = _cols(rx, ry, sz, sy)
    d = ctypes.c_uint64(0)
    c = _load().jpo_count(_p32(rx), _p32(ry), rx.size, _p32(sz), _p32(sy), sz.size,
                          threads or default_threads(), ctypes.byref(d))
    return int(c), int(d.value)


def join_project(rx, ry, sz, sy, threads: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Sorted (x, z) result as two int32 arrays."""
    rx, ry, sz, sy = _cols(rx, ry, sz, sy)
    lib = _load()
    cap = max(1, out_j(rx, ry, sz, sy))
    ox = np.empty(cap, dtype=np.int32)
    oz = np.empty(cap, dtype=np.int32)
    n = lib.jpo_list(_p32(rx), _p32(ry), rx.size, _p32(sz), _p32(sy), sz.size,
                     threads or default_threads(), _p32(ox), _p32(oz), cap)
    assert n <= cap
    return ox[:n].copy(), oz[:n].copy()


def rows(rx, ry, sz, sy, xs: Sequence[int], threads: Optional[int] = None) -> List[np.ndarray]:
    """Sorted distinct z's of each requested x value (empty if x has no match)."""
    rx, ry, sz, sy = _cols(rx, ry, sz, sy)
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    lib = _load()
    counts = np.zeros(max(1, xs.size), dtype=np.int64)
    # first pass sizes the rows, second fills them
    total = lib.jpo_rows(_p32(rx), _p32(ry), rx.size, _p32(sz), _p32(sy), sz.size, _p32(xs), xs.size,
                         threads or default_threads(),
                         counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p32(np.zeros(1, np.int32)), 0)
    out = np.empty(max(1, total), dtype=np.int32)
    lib.jpo_rows(_p32(rx), _p32(ry), rx.size, _p32(sz), _p32(sy), sz.size, _p32(xs), xs.size,
                 threads or default_threads(), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                 _p32(out), total)
    res = []
    pos = 0
    for i in range(xs.size):
        c = int(counts[i])
        res.append(out[pos:pos + c].copy())
        pos += c
    return res


def row_counts(rx, ry, sz, sy, threads: Optional[int] = None):
    """Per-row counts and digests by the matrix form (bit vector over z per x row).

    Returns (xs, counts, digests, total, digest): the distinct x values of R
    ascending, each row's number of pairs and digest (uint64), and the totals
    over the whole result.  Memory stays at |Z| bits per thread, so it scales
    to results far too large to list."""
    rx, ry, sz, sy = _cols(rx, ry, sz, sy)
    n = max(1, rx.size)
    xs = np.empty(n, dtype=np.int32)
    cnt = np.empty(n, dtype=np.int64)
    dig = np.empty(n, dtype=np.uint64)
    tot = ctypes.c_int64(0)
    d = ctypes.c_uint64(0)
    nx = _load().jpo_row_counts(_p32(rx), _p32(ry), rx.size, _p32(sz), _p32(sy), sz.size,
                                threads or default_threads(), _p32(xs),
                                cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                dig.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                ctypes.byref(tot), ctypes.byref(d))
    return xs[:nx].copy(), cnt[:nx].copy(), dig[:nx].copy(), int(tot.value), int(d.value)


def digest_pairs(xs: np.ndarray, zs: np.ndarray) -> int:
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    zs = np.ascontiguousarray(np.asarray(zs, dtype=np.int32))
    return int(_load().jpo_digest_pairs(_p32(xs), _p32(zs), xs.size))


# ------------------------------------------------------------ pure Python


def brute_force(rx: Iterable[int], ry: Iterable[int], sz: Iterable[int], sy: Iterable[int]):
    """Eq. 1 written out: every (R tuple, S tuple) pair with equal y contributes
    (x, z); the set removes duplicates.  Returns the sorted list of pairs."""
    r = list(zip((int(v) for v in rx), (int(v) for v in ry)))
    s = list(zip((int(v) for v in sz), (int(v) for v in sy)))
    out = set()
    for x, y in r:
        for z, y2 in s:
            if y == y2:
                out.add((x, z))
    return sorted(out)


def split_by_z(xs: np.ndarray, zs: np.ndarray, dense_z_values: np.ndarray):
    """Intersection-free partition of a result (Sec. 2.3): a pair is in the dense
    part iff its z value is one of the dense z values.  Returns
    ((dense_x, dense_z), (sparse_x, sparse_z)), each in input order."""
    mask = np.isin(zs, np.asarray(dense_z_values, dtype=np.int32))
    return (xs[mask], zs[mask]), (xs[~mask], zs[~mask])


# ------------------------------------------------------- composite keys


def _ranks(*cols_groups):
    """Lexicographic ranks of the row tuples of several column groups encoded
    together (np.unique over rows), one rank array per group, plus the sorted
    distinct tuples."""
    mats = [np.stack([np.asarray(c, dtype=np.int32) for c in g], axis=1) if len(g[0]) else
            np.zeros((0, len(g)), dtype=np.int32) for g in cols_groups]
    allm = np.concatenate(mats, axis=0)
    uniq, inv = np.unique(allm, axis=0, return_inverse=True)
    inv = inv.reshape(-1).astype(np.int32)
    out, at = [], 0
    for m in mats:
        out.append(inv[at:at + m.shape[0]])
        at += m.shape[0]
    return out, uniq


def join_project_composite(r_x, r_y, s_z, s_y):
    """Join-Project over multi-attribute keys (Sec. 2.2, wider range of
    operations): r_x, r_y, s_z, s_y are lists of int32 columns; x is the tuple of
    R's r_x columns, y the tuple of the join columns (equal arity on both sides),
    z the tuple of S's s_z columns.  Each tuple kind is replaced by its rank among
    the distinct tuples in lexicographic order (np.unique over rows; R.y and S.y
    ranked together), the single-column oracle runs on the ranks, and the ranks
    are mapped back.  Returns (x columns, z columns) of the distinct result
    pairs, sorted lexicographically by (x tuple, z tuple)."""
    (xr,), ux = _ranks(r_x)
    (yr, ys), _ = _ranks(r_y, s_y)
    (zr,), uz = _ranks(s_z)
    ox, oz = join_project(xr, yr, zr, ys)
    return [ux[ox, c].copy() for c in range(ux.shape[1])], [uz[oz, c].copy() for c in range(uz.shape[1])]


def brute_force_composite(r_x, r_y, s_z, s_y):
    """Eq. 1 over tuples, written out with nested loops (tiny inputs only):
    sorted list of distinct (x tuple, z tuple) pairs."""
    R = [(tuple(int(c[i]) for c in r_x), tuple(int(c[i]) for c in r_y)) for i in range(len(r_x[0]))]
    S = [(tuple(int(c[i]) for c in s_z), tuple(int(c[i]) for c in s_y)) for i in range(len(s_z[0]))]
    out = set()
    for x, y in R:
        for z, y2 in S:
            if y == y2:
                out.add((x, z))
    return sorted(out)


# ------------------------------------------------------- Join-Aggregate


def aggregate(rx, ry, rv, sz, sy, su, threads: Optional[int] = None):
    """Join-Aggregate (Sec. 4.1): groups (x, z) of R(x, y, v) JOIN_y S(z, y, u)
    with COUNT(*) and SUM(v * u) (int64, wrapping), sorted by (x, z).  Returns
    (x, z, count, sum) arrays."""
    rx, ry, sz, sy = _cols(rx, ry, sz, sy)
    rv = np.ascontiguousarray(np.asarray(rv, dtype=np.int32))
    su = np.ascontiguousarray(np.asarray(su, dtype=np.int32))
    if rv.shape != rx.shape or su.shape != sz.shape:
        raise ValueError("value column length mismatch")
    lib = _load()
    cap = max(1, out_j(rx, ry, sz, sy))
    ox = np.empty(cap, np.int32)
    oz = np.empty(cap, np.int32)
    oc = np.empty(cap, np.int64)
    osum = np.empty(cap, np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    n = lib.jpo_aggregate(_p32(rx), _p32(ry), _p32(rv), rx.size, _p32(sz), _p32(sy), _p32(su), sz.size,
                          threads or default_threads(), _p32(ox), _p32(oz), oc.ctypes.data_as(i64p),
                          osum.ctypes.data_as(i64p), cap)
    assert n <= cap
    return ox[:n].copy(), oz[:n].copy(), oc[:n].copy(), osum[:n].copy()


def brute_force_aggregate(rx, ry, rv, sz, sy, su):
    """Sec. 4.1's Join-Aggregate written out with nested loops (tiny inputs):
    sorted list of (x, z, count, sum of v * u)."""
    acc = {}
    for x, y, v in zip(rx, ry, rv):
        for z, y2, u in zip(sz, sy, su):
            if int(y) == int(y2):
                c, s = acc.get((int(x), int(z)), (0, 0))
                acc[(int(x), int(z))] = (c + 1, s + int(v) * int(u))
    return [(x, z, c, s) for (x, z), (c, s) in sorted(acc.items())]
