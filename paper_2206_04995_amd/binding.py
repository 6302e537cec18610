"""ctypes binding of the Join-Project C ABI (include/jp.h).

Argument marshalling only: every step of the Join-Project runs in the HIP
kernels of libjp.so.  Device columns are int32 torch tensors on a ROCm device;
streams are torch streams (the current one by default).  If the library is
missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("JP_LIB_PATH") or os.path.join(_HERE, "libjp.so")

JP_OK, JP_EINVAL, JP_ENOMEM, JP_EHIP, JP_ESTATE, JP_ERANGE, JP_EBUSY = range(7)
JP_PART_ALL, JP_PART_DENSE, JP_PART_SPARSE = 0, 1, 2
JP_TAU_AUTO, JP_TAU_FIXED = 0, 1
JP_DENSE_AUTO, JP_DENSE_BITS, JP_DENSE_MFMA = 0, 1, 2
JP_FLAG_TIMING = 1
JP_FLAG_GRAPH = 2
JP_FLAG_DIRECT_IDS = 4
JP_STRATEGY_AUTO, JP_STRATEGY_HYBRID, JP_STRATEGY_CLASSICAL = 0, 1, 2
JP_SERVER_DIGEST = 1
JP_SERVER_KEEP = 2
INT64_MAX = 2 ** 63 - 1

_STATUS = {0: "JP_OK", 1: "JP_EINVAL", 2: "JP_ENOMEM", 3: "JP_EHIP", 4: "JP_ESTATE", 5: "JP_ERANGE", 6: "JP_EBUSY"}

# every symbol include/jp.h declares
EXPORTS = [
    "jp_plan_create", "jp_execute", "jp_count", "jp_materialize", "jp_row_info", "jp_dense_z",
    "jp_plan_stats", "jp_plan_timings", "jp_plan_work", "jp_plan_destroy", "jp_last_error",
    "jp_batch_create", "jp_batch_execute", "jp_batch_counts", "jp_batch_materialize", "jp_batch_stats",
    "jp_batch_destroy", "jp_batch_timings", "jp_batch_work",
    "jp_server_create", "jp_server_submit", "jp_server_poll", "jp_server_wait", "jp_server_stats", "jp_server_destroy",
    "jp_server_materialize", "jp_server_release", "jp_digest_pairs",
    "jp_tune", "jp_tune_clear", "jp_count_static",
    "jp_dict_create", "jp_dict_size", "jp_dict_decode", "jp_dict_destroy",
    "jp_agg_create", "jp_agg_execute", "jp_agg_count", "jp_agg_materialize", "jp_agg_destroy",
    "jp_cache_build", "jp_cache_info", "jp_cache_z", "jp_plan_create_cached", "jp_cache_materialize",
    "jp_cache_destroy",
]


class JpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class jp_options(ctypes.Structure):
    _fields_ = [
        ("tau_mode", ctypes.c_int32),
        ("dense_kernel", ctypes.c_int32),
        ("dense_threshold", ctypes.c_int64),
        ("k_hot_max", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("workspace_limit_bytes", ctypes.c_int64),
        ("window_group", ctypes.c_int32),
        ("strategy", ctypes.c_int32),
        ("sparse_light_max", ctypes.c_int32),
        ("sparse_med_max", ctypes.c_int32),
        ("mfma_tile", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class jp_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_x", "n_y", "n_z", "n_r_kept", "out_j", "tau", "n_z_dense", "k_hot", "footprint_bytes",
                 "pivot_cover", "dense_mfma", "peak_bytes", "map_direct", "strategy")]


class jp_timings(ctypes.Structure):
    _fields_ = [("sparse_ms", ctypes.c_float), ("dense_ms", ctypes.c_float), ("execute_ms", ctypes.c_float),
                ("pad_", ctypes.c_float)] + [
        (n, ctypes.c_int64) for n in ("sparse_join_rows", "n_r_kept", "n_x", "dense_hot_words", "dense_row_words",
                                      "dense_cold_entries", "dense_mfma_ops")] + [
        ("map_ms", ctypes.c_float), ("partition_ms", ctypes.c_float), ("dense_mfma_issued_ops", ctypes.c_int64)]


class jp_tune_result(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_int64), ("model_tau", ctypes.c_int64), ("cost_ratio", ctypes.c_double),
                ("best_ms", ctypes.c_double), ("model_ms", ctypes.c_double), ("candidates", ctypes.c_int32),
                ("dense_kernel", ctypes.c_int32), ("k_hot_max", ctypes.c_int32), ("window_group", ctypes.c_int32),
                ("signature", ctypes.c_uint64), ("sparse_light_max", ctypes.c_int32), ("sparse_med_max", ctypes.c_int32),
                ("mfma_tile", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class jp_instance(ctypes.Structure):
    _fields_ = [
        ("r_x", ctypes.c_void_p), ("r_y", ctypes.c_void_p), ("s_z", ctypes.c_void_p), ("s_y", ctypes.c_void_p),
        ("n_r", ctypes.c_int64), ("n_s", ctypes.c_int64),
    ]


class jp_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("opt", jp_options), ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("chunk_pairs", ctypes.c_int64)]


class jp_query_result(ctypes.Structure):
    _fields_ = [("total", ctypes.c_int64), ("dense", ctypes.c_int64), ("sparse", ctypes.c_int64),
                ("digest", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("has_digest", ctypes.c_int32), ("kept", ctypes.c_int32), ("submit_us", ctypes.c_double),
                ("admit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class jp_server_summary(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "batches", "splits", "pairs",
                                              "peak_bytes", "budget_bytes", "charged_bytes")] + [
        (n, ctypes.c_double) for n in ("p50_us", "p99_us", "mean_us")]


def _load() -> ctypes.CDLL:
    # libjp.so must bind to the HIP runtime torch uses (both carry the soname
    # libamdhip64.so.7); a second runtime mapped into the process sees no device.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2206_04995_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    st = ctypes.c_int
    sig = {
        "jp_plan_create": (st, [vp, vp, i64, vp, vp, i64, ctypes.POINTER(jp_options), vp, ctypes.POINTER(vp)]),
        "jp_execute": (st, [vp, vp]),
        "jp_count": (st, [vp, i64p, i64p, i64p, vp]),
        "jp_materialize": (st, [vp, ctypes.c_int, i64, i64, vp, vp, i64p, vp]),
        "jp_row_info": (st, [vp, ctypes.c_int, i32p, i64p, vp]),
        "jp_dense_z": (st, [vp, i32p, vp]),
        "jp_plan_stats": (st, [vp, ctypes.POINTER(jp_stats)]),
        "jp_plan_timings": (st, [vp, ctypes.POINTER(jp_timings), vp]),
        "jp_plan_work": (st, [vp, ctypes.POINTER(jp_timings), vp]),
        "jp_plan_destroy": (None, [vp]),
        "jp_last_error": (ctypes.c_char_p, []),
        "jp_batch_create": (st, [ctypes.POINTER(jp_instance), i32, ctypes.POINTER(jp_options), vp, ctypes.POINTER(vp)]),
        "jp_batch_execute": (st, [vp, vp]),
        "jp_batch_counts": (st, [vp, i64p, vp]),
        "jp_batch_materialize": (st, [vp, i32, ctypes.c_int, i64, i64, vp, vp, i64p, vp]),
        "jp_batch_stats": (st, [vp, i32, ctypes.POINTER(jp_stats)]),
        "jp_batch_destroy": (None, [vp]),
        "jp_batch_timings": (st, [vp, ctypes.POINTER(jp_timings), vp]),
        "jp_batch_work": (st, [vp, ctypes.POINTER(jp_timings), vp]),
        "jp_server_create": (st, [ctypes.POINTER(jp_server_config), ctypes.POINTER(vp)]),
        "jp_server_submit": (st, [vp, ctypes.POINTER(jp_instance), ctypes.POINTER(ctypes.c_uint64)]),
        "jp_server_poll": (st, [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(jp_query_result)]),
        "jp_server_wait": (st, [vp, ctypes.c_uint64, ctypes.POINTER(jp_query_result)]),
        "jp_server_stats": (st, [vp, ctypes.POINTER(jp_server_summary)]),
        "jp_server_destroy": (None, [vp]),
        "jp_server_materialize": (st, [vp, ctypes.c_uint64, ctypes.c_int, i64, i64, vp, vp, i64p, vp]),
        "jp_server_release": (st, [vp, ctypes.c_uint64]),
        "jp_digest_pairs": (st, [vp, vp, i64, vp, vp]),
        "jp_tune": (st, [vp, vp, i64, vp, vp, i64, ctypes.POINTER(jp_options), vp, ctypes.POINTER(jp_tune_result)]),
        "jp_tune_clear": (st, []),
        "jp_count_static": (st, [vp, vp, i64, vp, vp, i64, ctypes.POINTER(jp_options), vp, i64p, i64p, i64p]),
        "jp_dict_create": (st, [i32, i32, ctypes.POINTER(vp), i64p, ctypes.POINTER(vp), vp, ctypes.POINTER(vp)]),
        "jp_dict_size": (st, [vp, i64p]),
        "jp_dict_decode": (st, [vp, vp, i64, ctypes.POINTER(vp), vp]),
        "jp_dict_destroy": (None, [vp]),
        "jp_agg_create": (st, [vp, vp, vp, i64, vp, vp, vp, i64, vp, ctypes.POINTER(vp)]),
        "jp_agg_execute": (st, [vp, vp]),
        "jp_agg_count": (st, [vp, i64p, i64p, vp]),
        "jp_agg_materialize": (st, [vp, i64, i64, vp, vp, vp, vp, i64p, vp]),
        "jp_agg_destroy": (None, [vp]),
        "jp_cache_build": (st, [vp, i64, vp, ctypes.POINTER(vp)]),
        "jp_cache_info": (st, [vp, i64p, i64p, i64p]),
        "jp_cache_z": (st, [vp, i32p]),
        "jp_plan_create_cached": (st, [vp, vp, i64, vp, vp, i64, vp, ctypes.POINTER(jp_options), vp,
                                       ctypes.POINTER(vp)]),
        "jp_cache_materialize": (st, [vp, i64, i64, vp, vp, i64p, vp]),
        "jp_cache_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    m = lib.jp_last_error()
    return m.decode() if m else ""


def _check(status: int):
    if status != JP_OK:
        raise JpError(status, last_error())


def _stream(stream) -> int:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> int:
    """Device pointer of an int32 tensor (None -> 0)."""
    if t is None:
        return 0
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("columns must be contiguous int32 tensors on a ROCm device")
    return t.data_ptr()


def make_options(tau_mode: int = JP_TAU_AUTO, dense_threshold: int = 0, dense_kernel: int = JP_DENSE_AUTO,
                 k_hot_max: int = 0, workspace_limit_bytes: int = 0, flags: int = 0,
                 window_group: int = 0, strategy: int = JP_STRATEGY_AUTO, sparse_light_max: int = 0,
                 sparse_med_max: int = 0, mfma_tile: int = 0) -> jp_options:
    o = jp_options()
    o.strategy = strategy
    o.sparse_light_max = sparse_light_max
    o.sparse_med_max = sparse_med_max
    o.mfma_tile = mfma_tile
    o.window_group = window_group
    o.tau_mode = tau_mode
    o.dense_kernel = dense_kernel
    o.dense_threshold = dense_threshold
    o.k_hot_max = k_hot_max
    o.flags = flags
    o.workspace_limit_bytes = workspace_limit_bytes
    return o


def _stats_dict(s: jp_stats) -> Dict[str, int]:
    return {name: int(getattr(s, name)) for name, _ in jp_stats._fields_}


# ------------------------------------------------------------------ plan


def jp_plan_create(r_x, r_y, s_z, s_y, opt: Optional[jp_options] = None, stream=None) -> int:
    h = ctypes.c_void_p()
    n_r = int(r_x.numel()) if r_x is not None else 0
    n_s = int(s_z.numel()) if s_z is not None else 0
    _check(lib.jp_plan_create(_ptr(r_x), _ptr(r_y), n_r, _ptr(s_z), _ptr(s_y), n_s,
                              ctypes.byref(opt) if opt is not None else None, _stream(stream), ctypes.byref(h)))
    return h.value


def jp_count_static(r_x, r_y, s_z, s_y, opt: Optional[jp_options] = None, stream=None) -> Tuple[int, int, int]:
    """(total, dense, sparse) of one query computed in the library's static device scratch (no allocation)."""
    n_r = int(r_x.numel()) if r_x is not None else 0
    n_s = int(s_z.numel()) if s_z is not None else 0
    t, d, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.jp_count_static(_ptr(r_x), _ptr(r_y), n_r, _ptr(s_z), _ptr(s_y), n_s,
                               ctypes.byref(opt) if opt is not None else None, _stream(stream),
                               ctypes.byref(t), ctypes.byref(d), ctypes.byref(s)))
    return t.value, d.value, s.value


def jp_tune(r_x, r_y, s_z, s_y, opt: Optional[jp_options] = None, stream=None) -> Dict[str, float]:
    """Time the candidate thresholds on this query and store the fastest one's cost ratio."""
    r = jp_tune_result()
    n_r = int(r_x.numel()) if r_x is not None else 0
    n_s = int(s_z.numel()) if s_z is not None else 0
    _check(lib.jp_tune(_ptr(r_x), _ptr(r_y), n_r, _ptr(s_z), _ptr(s_y), n_s,
                       ctypes.byref(opt) if opt is not None else None, _stream(stream), ctypes.byref(r)))
    return {name: getattr(r, name) for name, _ in jp_tune_result._fields_}


def jp_tune_clear():
    _check(lib.jp_tune_clear())


def jp_execute(plan: int, stream=None):
    _check(lib.jp_execute(plan, _stream(stream)))


def jp_count(plan: int, stream=None) -> Tuple[int, int, int]:
    t, d, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.jp_count(plan, ctypes.byref(t), ctypes.byref(d), ctypes.byref(s), _stream(stream)))
    return t.value, d.value, s.value


def jp_materialize(plan: int, part: int, first: int, max_pairs: int, out_x, out_z, stream=None) -> int:
    n = ctypes.c_int64()
    _check(lib.jp_materialize(plan, part, first, max_pairs, _ptr(out_x), _ptr(out_z), ctypes.byref(n),
                              _stream(stream)))
    return n.value


def jp_row_info(plan: int, part: int = JP_PART_ALL, stream=None) -> Tuple[np.ndarray, np.ndarray]:
    st = jp_plan_stats(plan)
    nx = st["n_x"]
    xv = np.zeros(max(nx, 1), dtype=np.int32)
    off = np.zeros(nx + 1, dtype=np.int64)
    _check(lib.jp_row_info(plan, part, xv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(stream)))
    return xv[:nx], off


def jp_dense_z(plan: int, stream=None) -> np.ndarray:
    nd = jp_plan_stats(plan)["n_z_dense"]
    z = np.zeros(max(nd, 1), dtype=np.int32)
    _check(lib.jp_dense_z(plan, z.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream(stream)))
    return z[:nd]


def jp_plan_stats(plan: int) -> Dict[str, int]:
    s = jp_stats()
    _check(lib.jp_plan_stats(plan, ctypes.byref(s)))
    return _stats_dict(s)


def jp_plan_timings(plan: int, stream=None) -> Dict[str, float]:
    """Kernel times (ms) of the last jp_execute of a plan built with JP_FLAG_TIMING."""
    t = jp_timings()
    _check(lib.jp_plan_timings(plan, ctypes.byref(t), _stream(stream)))
    return {name: float(getattr(t, name)) for name, _ in jp_timings._fields_ if name.endswith("_ms")}


def jp_plan_work(plan: int, stream=None) -> Dict[str, int]:
    """Algorithmic work counters of the execute kernels."""
    t = jp_timings()
    _check(lib.jp_plan_work(plan, ctypes.byref(t), _stream(stream)))
    return {name: int(getattr(t, name)) for name, _ in jp_timings._fields_
            if not name.endswith("_ms") and name != "pad_"}


def jp_plan_destroy(plan: int):
    lib.jp_plan_destroy(plan)


# ----------------------------------------------------------------- batch


def _instances(cols: Sequence[Tuple]) -> "ctypes.Array":
    arr = (jp_instance * len(cols))()
    for i, (rx, ry, sz, sy) in enumerate(cols):
        arr[i].r_x, arr[i].r_y = _ptr(rx), _ptr(ry)
        arr[i].s_z, arr[i].s_y = _ptr(sz), _ptr(sy)
        arr[i].n_r = int(rx.numel())
        arr[i].n_s = int(sz.numel())
    return arr


class Instances:
    """A batch's instance table (the jp_instance array of the C ABI), built once
    from (r_x, r_y, s_z, s_y) column tensors and reusable for every jp_batch_create
    over the same columns; it keeps the tensors referenced."""

    def __init__(self, cols: Sequence[Tuple]):
        self.cols = list(cols)
        self.arr = _instances(self.cols)

    def __len__(self) -> int:
        return len(self.cols)


def jp_batch_create(cols, opt: Optional[jp_options] = None, stream=None) -> int:
    """cols: a sequence of (r_x, r_y, s_z, s_y) tensors, or an Instances table."""
    arr = cols.arr if isinstance(cols, Instances) else _instances(cols)
    h = ctypes.c_void_p()
    _check(lib.jp_batch_create(arr, len(cols), ctypes.byref(opt) if opt is not None else None, _stream(stream),
                               ctypes.byref(h)))
    return h.value


def jp_batch_execute(batch: int, stream=None):
    _check(lib.jp_batch_execute(batch, _stream(stream)))


def jp_batch_counts(batch: int, n_inst: int, stream=None) -> np.ndarray:
    out = np.zeros(n_inst, dtype=np.int64)
    _check(lib.jp_batch_counts(batch, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(stream)))
    return out


def jp_batch_materialize(batch: int, inst: int, part: int, first: int, max_pairs: int, out_x, out_z,
                         stream=None) -> int:
    n = ctypes.c_int64()
    _check(lib.jp_batch_materialize(batch, inst, part, first, max_pairs, _ptr(out_x), _ptr(out_z),
                                    ctypes.byref(n), _stream(stream)))
    return n.value


def jp_batch_stats(batch: int, inst: int) -> Dict[str, int]:
    s = jp_stats()
    _check(lib.jp_batch_stats(batch, inst, ctypes.byref(s)))
    return _stats_dict(s)


def jp_batch_timings(batch: int, stream=None) -> Dict[str, float]:
    """Stage times (ms) of the plan and the last execute of a batch built with JP_FLAG_TIMING."""
    t = jp_timings()
    _check(lib.jp_batch_timings(batch, ctypes.byref(t), _stream(stream)))
    return {name: float(getattr(t, name)) for name, _ in jp_timings._fields_ if name.endswith("_ms")}


def jp_batch_work(batch: int, stream=None) -> Dict[str, int]:
    t = jp_timings()
    _check(lib.jp_batch_work(batch, ctypes.byref(t), _stream(stream)))
    return {name: int(getattr(t, name)) for name, _ in jp_timings._fields_
            if not name.endswith("_ms") and name != "pad_"}


def jp_batch_destroy(batch: int):
    lib.jp_batch_destroy(batch)


# ---------------------------------------------------------------- server


def _result_dict(r: jp_query_result) -> Dict[str, float]:
    return {name: getattr(r, name) for name, _ in jp_query_result._fields_}


def jp_server_create(device: int = 0, max_batch: int = 0, hbm_budget_bytes: int = 0,
                     opt: Optional[jp_options] = None, flags: int = 0, chunk_pairs: int = 0) -> int:
    cfg = jp_server_config()
    cfg.device = device
    cfg.max_batch = max_batch
    cfg.hbm_budget_bytes = hbm_budget_bytes
    cfg.opt = opt if opt is not None else make_options()
    cfg.flags = flags
    cfg.chunk_pairs = chunk_pairs
    h = ctypes.c_void_p()
    _check(lib.jp_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def jp_server_submit(server: int, r_x, r_y, s_z, s_y) -> int:
    arr = _instances([(r_x, r_y, s_z, s_y)])
    t = ctypes.c_uint64()
    _check(lib.jp_server_submit(server, arr, ctypes.byref(t)))
    return t.value


def jp_server_poll(server: int, ticket: int):
    done = ctypes.c_int()
    r = jp_query_result()
    _check(lib.jp_server_poll(server, ticket, ctypes.byref(done), ctypes.byref(r)))
    return (_result_dict(r) if done.value else None)


def jp_server_wait(server: int, ticket: int) -> Dict[str, float]:
    r = jp_query_result()
    _check(lib.jp_server_wait(server, ticket, ctypes.byref(r)))
    return _result_dict(r)


def jp_server_stats(server: int) -> Dict[str, float]:
    s = jp_server_summary()
    _check(lib.jp_server_stats(server, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in jp_server_summary._fields_}


def jp_server_materialize(server: int, ticket: int, part: int, first: int, max_pairs: int, out_x, out_z,
                          stream=None) -> int:
    n = ctypes.c_int64()
    _check(lib.jp_server_materialize(server, ticket, part, first, max_pairs, _ptr(out_x), _ptr(out_z),
                                     ctypes.byref(n), _stream(stream)))
    return n.value


def jp_server_release(server: int, ticket: int):
    _check(lib.jp_server_release(server, ticket))


def jp_server_destroy(server: int):
    lib.jp_server_destroy(server)


# ---------------------------------------------------------------- digest


def jp_digest_pairs(out_x, out_z, n: int, acc, stream=None):
    """acc (a one-element int64 device tensor, read as uint64) += digest of the first n pairs."""
    import torch

    if not isinstance(acc, torch.Tensor) or acc.dtype != torch.int64 or not acc.is_cuda or acc.numel() < 1:
        raise TypeError("acc must be an int64 tensor on a ROCm device")
    _check(lib.jp_digest_pairs(_ptr(out_x), _ptr(out_z), n, acc.data_ptr(), _stream(stream)))


# ------------------------------------------------------------ dictionaries


def jp_dict_create(parts: Sequence[Sequence], stream=None) -> Tuple[int, list]:
    """Encode the row tuples of several parts (each a list of equal-length int32
    device columns, the same number of columns in every part) with one
    dictionary.  Returns (handle, [ids of each part as an int32 device tensor])."""
    import torch

    n_cols = len(parts[0])
    if any(len(p) != n_cols for p in parts):
        raise ValueError("every part needs the same number of columns")
    cols = (ctypes.c_void_p * (n_cols * len(parts)))()
    ns = (ctypes.c_int64 * len(parts))()
    ids_t = []
    ids = (ctypes.c_void_p * len(parts))()
    for p, part in enumerate(parts):
        n = int(part[0].numel())
        ns[p] = n
        for c, col in enumerate(part):
            if int(col.numel()) != n:
                raise ValueError("columns of a part differ in length")
            cols[p * n_cols + c] = _ptr(col)
        t = torch.empty(max(n, 1), dtype=torch.int32, device=part[0].device)
        ids_t.append(t[:n])
        ids[p] = _ptr(t)
    h = ctypes.c_void_p()
    _check(lib.jp_dict_create(n_cols, len(parts), cols, ns, ids, _stream(stream), ctypes.byref(h)))
    return h.value, ids_t


def jp_dict_size(d: int) -> int:
    n = ctypes.c_int64()
    _check(lib.jp_dict_size(d, ctypes.byref(n)))
    return n.value


def jp_dict_decode(d: int, ids, n_cols: int, stream=None) -> list:
    """The tuples of the given ids as n_cols int32 device tensors."""
    import torch

    n = int(ids.numel())
    out = [torch.empty(max(n, 1), dtype=torch.int32, device=ids.device) for _ in range(n_cols)]
    arr = (ctypes.c_void_p * n_cols)(*[_ptr(t) for t in out])
    _check(lib.jp_dict_decode(d, _ptr(ids) if n else None, n, arr, _stream(stream)))
    return [t[:n] for t in out]


def jp_dict_destroy(d: int):
    lib.jp_dict_destroy(d)


# ---------------------------------------------------------- Join-Aggregate


def _ptr_any(t) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError("outputs must be contiguous tensors on a ROCm device")
    return t.data_ptr()


def jp_agg_create(r_x, r_y, r_v, s_z, s_y, s_u, stream=None) -> int:
    n_r, n_s = int(r_x.numel()), int(s_z.numel())
    if int(r_y.numel()) != n_r or int(r_v.numel()) != n_r or int(s_y.numel()) != n_s or int(s_u.numel()) != n_s:
        raise ValueError("column lengths differ")
    h = ctypes.c_void_p()
    _check(lib.jp_agg_create(_ptr(r_x), _ptr(r_y), _ptr(r_v), n_r, _ptr(s_z), _ptr(s_y), _ptr(s_u), n_s,
                             _stream(stream), ctypes.byref(h)))
    return h.value


def jp_agg_execute(a: int, stream=None):
    _check(lib.jp_agg_execute(a, _stream(stream)))


def jp_agg_count(a: int, stream=None) -> Tuple[int, int]:
    g, oj = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.jp_agg_count(a, ctypes.byref(g), ctypes.byref(oj), _stream(stream)))
    return g.value, oj.value


def jp_agg_materialize(a: int, first: int, max_groups: int, out_x, out_z, out_count, out_sum, stream=None) -> int:
    n = ctypes.c_int64()
    _check(lib.jp_agg_materialize(a, first, max_groups, _ptr(out_x), _ptr(out_z), _ptr_any(out_count),
                                  _ptr_any(out_sum), ctypes.byref(n), _stream(stream)))
    return n.value


def jp_agg_destroy(a: int):
    lib.jp_agg_destroy(a)


# ------------------------------------------------------ partial result cache


def jp_cache_build(plan: int, budget_bytes: int, stream=None) -> int:
    h = ctypes.c_void_p()
    _check(lib.jp_cache_build(plan, budget_bytes, _stream(stream), ctypes.byref(h)))
    return h.value


def jp_cache_info(cache: int) -> Dict[str, int]:
    nz, pairs, words = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.jp_cache_info(cache, ctypes.byref(nz), ctypes.byref(pairs), ctypes.byref(words)))
    return {"n_z": nz.value, "pairs": pairs.value, "words": words.value}


def jp_cache_z(cache: int) -> np.ndarray:
    n = jp_cache_info(cache)["n_z"]
    z = np.zeros(max(n, 1), dtype=np.int32)
    _check(lib.jp_cache_z(cache, z.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return z[:n]


def jp_plan_create_cached(r_x, r_y, s_z, s_y, cache: int, opt: Optional[jp_options] = None, stream=None) -> int:
    h = ctypes.c_void_p()
    _check(lib.jp_plan_create_cached(_ptr(r_x), _ptr(r_y), int(r_x.numel()), _ptr(s_z), _ptr(s_y),
                                     int(s_z.numel()), cache, ctypes.byref(opt) if opt is not None else None,
                                     _stream(stream), ctypes.byref(h)))
    return h.value


def jp_cache_materialize(cache: int, first: int, max_pairs: int, out_x, out_z, stream=None) -> int:
    n = ctypes.c_int64()
    _check(lib.jp_cache_materialize(cache, first, max_pairs, _ptr(out_x), _ptr(out_z), ctypes.byref(n),
                                    _stream(stream)))
    return n.value


def jp_cache_destroy(cache: int):
    lib.jp_cache_destroy(cache)
