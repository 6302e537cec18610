"""Small object wrappers over the C ABI (marshalling only)."""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

from . import binding as B


class Plan:
    """One planned query; frees its device memory on close()."""

    def __init__(self, r_x, r_y, s_z, s_y, opt: Optional[B.jp_options] = None, stream=None):
        self.stream = stream
        self.h = B.jp_plan_create(r_x, r_y, s_z, s_y, opt, stream)

    def execute(self):
        B.jp_execute(self.h, self.stream)
        return self

    def count(self) -> Tuple[int, int, int]:
        return B.jp_count(self.h, self.stream)

    def stats(self):
        return B.jp_plan_stats(self.h)

    def materialize(self, part: int = B.JP_PART_ALL, first: int = 0, max_pairs: Optional[int] = None,
                    out=None):
        """Pairs [first, first + max_pairs) of the sorted result as two int32 device tensors."""
        import torch

        total = self.count()[part]
        if max_pairs is None:
            max_pairs = max(0, total - first)
        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device())
            out = (torch.empty(max(max_pairs, 1), dtype=torch.int32, device=dev),
                   torch.empty(max(max_pairs, 1), dtype=torch.int32, device=dev))
        n = B.jp_materialize(self.h, part, first, max_pairs, out[0], out[1], self.stream)
        return out[0][:n], out[1][:n]

    def row_info(self, part: int = B.JP_PART_ALL):
        return B.jp_row_info(self.h, part, self.stream)

    def dense_z(self):
        return B.jp_dense_z(self.h, self.stream)

    def close(self):
        if self.h:
            B.jp_plan_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent queries planned and executed together."""

    def __init__(self, cols: Sequence[Tuple], opt: Optional[B.jp_options] = None, stream=None):
        self.stream = stream
        self.n = len(cols)
        self.h = B.jp_batch_create(cols, opt, stream)

    def execute(self):
        B.jp_batch_execute(self.h, self.stream)
        return self

    def counts(self):
        return B.jp_batch_counts(self.h, self.n, self.stream)

    def stats(self, i: int):
        return B.jp_batch_stats(self.h, i)

    def materialize(self, i: int, part: int = B.JP_PART_ALL, first: int = 0, max_pairs: Optional[int] = None):
        import torch

        total = int(self.counts()[i]) if part == B.JP_PART_ALL else None
        if max_pairs is None:
            if total is None:
                raise ValueError("max_pairs is required for a single part of a batch instance")
            max_pairs = max(0, total - first)
        dev = torch.device("cuda", torch.cuda.current_device())
        ox = torch.empty(max(max_pairs, 1), dtype=torch.int32, device=dev)
        oz = torch.empty(max(max_pairs, 1), dtype=torch.int32, device=dev)
        n = B.jp_batch_materialize(self.h, i, part, first, max_pairs, ox, oz, self.stream)
        return ox[:n], oz[:n]

    def close(self):
        if self.h:
            B.jp_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def join_project(r_x, r_y, s_z, s_y, opt: Optional[B.jp_options] = None, stream=None):
    """Plan, execute and materialise the whole sorted result (small inputs)."""
    with Plan(r_x, r_y, s_z, s_y, opt, stream) as p:
        p.execute()
        return p.materialize()


class Aggregate:
    """Join-Aggregate G_{x,z} COUNT(*), SUM(R.v * S.u) (jp_agg_* in include/jp.h)."""

    def __init__(self, r_x, r_y, r_v, s_z, s_y, s_u, stream=None):
        self.stream = stream
        self.h = B.jp_agg_create(r_x, r_y, r_v, s_z, s_y, s_u, stream)

    def execute(self):
        B.jp_agg_execute(self.h, self.stream)
        return self

    def count(self):
        """(number of groups, number of join rows)."""
        return B.jp_agg_count(self.h, self.stream)

    def materialize(self, first: int = 0, max_groups: Optional[int] = None):
        """Groups [first, first + max_groups) as (x, z, count, sum) device tensors."""
        import torch

        groups = self.count()[0]
        if max_groups is None:
            max_groups = max(0, groups - first)
        dev = torch.device("cuda", torch.cuda.current_device())
        m = max(max_groups, 1)
        ox = torch.empty(m, dtype=torch.int32, device=dev)
        oz = torch.empty(m, dtype=torch.int32, device=dev)
        oc = torch.empty(m, dtype=torch.int64, device=dev)
        osum = torch.empty(m, dtype=torch.int64, device=dev)
        n = B.jp_agg_materialize(self.h, first, max_groups, ox, oz, oc, osum, self.stream)
        return ox[:n], oz[:n], oc[:n], osum[:n]

    def close(self):
        if self.h:
            B.jp_agg_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Dict:
    """Dictionary of multi-column key tuples (jp_dict_* in include/jp.h)."""

    def __init__(self, parts: Sequence[Sequence], stream=None):
        self.stream = stream
        self.n_cols = len(parts[0])
        self.h, self.ids = B.jp_dict_create(parts, stream)

    def size(self) -> int:
        return B.jp_dict_size(self.h)

    def decode(self, ids):
        return B.jp_dict_decode(self.h, ids, self.n_cols, self.stream)

    def close(self):
        if self.h:
            B.jp_dict_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def join_project_composite(r_x: Sequence, r_y: Sequence, s_z: Sequence, s_y: Sequence,
                           opt: Optional[B.jp_options] = None, stream=None):
    """Join-Project over multi-attribute keys: x is the tuple of the r_x columns,
    y the tuple of the join columns (r_y and s_y, same arity), z the tuple of the
    s_z columns (lists of int32 device tensors).  Each kind is dictionary-encoded
    (R.y and S.y in one dictionary), the plan runs on the ids, and the id pairs
    are decoded.  Returns (x columns, z columns) of the distinct pairs, sorted
    lexicographically by (x tuple, z tuple)."""
    with Dict([r_x], stream) as dx, Dict([r_y, s_y], stream) as dy, Dict([s_z], stream) as dz:
        with Plan(dx.ids[0], dy.ids[0], dz.ids[0], dy.ids[1], opt, stream) as p:
            p.execute()
            ix, iz = p.materialize()
            return dx.decode(ix), dz.decode(iz)


class Server:
    """Continuous-batching query server, see jp_server_* in include/jp.h."""

    def __init__(self, device: int = 0, max_batch: int = 0, hbm_budget_bytes: int = 0,
                 opt: Optional[B.jp_options] = None, flags: int = 0, chunk_pairs: int = 0):
        self.h = B.jp_server_create(device, max_batch, hbm_budget_bytes, opt, flags, chunk_pairs)
        self._keep = {}

    def submit(self, r_x, r_y, s_z, s_y) -> int:
        t = B.jp_server_submit(self.h, r_x, r_y, s_z, s_y)
        self._keep[t] = (r_x, r_y, s_z, s_y)  # device columns stay alive until the query is done
        return t

    def poll(self, ticket: int):
        r = B.jp_server_poll(self.h, ticket)
        if r is not None:
            self._keep.pop(ticket, None)
        return r

    def wait(self, ticket: int):
        r = B.jp_server_wait(self.h, ticket)
        self._keep.pop(ticket, None)
        return r

    def materialize(self, ticket: int, total: int, part: int = B.JP_PART_ALL, first: int = 0,
                    max_pairs: Optional[int] = None):
        """Pairs [first, first + max_pairs) of a kept result as two device tensors."""
        import torch

        n = total - first if max_pairs is None else min(max_pairs, max(total - first, 0))
        ox = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        oz = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        w = B.jp_server_materialize(self.h, ticket, part, first, n, ox, oz)
        return ox[:w], oz[:w]

    def release(self, ticket: int):
        B.jp_server_release(self.h, ticket)

    def stats(self):
        return B.jp_server_stats(self.h)

    def close(self):
        if self.h:
            B.jp_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
