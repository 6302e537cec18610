"""MI355X (gfx950) Join-Project PI_{x,z}(R(x,y) JOIN_y S(z,y)) after DIM^3.

The compute path lives in libjp.so (HIP kernels behind the C ABI of
include/jp.h); this package only marshals arguments to it.
"""
from .binding import (  # noqa: F401
    EXPORTS,
    INT64_MAX,
    JP_DENSE_AUTO,
    JP_DENSE_BITS,
    JP_DENSE_MFMA,
    JP_FLAG_TIMING,
    JP_PART_ALL,
    JP_PART_DENSE,
    JP_PART_SPARSE,
    JP_TAU_AUTO,
    JP_TAU_FIXED,
    JpError,
    jp_batch_counts,
    jp_batch_create,
    jp_batch_destroy,
    jp_batch_execute,
    jp_batch_materialize,
    jp_batch_stats,
    jp_count,
    jp_dense_z,
    jp_execute,
    jp_materialize,
    jp_plan_create,
    jp_plan_destroy,
    jp_plan_stats,
    jp_plan_timings,
    jp_plan_work,
    jp_row_info,
    last_error,
    lib,
    make_options,
)
from .api import Plan, Batch, join_project  # noqa: F401
