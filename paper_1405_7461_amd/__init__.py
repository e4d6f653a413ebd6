"""Distance-threshold search over trajectory segments, native on MI355X.

The search itself runs in libtds.so (hand-written HIP for gfx950); this
package is its Python binding. See include/tds.h for the C ABI.
"""
from .api import (  # noqa: F401
    Hits,
    Index,
    NativeServer,
    Prepared,
    Query,
    TrajHits,
    build_index,
    fetch_results,
    plan_bins,
    plan_ranges,
    point_segments,
    prepare,
    query_batch,
    search,
    search_noalloc,
    use_torch_allocator,
)
from ._lib import TdsError, lib  # noqa: F401
