"""glint on MI355X: constant-cost spatio-angular range queries of a glint P-NDF
compressed by CP decomposition (Deng et al., "Constant-Cost Spatio-Angular
Prefiltering of Glinty Appearance Using Tensor Decomposition").

The compute path is libglint.so (C ABI in include/glint.h, HIP kernels for
gfx950 under csrc/); this package only binds it.  Build it in-tree with
``python -m paper_2109_14807_amd.build``.
"""
from . import _lib  # noqa: F401
from ._lib import GlintError, NdfDesc  # noqa: F401
from .api import (  # noqa: F401
    AlsResult, ClusteredTables, QueryTables, als_workspace, clustered_bf16, clustered_cumulative, cp_als_clustered,
    cp_als_clustered_map,
    query_clustered, sample_clustered, build_tensor, convert, cp_als, cumulative, cumulative_backward,
    cp_als_texel, desc_of, make_tables, mttkrp, mttkrp_texel, query, query_backward, query_grouped, query_trilinear,
    query_sg, query_wang, range_bruteforce, validate_queries, sample, texel_bins, texel_workspace, WangTables,
    wang_tables,
)
from .autograd import GlintQuery, glint_query_fn  # noqa: F401
from .refine import refine  # noqa: F401
