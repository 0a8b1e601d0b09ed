"""Seeded synthetic inputs for the glint P-NDF range-query path.

This package produces inputs only: normal maps, query batches and the
ALS initial factors.  It performs none of the method's arithmetic (no NDF
masses, no tensor, no decomposition, no query evaluation), so that both
the FP64 CPU oracle and the GPU library can be fed the very same arrays
without sharing any computation.
"""
from .inputs import (  # noqa: F401
    CONFIGS,
    GlintConfig,
    config,
    flake_map,
    scratch_map,
    normal_map,
    make_queries,
    make_grouped_queries,
    als_init,
    map_seed,
    query_seed,
)
