"""Oracle: constant-storage appearance synthesis with Wang tiles (Sec. 5.5), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed:
  * The plane is a grid of square cells of S texels; cell (i, j) holds the
    texels x in [i S, (i+1) S), y in [j S, (j+1) S) and shows one of the
    precomputed tiles.
  * No index map: vertex (i, j), the top-left corner of cell (i, j), draws
    two numbers from a hash of its index, and each becomes one of two edge
    colours; the first colours the edge to the vertex's right (the top edge
    of cell (i, j)), the second the edge below it (the left edge of cell
    (i, j)).  A cell's four edge colours pick its tile through an
    edge-to-tile map.
  * Each tile's NDF tensor is built with footprint centres reaching m texels
    past the tile on every side, and with only the tile's own texels
    contributing (the rest of the footprint is empty, weight still 1/k^2).
    The NDF of a footprint on the synthesized plane is then the sum, over the
    cells the footprint overlaps, of that cell's tile tensor at the
    footprint's centre in tile coordinates (Fig. wangTiles).
Readings:
  * hash: SplitMix64 used as a counter-based generator (as in the clustered
    layout) with counter ((i mod 2^32) 2^32 + (j mod 2^32)) 2 + e, e = 0 for
    the right edge and 1 for the edge below; colour = 1 if the number is
    >= 1/2, else 0;
  * edge code of cell (i, j) = 8 top + 4 right + 2 bottom + left, with
    top = right-edge colour of vertex (i, j), right = lower-edge colour of
    vertex (i+1, j), bottom = right-edge colour of vertex (i, j+1),
    left = lower-edge colour of vertex (i, j); tile = edge_to_tile[code];
  * a tile's tensor is the tensor of the tile padded with m absent texels
    (non-finite normals) on every side, so footprint centres run over the
    padded (S + 2m)^2 grid; m >= k_max / 2 keeps every overlapping cell's
    local centre inside it and lets toroidal wrap only reach the margins;
  * query records (x, y, l, s_lo, s_hi, t_lo, t_hi) use plane coordinates
    (any integers, no wrap); l and the bins are clamped as for the plain
    query.
"""
from __future__ import annotations

import numpy as np

from .cluster import uniform
from .ndf import box_sum, ndf_bruteforce
from .query import range_query

_M32 = (1 << 32) - 1


def edge_counter(i: int, j: int, e: int) -> int:
    return ((((i & _M32) << 32) | (j & _M32)) << 1 | e) & ((1 << 64) - 1)


def vertex_colours(seed: int, i: int, j: int):
    """(colour of the edge to the right of vertex (i, j), colour of the edge below it)."""
    u = uniform(seed, np.array([edge_counter(i, j, 0), edge_counter(i, j, 1)], dtype=np.uint64))
    return int(u[0] >= 0.5), int(u[1] >= 0.5)


def cell_tile(seed: int, edge_to_tile, i: int, j: int) -> int:
    top, left = vertex_colours(seed, i, j)
    right = vertex_colours(seed, i + 1, j)[1]
    bottom = vertex_colours(seed, i, j + 1)[0]
    return int(edge_to_tile[8 * top + 4 * right + 2 * bottom + left])


def explicit_map(tiles: np.ndarray, seed: int, edge_to_tile, i0: int, ni: int, j0: int, nj: int) -> np.ndarray:
    """The synthesized normal map over cells i0..i0+ni-1, j0..j0+nj-1, assembled explicitly."""
    S = tiles.shape[1]
    out = np.empty((ni * S, nj * S, 2))
    for a in range(ni):
        for b in range(nj):
            out[a * S:(a + 1) * S, b * S:(b + 1) * S] = tiles[cell_tile(seed, edge_to_tile, i0 + a, j0 + b)]
    return out


def padded_tile(tile: np.ndarray, m: int) -> np.ndarray:
    """The tile with m absent texels (NaN normals) on every side."""
    S = tile.shape[0]
    out = np.full((S + 2 * m, S + 2 * m, 2), np.nan)
    out[m:m + S, m:m + S] = tile
    return out


def tile_tensors(tiles: np.ndarray, m: int, nbins: int, sigma: float, nlevels: int):
    return [ndf_bruteforce(padded_tile(t, m), nbins, sigma, nlevels) for t in tiles]


def cells_of(x: int, y: int, l: int, S: int):
    """Cells overlapped by the level-l footprint centred on plane texel (x, y)."""
    k = 1 << l
    x0, y0 = x - k // 2, y - k // 2
    return [(i, j) for i in range(x0 // S, (x0 + k - 1) // S + 1) for j in range(y0 // S, (y0 + k - 1) // S + 1)]


def local_records(q, S: int, m: int, nlevels: int, nbins: int, seed: int, edge_to_tile):
    """Per query, the (tile, local record) pairs of the cells its footprint overlaps."""
    q = np.asarray(q, dtype=np.int64)
    out = []
    for x, y, l, slo, shi, tlo, thi in q:
        l = int(np.clip(l, 0, nlevels - 1))
        box = [int(np.clip(b, 0, nbins)) for b in (slo, shi, tlo, thi)]
        recs = []
        for i, j in cells_of(int(x), int(y), l, S):
            recs.append((cell_tile(seed, edge_to_tile, i, j), [int(x) - i * S + m, int(y) - j * S + m, l] + box))
        out.append(recs)
    return out


def wang_box_sum(tensors, q, S: int, m: int, seed: int, edge_to_tile):
    """Exact NDF box sums on the synthesized plane from the tile tensors."""
    nl, nbins = tensors[0].shape[2], tensors[0].shape[3]
    res = np.zeros(len(q))
    for n, recs in enumerate(local_records(q, S, m, nl, nbins, seed, edge_to_tile)):
        res[n] = sum(float(box_sum(tensors[t], np.array([r]))[0]) for t, r in recs)
    return res


def wang_range_query(factors, q, S: int, m: int, seed: int, edge_to_tile):
    """Range queries on the synthesized plane from per-tile CP factors
    (factors[t] = (U, V, L, CS, CT) of tile t)."""
    nl, nbins = factors[0][2].shape[0], factors[0][3].shape[0] - 1
    res = np.zeros(len(q))
    for n, recs in enumerate(local_records(q, S, m, nl, nbins, seed, edge_to_tile)):
        res[n] = sum(float(range_query(*factors[t], np.array([r]))[0]) for t, r in recs)
    return res
