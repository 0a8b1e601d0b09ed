"""Allocation and call sequencing over libglint (no arithmetic of its own).

Each helper allocates device tensors with torch and calls the C entry points
in ``_lib`` on the current stream; every value is computed by the library's
kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib as L
from ._lib import NdfDesc

_DEV = "cuda"


def desc_of(nu, nv, nlevels, nbins, sigma) -> NdfDesc:
    return NdfDesc.make(nu, nv, nlevels, nbins, sigma)


def _dev(x, dtype):
    if isinstance(x, torch.Tensor):
        return x.to(device=_DEV, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=_DEV)


def texel_bins(nxy, desc: NdfDesc):
    """Centre bins int32 [nu*nv*2] and window masses float64 [nu*nv*2*(2K+1)]."""
    nxy = _dev(nxy, torch.float32)
    K = L.glint_window_radius(desc)
    n2 = desc.nu * desc.nv * 2
    bins = torch.empty(n2, dtype=torch.int32, device=_DEV)
    mass = torch.empty(n2 * (2 * K + 1), dtype=torch.float64, device=_DEV)
    L.glint_texel_bins(desc, nxy, bins, mass)
    return bins, mass


def build_tensor(nxy, desc: NdfDesc, dtype=torch.float32, direct_levels: int = 0, out=None):
    """T[u][v][l][s][t] on the GPU."""
    nxy = _dev(nxy, torch.float32)
    shape = (desc.nu, desc.nv, desc.nlevels, desc.nbins, desc.nbins)
    T = torch.empty(shape, dtype=dtype, device=_DEV) if out is None else out
    ws = torch.empty(L.glint_build_tensor_workspace(desc), dtype=torch.uint8, device=_DEV)
    L.glint_build_tensor(desc, nxy, T, direct_levels, ws)
    return T


def range_bruteforce(nxy, desc: NdfDesc, q, bins_mass=None):
    """Exact box sums of the brute-force NDF for each query (FP64)."""
    bins, mass = texel_bins(nxy, desc) if bins_mass is None else bins_mass
    q = _dev(q, torch.int32)
    out = torch.empty(q.shape[0], dtype=torch.float64, device=_DEV)
    L.glint_range_bruteforce(desc, bins, mass, q, out)
    return out


@dataclasses.dataclass
class AlsResult:
    factors: tuple          # (U, V, L*lambda, S, T) FP64 device tensors
    fits: torch.Tensor      # [iters] FP64
    info: torch.Tensor      # int32 [4]: sweeps run, non-PD Gram updates, 0, 0


def als_workspace(desc: NdfDesc, R: int, T_dtype) -> torch.Tensor:
    n = L.glint_cp_als_workspace(desc, R, L.DTYPE_OF[T_dtype])
    if n == 0:
        raise ValueError("unsupported ALS configuration")
    return torch.empty(n, dtype=torch.uint8, device=_DEV)


def cp_als(T: torch.Tensor, desc: NdfDesc, init, iters: int, tol: float = 0.0,
           workspace=None) -> AlsResult:
    R = int(init[0].shape[1])
    F = tuple(_dev(a, torch.float64).clone() for a in init)
    fits = torch.zeros(iters, dtype=torch.float64, device=_DEV)
    info = torch.zeros(4, dtype=torch.int32, device=_DEV)
    ws = als_workspace(desc, R, T.dtype) if workspace is None else workspace
    L.glint_cp_als(desc, T, R, iters, tol, *F, fits, info, ws)
    return AlsResult(F, fits, info)


def mttkrp(T: torch.Tensor, desc: NdfDesc, factors, mode: int, workspace=None):
    """MTTKRP of one mode (FP64 [rows][R]) with the ALS matrix-core passes."""
    R = int(factors[0].shape[1])
    F = tuple(_dev(a, torch.float64) for a in factors)
    rows = (desc.nu, desc.nv, desc.nlevels, desc.nbins, desc.nbins)[mode]
    M = torch.empty((rows, R), dtype=torch.float64, device=_DEV)
    ws = als_workspace(desc, R, T.dtype) if workspace is None else workspace
    L.glint_mttkrp(desc, T, R, mode, *F, M, ws)
    return M


def texel_workspace(desc: NdfDesc, R: int) -> torch.Tensor:
    n = L.glint_cp_als_texel_workspace(desc, R)
    if n == 0:
        raise ValueError("unsupported texel-space ALS configuration")
    return torch.empty(n, dtype=torch.uint8, device=_DEV)


def mttkrp_texel(nxy, desc: NdfDesc, factors, mode: int, workspace=None):
    """MTTKRP of one mode evaluated from the normal map (T never formed)."""
    R = int(factors[0].shape[1])
    F = tuple(_dev(a, torch.float64) for a in factors)
    rows = (desc.nu, desc.nv, desc.nlevels, desc.nbins, desc.nbins)[mode]
    M = torch.empty((rows, R), dtype=torch.float64, device=_DEV)
    ws = texel_workspace(desc, R) if workspace is None else workspace
    L.glint_mttkrp_texel(desc, _dev(nxy, torch.float32), R, mode, *F, M, ws)
    return M


def cp_als_texel(nxy, desc: NdfDesc, init, iters: int, tol: float = 0.0, normT2: float = 0.0,
                 workspace=None) -> AlsResult:
    """CP-ALS from the normal map; fits are NaN unless ||T||^2 is supplied."""
    R = int(init[0].shape[1])
    F = tuple(_dev(a, torch.float64).clone() for a in init)
    fits = torch.zeros(iters, dtype=torch.float64, device=_DEV)
    info = torch.zeros(4, dtype=torch.int32, device=_DEV)
    ws = texel_workspace(desc, R) if workspace is None else workspace
    L.glint_cp_als_texel(desc, _dev(nxy, torch.float32), R, iters, tol, normT2, *F, fits, info, ws)
    return AlsResult(F, fits, info)


# ----------------------------------------------------------------------------
# query tables
# ----------------------------------------------------------------------------

_STORE = {"f32": torch.float32, "bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn,
          "f64": torch.float64}


@dataclasses.dataclass
class QueryTables:
    U: torch.Tensor
    V: torch.Tensor
    L: torch.Tensor
    CS: torch.Tensor
    CT: torch.Tensor
    scales: tuple           # five per-column FP32 scales or None

    def factors(self) -> L.Factors:
        return L.make_factors(self.U, self.V, self.L, self.CS, self.CT, self.scales)

    @property
    def R(self):
        return self.U.shape[1]


def convert(x, dtype: str):
    """Store a factor table as f32, bf16 or fp8 (+ per-column scales)."""
    x = x if isinstance(x, torch.Tensor) and x.is_cuda else _dev(x, torch.float64)
    if x.dtype not in (torch.float64, torch.float32):
        x = x.to(torch.float64)
    out = torch.empty(x.shape, dtype=_STORE[dtype], device=_DEV)
    sc = torch.empty(x.shape[1], dtype=torch.float32, device=_DEV) if dtype == "fp8" else None
    L.glint_convert(x.contiguous(), out, sc)
    return out, sc


def cumulative(S, dtype: str = "f32"):
    """Summed-area table [N+1][R] of S (FP64 accumulation) in a storage type."""
    S = S if isinstance(S, torch.Tensor) and S.is_cuda else _dev(S, torch.float64)
    if S.dtype not in (torch.float64, torch.float32):
        S = S.to(torch.float64)
    C = torch.empty((S.shape[0] + 1, S.shape[1]), dtype=_STORE[dtype], device=_DEV)
    sc = torch.empty(S.shape[1], dtype=torch.float32, device=_DEV) if dtype == "fp8" else None
    L.glint_make_cumulative(S.contiguous(), C, sc)
    return C, sc


def make_tables(U, V, Lf, S, Tf, dtype: str = "f32", cum_dtype: str = "f32") -> QueryTables:
    u, su = convert(U, dtype)
    v, sv = convert(V, dtype)
    l, sl = convert(Lf, dtype)
    cs, scs = cumulative(S, cum_dtype)
    ct, sct = cumulative(Tf, cum_dtype)
    return QueryTables(u, v, l, cs, ct, (su, sv, sl, scs, sct))


def query(tables: QueryTables, q, out=None):
    q = _dev(q, torch.int32)
    out = torch.empty(q.shape[0], dtype=torch.float32, device=_DEV) if out is None else out
    f = tables.factors()
    L.glint_query(f, q, out)
    return out


def query_grouped(tables: QueryTables, uvl, boxes, out=None):
    uvl = _dev(uvl, torch.int32)
    boxes = _dev(boxes, torch.int32)
    out = (torch.empty(boxes.shape[0], boxes.shape[1], dtype=torch.float32, device=_DEV)
           if out is None else out)
    f = tables.factors()
    L.glint_query_grouped(f, uvl, boxes, out)
    return out


def query_trilinear(tables: QueryTables, xyl, boxes, out=None):
    """Trilinear off-grid footprints: xyl float [nq][3] (x, y, level), boxes int [nq][4]."""
    xyl = _dev(xyl, torch.float32)
    boxes = _dev(boxes, torch.int32)
    out = torch.empty(xyl.shape[0], dtype=torch.float32, device=_DEV) if out is None else out
    L.glint_query_trilinear(tables.factors(), xyl, boxes, out)
    return out


def sample(tables: QueryTables, uvl, rnd):
    """Hierarchical importance samples: (h [n][2], pdf [n], bins [n][2])."""
    uvl = _dev(uvl, torch.int32)
    rnd = _dev(rnd, torch.float32)
    n = uvl.shape[0]
    levels = int(tables.CS.shape[0] - 1).bit_length() - 1
    if rnd.shape != (n, levels + 2):
        raise ValueError(f"rnd must be [n][{levels + 2}]")
    h = torch.empty((n, 2), dtype=torch.float32, device=_DEV)
    pdf = torch.empty(n, dtype=torch.float32, device=_DEV)
    bins = torch.empty((n, 2), dtype=torch.int32, device=_DEV)
    L.glint_sample(tables.factors(), uvl, rnd, h, pdf, bins)
    return h, pdf, bins


def query_sg(tables: QueryTables, uvl, h, sg, eps: float = 0.3):
    """Environment-light prefiltered lookups (Sec. 5.4): the average bin mass
    over each lookup's compact-eps box; returns (average [n], records [n][7])."""
    uvl = _dev(uvl, torch.int32)
    h = _dev(h, torch.float32)
    sg = _dev(sg, torch.float32)
    n = uvl.shape[0]
    q = torch.empty((n, 7), dtype=torch.int32, device=_DEV)
    out = torch.empty(n, dtype=torch.float32, device=_DEV)
    L.glint_query_sg(tables.factors(), uvl, h, sg, eps, q, out)
    return out, q


def validate_queries(tables: QueryTables, q) -> int:
    """Number of records the query's wrap/clamp rules would change."""
    q = _dev(q, torch.int32)
    nbad = torch.empty(1, dtype=torch.int64, device=_DEV)
    L.glint_validate_queries(tables.factors(), q, nbad)
    return int(nbad.item())


def query_backward(tables: QueryTables, q, gout):
    """Gradients (dU, dV, dL, dCS, dCT) of sum gout * q w.r.t. the stored tables."""
    R = tables.R
    z = lambda rows: torch.empty((rows, R), dtype=torch.float32, device=_DEV)
    dU, dV, dLt = z(tables.U.shape[0]), z(tables.V.shape[0]), z(tables.L.shape[0])
    dCS, dCT = z(tables.CS.shape[0]), z(tables.CT.shape[0])
    L.glint_query_backward(tables.factors(), _dev(q, torch.int32), gout.contiguous(),
                           dU, dV, dLt, dCS, dCT)
    return dU, dV, dLt, dCS, dCT


def cumulative_backward(dC):
    dS = torch.empty((dC.shape[0] - 1, dC.shape[1]), dtype=torch.float32, device=_DEV)
    L.glint_cumulative_backward(dC.contiguous(), dS)
    return dS


@dataclasses.dataclass
class ClusteredTables:
    """Per-(region, block) CP factors of the clustered layout (Sec. 4.2) and
    their block-local summed-area tables, FP32 on the device.  X, Y
    [ntensor][t][R], Z [ntensor][L][R] (weights absorbed), CX, CY
    [ntensor][t+1][R]; tensor = ((cu * ncv + cv) * nb + zs) * nb + zt."""
    desc: NdfDesc
    t: int
    cs: int
    X: torch.Tensor
    Y: torch.Tensor
    Z: torch.Tensor
    blank: torch.Tensor
    info: torch.Tensor
    CX: torch.Tensor = None
    CY: torch.Tensor = None
    zidx: torch.Tensor = None      # compact layout: [ntensor][L] row of Z or -1
    zbase: torch.Tensor = None     # compact layout: first row of each tensor, then the row count
    dtype: str = "f32"             # element type of CX, CY and Z as the query reads them

    @property
    def R(self):
        return self.X.shape[-1]

    def shape(self):
        d = self.desc
        return d.nu // self.cs, d.nv // self.cs, d.nbins // self.t

    def struct(self) -> L.Clustered:
        d = self.desc
        et = _STORE[self.dtype]
        return L.Clustered(self.t, self.cs, self.R, d.nu, d.nv, d.nlevels, d.nbins,
                           L._ptr(self.CX, et, "CX"), L._ptr(self.CY, et, "CY"),
                           L._ptr(self.Z, et, "Z"), L._ptr(self.zidx, torch.int32, "zidx"),
                           L._gdtype_of(et))

    def dense_z(self) -> torch.Tensor:
        """Z as [ntensor][L][R] with zero rows for blank image blocks."""
        if self.zidx is None:
            return self.Z
        n, Lr = self.zidx.shape
        out = torch.zeros((n * Lr, self.R), dtype=torch.float32, device=self.Z.device)
        keep = self.zidx.reshape(-1) >= 0
        out[keep] = self.Z[self.zidx.reshape(-1)[keep].long()]
        return out.reshape(n, Lr, self.R)


def cp_als_clustered(T: torch.Tensor, desc: NdfDesc, t: int, cs: int, R: int, iters: int,
                     seed: int = 0) -> ClusteredTables:
    """Clustered-layout CP of the built tensor T (F64 or F32) and its query
    tables.  `t` is the angular block side (min(t, nbins) is used), `cs`
    the region side in texels."""
    t = min(int(t), desc.nbins)
    ncu, ncv, nb = desc.nu // cs, desc.nv // cs, desc.nbins // t
    ntensor = ncu * ncv * nb * nb
    Lr = cs * cs * desc.nlevels
    f32 = dict(dtype=torch.float32, device=_DEV)
    X = torch.empty((ntensor, t, R), **f32)
    Y = torch.empty((ntensor, t, R), **f32)
    Z = torch.empty((ntensor, Lr, R), **f32)
    blank = torch.empty(ntensor, dtype=torch.uint8, device=_DEV)
    info = torch.empty(4, dtype=torch.int32, device=_DEV)
    L.glint_cp_als_clustered(desc, L.ClusterDesc(t, int(cs), int(R)), T.contiguous(), iters, seed,
                             X, Y, Z, blank, info)
    tab = ClusteredTables(desc, t, int(cs), X, Y, Z, blank, info)
    clustered_cumulative(tab)
    return tab


def cp_als_clustered_map(nxy: torch.Tensor, desc: NdfDesc, t: int, cs: int, R: int, iters: int,
                         seed: int = 0, dtype=torch.float32) -> ClusteredTables:
    """Clustered-layout CP straight from the normal map (no stored T): each
    angular block's tensor is built in `dtype` (F32 or F64) and fitted in
    turn; Z is compact (`zidx` gives each footprint's row)."""
    t = min(int(t), desc.nbins)
    ncu, ncv, nb = desc.nu // cs, desc.nv // cs, desc.nbins // t
    ntensor = ncu * ncv * nb * nb
    Lr = cs * cs * desc.nlevels
    cd = L.ClusterDesc(t, int(cs), int(R))
    ws = torch.empty(L.glint_cluster_map_workspace(desc, cd, dtype), dtype=torch.uint8, device=_DEV)
    nxy = nxy.to(_DEV, torch.float32).contiguous()
    zidx = torch.empty((ntensor, Lr), dtype=torch.int32, device=_DEV)
    zbase = torch.empty(ntensor + 1, dtype=torch.int64, device=_DEV)
    info = torch.empty(4, dtype=torch.int32, device=_DEV)
    L.glint_cluster_map_index(desc, cd, nxy, dtype, zidx, zbase, info, ws)
    rows = int(zbase[-1].item())
    f32 = dict(dtype=torch.float32, device=_DEV)
    X = torch.empty((ntensor, t, R), **f32)
    Y = torch.empty((ntensor, t, R), **f32)
    Z = torch.empty((max(rows, 1), R), **f32)
    blank = torch.empty(ntensor, dtype=torch.uint8, device=_DEV)
    L.glint_cp_als_clustered_map(desc, cd, nxy, dtype, iters, seed, zidx, X, Y, Z, blank, info, ws)
    del ws
    tab = ClusteredTables(desc, t, int(cs), X, Y, Z, blank, info, zidx=zidx, zbase=zbase)
    clustered_cumulative(tab)
    return tab


def clustered_cumulative(tab: ClusteredTables):
    """(Re)build the block-local summed-area tables CX, CY of `tab`."""
    n, t, R = tab.X.shape
    if tab.CX is None:
        tab.CX = torch.empty((n, t + 1, R), dtype=torch.float32, device=_DEV)
        tab.CY = torch.empty((n, t + 1, R), dtype=torch.float32, device=_DEV)
    L.glint_make_cumulative_batched(tab.X, tab.CX)
    L.glint_make_cumulative_batched(tab.Y, tab.CY)
    return tab


def clustered_bf16(tab: ClusteredTables) -> ClusteredTables:
    """The query tables of `tab` stored in BF16 (Sec. 4.4 storage): CX, CY
    and Z, each FP32 value rounded to nearest even by the library
    (glint_convert); X, Y, blank, zidx shared with `tab`.  Read by
    query_clustered; sampling takes the FP32 tables."""
    if tab.dtype != "f32":
        raise ValueError("clustered_bf16 converts FP32 tables")

    def bf(x):
        out = torch.empty(x.shape, dtype=torch.bfloat16, device=_DEV)
        L.glint_convert(x.reshape(-1, x.shape[-1]), out.view(-1, x.shape[-1]))
        return out

    return dataclasses.replace(tab, CX=bf(tab.CX), CY=bf(tab.CY), Z=bf(tab.Z), dtype="bf16")


def sample_clustered(tab: ClusteredTables, uvl, rnd):
    """Hierarchical importance samples on the clustered tables (block by mass,
    then quads): (h [n][2], pdf [n], bins [n][2]); rnd [n][log2(t) + 3]."""
    uvl = _dev(uvl, torch.int32)
    rnd = _dev(rnd, torch.float32)
    n = uvl.shape[0]
    levels = int(tab.t).bit_length() - 1
    if tuple(rnd.shape) != (n, levels + 3):
        raise ValueError(f"rnd must be [n][{levels + 3}]")
    h = torch.empty((n, 2), dtype=torch.float32, device=_DEV)
    pdf = torch.empty(n, dtype=torch.float32, device=_DEV)
    bins = torch.empty((n, 2), dtype=torch.int32, device=_DEV)
    L.glint_sample_clustered(tab.struct(), uvl, rnd, h, pdf, bins)
    return h, pdf, bins


def query_clustered(tab: ClusteredTables, q, out=None):
    q = _dev(q, torch.int32)
    out = torch.empty(q.shape[0], dtype=torch.float32, device=_DEV) if out is None else out
    L.glint_query_clustered(tab.struct(), q, out)
    return out


@dataclasses.dataclass
class WangTables:
    """Per-tile CP tables of a Wang-tile set (Sec. 5.5), FP32 on the device,
    stacked by tile: U, V [ntiles][S+2m][R], L [ntiles][nl][R],
    CS, CT [ntiles][N+1][R]."""
    S: int
    m: int
    seed: int
    edge_to_tile: tuple
    U: torch.Tensor
    V: torch.Tensor
    L: torch.Tensor
    CS: torch.Tensor
    CT: torch.Tensor

    def struct(self) -> L.Wang:
        ntiles, _, R = self.U.shape
        etl = (ctypes.c_uint8 * 16)(*[int(e) for e in self.edge_to_tile])
        return L.Wang(ntiles, self.S, self.m, R, self.L.shape[1], self.CS.shape[1] - 1, int(self.seed) & ((1 << 64) - 1),
                      etl, L._ptr(self.U, torch.float32, "U"), L._ptr(self.V, torch.float32, "V"),
                      L._ptr(self.L, torch.float32, "L"), L._ptr(self.CS, torch.float32, "CS"),
                      L._ptr(self.CT, torch.float32, "CT"))


def wang_tables(tile_factors, S: int, m: int, seed: int, edge_to_tile) -> WangTables:
    """Stack the CP factors (U, V, L, S, T) of every tile (each fitted on the
    tile padded with m absent texels) into query tables."""
    def stack(i):
        f64 = torch.stack([_dev(f[i], torch.float64) for f in tile_factors]).contiguous()
        out = torch.empty(f64.shape, dtype=torch.float32, device=_DEV)
        L.glint_convert(f64.view(-1, f64.shape[-1]), out.view(-1, f64.shape[-1]))
        return out
    U, V, Lf, Sf, Tf = (stack(i) for i in range(5))
    ntiles, N, R = Sf.shape
    CS = torch.empty((ntiles, N + 1, R), dtype=torch.float32, device=_DEV)
    CT = torch.empty((ntiles, N + 1, R), dtype=torch.float32, device=_DEV)
    L.glint_make_cumulative_batched(Sf, CS)
    L.glint_make_cumulative_batched(Tf, CT)
    return WangTables(int(S), int(m), int(seed), tuple(int(e) for e in edge_to_tile), U, V, Lf, CS, CT)


def query_wang(tab: WangTables, q, out=None):
    """Range queries at plane coordinates on the Wang-tile synthesized map."""
    q = _dev(q, torch.int32)
    out = torch.empty(q.shape[0], dtype=torch.float32, device=_DEV) if out is None else out
    L.glint_query_wang(tab.struct(), q, out)
    return out
