"""Seeded input generators: normal maps, query batches, ALS initial factors.

Every function is a pure function of its arguments (seeds included) and
returns NumPy arrays.  Nothing here evaluates the NDF, the tensor, its
decomposition or a query: these are inputs to both the CPU oracle and the
GPU library.

Workload recipes (the paper's textures and scenes are not available, so
these synthetic maps take their place with the sizes of the configurations):

* Flake map: periodic Voronoi cells ("metallic flakes").  ``nsites``
  sites uniform on the torus; each texel centre takes the nearest site by
  toroidal distance.  Each site draws a Beckmann-distributed normal with
  roughness ``alpha`` by the standard microfacet sampling rule
  (phi = 2*pi*xi1, tan^2(theta) = -alpha^2 * ln(1 - xi2)); the map stores
  the projected normal (n_x, n_y) = sin(theta) * (cos phi, sin phi).
* Scratch map: flat background (projected normal 0) with random line
  segments; a texel within half a width of a segment takes the segment's
  tilted normal sin(tilt) * p, p the in-plane unit vector perpendicular
  to the segment.  Later scratches overwrite earlier ones.
* Query boxes: a footprint centre (u, v), a level l and an angular box in
  projected half-vector space converted to half-open bin ranges.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class GlintConfig:
    name: str
    map_kind: str          # "flake" | "scratch"
    nu: int
    nv: int
    nsites: int            # flakes: Voronoi sites; scratch: segments
    alpha: float           # flake Beckmann roughness (unused for scratches)
    sigma: float           # intrinsic roughness of every texel's Gaussian
    nbins: int             # NDF bins per axis over [-1, 1]
    nlevels: int           # footprint levels, level l is a 2^l x 2^l box
    rank: int
    iters: int             # ALS sweeps
    query_kind: str        # "uniform" | "frame" | "footprints" | "sg_grouped"
    nqueries: int          # total queries (or boxes for grouped)
    side_lo: float
    side_hi: float
    side_log: bool
    boxes_per_point: int = 1
    dtype: str = "f32"     # storage type of the factor tables on the query path
    cum_dtype: str = "f32"

    @property
    def index(self) -> int:
        return int(self.name[1:]) if self.name[1:].isdigit() else 0


CONFIGS = {
    # Plain method at small size; 10^4 uniform queries, box side U[0.02, 0.5].
    "c1": GlintConfig("c1", "flake", 64, 64, 200, 0.10, 0.010, 32, 5, 16, 50,
                      "uniform", 10_000, 0.02, 0.5, False),
    # Plain FP32 query at scale: 8 boxes per pixel of a 1920x1080 frame.
    "c2": GlintConfig("c2", "flake", 512, 512, 5000, 0.15, 0.005, 64, 8, 64, 50,
                      "frame", 1920 * 1080 * 8, 0.005, 0.3, True, boxes_per_point=8),
    # Precision: BF16 factors and cumulative tables.
    "c3": GlintConfig("c3", "flake", 2048, 2048, 80_000, 0.20, 0.005, 64, 10, 128, 50,
                      "footprints", 8_000_000 * 8, 0.005, 0.3, True, boxes_per_point=8,
                      dtype="bf16", cum_dtype="bf16"),
    # Differentiation: 2^24 queries per refinement step, FP32.
    "c4": GlintConfig("c4", "flake", 2048, 2048, 80_000, 0.20, 0.005, 64, 10, 128, 50,
                      "footprints", 1 << 24, 0.005, 0.3, True, boxes_per_point=8),
    # Scratch map, FP8 factors, 32 SG-derived boxes per shading point.
    "c5": GlintConfig("c5", "scratch", 4096, 4096, 20_000, 0.0, 0.005, 128, 12, 256, 50,
                      "sg_grouped", (1 << 20) * 32, 0.0, 0.0, False, boxes_per_point=32,
                      dtype="fp8", cum_dtype="bf16"),
}


def config(name: str, **overrides) -> GlintConfig:
    """Named configuration, optionally with fields replaced (tests use small copies)."""
    return dataclasses.replace(CONFIGS[name], **overrides)


def map_seed(cfg: GlintConfig) -> int:
    return 0x2109_14807 + cfg.index


def query_seed(cfg: GlintConfig) -> int:
    return map_seed(cfg) + 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# normal maps
# ----------------------------------------------------------------------------


def flake_map(nu: int, nv: int, nsites: int, alpha: float, seed: int) -> np.ndarray:
    """Periodic Voronoi flake map; returns float32 [nu][nv][2] projected normals."""
    from scipy.spatial import cKDTree

    rng = _rng(seed)
    sites = np.empty((nsites, 2))
    sites[:, 0] = rng.random(nsites) * nu
    sites[:, 1] = rng.random(nsites) * nv
    xi1 = rng.random(nsites)
    xi2 = rng.random(nsites)
    phi = 2.0 * np.pi * xi1
    tan2 = -(alpha * alpha) * np.log1p(-xi2)
    sin_t = np.sqrt(tan2 / (1.0 + tan2))
    site_n = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi)], axis=1)

    # cKDTree's boxsize gives toroidal distances; sites must lie in [0, box).
    sites[:, 0] = np.mod(sites[:, 0], nu)
    sites[:, 1] = np.mod(sites[:, 1], nv)
    tree = cKDTree(sites, boxsize=(float(nu), float(nv)))
    out = np.empty((nu, nv, 2), dtype=np.float32)
    ys = np.arange(nv) + 0.5
    chunk = max(1, (1 << 22) // nv)
    for u0 in range(0, nu, chunk):
        u1 = min(nu, u0 + chunk)
        xs = np.arange(u0, u1) + 0.5
        pts = np.stack(np.meshgrid(xs, ys, indexing="ij"), axis=-1).reshape(-1, 2)
        _, idx = tree.query(pts, k=1)
        out[u0:u1] = site_n[idx].reshape(u1 - u0, nv, 2).astype(np.float32)
    return out


def scratch_map(nu: int, nv: int, nscratch: int, seed: int,
                len_lo: float = 32.0, len_hi: float = 1024.0,
                width_lo: float = 1.0, width_hi: float = 3.0,
                tilt_sd: float = 0.3) -> np.ndarray:
    """Random-scratch map; returns float32 [nu][nv][2] projected normals."""
    rng = _rng(seed)
    out = np.zeros((nu, nv, 2), dtype=np.float32)
    x0 = rng.random(nscratch) * nu
    y0 = rng.random(nscratch) * nv
    ang = rng.random(nscratch) * 2.0 * np.pi
    length = np.exp(np.log(len_lo) + rng.random(nscratch) * (np.log(len_hi) - np.log(len_lo)))
    width = width_lo + rng.random(nscratch) * (width_hi - width_lo)
    tilt = rng.normal(0.0, tilt_sd, nscratch)
    for i in range(nscratch):
        dx, dy = math.cos(ang[i]), math.sin(ang[i])
        px, py = -dy, dx                      # in-plane perpendicular
        half = 0.5 * width[i]
        # candidate texels: a rotated rectangle swept along the segment
        ts = np.arange(-1.0, length[i] + 1.0, 0.5)
        os_ = np.arange(-half - 1.0, half + 1.0, 0.5)
        tt, oo = np.meshgrid(ts, os_, indexing="ij")
        cx = np.floor(x0[i] + tt * dx + oo * px).astype(np.int64).ravel()
        cy = np.floor(y0[i] + tt * dy + oo * py).astype(np.int64).ravel()
        # distinct candidates through one int64 key (|cx|, |cy| < 2^20 here)
        key = np.unique((cx + (1 << 20)) * (1 << 21) + (cy + (1 << 20)))
        cand_x = key // (1 << 21) - (1 << 20)
        cand_y = key % (1 << 21) - (1 << 20)
        # exact test: distance from the texel centre to the segment <= half width
        rx = cand_x + 0.5 - x0[i]
        ry = cand_y + 0.5 - y0[i]
        along = np.clip(rx * dx + ry * dy, 0.0, length[i])
        ex = rx - along * dx
        ey = ry - along * dy
        keep = ex * ex + ey * ey <= half * half
        cu = np.mod(cand_x[keep], nu)
        cv = np.mod(cand_y[keep], nv)
        s = math.sin(tilt[i])
        out[cu, cv, 0] = np.float32(s * px)
        out[cu, cv, 1] = np.float32(s * py)
    return out


def normal_map(cfg: GlintConfig) -> np.ndarray:
    if cfg.map_kind == "flake":
        return flake_map(cfg.nu, cfg.nv, cfg.nsites, cfg.alpha, map_seed(cfg))
    if cfg.map_kind == "scratch":
        return scratch_map(cfg.nu, cfg.nv, cfg.nsites, map_seed(cfg))
    raise ValueError(cfg.map_kind)


# ----------------------------------------------------------------------------
# queries
# ----------------------------------------------------------------------------


def _footprint_texel(rng, u, v, l, nu, nv):
    """A uniformly chosen texel of the 2^l box footprint anchored at (u, v)."""
    k = np.left_shift(1, l)
    i = (rng.random(u.shape) * k).astype(np.int64)
    j = (rng.random(u.shape) * k).astype(np.int64)
    return np.mod(u - k // 2 + i, nu), np.mod(v - k // 2 + j, nv)


def _sides(rng, n, lo, hi, log):
    if log:
        return np.exp(np.log(lo) + rng.random(n) * (np.log(hi) - np.log(lo)))
    return lo + rng.random(n) * (hi - lo)


def _centres(rng, side, normal_comp):
    """50/50 mixture: uniform in the domain, or a footprint texel's normal + N(0, side/4)."""
    n = side.shape[0]
    lo = -1.0 + 0.5 * side
    hi = 1.0 - 0.5 * side
    uni = lo + rng.random(n) * (hi - lo)
    jit = normal_comp + rng.normal(0.0, 1.0, n) * (0.25 * side)
    pick = rng.random(n) < 0.5
    c = np.where(pick, uni, jit)
    return np.clip(c, lo, hi)


def box_to_bins(centre, side, nbins):
    """Continuous box [c - w/2, c + w/2] to a half-open bin range, always >= 1 bin."""
    half_n = nbins / 2.0
    lo = np.floor((centre - 0.5 * side + 1.0) * half_n).astype(np.int64)
    hi = np.floor((centre + 0.5 * side + 1.0) * half_n).astype(np.int64)
    lo = np.clip(lo, 0, nbins - 1)
    hi = np.clip(hi, 0, nbins - 1) + 1
    return lo, hi


def _boxes_for(rng, nxy, u, v, l, cfg, side_lo, side_hi, side_log):
    n = u.shape[0]
    tx, ty = _footprint_texel(rng, u, v, l, cfg.nu, cfg.nv)
    ws = _sides(rng, n, side_lo, side_hi, side_log)
    wt = _sides(rng, n, side_lo, side_hi, side_log)
    cs = _centres(rng, ws, nxy[tx, ty, 0].astype(np.float64))
    ct = _centres(rng, wt, nxy[tx, ty, 1].astype(np.float64))
    slo, shi = box_to_bins(cs, ws, cfg.nbins)
    tlo, thi = box_to_bins(ct, wt, cfg.nbins)
    return slo, shi, tlo, thi


def make_queries(cfg: GlintConfig, nxy: np.ndarray, nq: int | None = None,
                 seed: int | None = None, shuffle: bool = False) -> np.ndarray:
    """Query records int32 [nq][7] = (u, v, l, s_lo, s_hi, t_lo, t_hi).

    ``nq`` defaults to the configuration's batch; a smaller ``nq`` takes the
    leading queries of the same recipe (pixel-major for "frame").
    """
    nq = cfg.nqueries if nq is None else nq
    rng = _rng(query_seed(cfg) if seed is None else seed)
    out = np.empty((nq, 7), dtype=np.int32)
    chunk = 1 << 22
    for q0 in range(0, nq, chunk):
        q1 = min(nq, q0 + chunk)
        idx = np.arange(q0, q1, dtype=np.int64)
        if cfg.query_kind == "uniform":
            n = q1 - q0
            u = (rng.random(n) * cfg.nu).astype(np.int64)
            v = (rng.random(n) * cfg.nv).astype(np.int64)
            l = (rng.random(n) * cfg.nlevels).astype(np.int64)
        elif cfg.query_kind == "frame":
            # 1920x1080 pixels, boxes_per_point boxes per pixel, pixel-major;
            # band level l(y) = floor(nlevels*y/1080); footprint-coherent centres.
            pix = idx // cfg.boxes_per_point
            x = pix % 1920
            y = pix // 1920
            l = (cfg.nlevels * y) // 1080
            u = np.mod(np.floor((x + 0.5) * np.left_shift(1, l)).astype(np.int64), cfg.nu)
            v = np.mod(np.floor((y + 0.5) * np.left_shift(1, l)).astype(np.int64), cfg.nv)
        elif cfg.query_kind in ("footprints", "sg_grouped"):
            # boxes_per_point consecutive boxes share one random footprint
            fp = idx // cfg.boxes_per_point
            first = np.unique(fp)
            n_fp = first.shape[0]
            fu = (rng.random(n_fp) * cfg.nu).astype(np.int64)
            fv = (rng.random(n_fp) * cfg.nv).astype(np.int64)
            fl = (rng.random(n_fp) * cfg.nlevels).astype(np.int64)
            pos = fp - first[0]
            u, v, l = fu[pos], fv[pos], fl[pos]
        else:
            raise ValueError(cfg.query_kind)
        if cfg.query_kind == "sg_grouped":
            slo, shi, tlo, thi = _sg_boxes(rng, nxy, u, v, l, cfg)
        else:
            slo, shi, tlo, thi = _boxes_for(rng, nxy, u, v, l, cfg,
                                            cfg.side_lo, cfg.side_hi, cfg.side_log)
        out[q0:q1] = np.stack([u, v, l, slo, shi, tlo, thi], axis=1).astype(np.int32)
    if shuffle:
        perm = _rng(query_seed(cfg) + 99).permutation(nq)
        out = out[perm]
    return out


def _sg_boxes(rng, nxy, u, v, l, cfg):
    """Environment-light boxes: a spherical Gaussian per box with bandwidth
    lambda ~ logU[10, 1000] and amplitude A ~ U[1, 10]; its compact-eps support
    angle (eps = 0.3) gives a square box of N*theta/pi bins (Sec. 5.4)."""
    n = u.shape[0]
    lam = np.exp(np.log(10.0) + rng.random(n) * (np.log(1000.0) - np.log(10.0)))
    amp = 1.0 + rng.random(n) * 9.0
    theta = np.arccos(np.clip((np.log(0.3) - np.log(amp)) / lam + 1.0, -1.0, 1.0))
    side = np.minimum(2.0 * theta / np.pi, 2.0)    # N*theta/pi bins of width 2/N
    tx, ty = _footprint_texel(rng, u, v, l, cfg.nu, cfg.nv)
    cs = _centres(rng, side, nxy[tx, ty, 0].astype(np.float64))
    ct = _centres(rng, side, nxy[tx, ty, 1].astype(np.float64))
    slo, shi = box_to_bins(cs, side, cfg.nbins)
    tlo, thi = box_to_bins(ct, side, cfg.nbins)
    return slo, shi, tlo, thi


def make_grouped_queries(cfg: GlintConfig, nxy: np.ndarray, npts: int | None = None,
                         seed: int | None = None):
    """Grouped form: uvl int32 [npts][3] and boxes int32 [npts][K][4] = (s_lo, s_hi, t_lo, t_hi)."""
    K = cfg.boxes_per_point
    npts = cfg.nqueries // K if npts is None else npts
    flat = make_queries(cfg, nxy, nq=npts * K, seed=seed)
    uvl = flat[::K, 0:3].copy()
    boxes = flat[:, 3:7].reshape(npts, K, 4).copy()
    return uvl, boxes


# ----------------------------------------------------------------------------
# ALS initial factors (the random numbers the method draws, passed as input)
# ----------------------------------------------------------------------------


def als_init(cfg_or_dims, rank: int | None = None, seed: int | None = None):
    """I.i.d. U[0,1) initial factors (U, V, L, S, T) from PCG64(seed), FP64.

    ``cfg_or_dims`` is a GlintConfig or a tuple (nu, nv, nlevels, nbins).
    """
    if isinstance(cfg_or_dims, GlintConfig):
        cfg = cfg_or_dims
        dims = (cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.nbins)
        rank = cfg.rank if rank is None else rank
        seed = map_seed(cfg) + 2 if seed is None else seed
    else:
        nu, nv, nl, nb = cfg_or_dims
        dims = (nu, nv, nl, nb, nb)
        assert rank is not None and seed is not None
    rng = _rng(seed)
    return tuple(rng.random((d, rank)) for d in dims)
