#!/usr/bin/env python3
"""Benchmark: batched P-NDF range queries (Sec. 4.4, Eq. rangeDecom) on one GPU.

Headline workload (one step = one glint_query launch over the whole batch):
a 2048x2048 periodic Voronoi flake map (80 000 sites, Beckmann alpha 0.2),
intrinsic roughness 0.005, a 64x64 NDF grid, 10 footprint levels (1..512
texels), CP rank 128 fitted by 50 texel-space ALS sweeps (FP64), FP32 factor
and summed-area tables, and a batch of 2^24 range queries (8 angular boxes per
random footprint, box sides log-uniform in [0.005, 0.3]).  Inputs are
synthetic and seeded and resident in HBM before timing starts.

value = queries answered per second over the timed steps.  roofline = the
query kernel's HBM rate (32 algorithmic bytes per query: the 28-byte record
and the 4-byte result) against the 8 TB/s peak, with the on-chip roof that
binds it beside it.

Further legs, each reported with its own rate, its error against brute-force
range integrals and (in the cpu_baseline leg) its error against the FP64
oracle on sampled outputs:
  c3      the same map recipe, rank 128, BF16 tables, 6.4e7 queries
  c5      4096^2 scratch map, rank 256, FP8 factors (BF16 and FP8 summed-area
          tables), 2^20 shading points x 32 boxes (grouped query)
  r16     the 64^2 map's rank-16 factors on a 1.66e7-record batch (the regime
          where HBM binds)
  c2      512^2 map, rank 64 FP32, the 1920x1080x8 frame batch; the FP32 tensor
          build, the dense matrix-core ALS, the query backward and the
          section 4/5 front-ends (off-grid, sampling, SG, Wang tiles, the
          clustered layout)
  refine  Adam refinement of the headline factors (FP32, and BF16 straight
          through) against brute-force range integrals; error on a held-out
          batch and the refined BF16 query's speed against the plain FP32 one
  sweep   query time over levels x box widths (constant cost)
  cpu_baseline  the FP64 oracle on the host: its 1-core query rate, brute
          force per level, and the parity samples of every leg
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix
VALU_LANE_OPS = 256 * 2.4e9 * 64   # unpacked FP32 lane operations per second: 256 CUs x 2.4 GHz x 64 lanes
# on-chip ceilings measured on this part with plain loops (no other work): conflict-free 16-byte
# LDS reads by 32 waves per CU, and independent FP32 FMA chains (wave instructions per second)
LDS_READ_TBS_MEASURED = 124.0
VALU_FP32_WAVE_INSTR_MEASURED = 8.7e11
Q_BYTES = 32                   # algorithmic HBM bytes per flat query: 28-byte record + 4-byte result

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE on the named
# launch, scaled by what the counters read for a plain 2 GiB copy in the same
# run (profiles/*_counters.md).  Valid only for the source file they were
# taken with (sha1 of the whole file: a kernel's instantiation depends on
# helpers and constants outside its own text); otherwise traffic is null.
MEASURED_TRAFFIC = {
    "k_mttkrp_y": ("paper_2109_14807_amd/csrc/cp_als.hip", "fc21e4c6223d0b00e6b413af67d951920b9cea9a", 36577139135),
    "k_mttkrp_z": ("paper_2109_14807_amd/csrc/cp_als.hip", "fc21e4c6223d0b00e6b413af67d951920b9cea9a", 34934241770),
    "k_query_c4": ("paper_2109_14807_amd/csrc/query.hip", "a1e2724f94e86b56b0967e488a072eeaab4adb8a", 554306304),
    "k_query_r16": ("paper_2109_14807_amd/csrc/query.hip", "a1e2724f94e86b56b0967e488a072eeaab4adb8a", 532277504),
    "k_query_clustered": ("paper_2109_14807_amd/csrc/cluster.hip", "08645f6f9e0410b9481c4a048e056380329dbfe0", 9302617408),
    "k_query_clustered_bf16": ("paper_2109_14807_amd/csrc/cluster.hip", "08645f6f9e0410b9481c4a048e056380329dbfe0",
                               8402666272),
    "k_query_c3": ("paper_2109_14807_amd/csrc/query.hip", "a1e2724f94e86b56b0967e488a072eeaab4adb8a", 2056795136),
    "k_query_grouped_c5_bf16": ("paper_2109_14807_amd/csrc/query.hip", "a1e2724f94e86b56b0967e488a072eeaab4adb8a",
                                966130304),
    "k_query_grouped_c5_fp8": ("paper_2109_14807_amd/csrc/query.hip", "a1e2724f94e86b56b0967e488a072eeaab4adb8a",
                               965127168),
}

LEGS = ("c3", "c5", "r16", "c2", "clustered", "refine", "sweep", "cpu_baseline")


def source_sha(path):
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def measured_traffic(key):
    """HBM bytes per launch from the committed counter runs, or None once the
    kernel's source file has changed since they were taken."""
    src, sha, nbytes = MEASURED_TRAFFIC[key]
    try:
        cur = source_sha(src)
    except OSError:
        return None
    return nbytes if cur == sha and nbytes > 0 else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sweeps", type=int, default=50, help="ALS sweeps of every workload")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs after the headline: " + ",".join(LEGS) + " (or 'none')")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="same as leaving cpu_baseline out of --legs")
    ap.add_argument("--reps", type=int, default=10, help="event-timed launches per kernel figure")
    ap.add_argument("--refine-steps", type=int, default=200)
    ap.add_argument("--cluster-sweeps", type=int, default=20, help="ALS sweeps per region tensor (clustered leg)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 2 GiB device copy (read 2 GiB, write 2 GiB), the reference "
                         "for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def timed(fn, reps, spin_s=0.2):
    """Mean duration (ms) of fn's launches: `reps` launches back to back
    between two HIP events on the current stream (the stream the library
    calls enqueue on), after untimed launches for about `spin_s` seconds (at
    least one), so that the GPU has left the clocks it idles at while a leg
    prepares its inputs on the host."""
    import torch
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    n, calls = 1, 0
    while True:
        for _ in range(n):
            fn()
        calls += n
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= spin_s:
            break
        n = min(2 * n, 64)
    if calls > 1:
        # a short launch: one more is queued ahead of the first event, so that
        # the timed launches run back to back from it (without it the host's
        # latency to the first launch is timed too)
        fn()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def stored_tables(tabs):
    """Host FP64 copies of the values a table set stores (decoded exactly) and
    the per-rank folded scale (None if no scales), for the parity samples."""
    import numpy as np
    import torch

    def dec(t):
        if t.dtype == torch.float8_e4m3fn or t.dtype == torch.uint8:
            return t.view(torch.float8_e4m3fn).float().double().cpu().numpy()
        if t.dtype == torch.bfloat16 or t.dtype == torch.int16:
            return t.view(torch.bfloat16).float().double().cpu().numpy()
        return t.double().cpu().numpy()
    vals = [dec(t) for t in (tabs.U, tabs.V, tabs.L, tabs.CS, tabs.CT)]
    scale = None
    for s in tabs.scales:
        if s is not None:
            s = s.cpu().numpy().astype(np.float64)
            scale = s if scale is None else scale * s
    return vals, scale


def sample_idx(n, k, seed):
    import numpy as np
    rng = np.random.default_rng(seed)
    k = min(n, k)
    idx = np.sort(rng.choice(n, k, replace=False))
    idx[-1] = n - 1
    return idx


def error_vs_bruteforce(desc, nxy, recs, out, levels=None):
    """Relative L2 error of query outputs against brute-force range integrals
    (GPU, FP64) of the same records; per level when ``levels`` is given."""
    import torch
    import paper_2109_14807_amd as G
    bf = G.range_bruteforce(nxy, desc, recs)
    d = out.double() - bf
    res = {"all": float((torch.linalg.vector_norm(d) / torch.linalg.vector_norm(bf)).item())}
    if levels:
        lv = torch.clamp(recs[:, 2].long(), 0, levels - 1)
        per = []
        for l in range(levels):
            m = lv == l
            nb = torch.linalg.vector_norm(bf[m])
            per.append(float((torch.linalg.vector_norm(d[m]) / nb).item()) if float(nb) > 0 else None)
        res["per_level"] = per
    return res, bf


def flat_rate(nq, ms):
    gbs = Q_BYTES * nq / (ms * 1e-3) / 1e9
    return {"ms": ms, "queries_per_s": nq / (ms * 1e-3), "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}


def table_onchip_bytes(R, elt_fac, elt_cum, boxes_per_footprint):
    """Bytes a flat query gathers from on-chip memories: four summed-area rows
    (LDS) and, once per footprint, the U, V (L2) and L (LDS) rows."""
    return 4 * R * elt_cum + 3 * R * elt_fac / boxes_per_footprint


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def fit_workload(name, sweeps, dev):
    """Map, batch, and the CP factors of a workload: dense FP64 ALS on the
    materialised tensor for the 64^2 map, texel-space FP64 ALS otherwise."""
    import torch
    import gen
    import paper_2109_14807_amd as G

    cfg = gen.config(name)
    t0 = time.time()
    nxy_h = gen.normal_map(cfg)
    desc = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    init = [torch.tensor(a, device=dev) for a in gen.als_init(cfg)]
    nxy = torch.tensor(nxy_h, device=dev)
    gen_s = time.time() - t0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if cfg.nu * cfg.nv <= 64 * 64:
        T = G.build_tensor(nxy, desc, dtype=torch.float64)
        e0.record()
        res = G.cp_als(T, desc, init, sweeps)
        e1.record()
        kind = "dense FP64 (matrix cores)"
        del T
    else:
        ws = G.texel_workspace(desc, cfg.rank)
        e0.record()
        res = G.cp_als_texel(nxy, desc, init, sweeps, workspace=ws)
        e1.record()
        kind = "texel-space FP64"
        del ws
    torch.cuda.synchronize()
    info = res.info.cpu().tolist()
    als = {"kind": kind, "sweeps": sweeps, "ms": e0.elapsed_time(e1), "solve_fallbacks": info[1],
           "map_seconds": gen_s}
    return cfg, nxy_h, nxy, desc, res.factors, als


def tables_report(tabs):
    name = lambda t: str(t.dtype).replace("torch.", "")
    return {"U_V_L": name(tabs.U), "CS_CT": name(tabs.CS), "R": tabs.R,
            "bytes": int(sum(t.numel() * t.element_size() for t in (tabs.U, tabs.V, tabs.L, tabs.CS, tabs.CT)))}


# ---------------------------------------------------------------------------
# headline: the 2048^2 rank-128 FP32 batch
# ---------------------------------------------------------------------------

def headline(args, dev, keep):
    import numpy as np
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    cfg, nxy_h, nxy, desc, F, als = fit_workload("c4", args.sweeps, dev)
    log(f"c4: map and {als['kind']} ALS ({als['ms']:.0f} ms)")
    t0 = time.time()
    q_h = gen.make_queries(cfg, nxy_h)
    q = torch.tensor(q_h, device=dev)
    nq = q.shape[0]
    log(f"c4: {nq} queries generated in {time.time() - t0:.1f}s")
    tabs = G.make_tables(*F, dtype="f32", cum_dtype="f32")
    fac = tabs.factors()
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    # bring the GPU out of its idle clocks (the map and batch were built on the
    # host) with about 0.3 s of the same launches, untimed, before the warm-up
    t_spin = time.perf_counter()
    while time.perf_counter() - t_spin < 0.3:
        for _ in range(20):
            L.glint_query(fac, q, out)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        L.glint_query(fac, q, out)
    torch.cuda.synchronize()
    # HIP events on the library's stream around the K back-to-back launches
    # of the timed region: their mean launch duration is the roofline's
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        L.glint_query(fac, q, out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kernel_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    log(f"c4: {args.steps} timed steps in {wall * 1e3:.2f} ms (kernel {kernel_ms:.4f} ms)")

    R = cfg.rank
    achieved = Q_BYTES * nq / (kernel_ms * 1e-3) / 1e9
    onchip = table_onchip_bytes(R, 4, 4, cfg.boxes_per_point)
    lds_per_q = 4 * R * 4 + R * 4 / cfg.boxes_per_point
    # FP32 lane operations per query: 2 differences, one product and one FMA per rank
    ops_per_q = 4 * R
    roofline = {
        "kernel": "k_query<float,float,float,128,16,false,512> (glint_query, FP32 rank-128 tables in LDS, 16 ranks a lane)",
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("k_query_c4"),
        "per_launch": {"queries": nq, "algorithmic_bytes": Q_BYTES * nq, "ms": kernel_ms,
                       "launches_timed": args.steps},
        "on_chip": {
            "what": "the roofs that bind at rank 128: per query four 512-byte summed-area rows and (once per "
                    "8-box footprint) one L row from LDS, the U and V rows from L2; 4R FP32 lane operations",
            "lds_bytes_per_query": lds_per_q, "gathered_bytes_per_query": onchip,
            "lds_tbs": lds_per_q * nq / (kernel_ms * 1e-3) / 1e12,
            "lds_frac_of_measured_read_rate": lds_per_q * nq / (kernel_ms * 1e-3) / 1e12 / LDS_READ_TBS_MEASURED,
            "valu_lane_ops_per_query": ops_per_q,
            "valu_frac_of_nominal_lane_ops": ops_per_q * nq / (kernel_ms * 1e-3) / VALU_LANE_OPS,
            "note": "the VALU instruction count per query (all of the kernel's work, not only the 4R "
                    "arithmetic) and its issue rate come from the SQ counters in profiles/",
        },
    }
    # error against brute-force range integrals on a 2^18-record sample, per level
    idx = sample_idx(nq, 1 << 18, 11)
    idx_d = torch.tensor(idx, device=dev)
    ebf, _ = error_vs_bruteforce(desc, nxy, q[idx_d], out[idx_d], levels=cfg.nlevels)
    pidx = sample_idx(nq, 100_000, 5)
    keep["parity"].append({"leg": "c4 (headline, FP32 rank 128)", "tables": stored_tables(tabs),
                           "records": q_h[pidx], "got": out[torch.tensor(pidx, device=dev)].cpu().numpy()})
    keep["c4"] = {"cfg": cfg, "nxy_h": nxy_h, "nxy": nxy, "desc": desc, "F": F, "q": q, "q_h": q_h,
                  "tabs": tabs, "kernel_ms": kernel_ms}
    head = {
        "value": nq / (ms_per_step * 1e-3), "ms_per_step": ms_per_step, "kernel_ms": kernel_ms,
        "roofline": roofline,
        "workload": {
            "workload": "c4: 2048x2048 flake map (80000 sites, alpha 0.2), sigma 0.005, 64x64 NDF bins, "
                        "10 levels (1..512), CP rank 128 (50 texel-space FP64 ALS sweeps), FP32 tables, "
                        "2^24 range queries (8 boxes per random footprint, sides log-U[0.005, 0.3])",
            "queries_per_step": nq, "rank": R, "nbins": cfg.nbins, "levels": cfg.nlevels,
            "tables": tables_report(tabs), "als": als},
        "error_vs_bruteforce": ebf,
    }
    log(f"c4: {head['value'] / 1e9:.2f} G q/s, {achieved:.0f} GB/s, E_bf {ebf['all']:.4f}")
    return head


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------

def leg_c3(args, dev, keep):
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    cfg, nxy_h, nxy, desc, F, als = fit_workload("c3", args.sweeps, dev)
    t0 = time.time()
    q_h = gen.make_queries(cfg, nxy_h)
    q = torch.tensor(q_h, device=dev)
    nq = q.shape[0]
    log(f"c3: {nq} queries in {time.time() - t0:.1f}s")
    tabs = G.make_tables(*F, dtype="bf16", cum_dtype="bf16")
    master = G.make_tables(*F, dtype="f32", cum_dtype="f32")
    fac = tabs.factors()
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    ms = timed(lambda: L.glint_query(fac, q, out), args.reps)
    idx = torch.tensor(sample_idx(nq, 1 << 18, 12), device=dev)
    ebf, bf = error_vs_bruteforce(desc, nxy, q[idx], out[idx])
    o32 = G.query(master, q[idx])
    ebf32 = float((torch.linalg.vector_norm(o32.double() - bf) / torch.linalg.vector_norm(bf)).item())
    pidx = sample_idx(nq, 100_000, 6)
    keep["parity"].append({"leg": "c3 (BF16 rank 128)", "tables": stored_tables(tabs),
                           "master": stored_tables(master), "records": q_h[pidx],
                           "got": out[torch.tensor(pidx, device=dev)].cpu().numpy()})
    rep = {"workload": "2048x2048 flake map (80000 sites, alpha 0.2), rank 128, BF16 factor and summed-area "
                       "tables, 6.4e7 queries (8 boxes per random footprint)",
           "queries": nq, "tables": tables_report(tabs), "als": als, **flat_rate(nq, ms),
           "traffic": measured_traffic("k_query_c3"),
           "error_vs_bruteforce": ebf["all"], "error_vs_bruteforce_f32_tables": ebf32}
    log(f"c3: {rep['queries_per_s'] / 1e9:.2f} G q/s, E_bf {ebf['all']:.4f}")
    return rep


def leg_c5(args, dev, keep):
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    cfg, nxy_h, nxy, desc, F, als = fit_workload("c5", args.sweeps, dev)
    t0 = time.time()
    uvl_h, boxes_h = gen.make_grouped_queries(cfg, nxy_h)
    uvl, boxes = torch.tensor(uvl_h, device=dev), torch.tensor(boxes_h, device=dev)
    npts, K = boxes_h.shape[:2]
    nq = npts * K
    log(f"c5: {npts} x {K} boxes in {time.time() - t0:.1f}s")
    idx = sample_idx(nq, 1 << 18, 13)
    idx_d = torch.tensor(idx, device=dev)
    flat = torch.cat([uvl[idx_d // K], boxes.reshape(-1, 4)[idx_d]], dim=1).contiguous()
    bf = G.range_bruteforce(nxy, desc, flat)
    master = G.make_tables(*F, dtype="f32", cum_dtype="f32")
    pidx = sample_idx(nq, 100_000, 7)
    prec = torch.tensor(pidx, device=dev)
    rec_p = torch.cat([uvl[prec // K], boxes.reshape(-1, 4)[prec]], dim=1).cpu().numpy()
    rep = {"workload": "4096x4096 scratch map (20000 segments), N 128, 12 levels (1..2048), rank 256, FP8 "
                       "factors with per-column scales, 2^20 shading points x 32 SG boxes (grouped query)",
           "boxes": nq, "als": als}
    out = torch.empty((npts, K), dtype=torch.float32, device=dev)
    o32 = G.query(master, flat)
    rep["error_vs_bruteforce_f32_tables"] = float(
        (torch.linalg.vector_norm(o32.double() - bf) / torch.linalg.vector_norm(bf)).item())
    for cum in ("bf16", "fp8"):
        tabs = G.make_tables(*F, dtype="fp8", cum_dtype=cum)
        fac = tabs.factors()
        ms = timed(lambda: L.glint_query_grouped(fac, uvl, boxes, out), args.reps)
        o = out.reshape(-1)
        e = float((torch.linalg.vector_norm(o[idx_d].double() - bf) / torch.linalg.vector_norm(bf)).item())
        # per box: 16-byte box record + 4-byte result, plus the 12-byte shading point once per 32 boxes
        gbs = (20.0 + 12.0 / K) * nq / (ms * 1e-3) / 1e9
        name = "fp8_factors_bf16_sat" if cum == "bf16" else "all_fp8"
        rep[name] = {"tables": tables_report(tabs), "ms": ms, "boxes_per_s": nq / (ms * 1e-3), "hbm_gbs": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS, "error_vs_bruteforce": e,
                     "traffic": measured_traffic("k_query_grouped_c5_" + cum)}
        keep["parity"].append({"leg": f"c5 (FP8 factors, {cum.upper()} summed-area tables, grouped)",
                               "tables": stored_tables(tabs), "master": stored_tables(master), "records": rec_p,
                               "got": o[prec].cpu().numpy()})
        log(f"c5 {name}: {rep[name]['boxes_per_s'] / 1e9:.2f} G boxes/s, E_bf {e:.4f}")
    return rep


def leg_r16(args, dev, keep):
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    cfg, nxy_h, nxy, desc, F, als = fit_workload("c1", args.sweeps, dev)
    nq = 16_588_800
    t0 = time.time()
    q_h = gen.make_queries(cfg, nxy_h, nq=nq)
    q = torch.tensor(q_h, device=dev)
    log(f"r16: {nq} queries in {time.time() - t0:.1f}s")
    tabs = G.make_tables(*F, dtype="f32", cum_dtype="f32")
    fac = tabs.factors()
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    ms = timed(lambda: L.glint_query(fac, q, out), args.reps)
    idx = torch.tensor(sample_idx(nq, 1 << 18, 14), device=dev)
    ebf, _ = error_vs_bruteforce(desc, nxy, q[idx], out[idx])
    pidx = sample_idx(nq, 100_000, 8)
    keep["parity"].append({"leg": "r16 (64^2 map, rank 16 FP32)", "tables": stored_tables(tabs),
                           "records": q_h[pidx], "got": out[torch.tensor(pidx, device=dev)].cpu().numpy()})
    rep = {"workload": "64x64 flake map (200 sites, alpha 0.1), sigma 0.01, 32x32 bins, 5 levels, rank 16 "
                       "(50 dense FP64 ALS sweeps), FP32 tables, 16,588,800 uniform queries (box sides U[0.02, 0.5])",
           "queries": nq, "tables": tables_report(tabs), "als": als, **flat_rate(nq, ms),
           "traffic": measured_traffic("k_query_r16"), "error_vs_bruteforce": ebf["all"]}
    log(f"r16: {rep['queries_per_s'] / 1e9:.1f} G q/s = {rep['hbm_frac']:.3f} of HBM")
    return rep


def leg_clustered(args, dev, keep):
    """The paper's own layout at its own scale (Sec. 4.2 practical choices):
    the 2048^2 flake map of the headline in 16 x 16 angular blocks and 8 x 8
    texel regions, rank 32 per region tensor, built block by block from the
    map (no stored T), compact Z; its range query on the headline batch."""
    import numpy as np
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    cfg = gen.config("c4")
    nxy_h = gen.normal_map(cfg)
    desc = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    nxy = torch.tensor(nxy_h, device=dev)
    t, cs, R = 16, 8, 32
    ncu, ncv, nb = cfg.nu // cs, cfg.nv // cs, cfg.nbins // t
    ntensor, Lr = ncu * ncv * nb * nb, cs * cs * cfg.nlevels
    cd = L.ClusterDesc(t, cs, R)
    ws = torch.empty(L.glint_cluster_map_workspace(desc, cd, torch.float32), dtype=torch.uint8, device=dev)
    zidx = torch.empty((ntensor, Lr), dtype=torch.int32, device=dev)
    zbase = torch.empty(ntensor + 1, dtype=torch.int64, device=dev)
    info = torch.empty(4, dtype=torch.int32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    L.glint_cluster_map_index(desc, cd, nxy, torch.float32, zidx, zbase, info, ws)
    ev[1].record()
    rows = int(zbase[-1].item())
    f32 = dict(dtype=torch.float32, device=dev)
    X, Y = torch.empty((ntensor, t, R), **f32), torch.empty((ntensor, t, R), **f32)
    Z = torch.empty((max(rows, 1), R), **f32)
    blank = torch.empty(ntensor, dtype=torch.uint8, device=dev)
    ev[2].record()
    L.glint_cp_als_clustered_map(desc, cd, nxy, torch.float32, args.cluster_sweeps, 5, zidx, X, Y, Z, blank, info, ws)
    ev[3].record()
    torch.cuda.synchronize()
    index_ms, als_ms = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    inf = info.cpu().tolist()
    del ws
    tab = G.ClusteredTables(desc, t, cs, X, Y, Z, blank, info, zidx=zidx, zbase=zbase)
    G.clustered_cumulative(tab)
    log(f"clustered: index {index_ms:.0f} ms, ALS {als_ms:.0f} ms, {rows} of {ntensor * Lr} image blocks stacked")
    q_h = gen.make_queries(cfg, nxy_h)
    q = torch.tensor(q_h, device=dev)
    nq = q.shape[0]
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    ms = timed(lambda: L.glint_query_clustered(tab.struct(), q, out), args.reps)
    idx = torch.tensor(sample_idx(nq, 1 << 18, 12), device=dev)
    ebf, _ = error_vs_bruteforce(desc, nxy, q[idx], out[idx], levels=cfg.nlevels)
    nonblank_tensors = ntensor - inf[1]
    full = cfg.nu * cfg.nv * cfg.nlevels * cfg.nbins ** 2
    stored = nonblank_tensors * 2 * t * R + rows * R
    # parity sample: every record's region (its nb^2 tensors, FP32 factors
    # and the Z rows of its footprint) goes to the oracle as a one-region,
    # one-footprint layout
    pidx = sample_idx(nq, 2000, 8)
    recs = q_h[pidx].astype(np.int64)
    u = np.mod(recs[:, 0], cfg.nu)
    v = np.mod(recs[:, 1], cfg.nv)
    l = np.clip(recs[:, 2], 0, cfg.nlevels - 1)
    t0 = ((u // cs) * ncv + v // cs) * nb * nb
    tens = torch.tensor(t0[:, None] + np.arange(nb * nb)[None, :], device=dev)
    f = torch.tensor(((u % cs) * cs + v % cs) * cfg.nlevels + l, device=dev)
    rowsel = zidx[tens, f[:, None]]
    Zs = torch.where(rowsel[..., None] >= 0, Z[rowsel.clamp(min=0).long()], torch.zeros((), **f32))
    keep["parity"].append({"leg": "clustered (2048^2, t 16, 8x8 regions, rank 32, compact Z)", "kind": "clustered",
                           "X": X[tens].cpu().numpy(), "Y": Y[tens].cpu().numpy(), "Z": Zs.cpu().numpy(),
                           "records": recs, "got": out[torch.tensor(pidx, device=dev)].cpu().numpy(),
                           "nb": nb, "t": t})
    rep = {"workload": "2048x2048 flake map (80000 sites, alpha 0.2) of the headline, clustered layout: 16x16 "
                       "angular blocks, 8x8 texel regions, 10 levels, rank 32 per region tensor, "
                       f"{args.cluster_sweeps} FP64 ALS sweeps, FP32 block tensors built from the map one angular "
                       "block at a time (no stored T), compact Z; queries: the headline's 2^24 records",
           "index_ms": index_ms, "als_ms": als_ms, "als_ms_per_sweep": als_ms / args.cluster_sweeps,
           "region_tensors": ntensor, "blank_tensors": inf[1], "solve_failures": inf[0],
           "stacked_image_blocks": rows, "image_blocks": ntensor * Lr,
           "compression": {"stored_floats": stored, "tensor_floats": full, "ratio": stored / full,
                           "what": "X, Y of the non-blank tensors and the stacked Z rows, over the entries of T"},
           **flat_rate(nq, ms), "error_vs_bruteforce": ebf["all"], "error_vs_bruteforce_per_level": ebf["per_level"]}
    # the tables (31 GB) stay in HBM: the gathers are HBM traffic too
    tr = measured_traffic("k_query_clustered")
    rep["traffic"] = tr
    if tr:
        rep["traffic_gbs"] = tr / (ms * 1e-3) / 1e9
        rep["traffic_frac"] = rep["traffic_gbs"] / HBM_PEAK_GBS
    log(f"clustered: query {rep['queries_per_s'] / 1e9:.2f} G q/s, E_bf {ebf['all']:.4f}")
    # the same tables stored in BF16 (CX, CY and Z rounded to nearest even)
    bt = G.clustered_bf16(tab)
    outb = torch.empty(nq, dtype=torch.float32, device=dev)
    msb = timed(lambda: L.glint_query_clustered(bt.struct(), q, outb), args.reps)
    ebfb, _ = error_vs_bruteforce(desc, nxy, q[idx], outb[idx], levels=cfg.nlevels)
    d32 = float(torch.linalg.vector_norm((outb - out).double()) / torch.linalg.vector_norm(out.double()))
    bsel = bt.Z[rowsel.clamp(min=0).long()]
    Zb = torch.where(rowsel[..., None] >= 0, bsel, torch.zeros((), dtype=torch.bfloat16, device=dev))
    keep["parity"].append({"leg": "clustered BF16 tables (2048^2, t 16, 8x8 regions, rank 32, compact Z)",
                           "kind": "clustered_tables", "CX": bt.CX[tens].float().cpu().numpy(),
                           "CY": bt.CY[tens].float().cpu().numpy(), "Z": Zb.float().cpu().numpy(),
                           "records": recs, "got": outb[torch.tensor(pidx, device=dev)].cpu().numpy(),
                           "nb": nb, "t": t})
    rep["bf16_tables"] = {"what": "CX, CY and Z stored in BF16 (each FP32 value rounded to nearest even), "
                                  "FP32 arithmetic on the decoded values",
                          "table_bytes": int(sum(x.numel() * 2 for x in (bt.CX, bt.CY, bt.Z))),
                          "fp32_table_bytes": int(sum(x.numel() * 4 for x in (tab.CX, tab.CY, tab.Z))),
                          **flat_rate(nq, msb), "speedup_over_fp32_tables": ms / msb,
                          "error_vs_bruteforce": ebfb["all"], "rel_l2_vs_fp32_tables": d32}
    trb = measured_traffic("k_query_clustered_bf16")
    rep["bf16_tables"]["traffic"] = trb
    if trb:
        rep["bf16_tables"]["traffic_gbs"] = trb / (msb * 1e-3) / 1e9
        rep["bf16_tables"]["traffic_frac"] = rep["bf16_tables"]["traffic_gbs"] / HBM_PEAK_GBS
    log(f"clustered BF16: query {rep['bf16_tables']['queries_per_s'] / 1e9:.2f} G q/s, E_bf {ebfb['all']:.4f}")
    return rep


def leg_refine(args, dev, keep):
    """Adam refinement of the headline factors against brute-force range
    integrals of the headline batch; held-out error on a separate batch of the
    same recipe; the refined BF16 query against the plain FP32 one."""
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    h = keep["c4"]
    cfg, desc, nxy, q, F = h["cfg"], h["desc"], h["nxy"], h["q"], h["F"]
    nq = q.shape[0]
    t0 = time.time()
    tgt = G.range_bruteforce(nxy, desc, q)
    q_ev = torch.tensor(gen.make_queries(cfg, h["nxy_h"], nq=1 << 20, seed=gen.query_seed(cfg) + 7, shuffle=True),
                        device=dev)
    bf_ev = G.range_bruteforce(nxy, desc, q_ev)
    torch.cuda.synchronize()
    tgt_s = time.time() - t0
    log(f"refine: brute-force targets in {tgt_s:.1f}s")

    def heldout(tables):
        o = G.query(tables, q_ev)
        return float((torch.linalg.vector_norm(o.double() - bf_ev) / torch.linalg.vector_norm(bf_ev)).item())

    masters = [f.float() for f in F]
    rms = float(torch.sqrt(torch.mean(torch.cat([m.flatten() for m in masters]) ** 2)).item())
    lr = 1e-4 * rms
    plain = h["tabs"]
    rep = {"what": f"{args.refine_steps} Adam steps (lr 1e-4 x rms of the factors, betas 0.9/0.999) on the "
                   "2^24-record batch, each step: tables, query, MSE gradient, query backward, summed-area chain "
                   "rule, Adam; error on a held-out 2^20-record batch",
           "targets_seconds": tgt_s, "lr": lr, "heldout_error_plain_f32": heldout(plain)}
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    f_plain = plain.factors()
    for dt in ("f32", "bf16"):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        refined, losses = G.refine(*masters, q, tgt, steps=args.refine_steps, lr=lr, dtype=dt)
        e1.record()
        torch.cuda.synchronize()
        ls = losses.cpu().numpy()
        tabs = G.make_tables(*refined, dtype=dt, cum_dtype=dt)
        f_ref = tabs.factors()
        ms_ref = timed(lambda: L.glint_query(f_ref, q, out), args.reps)
        ms_plain = timed(lambda: L.glint_query(f_plain, q, out), args.reps)
        rep[dt] = {"ms_per_adam_step": e0.elapsed_time(e1) / args.refine_steps,
                   "train_loss_first_last": [float(ls[0]), float(ls[-1])],
                   "heldout_error": heldout(tabs), "query_ms": ms_ref, "plain_f32_query_ms_same_run": ms_plain,
                   "speedup_over_plain_f32": ms_plain / ms_ref}
        log(f"refine {dt}: {rep[dt]}")
    # the same refinement at half the rank: a rank-64 texel-space ALS of the same map
    # and batch targets, refined in BF16, against the plain rank-128 FP32 query
    init64 = [torch.tensor(a, device=dev) for a in gen.als_init((cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins), rank=64,
                                                                  seed=gen.map_seed(cfg) + 2)]
    ws64 = G.texel_workspace(desc, 64)
    F64 = G.cp_als_texel(nxy, desc, init64, args.sweeps, workspace=ws64).factors
    del ws64
    m64 = [f.float() for f in F64]
    rms64 = float(torch.sqrt(torch.mean(torch.cat([m.flatten() for m in m64]) ** 2)).item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ref64, losses64 = G.refine(*m64, q, tgt, steps=args.refine_steps, lr=1e-4 * rms64, dtype="bf16")
    e1.record()
    torch.cuda.synchronize()
    t64 = G.make_tables(*ref64, dtype="bf16", cum_dtype="bf16")
    f64 = t64.factors()
    ms64 = timed(lambda: L.glint_query(f64, q, out), args.reps)
    ms_plain = timed(lambda: L.glint_query(f_plain, q, out), args.reps)
    rep["rank64_bf16"] = {"what": "rank-64 texel-space ALS of the same map, refined in BF16 the same way",
                          "heldout_error_plain_f32_rank64": heldout(G.make_tables(*m64)),
                          "ms_per_adam_step": e0.elapsed_time(e1) / args.refine_steps,
                          "heldout_error": heldout(t64), "query_ms": ms64,
                          "plain_f32_rank128_query_ms_same_run": ms_plain,
                          "speedup_over_plain_f32_rank128": ms_plain / ms64}
    log(f"refine rank-64 bf16: {rep['rank64_bf16']}")
    b = rep["bf16"]
    c = rep["rank64_bf16"]
    rep["bf16_refined_vs_plain_f32"] = {
        "same_rank_128": {"speedup": b["speedup_over_plain_f32"], "error_refined_bf16": b["heldout_error"],
                          "error_plain_f32": rep["heldout_error_plain_f32"],
                          "equal_or_lower_error": bool(b["heldout_error"] <= rep["heldout_error_plain_f32"])},
        "rank_64": {"speedup": c["speedup_over_plain_f32_rank128"], "error_refined_bf16": c["heldout_error"],
                    "error_plain_f32_rank128": rep["heldout_error_plain_f32"],
                    "equal_or_lower_error": bool(c["heldout_error"] <= rep["heldout_error_plain_f32"])}}
    # one query backward on the batch (the refinement's gradient kernel)
    g = torch.randn(nq, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
    bufs = [torch.empty((n, cfg.rank), dtype=torch.float32, device=dev)
            for n in (cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins + 1, cfg.nbins + 1)]
    rep["backward_ms"] = timed(lambda: L.glint_query_backward(f_plain, q, g, *bufs), args.reps)
    return rep


def leg_sweep(args, dev, keep):
    """Query time at fixed level and fixed box width (both axes) on the
    headline tables, each cell a 2^24-record batch (8 boxes per random
    footprint, drawn on the GPU): the constant-cost claim."""
    import numpy as np
    import torch
    from paper_2109_14807_amd import _lib as L

    h = keep["c4"]
    cfg, fac = h["cfg"], h["tabs"].factors()
    n = h["q"].shape[0]
    gen_ = torch.Generator(device=dev).manual_seed(21)
    widths = (1, 4, 16, 64)
    table = []
    out = torch.empty(n, dtype=torch.float32, device=dev)
    q = torch.empty((n, 7), dtype=torch.int32, device=dev)
    for l in range(cfg.nlevels):
        row = []
        for w in widths:
            fu = torch.randint(0, cfg.nu, (n // 8,), device=dev, generator=gen_, dtype=torch.int32)
            fv = torch.randint(0, cfg.nv, (n // 8,), device=dev, generator=gen_, dtype=torch.int32)
            q[:, 0] = fu.repeat_interleave(8)
            q[:, 1] = fv.repeat_interleave(8)
            q[:, 2] = l
            q[:, 3] = torch.randint(0, cfg.nbins - w + 1, (n,), device=dev, generator=gen_, dtype=torch.int32)
            q[:, 4] = q[:, 3] + w
            q[:, 5] = torch.randint(0, cfg.nbins - w + 1, (n,), device=dev, generator=gen_, dtype=torch.int32)
            q[:, 6] = q[:, 5] + w
            row.append(timed(lambda: L.glint_query(fac, q, out), 5))
        table.append(row)
    t = np.array(table)
    return {"what": "glint_query on the headline tables, 2^24 records per cell (8 boxes per random footprint), "
                    "all records at one level and one box width (bins per axis)",
            "levels": list(range(cfg.nlevels)), "widths_bins": list(widths), "ms": table,
            "max_over_min": float(t.max() / t.min()), "queries_per_s_mean": float(n / (t.mean() * 1e-3))}


def leg_c2(args, dev, keep):
    """The 512^2 rank-64 workload end to end: FP32 tensor build, dense
    matrix-core ALS (and the texel-space ALS beside it), FP32 tables, the
    frame batch, the backward, and the section-5 front-ends."""
    import numpy as np
    import torch
    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    cfg = gen.config("c2")
    R, N, nl = cfg.rank, cfg.nbins, cfg.nlevels
    nxy_h = gen.normal_map(cfg)
    q_h = gen.make_queries(cfg, nxy_h)
    nq = q_h.shape[0]
    desc = G.desc_of(cfg.nu, cfg.nv, nl, N, cfg.sigma)
    nxy = torch.tensor(nxy_h, device=dev)
    q = torch.tensor(q_h, device=dev)
    init = [torch.tensor(a, device=dev) for a in gen.als_init(cfg)]
    rep = {"workload": "512x512 flake map (5000 sites, alpha 0.15), sigma 0.005, 64x64 bins, 8 levels, rank 64, "
                       "1920x1080x8 frame queries"}
    # build: T FP32 (34.4 GB); the default plan builds levels 0-2 directly
    # (writes only) and doubles the rest (each doubled level reads the level
    # below once at least): algorithmic bytes = T + the doubled levels' sources
    T = torch.empty((cfg.nu, cfg.nv, nl, N, N), dtype=torch.float32, device=dev)
    ws_b = torch.empty(L.glint_build_tensor_workspace(desc), dtype=torch.uint8, device=dev)
    b_ms = timed(lambda: L.glint_build_tensor(desc, nxy, T, 0, ws_b), 3)
    tb = T.numel() * 4
    direct = min(3, nl)
    alg = tb + tb // nl * (nl - direct)
    rep["build"] = {"ms": b_ms, "tensor_bytes": tb, "written_gbs": tb / (b_ms * 1e-3) / 1e9,
                    "written_frac": tb / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "direct_levels": direct, "algorithmic_bytes": alg,
                    "hbm_gbs": alg / (b_ms * 1e-3) / 1e9, "hbm_frac": alg / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del ws_b
    # dense ALS on the matrix cores
    ws = torch.empty(L.glint_cp_als_workspace(desc, R, L.GLINT_F32), dtype=torch.uint8, device=dev)
    F = [torch.empty_like(a) for a in init]
    fits = torch.zeros(args.sweeps, dtype=torch.float64, device=dev)
    info = torch.zeros(4, dtype=torch.int32, device=dev)

    def als():
        for a, b in zip(F, init):
            a.copy_(b)
        L.glint_cp_als(desc, T, R, args.sweeps, 0.0, *F, fits, info, ws)
    als_ms = timed(als, 1)
    M_u = torch.empty((cfg.nu, R), dtype=torch.float64, device=dev)
    M_s = torch.empty((N, R), dtype=torch.float64, device=dev)
    y_ms = timed(lambda: L.glint_mttkrp(desc, T, R, 3, *F, M_s, ws), args.reps)
    z_ms = timed(lambda: L.glint_mttkrp(desc, T, R, 0, *F, M_u, ws), args.reps)
    flops = 2.0 * T.numel() * R
    rep["als_dense"] = {
        "sweeps": args.sweeps, "ms": als_ms, "fit": float(fits[-1]), "solve_fallbacks": int(info[1]),
        "mttkrp_y": {"kernel": "k_mttkrp_y (timed as glint_mttkrp mode s)", "ms": y_ms,
                     "tflops": flops / (y_ms * 1e-3) / 1e12, "mfma_frac": flops / (y_ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS,
                     "traffic": measured_traffic("k_mttkrp_y"), "algorithmic_bytes": tb},
        "mttkrp_z": {"kernel": "k_mttkrp_z (timed as glint_mttkrp mode u)", "ms": z_ms,
                     "tflops": flops / (z_ms * 1e-3) / 1e12, "mfma_frac": flops / (z_ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS,
                     "traffic": measured_traffic("k_mttkrp_z"), "algorithmic_bytes": tb},
    }
    normT2 = float(torch.sum(T.double() ** 2).item())
    ws_t = G.texel_workspace(desc, R)
    Ft = [torch.empty_like(a) for a in init]
    fits_t = torch.zeros(args.sweeps, dtype=torch.float64, device=dev)

    def tex():
        for a, b in zip(Ft, init):
            a.copy_(b)
        L.glint_cp_als_texel(desc, nxy, R, args.sweeps, 0.0, normT2, *Ft, fits_t, info, ws_t)
    rep["als_texel"] = {"sweeps": args.sweeps, "ms": timed(tex, 1), "fit": float(fits_t[-1])}
    del ws_t, Ft
    log(f"c2: build {b_ms:.1f} ms, dense ALS {als_ms:.0f} ms, texel ALS {rep['als_texel']['ms']:.0f} ms")

    # clustered layout of the same tensor (before T is freed)
    rep["clustered"] = clustered_report(desc, T, q, nxy, args.reps)
    del T, ws
    torch.cuda.empty_cache()

    tabs = G.make_tables(*F, dtype="f32", cum_dtype="f32")
    fac = tabs.factors()
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    q_ms = timed(lambda: L.glint_query(fac, q, out), args.reps)
    idx = torch.tensor(sample_idx(nq, 1 << 18, 15), device=dev)
    ebf, _ = error_vs_bruteforce(desc, nxy, q[idx], out[idx])
    rep["query"] = {"tables": tables_report(tabs), **flat_rate(nq, q_ms), "error_vs_bruteforce": ebf["all"]}
    pidx = sample_idx(nq, 100_000, 9)
    keep["parity"].append({"leg": "c2 (FP32 rank 64, frame batch)", "tables": stored_tables(tabs),
                           "records": q_h[pidx], "got": out[torch.tensor(pidx, device=dev)].cpu().numpy()})
    g = torch.randn(nq, device=dev, generator=torch.Generator(device=dev).manual_seed(4))
    bufs = [torch.empty((n, R), dtype=torch.float32, device=dev) for n in (cfg.nu, cfg.nv, nl, N + 1, N + 1)]
    rep["backward_ms"] = timed(lambda: L.glint_query_backward(fac, q, g, *bufs), args.reps)
    del bufs, g

    # front-ends (section 4.1/4.3 off-grid footprints, 5.2 sampling, 5.4 SG, 5.5 Wang tiles)
    frac = torch.tensor([0.37, 0.61, 0.25], dtype=torch.float32, device=dev)
    xyl = (q[:, :3].float() + frac).contiguous()
    boxes = q[:, 3:7].contiguous()
    o2 = torch.empty_like(out)
    rep["trilinear"] = {"queries_per_s": nq / (timed(lambda: L.glint_query_trilinear(fac, xyl, boxes, o2),
                                                     args.reps) * 1e-3)}
    del xyl, boxes
    npix = nq // cfg.boxes_per_point
    s_uvl = q[::cfg.boxes_per_point, :3].contiguous()
    levels = N.bit_length() - 1
    s_rnd = torch.rand((npix, levels + 2), device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    s_h = torch.empty((npix, 2), dtype=torch.float32, device=dev)
    s_pdf = torch.empty(npix, dtype=torch.float32, device=dev)
    s_bins = torch.empty((npix, 2), dtype=torch.int32, device=dev)
    rep["sampling"] = {"samples_per_s": npix / (timed(lambda: L.glint_sample(fac, s_uvl, s_rnd, s_h, s_pdf, s_bins),
                                                      args.reps) * 1e-3)}
    gsg = torch.Generator(device=dev).manual_seed(6)
    sg_h = (torch.rand((npix, 2), device=dev, generator=gsg) * 1.2 - 0.6).contiguous()
    sg_p = torch.stack([torch.exp(math.log(10.0) + torch.rand(npix, device=dev, generator=gsg) * math.log(100.0)),
                        1.0 + 9.0 * torch.rand(npix, device=dev, generator=gsg)], 1).contiguous()
    sg_q = torch.empty((npix, 7), dtype=torch.int32, device=dev)
    sg_out = torch.empty(npix, dtype=torch.float32, device=dev)
    rep["sg_prefilter"] = {"lookups_per_s": npix / (timed(
        lambda: L.glint_query_sg(fac, s_uvl, sg_h, sg_p, 0.3, sg_q, sg_out), args.reps) * 1e-3)}
    del s_uvl, s_rnd, s_h, s_pdf, s_bins, sg_h, sg_p, sg_q, sg_out
    gw = np.random.default_rng(8)
    wS, wm, wnl, wR = 64, 8, 5, 16
    wF = [[torch.tensor(gw.random((n, wR)) * 0.1, device=dev) for n in (wS + 2 * wm, wS + 2 * wm, wnl, N, N)]
          for _ in range(16)]
    wtab = G.wang_tables(wF, wS, wm, 2024, gw.permutation(16))
    wq = q.clone()
    wq[:, 2] = torch.remainder(q[:, 2], wnl)
    wstruct = wtab.struct()
    rep["wang"] = {"what": "16 tiles of 64^2 texels, 8-texel margins, 5 levels, rank 16, the frame's records as "
                           "plane coordinates",
                   "queries_per_s": nq / (timed(lambda: L.glint_query_wang(wstruct, wq, o2), args.reps) * 1e-3)}
    log(f"c2: query {rep['query']['queries_per_s'] / 1e9:.1f} G q/s, front-ends done")
    return rep


def clustered_report(desc, T, q, nxy, reps, t=16, cs=8, R=16, sweeps=20):
    """The clustered layout of the same tensor (Sec. 4.2 practical choices):
    16 x 16 angular blocks, 8 x 8 texel regions, rank 16 per region and block,
    FP64 ALS per block tensor; its batch query time and error against the
    brute-force range integrals."""
    import torch
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    G.cp_als_clustered(T, desc, t, cs, R, iters=1)          # warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def run(iters):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tab = G.cp_als_clustered(T, desc, t, cs, R, iters=iters)
        e1.record(stream)
        torch.cuda.synchronize()
        return tab, e0.elapsed_time(e1)

    _, one_ms = run(1)
    tab, als_ms = run(sweeps)
    sweep_ms = (als_ms - one_ms) / max(sweeps - 1, 1)
    out = torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
    st = tab.struct()
    query_ms = timed(lambda: L.glint_query_clustered(st, q, out), reps)
    idx = torch.tensor(sample_idx(q.shape[0], 1 << 18, 16), device=q.device)
    ebf, _ = error_vs_bruteforce(desc, nxy, q[idx], out[idx])
    npix = q.shape[0] // 8
    s_uvl = q[::8, :3].contiguous()
    s_rnd = torch.rand((npix, (t.bit_length() - 1) + 3), device=q.device,
                       generator=torch.Generator(device=q.device).manual_seed(8))
    s_h = torch.empty((npix, 2), dtype=torch.float32, device=q.device)
    s_pdf = torch.empty(npix, dtype=torch.float32, device=q.device)
    s_bins = torch.empty((npix, 2), dtype=torch.int32, device=q.device)
    sample_ms = timed(lambda: L.glint_sample_clustered(st, s_uvl, s_rnd, s_h, s_pdf, s_bins), reps)
    info = tab.info.cpu().tolist()
    stacked = info[3]
    tt = t * t
    flops = 2 * 2.0 * tt * stacked * R
    dbytes = 2 * 4.0 * tt * stacked
    gbs = dbytes / (sweep_ms * 1e-3) / 1e9
    return {
        "what": f"per-(region, angular block) rank-{R} CP: {t}x{t} bin blocks, {cs}x{cs} texel regions, "
                f"{sweeps} FP64 ALS sweeps per block tensor (blank blocks skipped), FP32 tables",
        "block_tensors": tab.X.shape[0], "blank": info[1], "solve_failures": info[0], "stacked_blocks": stacked,
        "als_ms": als_ms, "als_ms_per_sweep": sweep_ms,
        "als_roofline": {"kernel": f"k_cluster_als<float,{R}>", "bound": "hbm", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "fp64_mfma_frac": flops / (sweep_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS},
        "query_ms": query_ms, "queries_per_s": q.shape[0] / (query_ms * 1e-3),
        "samples_per_s": npix / (sample_ms * 1e-3),
        "error_vs_bruteforce": ebf["all"],
        "table_bytes": int(4 * (tab.CX.numel() + tab.CY.numel() + tab.Z.numel())),
    }


# ---------------------------------------------------------------------------
# cpu_baseline leg: the FP64 oracle on the host (timing and the parity samples);
# the only part of the benchmark that runs the oracle
# ---------------------------------------------------------------------------

def clustered_tables_parity(p):
    """Each sampled record against the oracle's block-split query on the
    stored tables (oracle.cluster.clustered_range_query_tables) of its
    region, as one region of one texel and one level; M_q = the sum of the
    query's |rank terms| on those tables (the scale of its FP32 rounding)."""
    import numpy as np
    from oracle import cluster
    got = p["got"].astype(np.float64)
    want = np.empty(got.size)
    mag = np.zeros(got.size)
    nb, t = p["nb"], p["t"]
    N = nb * t
    for i, r in enumerate(p["records"]):
        CX = p["CX"][i].astype(np.float64).reshape(1, 1, nb, nb, t + 1, -1)
        CY = p["CY"][i].astype(np.float64).reshape(1, 1, nb, nb, t + 1, -1)
        Z = p["Z"][i].astype(np.float64).reshape(1, 1, nb, nb, 1, -1)
        q1 = np.array([[0, 0, 0, r[3], r[4], r[5], r[6]]], dtype=np.int64)
        want[i] = cluster.clustered_range_query_tables(CX, CY, Z, q1, 1, 1)[0]
        slo, shi, tlo, thi = (min(max(int(x), 0), N) for x in r[3:7])
        if slo < shi and tlo < thi:
            for zs in range(slo // t, (shi - 1) // t + 1):
                a0, a1 = max(slo, zs * t) - zs * t, min(shi, (zs + 1) * t) - zs * t
                for zt in range(tlo // t, (thi - 1) // t + 1):
                    b0, b1 = max(tlo, zt * t) - zt * t, min(thi, (zt + 1) * t) - zt * t
                    cx, cy = CX[0, 0, zs, zt], CY[0, 0, zs, zt]
                    mag[i] += float(np.sum(np.abs(Z[0, 0, zs, zt, 0] * (cx[a1] - cx[a0]) * (cy[b1] - cy[b0]))))
    err = np.abs(got - want)
    normal = mag >= 1e-30
    ent = {"leg": p["leg"], "n": int(got.size),
           "max_err_over_Mq": float(np.max(err[normal] / mag[normal])) if normal.any() else 0.0,
           "records_with_Mq_below_1e-30": int((~normal).sum()),
           "max_abs_err_there": float(np.max(err[~normal])) if (~normal).any() else 0.0,
           "tolerance": "|q_gpu - q_64| <= 1e-5 M_q + 1e-30"}
    ent["pass"] = bool(np.all(err <= 1e-5 * mag + 1e-30))
    return ent


def clustered_parity(p):
    """Each sampled record against the oracle's block-split query
    (oracle.cluster.clustered_range_query) over its region's downloaded FP32
    factors, laid out as one region of one texel and one level.  The oracle
    forms the blocks' cumulative sums of X and Y in FP64, the GPU reads them
    rounded to FP32, each off by up to 2^-24 of the block's absolute sum: the
    error scale M_q is the same query over |X|, |Y|, |Z| with the box widened
    to the whole blocks it touches."""
    import numpy as np
    from oracle import cluster
    got = p["got"].astype(np.float64)
    want = np.empty(got.size)
    mag = np.empty(got.size)
    nb, t = p["nb"], p["t"]
    N = nb * t
    for i, r in enumerate(p["records"]):
        X = p["X"][i].astype(np.float64).reshape(1, 1, nb, nb, t, -1)
        Y = p["Y"][i].astype(np.float64).reshape(1, 1, nb, nb, t, -1)
        Z = p["Z"][i].astype(np.float64).reshape(1, 1, nb, nb, 1, -1)
        q1 = np.array([[0, 0, 0, r[3], r[4], r[5], r[6]]], dtype=np.int64)
        want[i] = cluster.clustered_range_query(X, Y, Z, q1, 1, 1)[0]
        slo, shi, tlo, thi = (min(max(int(x), 0), N) for x in r[3:7])
        if slo < shi and tlo < thi:
            w = np.array([[0, 0, 0, slo // t * t, ((shi - 1) // t + 1) * t, tlo // t * t, ((thi - 1) // t + 1) * t]])
            mag[i] = cluster.clustered_range_query(np.abs(X), np.abs(Y), np.abs(Z), w, 1, 1)[0]
        else:
            mag[i] = 0.0
    err = np.abs(got - want)
    normal = mag >= 1e-30
    ent = {"leg": p["leg"], "n": int(got.size),
           "max_err_over_Mq": float(np.max(err[normal] / mag[normal])) if normal.any() else 0.0,
           "records_with_Mq_below_1e-30": int((~normal).sum()),
           "max_abs_err_there": float(np.max(err[~normal])) if (~normal).any() else 0.0,
           "tolerance": "|q_gpu - q_64| <= 1e-5 M_q + 1e-30 (M_q over whole blocks)"}
    ent["pass"] = bool(np.all(err <= 1e-5 * mag + 1e-30))
    return ent


def leg_cpu_baseline(args, keep):
    """The oracle as it stands, timed on the host: its range query on a
    sample of the headline batch on one core (the baseline), and its
    brute-force range integral per level
    (the O(k^2) work the method removes).  Then the parity samples of every
    leg: the GPU's outputs against the oracle's FP64 query on the same stored
    tables, |q_gpu - q_64| <= 1e-5 M_q with M_q the sum of the rank terms'
    magnitudes (plus 1e-30 for terms that underflow FP32)."""
    import numpy as np
    from oracle import ndf, query

    try:
        from threadpoolctl import threadpool_limits
    except Exception:      # pragma: no cover
        threadpool_limits = None
    h = keep["c4"]
    vals, scale = stored_tables(h["tabs"])
    q_h = h["q_h"]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    res = {"host_cores": cores}

    def one_core(n):
        ctx = threadpool_limits(1) if threadpool_limits else None
        t0 = time.perf_counter()
        query.range_query(*vals, q_h[:n], scale=scale)
        dt = time.perf_counter() - t0
        if ctx is not None:
            ctx.unregister()
        return dt
    n = 1 << 18
    dt = one_core(n)
    n = int(min(q_h.shape[0], max(n, n * 12.0 / max(dt, 1e-3))))   # about 12 s of work
    dt = one_core(n)
    res["cpu_baseline"] = {"value": n / dt, "unit": "queries/s", "cores": 1, "kind": "oracle",
                           "sample": f"FP64 NumPy oracle range query (oracle.query.range_query) on the first {n} "
                                     "records of the headline batch with its stored FP32 tables, one thread",
                           "seconds": dt}
    log(f"cpu: 1-core oracle {n / dt:.3g} q/s")
    # brute force per level: the cost the constant-cost query removes
    cfg, nxy_h = h["cfg"], h["nxy_h"]
    bfl = []
    rng = np.random.default_rng(31)
    for l in range(cfg.nlevels):
        k = 1 << l
        m = int(max(2, min(2000, 2e6 / (k * k))))
        recs = q_h[rng.choice(q_h.shape[0], m, replace=False)].copy()
        recs[:, 2] = l
        t0 = time.perf_counter()
        ndf.range_bruteforce(nxy_h, cfg.nbins, cfg.sigma, cfg.nlevels, recs)
        dt = time.perf_counter() - t0
        bfl.append({"level": l, "footprint_texels": k * k, "queries": m, "queries_per_s": m / dt})
    res["bruteforce_per_level"] = bfl
    log("cpu: brute force per level done")

    # parity samples
    par = []
    for p in keep["parity"]:
        if p.get("kind") in ("clustered", "clustered_tables"):
            par.append(clustered_parity(p) if p["kind"] == "clustered" else clustered_tables_parity(p))
            log(f"parity {p['leg']}: max |err|/M_q {par[-1]['max_err_over_Mq']:.2e}")
            continue
        v, s = p["tables"]
        want = query.range_query(*v, p["records"], scale=s)
        mag = query.range_query_term_magnitude(*v, p["records"], scale=s)
        nmag = query.range_query_magnitude(*v, p["records"], scale=s)
        got = p["got"].astype(np.float64).reshape(-1)
        err = np.abs(got - want)
        big = np.abs(want) >= 1e-3 * np.max(np.abs(want))
        # terms below the FP32 normal range round absolutely, not relatively:
        # records whose M_q is under 1e-30 are checked against that floor alone
        normal = mag >= 1e-30
        ent = {"leg": p["leg"], "n": int(got.size),
               "max_err_over_Mq": float(np.max(err[normal] / mag[normal])),
               "max_err_over_Nq": float(np.max(err[normal] / np.maximum(nmag[normal], 1e-300))),
               "max_rel_err_where_q_ge_1e-3_max": float(np.max(err[big] / np.abs(want[big]))),
               "records_with_Mq_below_1e-30": int((~normal).sum()),
               "max_abs_err_there": float(np.max(err[~normal])) if (~normal).any() else 0.0,
               "tolerance": "|q_gpu - q_64| <= 1e-5 M_q + 1e-30"}
        ent["pass"] = bool(np.all(err <= 1e-5 * mag + 1e-30))
        if "master" in p:
            vm, sm = p["master"]
            wm = query.range_query(*vm, p["records"], scale=sm)
            ent["vs_fp32_master_rel_l2"] = float(np.linalg.norm(got - wm) / np.linalg.norm(wm))
            ent["vs_fp32_master_max_err_over_Mq"] = float(np.max(np.abs(got - wm) / np.maximum(
                query.range_query_term_magnitude(*vm, p["records"], scale=sm), 1e-300)))
        par.append(ent)
        log(f"parity {p['leg']}: max |err|/M_q {ent['max_err_over_Mq']:.2e}")
    res["parity"] = par
    return res


# ---------------------------------------------------------------------------

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    legs = [] if args.legs.strip() in ("", "none") else [x.strip() for x in args.legs.split(",") if x.strip()]
    for x in legs:
        if x not in LEGS:
            raise SystemExit(f"unknown leg {x!r}; legs are {', '.join(LEGS)}")
    if args.no_cpu_baseline and "cpu_baseline" in legs:
        legs.remove("cpu_baseline")
    keep = {"parity": []}
    head = headline(args, dev, keep)
    res = {
        "metric": "P-NDF range queries/sec + %HBM peak at stated rel. error vs brute-force NDF",
        "value": head["value"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic", "config": head["workload"],
        "roofline": head["roofline"], "error_vs_bruteforce": head["error_vs_bruteforce"],
    }
    fns = {"c3": leg_c3, "c5": leg_c5, "r16": leg_r16, "c2": leg_c2, "clustered": leg_clustered,
           "refine": leg_refine, "sweep": leg_sweep}
    res["legs"] = {}
    for name in legs:
        if name == "cpu_baseline":
            continue
        log(f"leg {name}")
        res["legs"][name] = fns[name](args, dev, keep)
        torch.cuda.empty_cache()
    if args.copy_calibration:
        src = torch.ones(1 << 29, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration done (2 GiB read, 2 GiB written)")
    if "cpu_baseline" in legs:
        log("leg cpu_baseline")
        cpu = leg_cpu_baseline(args, keep)
        res["cpu_baseline"] = cpu.pop("cpu_baseline")
        res["legs"]["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
