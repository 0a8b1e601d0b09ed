#!/usr/bin/env python3
"""Benchmark: one step = the whole glint path on one batch, on one GPU.

Workload (the plain FP32 query at scale): a 512x512 periodic Voronoi flake
map (5000 sites, Beckmann alpha 0.15), intrinsic roughness 0.005, a 64x64
NDF grid, 8 footprint levels (1..128 texels), CP rank 64 fitted by 50 ALS
sweeps, and 1920x1080x8 = 16,588,800 range queries (8 angular boxes per pixel,
pixel-major, box sides log-uniform in [0.005, 0.3]).  Inputs are synthetic and
seeded; they are resident on the GPU before timing starts.

A step runs, in order, every stage of the path:
  build   per-texel binning and the FP32 NDF tensor T[u,v,l,s,t] (34 GB)
  als     50 CP-ALS sweeps on the matrix cores (FP32 MTTKRP, FP64 solves)
  tables  FP32 factor tables and summed-area tables (FP64 prefix sums)
  query   the range query over the whole batch
  grad    MSE gradient against the brute-force range integrals (computed
          once, untimed, as the refinement targets) and the query backward
  adam    one Adam step on the five FP32 factor tables

Prints one JSON line.  value = queries answered per second of whole-step time.
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

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE on this workload,
# scaled by the counters' reading for a plain 2 GiB copy (fetch x2.0, write x1.0);
# see profiles/<kernel>_c2_hbm_traffic.md.  Valid only for the source file they
# were taken with (sha1 of the whole file: a kernel's instantiation depends on
# helpers and constants outside its own text); otherwise traffic is null.
MEASURED_TRAFFIC = {
    "k_mttkrp_y": ("paper_2109_14807_amd/csrc/cp_als.hip", "8f1fc0087c76e7f0be86b1f48cccf40f66e4460d", 36580068392),
    "k_mttkrp_z": ("paper_2109_14807_amd/csrc/cp_als.hip", "8f1fc0087c76e7f0be86b1f48cccf40f66e4460d", 34936702917),
    "k_query": ("paper_2109_14807_amd/csrc/query.hip", "62bcaefe675668a679f218db5c4c145c6ceefd8e", 538682213),
}


def source_sha(path):
    """SHA-1 of a source file's text."""
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter runs, or None once the
    kernel's source file has changed since they were taken."""
    src, sha, nbytes = MEASURED_TRAFFIC[kernel]
    try:
        cur = source_sha(src)
    except OSError:
        return None
    return nbytes if cur == sha and nbytes > 0 else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=10,
                    help="events-timed launches of the MTTKRP and query kernels")
    ap.add_argument("--refine-steps", type=int, default=100,
                    help="Adam steps of the BF16 refinement report (0 to skip)")
    ap.add_argument("--cluster-sweeps", type=int, default=20,
                    help="ALS sweeps of the clustered layout's report (0 skips it)")
    ap.add_argument("--configs", default="",
                    help="comma-separated extra workloads (c1, c3, c4, c5) run end to end on their own "
                         "ALS factors after the step, reported under 'configs'")
    ap.add_argument("--als-only", default="",
                    help="instead of the step: run only the named workload's CP-ALS (--sweeps sweeps, "
                         "texel-space for maps whose tensor does not fit) and print its timing; "
                         "used to profile the ALS kernels at that shape")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 2 GiB device copy (read 2 GiB, write 2 GiB) after the "
                         "steps, the reference for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.als_only:
        print(json.dumps(als_only(args.als_only, args.sweeps)), flush=True)
        return
    cfg = gen.config("c2")
    R, N, nl = cfg.rank, cfg.nbins, cfg.nlevels
    desc = G.desc_of(cfg.nu, cfg.nv, nl, N, cfg.sigma)

    t0 = time.time()
    nxy_h = gen.normal_map(cfg)
    q_h = gen.make_queries(cfg, nxy_h)
    init_h = gen.als_init(cfg)
    nq = q_h.shape[0]
    log(f"inputs generated in {time.time() - t0:.1f}s: {nq} queries")

    nxy = torch.tensor(nxy_h, device=dev)
    q = torch.tensor(q_h, device=dev)
    init = [torch.tensor(a, device=dev) for a in init_h]

    # ---- buffers (allocated once, outside the timed region) ----
    T = torch.empty((cfg.nu, cfg.nv, nl, N, N), dtype=torch.float32, device=dev)
    ws_build = torch.empty(L.glint_build_tensor_workspace(desc), dtype=torch.uint8, device=dev)
    ws_als = torch.empty(L.glint_cp_als_workspace(desc, R, L.GLINT_F32), dtype=torch.uint8, device=dev)
    F = [torch.empty_like(a) for a in init]
    fits = torch.zeros(args.sweeps, dtype=torch.float64, device=dev)
    info = torch.zeros(4, dtype=torch.int32, device=dev)
    rows = (cfg.nu, cfg.nv, nl, N, N)
    P = [torch.empty((r, R), dtype=torch.float32, device=dev) for r in rows]   # FP32 masters
    CS = torch.empty((N + 1, R), dtype=torch.float32, device=dev)
    CT = torch.empty((N + 1, R), dtype=torch.float32, device=dev)
    out = torch.empty(nq, dtype=torch.float32, device=dev)
    gout = torch.empty(nq, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    dT = [torch.empty((r, R), dtype=torch.float32, device=dev) for r in (cfg.nu, cfg.nv, nl, N + 1, N + 1)]
    dS = torch.empty((N, R), dtype=torch.float32, device=dev)
    dTt = torch.empty((N, R), dtype=torch.float32, device=dev)
    adam_m = [torch.zeros_like(p) for p in P]
    adam_v = [torch.zeros_like(p) for p in P]
    fac = L.make_factors(P[0], P[1], P[2], CS, CT)

    # ---- refinement targets: brute-force range integrals, once, untimed ----
    t0 = time.time()
    bins, mass = G.texel_bins(nxy, desc)
    q_bf = torch.empty(nq, dtype=torch.float64, device=dev)
    L.glint_range_bruteforce(desc, bins, mass, q, q_bf)
    torch.cuda.synchronize()
    log(f"brute-force targets in {time.time() - t0:.1f}s")

    stream = torch.cuda.current_stream()
    stages = ["build", "als", "tables", "query", "grad", "adam"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record(stream)
        mark(0)
        L.glint_build_tensor(desc, nxy, T, 0, ws_build)
        mark(1)
        for a, b in zip(F, init):
            a.copy_(b)
        L.glint_cp_als(desc, T, R, args.sweeps, 0.0, *F, fits, info, ws_als)
        mark(2)
        for a, p in zip(F, P):
            L.glint_convert(a, p)
        L.glint_make_cumulative(P[3], CS)
        L.glint_make_cumulative(P[4], CT)
        mark(3)
        L.glint_query(fac, q, out)
        mark(4)
        L.glint_mse_grad(out, q_bf, gout, loss)
        L.glint_query_backward(fac, q, gout, *dT)
        L.glint_cumulative_backward(dT[3], dS)
        L.glint_cumulative_backward(dT[4], dTt)
        mark(5)
        grads = (dT[0], dT[1], dT[2], dS, dTt)
        for k, (p, g) in enumerate(zip(P, grads)):
            L.glint_adam_step(p, g, adam_m[k], adam_v[k], 1e-4, 0.9, 0.999, 1e-8, 1)
        mark(6)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    log(f"{args.steps} timed steps done in {wall:.2f}s")
    stage_ms = {s: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)]))
                for i, s in enumerate(stages)}
    ev_total = float(np.mean([evs[k][0].elapsed_time(evs[k][6]) for k in range(args.steps)]))
    ms_per_step = wall * 1e3 / args.steps
    value = nq / (ms_per_step * 1e-3)

    # ---- quality of this step's result ----
    fit_last = float(fits[-1].item())
    ebf = float((torch.linalg.vector_norm(out.double() - q_bf) / torch.linalg.vector_norm(q_bf)).item())
    # the query as answered before this step's Adam update: re-run the step's query on its tables
    # (out holds it already; P now holds the updated masters, so ebf above is the ALS form's error)

    # ---- per-kernel timing with events (same launches as in the step) ----
    reps = args.kernel_reps
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]

    def timed(fn):
        for i in range(reps):
            e0[i].record(stream)
            fn()
            e1[i].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([e0[i].elapsed_time(e1[i]) for i in range(reps)]))

    M_u = torch.empty((cfg.nu, R), dtype=torch.float64, device=dev)
    M_s = torch.empty((N, R), dtype=torch.float64, device=dev)
    # mode s: U*V table + cell pass (k_mttkrp_y) + split reduction + (s) contraction
    mttkrp_y_ms = timed(lambda: L.glint_mttkrp(desc, T, R, 3, *F, M_s, ws_als))
    # mode u: (s,t) pass (k_mttkrp_z) + u reduction
    mttkrp_z_ms = timed(lambda: L.glint_mttkrp(desc, T, R, 0, *F, M_u, ws_als))
    query_ms = timed(lambda: L.glint_query(fac, q, out))
    # off-grid footprints: the same records at fractional centres and levels
    frac = torch.tensor([0.37, 0.61, 0.25], dtype=torch.float32, device=dev)
    xyl = (q[:, :3].float() + frac).contiguous()
    boxes = q[:, 3:7].contiguous()
    out_tri = torch.empty_like(out)      # `out` keeps the step's query for the parity sample
    tri_ms = timed(lambda: L.glint_query_trilinear(fac, xyl, boxes, out_tri))
    del xyl, boxes, out_tri
    # hierarchical importance sampling: one sample per pixel footprint of the frame
    npix = nq // cfg.boxes_per_point
    s_uvl = q[::cfg.boxes_per_point, :3].contiguous()
    levels = N.bit_length() - 1
    s_rnd = torch.rand((npix, levels + 2), device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    s_h = torch.empty((npix, 2), dtype=torch.float32, device=dev)
    s_pdf = torch.empty(npix, dtype=torch.float32, device=dev)
    s_bins = torch.empty((npix, 2), dtype=torch.int32, device=dev)
    sample_ms = timed(lambda: L.glint_sample(fac, s_uvl, s_rnd, s_h, s_pdf, s_bins))
    # environment-light prefiltering: one SG lobe per pixel footprint (lambda logU[10, 1000],
    # A U[1, 10]) around a half vector near the footprint's normals
    gsg = torch.Generator(device=dev).manual_seed(6)
    sg_h = (torch.rand((npix, 2), device=dev, generator=gsg) * 1.2 - 0.6).contiguous()
    sg_p = torch.stack([torch.exp(math.log(10.0) + torch.rand(npix, device=dev, generator=gsg) * math.log(100.0)),
                        1.0 + 9.0 * torch.rand(npix, device=dev, generator=gsg)], 1).contiguous()
    sg_q = torch.empty((npix, 7), dtype=torch.int32, device=dev)
    sg_out = torch.empty(npix, dtype=torch.float32, device=dev)
    sg_ms = timed(lambda: L.glint_query_sg(fac, s_uvl, sg_h, sg_p, 0.3, sg_q, sg_out))
    del s_uvl, s_rnd, s_h, s_pdf, s_bins, sg_h, sg_p, sg_q, sg_out
    # Wang-tile synthesis: 16 tiles of 64^2 texels (8-texel margins, 5 levels, rank 16,
    # random FP32 tables: the query's cost does not depend on their values); the frame's
    # records read as plane coordinates, levels taken mod 5
    gw = np.random.default_rng(8)
    wS, wm, wnl, wR = 64, 8, 5, 16
    wF = [[torch.tensor(gw.random((n, wR)) * 0.1, device=dev) for n in (wS + 2 * wm, wS + 2 * wm, wnl, N, N)]
          for _ in range(16)]
    wtab = G.wang_tables(wF, wS, wm, 2024, gw.permutation(16))
    wq = q.clone()
    wq[:, 2] = torch.remainder(q[:, 2], wnl)
    wout = torch.empty(nq, dtype=torch.float32, device=dev)
    wstruct = wtab.struct()
    wang_ms = timed(lambda: L.glint_query_wang(wstruct, wq, wout))
    del wF, wtab, wq, wout

    ncells = cfg.nu * cfg.nv * nl
    t_elems = ncells * N * N
    mttkrp_flops = 2.0 * t_elems * R                 # one pass over T, 2R flops per element
    y_tflops = mttkrp_flops / (mttkrp_y_ms * 1e-3) / 1e12
    z_tflops = mttkrp_flops / (mttkrp_z_ms * 1e-3) / 1e12
    q_bytes = nq * (7 * 4 + 4)                       # record in, value out
    q_gbs = q_bytes / (query_ms * 1e-3) / 1e9
    mttkrp_ms = mttkrp_y_ms

    res = {
        "metric": "P-NDF range queries/sec + %HBM peak at stated rel. error vs brute-force NDF",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "c2: 512x512 flake map (5000 sites, alpha 0.15), sigma 0.005, 64x64 NDF bins, "
                        "8 levels (1..128), rank 64, 50 ALS sweeps, 1920x1080x8 frame queries",
            "queries_per_step": nq, "rank": R, "nbins": N, "levels": nl, "als_sweeps": args.sweeps,
            "tensor": "FP32 34.4 GB", "query_tables": "FP32",
        },
        "roofline": {
            "kernel": "k_mttkrp_y, the ALS cell-contraction pass (timed as glint_mttkrp mode s: "
                      "U*V table + k_mttkrp_y + split reduction + s contraction)",
            "bound": "mfma", "achieved": y_tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": y_tflops / FP32_MFMA_PEAK_TFLOPS,
            "traffic": measured_traffic("k_mttkrp_y"),
            "per_launch": {"flops": mttkrp_flops, "ms": mttkrp_y_ms, "algorithmic_bytes": t_elems * 4,
                           "launches_per_step": args.sweeps},
        },
        "mttkrp_z": {
            "kernel": "k_mttkrp_z, the ALS (s,t)-contraction pass (timed as glint_mttkrp mode u)",
            "ms": mttkrp_z_ms, "achieved_tflops": z_tflops, "frac": z_tflops / FP32_MFMA_PEAK_TFLOPS,
            "traffic": measured_traffic("k_mttkrp_z"), "launches_per_step": args.sweeps,
        },
        "query_kernel": {
            "kernel": "k_query<float,float,float,64,8,1024>", "ms": query_ms, "queries_per_s": nq / (query_ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": q_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": q_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("k_query"),
                         "algorithmic_bytes_per_query": 32,
                         "note": "HBM is the nominal bound; the counters in profiles/k_query_c2_lds_counters.md "
                                 "show the on-chip gathers (LDS issue, 7R values per query) binding instead"},
        },
        "query_trilinear_kernel": {
            "kernel": "k_query_trilinear<float,float,64,8>: the batch at fractional centres and levels "
                      "(eight-footprint trilinear blend, two rows per factor)",
            "ms": tri_ms, "queries_per_s": nq / (tri_ms * 1e-3),
        },
        "sample_kernel": {
            "kernel": f"k_sample<float,float,64,8>: one hierarchical NDF importance sample ({levels} levels of "
                      "four-quad range queries) per pixel footprint of the frame",
            "samples": npix, "ms": sample_ms, "samples_per_s": npix / (sample_ms * 1e-3),
        },
        "sg_prefilter_kernel": {
            "kernel": "glint_query_sg: k_sg_records + k_query<float,float,float,64,8,1024> + k_box_average, one "
                      "compact-eps SG box per pixel footprint of the frame, averaged",
            "lookups": npix, "ms": sg_ms, "lookups_per_s": npix / (sg_ms * 1e-3),
        },
        "wang_query_kernel": {
            "kernel": "k_query_wang: range queries on the Wang-tile synthesized plane (16 tiles of 64^2 texels, "
                      "8-texel margins, 5 levels, rank 16 FP32; per record the tile of every overlapped cell "
                      "from the hashed edge colours, summed), the frame's records as plane coordinates",
            "queries": nq, "ms": wang_ms, "queries_per_s": nq / (wang_ms * 1e-3),
        },
        "stages_ms": stage_ms,
        "events_ms_per_step": ev_total,
        "fit_after_als": fit_last,
        "error_vs_bruteforce": ebf,
    }

    log(f"kernels timed: mttkrp cell pass {mttkrp_y_ms:.3f} ms, (s,t) pass {mttkrp_z_ms:.3f} ms, "
        f"query {query_ms:.3f} ms")

    # ---- the same decomposition by the texel-space ALS (T never read) ----
    normT2 = float(torch.sum(T.double() ** 2).item())
    ws_tex = G.texel_workspace(desc, R)
    Ftex = [torch.empty_like(a) for a in init]
    fits_tex = torch.zeros(args.sweeps, dtype=torch.float64, device=dev)

    def texel_als():
        for a, b in zip(Ftex, init):
            a.copy_(b)
        L.glint_cp_als_texel(desc, nxy, R, args.sweeps, 0.0, normT2, *Ftex, fits_tex, info, ws_tex)

    texel_als()
    tex_ms = timed(texel_als)
    als_ms = stage_ms["als"]
    res["als_texel"] = {
        "what": f"glint_cp_als_texel, {args.sweeps} sweeps on the same map and initial factors: the same "
                "contractions evaluated from per-texel bin windows in FP64 (no tensor read)",
        "ms": tex_ms, "dense_als_ms": als_ms, "speedup_over_dense": als_ms / tex_ms,
        "fit": float(fits_tex[-1].item()), "dense_fit_fp32_tensor": fit_last,
        "step_queries_per_s_with_texel_als": nq / ((ms_per_step - als_ms + tex_ms) * 1e-3),
    }
    log(f"texel-space ALS: {tex_ms:.1f} ms vs dense {als_ms:.1f} ms; fit {res['als_texel']['fit']:.6f} "
        f"vs {fit_last:.6f}")
    del ws_tex
    if args.cluster_sweeps > 0:
        res["clustered"] = clustered_report(desc, T, q, q_bf, args.cluster_sweeps, timed)
        log(f"clustered layout: {res['clustered']}")
    if args.refine_steps > 0:
        res["refinement"] = refine_report(cfg, nxy_h, desc, F, q, q_bf, args.refine_steps, timed)
        log(f"refinement report done: {res['refinement']}")
    if args.configs:
        res["configs"] = {}
        for name in [c.strip() for c in args.configs.split(",") if c.strip()]:
            log(f"workload {name}")
            res["configs"][name] = config_report(name, args.sweeps, timed)
            log(f"workload {name}: {res['configs'][name]}")
            torch.cuda.empty_cache()
    if args.copy_calibration:
        src = torch.ones(1 << 29, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration done (2 GiB read, 2 GiB written)")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle samples)")
        res["cpu_baseline"], res["parity_sample"] = cpu_baseline(cfg, nxy_h, q_h, out, P, F, CS, CT,
                                                                  args.sweeps, nq)
    print(json.dumps(res), flush=True)


def refine_report(cfg, nxy_h, desc, F, q, q_bf, steps, timed):
    """BF16 straight-through refinement of this step's ALS factors against the
    brute-force range integrals of the batch, evaluated on a held-out batch:
    error against brute force and query throughput, plain FP32 vs refined BF16."""
    import torch

    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    dev = q.device
    q_ev_h = gen.make_queries(cfg, nxy_h, nq=1 << 21, seed=gen.query_seed(cfg) + 7, shuffle=True)
    q_ev = torch.tensor(q_ev_h, device=dev)
    bins, mass = G.texel_bins(torch.tensor(nxy_h, device=dev), desc)
    bf_ev = torch.empty(q_ev.shape[0], dtype=torch.float64, device=dev)
    L.glint_range_bruteforce(desc, bins, mass, q_ev, bf_ev)

    def ebf(tables):
        out = G.query(tables, q_ev)
        return float((torch.linalg.vector_norm(out.double() - bf_ev) / torch.linalg.vector_norm(bf_ev)).item())

    masters = [f.float() for f in F]
    plain = G.make_tables(*masters, dtype="f32", cum_dtype="f32")
    rms = float(torch.sqrt(torch.mean(torch.cat([m.flatten() for m in masters]) ** 2)).item())
    lr = 1e-3 * rms
    t0 = time.perf_counter()
    refined, losses = G.refine(*masters, q, q_bf, steps=steps, lr=lr, dtype="bf16")
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    bf16 = G.make_tables(*refined, dtype="bf16", cum_dtype="bf16")
    plain_bf16 = G.make_tables(*masters, dtype="bf16", cum_dtype="bf16")
    out = torch.empty(q.shape[0], dtype=torch.float32, device=dev)
    f_plain, f_bf16, f_pb = plain.factors(), bf16.factors(), plain_bf16.factors()
    ms_plain = timed(lambda: L.glint_query(f_plain, q, out))
    ms_bf16 = timed(lambda: L.glint_query(f_bf16, q, out))
    ms_pb = timed(lambda: L.glint_query(f_pb, q, out))
    ms_plain2 = timed(lambda: L.glint_query(f_plain, q, out))

    def subnormal(tabs):
        n = 0
        for t in (tabs.U, tabs.V, tabs.L, tabs.CS, tabs.CT):
            x = t.float().abs()
            n += int(((x > 0) & (x < torch.finfo(torch.float32).tiny)).sum().item())
        return n
    e_plain, e_bf16 = ebf(plain), ebf(bf16)
    ls = losses.cpu().numpy()
    return {
        "adam_steps": steps, "lr": lr, "seconds": t_ref,
        "train_loss_first_last": [float(ls[0]), float(ls[-1])],
        "heldout_queries": int(q_ev.shape[0]),
        "error_vs_bruteforce_plain_f32": e_plain,
        "error_vs_bruteforce_refined_bf16": e_bf16,
        "query_ms_plain_f32": ms_plain, "query_ms_refined_bf16": ms_bf16,
        "query_ms_plain_bf16": ms_pb, "query_ms_plain_f32_again": ms_plain2,
        "subnormal_entries_refined_bf16": subnormal(bf16),
        "speedup_bf16_over_f32": ms_plain / ms_bf16,
        "equal_or_lower_error": bool(e_bf16 <= e_plain),
    }


def clustered_report(desc, T, q, q_bf, sweeps, timed, t=16, cs=8, R=16):
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
    query_ms = timed(lambda: L.glint_query_clustered(st, q, out))
    ebf = float((torch.linalg.vector_norm(out.double() - q_bf) / torch.linalg.vector_norm(q_bf)).item())
    # importance sampling on these tables (block by mass, then quads): one sample per pixel footprint
    npix = q.shape[0] // 8
    s_uvl = q[::8, :3].contiguous()
    s_rnd = torch.rand((npix, (t.bit_length() - 1) + 3), device=q.device,
                       generator=torch.Generator(device=q.device).manual_seed(8))
    s_h = torch.empty((npix, 2), dtype=torch.float32, device=q.device)
    s_pdf = torch.empty(npix, dtype=torch.float32, device=q.device)
    s_bins = torch.empty((npix, 2), dtype=torch.int32, device=q.device)
    sample_ms = timed(lambda: L.glint_sample_clustered(st, s_uvl, s_rnd, s_h, s_pdf, s_bins))
    del s_uvl, s_rnd, s_h, s_pdf, s_bins
    info = tab.info.cpu().tolist()
    ntensor = tab.X.shape[0]
    stacked = info[3]                                 # non-blank image blocks over all block tensors
    tt = t * t
    flops = 2 * 2.0 * tt * stacked * R                # P = D Z and Z = D^T (X kr Y), per sweep
    dbytes = 2 * 4.0 * tt * stacked                   # the two streams over the stacked blocks
    tf = flops / (sweep_ms * 1e-3) / 1e12
    gbs = dbytes / (sweep_ms * 1e-3) / 1e9
    return {
        "what": f"per-(region, angular block) rank-{R} CP: {t}x{t} bin blocks, {cs}x{cs} texel regions, "
                f"{sweeps} FP64 ALS sweeps per block tensor (blank blocks skipped), FP32 tables",
        "block_tensors": ntensor, "blank": info[1], "solve_failures": info[0],
        "als_ms_incl_tables": als_ms, "one_sweep_call_ms": one_ms, "als_ms_per_sweep": sweep_ms,
        # R/2 flop per streamed byte (8 at rank 16) sits under the FP64 matrix balance
        # (78.6 TFLOP/s / 8 TB/s = 9.8): HBM is the nearer bound
        "roofline": {"kernel": f"k_cluster_als<float,{R}> (two FP64 MFMA streams over the stacked D per sweep)",
                     "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "per_sweep": {"stream_bytes": dbytes, "flops": flops, "fp64_tflops": tf,
                                   "fp64_frac": tf / FP64_MFMA_PEAK_TFLOPS}},
        "stacked_blocks": info[3],
        "query_ms": query_ms, "queries_per_s": q.shape[0] / (query_ms * 1e-3),
        "sample_ms": sample_ms, "samples_per_s": npix / (sample_ms * 1e-3),
        "error_vs_bruteforce": ebf,
        "table_bytes": int(4 * (tab.CX.numel() + tab.CY.numel() + tab.Z.numel())),
    }


def als_only(name, sweeps):
    """CP-ALS of one workload alone (one untimed warm-up run of 1 sweep first)."""
    import torch

    import gen
    import paper_2109_14807_amd as G

    dev = torch.device("cuda:0")
    cfg = gen.config(name)
    nxy = torch.tensor(gen.normal_map(cfg), device=dev)
    desc = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    init = [torch.tensor(a, device=dev) for a in gen.als_init(cfg)]
    dense = cfg.nu * cfg.nv <= 64 * 64
    if dense:
        T = G.build_tensor(nxy, desc, dtype=torch.float64)
        ws = G.als_workspace(desc, cfg.rank, T.dtype)
        run = lambda k: G.cp_als(T, desc, init, k, workspace=ws)
    else:
        ws = G.texel_workspace(desc, cfg.rank)
        run = lambda k: G.cp_als_texel(nxy, desc, init, k, workspace=ws)
    run(1)
    torch.cuda.synchronize()
    log(f"{name}: warm-up done; {sweeps} sweeps")
    t0 = time.perf_counter()
    res = run(sweeps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    return {"workload": name, "als": "dense FP64" if dense else "texel-space FP64", "rank": cfg.rank,
            "sweeps": sweeps, "ms": ms, "ms_per_sweep": ms / sweeps, "workspace_bytes": int(ws.numel()),
            "info": res.info.cpu().tolist()}


def config_report(name, sweeps, timed):
    """One workload end to end on its own inputs: CP-ALS (dense FP64 tensor for
    the 64x64 map, texel-space ALS for the maps whose tensor does not fit),
    query tables in the workload's storage types, the batch's query time, and
    the relative L2 error against brute-force range integrals on a sample of
    the batch (the FP32 tables' error beside it).  The 2048x2048 FP32 workload
    adds Adam refinement of the factors over its 2^24-record batch."""
    import numpy as np
    import torch

    import gen
    import paper_2109_14807_amd as G
    from paper_2109_14807_amd import _lib as L

    dev = torch.device("cuda:0")
    cfg = gen.config(name)
    t0 = time.time()
    nxy_h = gen.normal_map(cfg)
    nxy = torch.tensor(nxy_h, device=dev)
    desc = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    grouped = cfg.query_kind == "sg_grouped"
    if grouped:
        uvl_h, boxes_h = gen.make_grouped_queries(cfg, nxy_h)
        uvl, boxes = torch.tensor(uvl_h, device=dev), torch.tensor(boxes_h, device=dev)
        nq = boxes_h.shape[0] * boxes_h.shape[1]
    else:
        q_h = gen.make_queries(cfg, nxy_h)
        q = torch.tensor(q_h, device=dev)
        nq = q_h.shape[0]
    rep = {"inputs_s": time.time() - t0, "queries": nq, "rank": cfg.rank, "sweeps": sweeps,
           "storage": f"{cfg.dtype}/{cfg.cum_dtype}"}
    log(f"  {name}: inputs ready ({nq} queries)")
    init = [torch.tensor(a, device=dev) for a in gen.als_init(cfg)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if cfg.nu * cfg.nv <= 64 * 64:
        T = G.build_tensor(nxy, desc, dtype=torch.float64)
        res = G.cp_als(T, desc, init, sweeps)
        rep["als"] = "dense FP64"
        torch.cuda.synchronize()
        rep["fit"] = float(res.fits[-1])
        del T
    else:
        res = G.cp_als_texel(nxy, desc, init, sweeps)
        rep["als"] = "texel-space FP64"
        torch.cuda.synchronize()
        rep["fit"] = None
    rep["als_s"] = time.perf_counter() - t0
    F = res.factors
    log(f"  {name}: ALS done in {rep['als_s']:.2f}s")

    # brute-force sample of the batch
    rng = np.random.default_rng(11)
    ns = min(nq, 1 << 18)
    idx = torch.tensor(np.sort(rng.choice(nq, ns, replace=False)), device=dev)
    if grouped:
        K = boxes.shape[1]
        flat = torch.cat([uvl[idx // K], boxes.reshape(-1, 4)[idx]], dim=1).contiguous()
    else:
        flat = q[idx].contiguous()
    bins, mass = G.texel_bins(nxy, desc)
    bf = torch.empty(ns, dtype=torch.float64, device=dev)
    L.glint_range_bruteforce(desc, bins, mass, flat, bf)

    def ebf(tables):
        out = G.query(tables, flat)
        return float((torch.linalg.vector_norm(out.double() - bf) / torch.linalg.vector_norm(bf)).item())

    tabs = G.make_tables(*F, dtype=cfg.dtype, cum_dtype=cfg.cum_dtype)
    f32 = G.make_tables(*F)
    rep["error_vs_bruteforce"] = ebf(tabs)
    rep["error_vs_bruteforce_f32_tables"] = ebf(f32)
    fac = tabs.factors()
    if grouped:
        out = torch.empty(boxes.shape[:2], dtype=torch.float32, device=dev)
        ms = timed(lambda: L.glint_query_grouped(fac, uvl, boxes, out))
    else:
        out = torch.empty(nq, dtype=torch.float32, device=dev)
        ms = timed(lambda: L.glint_query(fac, q, out))
    rep["query_ms"] = ms
    rep["queries_per_s"] = nq / (ms * 1e-3)
    if name == "c4":
        # Adam refinement of the FP32 factors over the whole batch, against its
        # brute-force integrals; error on a held-out batch of the same recipe
        t0 = time.time()
        tgt = torch.empty(nq, dtype=torch.float64, device=dev)
        L.glint_range_bruteforce(desc, bins, mass, q, tgt)
        q_ev = torch.tensor(gen.make_queries(cfg, nxy_h, nq=1 << 18, seed=gen.query_seed(cfg) + 7,
                                             shuffle=True), device=dev)
        bf_ev = torch.empty(q_ev.shape[0], dtype=torch.float64, device=dev)
        L.glint_range_bruteforce(desc, bins, mass, q_ev, bf_ev)
        torch.cuda.synchronize()
        rep["refine_targets_s"] = time.time() - t0
        log(f"  {name}: brute-force targets in {rep['refine_targets_s']:.1f}s; refining")
        masters = [f.float() for f in F]
        rms = float(torch.sqrt(torch.mean(torch.cat([m.flatten() for m in masters]) ** 2)).item())
        steps = 200

        def ebf_ev(tables):
            o = G.query(tables, q_ev)
            return float((torch.linalg.vector_norm(o.double() - bf_ev) / torch.linalg.vector_norm(bf_ev)).item())

        rep["heldout_error_before"] = ebf_ev(f32)
        rep["refinement"] = []
        for rel_lr in (1e-4, 3e-4, 1e-3):
            t0 = time.perf_counter()
            refined, losses = G.refine(*masters, q, tgt, steps=steps, lr=rel_lr * rms, dtype="f32")
            torch.cuda.synchronize()
            ls = losses.cpu().numpy()
            rep["refinement"].append({
                "adam_steps": steps, "lr": rel_lr * rms, "ms_per_step": (time.perf_counter() - t0) * 1e3 / steps,
                "train_loss_first_last": [float(ls[0]), float(ls[-1])],
                "heldout_error_after": ebf_ev(G.make_tables(*refined))})
            log(f"  {name}: refinement lr {rel_lr:g} x rms: {rep['refinement'][-1]}")
    return rep


def cpu_baseline(cfg, nxy_h, q_h, out_dev, P, F, CS, CT, sweeps, nq):
    """The FP64 oracle timed on bounded samples of each stage and scaled to
    the whole step (plus a parity check of sampled outputs of this step)."""
    import numpy as np
    import torch

    from oracle import cp_als, ndf, query

    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        threads = 1
    cores = os.cpu_count() or 1
    t_total = 0.0
    parts = {}
    N, R, nl = cfg.nbins, cfg.rank, cfg.nlevels

    # build: brute force on a 32x32 crop of the map, 5 levels, scaled by texel-visit count
    crop = np.ascontiguousarray(nxy_h[:32, :32])
    t0 = time.perf_counter()
    ndf.ndf_bruteforce(crop, N, cfg.sigma, 5)
    dt = time.perf_counter() - t0
    scale = (cfg.nu * cfg.nv * sum(4 ** l for l in range(nl))) / (32 * 32 * sum(4 ** l for l in range(5)))
    parts["build_s"] = dt * scale

    # ALS: one plain sweep on a 16x16x8 tensor of the same cell shape, scaled by |T| and sweeps
    Ts = np.random.default_rng(0).random((16, 16, nl, N, N))
    init = [np.random.default_rng(1).random((d, R)) for d in (16, 16, nl, N, N)]
    t0 = time.perf_counter()
    cp_als.cp_als(Ts, init, iters=1)
    dt = time.perf_counter() - t0
    parts["als_s"] = dt * (cfg.nu * cfg.nv) / (16 * 16) * sweeps

    # query and its gradient on the FP32 tables of this step
    tabs = [p.double().cpu().numpy() for p in P[:3]] + [CS.double().cpu().numpy(), CT.double().cpu().numpy()]
    ns = 1_000_000
    qs = q_h[:ns]
    t0 = time.perf_counter()
    qv = query.range_query(*tabs, qs)
    dt = time.perf_counter() - t0
    parts["query_s"] = dt * nq / ns
    t0 = time.perf_counter()
    query.range_query_grad(*tabs, qs[:200_000], np.ones(200_000))
    dt = time.perf_counter() - t0
    parts["grad_s"] = dt * nq / 200_000
    t_total = sum(parts.values())

    # parity: 10^5 sampled outputs of this step's query against the oracle on the same tables
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(nq, 100_000, replace=False))
    got = out_dev.double().cpu().numpy()  # out holds the last query over these tables
    want = query.range_query(*tabs, q_h[idx])
    mag = query.range_query_magnitude(*tabs, q_h[idx])
    rel = np.abs(got[idx] - want) / np.maximum(mag, 1e-300)
    del qv
    cpu = {"value": nq / t_total, "unit": "queries/s", "cores": int(threads), "host_cores": int(cores),
           "kind": "oracle",
           "sample": "FP64 NumPy oracle per stage, scaled to the step: brute-force NDF on a 32x32 crop "
                     "(5 levels) x texel visits; one plain ALS sweep on a 16x16x8x64x64 tensor x |T| x "
                     f"{sweeps}; range query on 1e6 and its gradient on 2e5 of the batch x batch size",
           "stage_seconds": parts}
    parity = {"n": int(idx.size), "max_err_over_Nq": float(rel.max()), "tolerance": 1e-5,
              "pass": bool(rel.max() <= 1e-5)}
    return cpu, parity


if __name__ == "__main__":
    main()
