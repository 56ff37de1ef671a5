"""Throughput of the APC hot path on one MI355X.

One step = one frame of the whole path on the largest single-GPU workload:
stage one (boundary-face binning + tet walk + power moments) for all 72
subdomains, the canonical-order moment sum, and stage two (the same walk with
the FP64 moment bound) with the final renormalised image.  Inputs (mesh,
transfer function, camera) are resident in HBM before timing starts.

Prints ONE JSON line.  `value` is ray samples per second (pieces generated
per frame / frame time); frames/s, per-kernel times, the roofline figure of
the dominant kernel, sampled parity against the FP64 oracle, and the oracle's
own throughput on a bounded pixel sample of the same frame are reported beside
it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray samples/s + frames/s at 2560², m=8; p50/p99 frame latency (served)"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic work per unit: FP64 flops of one sample's moment bound, bytes of one tet, vertex and piece
FP64_FLOPS_PER_PIECE_M8 = 250.0   # per-sample moment bound at m = 8
TET_BYTES = 32.0                  # vertex ids + neighbour codes of one tet
VERT_BYTES = 16.0                 # x, y, z, scalar
STAGE_BYTES = 12.0                # one staged piece of stage two: z, a, s


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_large_2560_m8.json")


def measured_traffic(args, kernel):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) of `kernel` from the committed
    rocprofv3 record of the default large workload, or None when the workload differs or the kernel
    sources changed since the counters were taken."""
    import hashlib
    if args.workload != "large" or args.size or args.grid or args.m or not os.path.exists(TRAFFIC_RECORD):
        return None, "no counter record for this workload"
    rec = json.load(open(TRAFFIC_RECORD))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None, "kernel sources changed since the counters were taken"
    b = rec["bytes_per_launch"].get(kernel)
    if b is None:
        return None, "kernel not in the counter record"
    return int(b["fetch_bytes"] + b["write_bytes"]), "profiles/traffic_large_2560_m8.json (read %.3g B + write %.3g B)" % (
        b["fetch_bytes"], b["write_bytes"])


def batching_frames(sc, steps=3):
    """Frames of the batching configuration (its adaptive mesh, 72 uneven subdomains, 2560^2, m = 8, stage one
    summing the subdomains): two untimed frames (the first sizes the piece store), then `steps` timed ones."""
    import torch
    import paper_2501_12581_amd as apc
    ctx = apc.Context(0)
    r = apc.Renderer(ctx, sc)
    for _ in range(2):
        r.frame(fused=True)
    torch.cuda.synchronize()
    ctx.counters(reset=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    kern = {"moments_ms": 0.0, "eval_ms": 0.0, "stage_ms": 0.0}
    for _ in range(steps):
        r.frame(fused=True)
        tk = ctx.timings()
        for key in kern:
            kern[key] += tk[key] / steps
    stream.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    cnt = ctx.counters()
    walks = 1 if kern["stage_ms"] == 0.0 else 2
    pieces = cnt["pieces"] / (walks * float(steps))
    del r
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out = {"workload": "batching: %d tets (32^3 base refined 0-3 levels, cone decomposition), 72 Morton subdomains "
                       "of tet-count ratio 12, %dx%d perspective view, m=%d" % (
                           sc.mesh.n_tets, sc.view["width"], sc.view["height"], sc.m),
           "steps": steps, "ms_per_step": round(ms, 3), "frames_per_s": round(1e3 / ms, 3),
           "samples_per_s": round(pieces / (ms / 1e3), 1), "samples_per_frame": int(pieces),
           "kernels_ms": {k: round(v, 3) for k, v in kern.items()}}
    log("batching frames: %s" % out)
    return out


def serve_run(n_requests, slots=4, workspace_limit=40 << 30, small_slots=0, small_workspace_limit=12 << 30,
              sc=None):
    """p50/p99 frame latency of a served request stream, batched (`slots` slots for any size and `small_slots`
    for sizes up to 1024^2) and one at a time, on the batching configuration's mesh (`sc`, else generated)."""
    import synth
    from paper_2501_12581_amd.serve import Server
    t0 = time.time()
    if sc is None:
        sc = synth.scene_batching(size=1024)
    m = sc.mesh
    tfs = [synth.make_tf(s) for s in (21, 22, 23)]
    srv = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=slots,
                 workspace_limit=workspace_limit, hbm_budget=64 << 30, small_slots=small_slots, small_size=1024,
                 small_workspace_limit=small_workspace_limit)
    srv.warm()  # every slot's library buffers at the largest request's size before serving
    log("serving: %d tets (adaptive), 72 uneven subdomains, generated, resident and warm in %.1fs" % (
        m.n_tets, time.time() - t0))
    warm = synth.request_stream(8, rate=1000.0, seed=99)
    srv.run(warm, "batched")
    srv.run(warm, "fifo")
    res = {}
    for rate in (50.0, 30.0):  # the specified rate, and one below what this GPU sustains for this mix
        reqs = synth.request_stream(n_requests, rate=rate, seed=12)
        for mode in ("batched", "fifo"):
            st = srv.run(reqs, mode)
            st.pop("records")
            res["%s_%g" % (mode, rate)] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            log("serving %g/s %s: %s" % (rate, mode, res["%s_%g" % (mode, rate)]))
    srv.close()
    return {"workload": "batching mesh: %d tets (32^3 base refined 0-3 levels, cone decomposition), 72 Morton "
                        "subdomains of tet-count ratio 12; "
                        "%d requests per run, Poisson arrivals, sizes {256,512,1024,2048}^2, m in {4,6,8}, "
                        "3 transfer functions, cameras on the radius-2 sphere" % (m.n_tets, n_requests),
            "rate_50_per_s": {"batched": res["batched_50"], "one_at_a_time": res["fifo_50"]},
            "rate_30_per_s": {"batched": res["batched_30"], "one_at_a_time": res["fifo_30"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["large", "batching", "medium", "tiny", "slabs"])
    ap.add_argument("--ranks", type=int, default=16, help="slabs workload: subdomains (4 slabs each)")
    ap.add_argument("--m", type=int, default=None, help="override the number of moments (4, 6, 8)")
    ap.add_argument("--tile-width", type=int, default=None, help="pixels per tile row (tile = w x 64/w)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the tile shape with the autotuner first (on by default for the batching workload)")
    ap.add_argument("--size", type=int, default=None, help="override the image size (square)")
    ap.add_argument("--grid", type=int, default=None, help="override cubes per axis (large workload)")
    ap.add_argument("--cpu-pixels", type=int, default=65536, help="oracle sample size (0 = skip)")
    ap.add_argument("--profile-steps", action="store_true", help="no oracle leg and no serving run (for profiler runs)")
    ap.add_argument("--separate-sum", action="store_true",
                    help="time frames with per-subdomain moment images + apc_sum_moments (the form several GPUs "
                         "would run) instead of stage one summing the subdomains itself")
    ap.add_argument("--serve-requests", type=int, default=120,
                    help="requests of the serving run (Poisson, 50/s, batching mesh); 0 = skip")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU path (subdomains sharded over GPUs with an "
              "all-reduce of the moment image) is not implemented; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 256 << 20
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 3}), flush=True)
        return

    import paper_2501_12581_amd as apc
    import synth

    t0 = time.time()
    if args.workload == "large":
        kw = {}
        if args.size:
            kw["size"] = args.size
        if args.grid:
            kw["n"] = args.grid
        sc = synth.scene_large(**kw)
    elif args.workload == "batching":
        sc = synth.scene_batching(**({"size": args.size} if args.size else {}))
    elif args.workload == "medium":
        sc = synth.scene_medium(**({"size": args.size} if args.size else {}))
    elif args.workload == "slabs":
        sc = synth.scene_slabs(n_ranks=args.ranks, size=args.size or 2560)
    else:
        sc = synth.scene_tiny()
    if args.m:
        sc.m = args.m
        sc.bias = synth.default_bias(args.m)
    mesh = sc.mesh
    log("generated %s: %d tets, %d vertices, %d subdomains in %.1fs" % (
        sc.name, mesh.n_tets, mesh.n_vertices, mesh.n_sub, time.time() - t0))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = apc.Context(0)
    t0 = time.time()
    r = apc.Renderer(ctx, sc, device=dev)
    torch.cuda.synchronize()
    info = r.mesh.info()
    log("mesh resident in %.1fs: %d boundary faces, %.2f GB" % (
        time.time() - t0, info["n_boundary_faces"], info["device_bytes"] / 1e9))

    tuned = None
    if args.tile_width:
        ctx.set_tile_shape(args.tile_width)
    if args.autotune or (args.workload == "batching" and not args.tile_width):
        best, ms = ctx.autotune_tile_shape(r.mesh, r.view, r.tf, r.mboit, r.subs, r.moments, r.rgba, repeats=1)
        tuned = {"best_width": best, "frame_ms_by_width": {str(k): round(v, 3) for k, v in ms.items()}}
        log("autotuned tile: %s" % tuned)
    fused = not args.separate_sum  # one GPU holds every subdomain: stage one sums them (APC_MOMENTS_GLOBAL)
    for _ in range(args.warmup):
        r.frame(fused=fused)
    torch.cuda.synchronize()
    log("warmup done")
    ctx.counters(reset=True)
    kern = {"bin_ms": 0.0, "moments_ms": 0.0, "sum_ms": 0.0, "resolve_ms": 0.0, "stage_ms": 0.0, "eval_ms": 0.0}
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    frame_ms = []
    for k in range(args.steps):
        f0 = time.perf_counter()
        r.frame(fused=fused)
        # the library records HIP events around each kernel on this stream; reading them waits for the frame
        tk = ctx.timings()
        stream.synchronize()
        frame_ms.append((time.perf_counter() - f0) * 1e3)
        for key in kern:
            kern[key] += tk[key]
        log("step %d: %.1f ms (moments %.1f, resolve %.1f = re-walk %.1f + evaluation %.1f)" % (
            k, frame_ms[-1], tk["moments_ms"], tk["resolve_ms"], tk["stage_ms"], tk["eval_ms"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    tile_shape = list(ctx.tile_shape())
    ms_per_step = elapsed * 1e3 / args.steps
    cnt = ctx.counters()
    walks = 1 if kern["stage_ms"] == 0.0 else 2  # stage two walks again unless stage one kept the pieces
    pieces_per_frame = cnt["pieces"] / (walks * float(args.steps))   # every walk counts its pieces
    steps_per_frame = cnt["tet_steps"] / (walks * float(args.steps))
    for key in kern:
        kern[key] /= args.steps
    samples_per_s = pieces_per_frame / (ms_per_step / 1e3)

    # ---- segments per pixel (what a sort-last compositor would exchange) vs APC's fixed exchange
    segs = ctx.segment_counts(r.view.height, r.view.width).reshape(2, -1)
    met = segs[1]
    cov = met > 0
    n_cov = int(cov.sum().item())
    seg_stats = {"covered_pixels": n_cov,
                 "segments_mean": round(segs[0][cov].double().mean().item(), 4) if n_cov else 0.0,
                 "segments_max": int(segs[0].max().item()),
                 "subdomains_met_mean": round(met[cov].double().mean().item(), 4) if n_cov else 0.0,
                 "apc_exchanged_per_pixel_mean": round(2.0 * met[cov].double().mean().item(), 4) if n_cov else 0.0,
                 "apc_exchanged_upper_bound": 2 * mesh.n_sub}

    # ---- roofline of the dominant kernel
    H, W, m = r.view.height, r.view.width, sc.m
    S = mesh.n_sub
    mesh_bytes = mesh.n_tets * TET_BYTES + mesh.n_vertices * VERT_BYTES
    pairs = int(met.sum().item())  # (pixel, subdomain) pairs with pieces
    if fused:  # each pair's moments enter the sum once; the global image is written once
        mom_bytes = (pairs + H * W) * (m + 1) * 4.0
        mom_label = "per-pair moments + global image"
    else:  # the API's dense per-subdomain images
        mom_bytes = S * (m + 1) * H * W * 4.0
        mom_label = "dense per-subdomain moments"
    kept = kern["stage_ms"] == 0.0  # stage one kept its pieces: no second walk
    kept_bytes = pieces_per_frame * STAGE_BYTES if kept else 0.0
    rooflines = {
        "k_moments": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                      "achieved": (mesh_bytes + mom_bytes + kept_bytes) / (kern["moments_ms"] / 1e3) / 1e9,
                      "per_launch": "mesh %.3g B + %s %.3g B + kept pieces %.3g B" % (
                          mesh_bytes, mom_label, mom_bytes, kept_bytes)},
        "k_stage": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                    "achieved": (mesh_bytes + pieces_per_frame * STAGE_BYTES) / (max(kern["stage_ms"], 1e-9) / 1e3) / 1e9,
                    "per_launch": "mesh %.3g B + staged pieces %.3g B" % (mesh_bytes, pieces_per_frame * STAGE_BYTES)},
        "k_eval": {"bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
                   "achieved": FP64_FLOPS_PER_PIECE_M8 * pieces_per_frame / (kern["eval_ms"] / 1e3) / 1e12,
                   "per_launch": "%d FP64 flops x %.4g pieces" % (FP64_FLOPS_PER_PIECE_M8, pieces_per_frame)},
    }
    timed = {"k_moments": kern["moments_ms"], "k_stage": kern["stage_ms"], "k_eval": kern["eval_ms"]}
    if kept:
        del rooflines["k_stage"], timed["k_stage"]
    dom = max(timed, key=timed.get)
    rf = rooflines[dom]
    traffic, traffic_note = measured_traffic(args, dom)
    roofline = {"kernel": dom, "kernel_ms": round(timed[dom], 3), "bound": rf["bound"], "achieved": round(rf["achieved"], 4), "peak": rf["peak"],
                "unit": rf["unit"], "frac": round(rf["achieved"] / rf["peak"], 5), "traffic": traffic,
                "traffic_source": traffic_note,
                "work_per_launch": rf["per_launch"],
                "other": {k: {"bound": v["bound"], "achieved": round(v["achieved"], 4), "unit": v["unit"],
                              "frac": round(v["achieved"] / v["peak"], 5)} for k, v in rooflines.items()
                          if k != dom}}

    # ---- sampled parity + CPU baseline (FP64 oracle on a bounded pixel sample)
    cpu = None
    parity = None
    variants = None
    if args.cpu_pixels > 0 and not args.profile_steps:
        import oracle
        pix = np.sort(np.random.default_rng(11).choice(H * W, min(args.cpu_pixels, H * W), replace=False))
        threads = min(16, os.cpu_count() or 1)  # the host share of one GPU
        log("oracle on %d sampled pixels with %d threads" % (len(pix), threads))
        t0 = time.perf_counter()
        ref = oracle.render(sc, pixels=pix, threads=threads)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(ref["n_pieces"] / cpu_s, 1), "unit": "samples/s", "cores": threads, "kind": "oracle",
               "sample": "%d seeded pixels of the same %dx%d frame (%d samples, both passes, %.1f s)" % (
                   len(pix), W, H, ref["n_pieces"], cpu_s)}
        mom = r.moments.reshape(m + 1, -1)[:, torch.as_tensor(pix, device=dev)].double().cpu().numpy()
        rgba = r.rgba.reshape(-1, 4)[torch.as_tensor(pix, device=dev)].double().cpu().numpy()
        from oracle.parity import moment_parity
        mp = moment_parity(sc, pix, mom, ref, tol=1e-5, floor=1e-3, threads=threads)
        d = rgba - ref["rgba"]
        parity = {"pixels": int(len(pix)), "covered": mp["covered"], "background_exact": mp["background_exact"],
                  "moments_rel_max_forward": mp["forward_max"],
                  "moments_backward_bar_pixels": mp["backward_bar_pixels"],
                  "moments_outside_backward_band": mp["outside_backward_band"],
                  "rgba_max_abs": float(np.abs(d).max()), "rgba_rmse": float(math.sqrt(np.mean(d ** 2)))}
        log("parity %s" % parity)
        # FP16 moment-image variant (ln b0, b_j / b0), run after the timed frames on the same sample
        mom_timed = r.moments.clone()
        r.frame(moments_f16=True, fused=fused)
        rgba16 = r.rgba.reshape(-1, 4)[torch.as_tensor(pix, device=dev)].double().cpu().numpy()
        d16 = rgba16 - ref["rgba"]
        variants = {"fp16_moments": {
            "rgba_max_abs": float(np.abs(d16).max()), "rgba_rmse": float(math.sqrt(np.mean(d16 ** 2))),
            "moment_image_bytes": int(r.moments_h.numel() * 2), "fp32_moment_image_bytes": int(r.moments.numel() * 4)}}
        # the other form of stage one + sum: its frames' time and whether its global moments are bitwise equal
        other = []
        for _ in range(2):
            f0 = time.perf_counter()
            r.frame(fused=not fused)
            tk = ctx.timings()
            torch.cuda.synchronize()
            other.append(((time.perf_counter() - f0) * 1e3, tk["moments_ms"], tk["sum_ms"]))
        variants["separate_sum" if fused else "fused_sum"] = {
            "frame_ms": round(other[-1][0], 2), "moments_ms": round(other[-1][1], 3),
            "sum_ms": round(other[-1][2], 3) if fused else 0.0,
            "global_moments_bitwise_equal": bool(torch.equal(r.moments, mom_timed))}
        log("variants %s" % variants)

    # ---- serving: continuous batching vs one request at a time (after the frame buffers are released)
    serving = batching = None
    if args.serve_requests > 0 and not args.profile_steps:
        del r
        import gc
        gc.collect()
        ctx.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        t0 = time.time()
        bsc = synth.scene_batching() if args.workload != "batching" else sc
        log("batching mesh: %d tets in %.1fs" % (bsc.mesh.n_tets, time.time() - t0))
        if args.workload != "batching":  # the batching configuration's frames, beside the headline workload's
            batching = batching_frames(bsc)
        serving = serve_run(args.serve_requests, sc=bsc)

    out = {
        "metric": METRIC, "value": round(samples_per_s, 1), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d tets (%s), %d %s subdomains, %dx%d %s view, m=%d" % (
            sc.name, mesh.n_tets, "adaptive: 32^3 base refined 0-3 levels, cone decomposition"
            if args.workload == "batching" else "jittered Kuhn grid", S,
            {"slabs": "interleaved-slab (4 slabs each)", "batching": "Morton (tet-count ratio 12)"}.get(
                args.workload, "Morton"),
            W, H, "perspective" if sc.view["projection"] else "orthographic", m),
            "global_batch": 1, "seq_len": None, "parallelism": "single GPU, all subdomains on device"},
        "frames_per_s": round(1e3 / ms_per_step, 4),
        "samples_per_frame": int(pieces_per_frame), "tet_steps_per_frame": int(steps_per_frame),
        "kernels_ms": {k: round(v, 3) for k, v in kern.items()},
        "stage_one_sums_subdomains": fused,
        "frame_ms_each": [round(x, 2) for x in frame_ms],
        "tile_shape": tile_shape, "autotune": tuned,
        "segments": seg_stats, "counters": cnt, "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "variants": variants,
        "batching": batching, "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
