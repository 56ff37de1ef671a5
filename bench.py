"""Throughput of the APC hot path on one MI355X.

One step = one frame of the whole path in its plain form on the largest
single-GPU workload (256^3 x 6 = 100,663,296 tets, 72 Morton subdomains,
2560^2, m = 8): stage one (boundary-face binning, tet walk, power moments) for
all 72 subdomains with the canonical-order moment sum, then stage two (the
same walk again, every piece weighted at once by the FP64 moment bound) with
the final renormalised image.  Frames cycle over the workload's 5 seeded orbit
cameras.  Inputs (mesh, transfer function, cameras) are resident in HBM before
timing starts.

Prints ONE JSON line.  `value` is ray samples per second over the timed frames
(pieces generated per frame / frame time); frames/s is 1 / the median over the
cameras of their mean frame time.  Reported beside it: per-kernel times, the
roofline figure of the dominant kernel (algorithmic bytes or flops of the
method only), sampled parity against the FP64 oracle, the oracle's own
throughput on a bounded pixel sample, labelled variants (kept pieces, the
separate moment sum, FP16 moment images, a HIP-graph replay, the RGBA copy to
the host), the batching configuration and the serving run.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray samples/s + frames/s at 2560², m=8; p50/p99 frame latency (served)"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic work per unit: FP64 flops of one sample's moment bound at m = 8, bytes of one tet and vertex
FP64_FLOPS_PER_PIECE_M8 = 250.0
TET_BYTES = 32.0                  # vertex ids + neighbour codes of one tet
VERT_BYTES = 16.0                 # x, y, z, scalar
PIECE_BYTES = 12.0                # one kept piece: z, a, s
N_CAMERAS = 5


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
    return int(b["fetch_bytes"] + b["write_bytes"]), "%s (read %.3g B + write %.3g B)" % (
        os.path.relpath(TRAFFIC_RECORD, ROOT), b["fetch_bytes"], b["write_bytes"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads():
    """Threads for the oracle: the job's CPU share (OMP_NUM_THREADS where the host sets it, else the CPUs
    this process may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def camera_views(args, sc):
    import synth
    seed = {"large": synth.LARGE_SEED, "batching": synth.BATCHING_SEED}.get(args.workload)
    if seed is None:  # the other workloads have one camera
        return [sc.view]
    W = sc.view["width"]
    return [synth.orbit_view(seed, c, W) for c in range(N_CAMERAS)]


class Frames:
    """Frames of one renderer over a list of cameras, in the plain form unless `keep`.  by_pair: both passes
    walk the (tile, subdomain) pairs in parallel -- stage one into the tiles form, summed in order (the same
    global moments, bit for bit), stage two into per-pair colour sums, summed in order and finalised (the
    image to FP32 rounding); else one workgroup per tile walks all its subdomains in each pass."""

    def __init__(self, r, ctx, views, global_sum=True, keep=False, by_pair=False):
        """views: camera dicts, or the apc_view structures of another Frames."""
        import paper_2501_12581_amd as apc
        self.r, self.ctx, self.global_sum, self.keep = r, ctx, global_sum, keep
        self.by_pair = by_pair and global_sum and not keep
        self.views = [apc.make_view(v, r.scene.step) if isinstance(v, dict) else v for v in views]

    def frame(self, c, by_tile=False, **kw):
        """by_tile: this frame's stage one one workgroup per tile whatever self.by_pair says (it keeps the
        per-pixel segment statistics the pair form does not)."""
        self.r.view = self.views[c]
        bp = self.by_pair and not by_tile
        return self.r.frame(global_sum=self.global_sum, keep=self.keep, by_pair=bp, resolve_by_pair=bp, **kw)

    def survey(self):
        """One untimed frame per camera (sizes the library's buffers): pieces, segment statistics and
        (pixel, subdomain) pairs of every camera."""
        import torch
        out = []
        for c in range(len(self.views)):
            self.ctx.counters(reset=True)
            self.frame(c, by_tile=True)
            torch.cuda.synchronize()
            cnt = self.ctx.counters()
            walks = 2 if self.ctx.timings()["rewalk_ms"] > 0 else 1
            v = self.views[c]
            segs = self.ctx.segment_counts(v.height, v.width).reshape(2, -1)
            met = segs[1]
            cov = met > 0
            n_cov = int(cov.sum().item())
            out.append({"pieces": cnt["pieces"] / walks, "tet_steps": cnt["tet_steps"] / walks,
                        "pairs": int(met.sum().item()), "covered_pixels": n_cov,
                        "segments_mean": segs[0][cov].double().mean().item() if n_cov else 0.0,
                        "segments_max": int(segs[0].max().item()),
                        "subdomains_met_mean": met[cov].double().mean().item() if n_cov else 0.0,
                        "counters": cnt})
        return out

    def timed(self, steps, first=0):
        """`steps` frames, camera (first + k) mod n for frame k, each timed from the host (the library's
        HIP events are read after each frame, which waits for it)."""
        import torch
        keys = ("bin_ms", "moments_ms", "sum_ms", "resolve_ms", "rewalk_ms", "eval_ms")
        kern = {k: [] for k in keys}
        frame_ms, cams = [], []
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(steps):
            c = (first + k) % len(self.views)
            f0 = time.perf_counter()
            self.frame(c)
            tk = self.ctx.timings()
            stream.synchronize()
            frame_ms.append((time.perf_counter() - f0) * 1e3)
            cams.append(c)
            for key in keys:
                kern[key].append(tk[key])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        per_cam = {}
        for c, ms in zip(cams, frame_ms):
            per_cam.setdefault(c, []).append(ms)
        cam_mean = {c: float(np.mean(v)) for c, v in per_cam.items()}
        return {"elapsed_s": elapsed, "frame_ms": frame_ms, "cameras": cams, "kernels": kern,
                "camera_mean_ms": cam_mean, "median_camera_ms": float(np.median(list(cam_mean.values())))}


def roofline_figures(mesh, m, H, W, survey, run, by_pair=False):
    """Per-kernel rooflines from the method's own work (algorithmic bytes and flops): stage one
    reads each touched tet and vertex once and writes each (pixel, subdomain) pair's m+1 moments (by_pair:
    into the tiles, which the ordered sum reads back into the global image; else into the sum plus the
    global image); stage two reads the mesh again and the global image and writes the colour; its dominant
    cost is the moment bound, ~250 FP64 flops per piece at m = 8."""
    mesh_bytes = mesh.n_tets * TET_BYTES + mesh.n_vertices * VERT_BYTES
    cams, kern = run["cameras"], run["kernels"]
    img = 0 if by_pair else H * W
    mom_bytes = sum(mesh_bytes + (survey[c]["pairs"] + img) * (m + 1) * 4.0 for c in cams)
    res_bytes = sum(mesh_bytes + H * W * ((m + 1) * 4.0 + 16.0) for c in cams)
    flops = sum(FP64_FLOPS_PER_PIECE_M8 * survey[c]["pieces"] for c in cams) if m == 8 else None
    t_mom = sum(kern["moments_ms"]) / 1e3
    t_res = sum(kern["rewalk_ms"]) / 1e3
    n = len(cams)
    out = {
        "k_moments": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "kernel_ms": 1e3 * t_mom / n,
                      "achieved": mom_bytes / t_mom / 1e9,
                      "work_per_launch": "mesh %%.3g B (each tet 32 B + each vertex 16 B) + %s x "
                                         "(m+1) x 4 B moments, %%.3g B on average" % (
                                             "(pixel, subdomain) pairs" if by_pair else "(pairs + pixels)") % (
                                             mesh_bytes, mom_bytes / n)},
    }
    t_sum = sum(kern["sum_ms"]) / 1e3
    if by_pair and t_sum > 0:
        sum_bytes = sum((survey[c]["pairs"] + H * W) * (m + 1) * 4.0 for c in cams)
        out["k_sum_tiles"] = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "kernel_ms": 1e3 * t_sum / n,
                              "achieved": sum_bytes / t_sum / 1e9,
                              "work_per_launch": "(pixel, subdomain) pairs read + pixels written, x (m+1) x 4 B, "
                                                 "%.3g B on average" % (sum_bytes / n)}
    if t_res > 0 and flops is not None:
        out["k_resolve"] = {"bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS, "kernel_ms": 1e3 * t_res / n,
                            "achieved": flops / t_res / 1e12,
                            "work_per_launch": "%d FP64 flops x %.4g pieces (moment bound per piece, m = 8)" % (
                                FP64_FLOPS_PER_PIECE_M8, flops / n / FP64_FLOPS_PER_PIECE_M8),
                            "hbm_view": {"achieved_gbs": res_bytes / t_res / 1e9,
                                         "frac": res_bytes / t_res / 1e9 / HBM_PEAK_GBS,
                                         "bytes_per_launch": res_bytes / n}}
    for v in out.values():
        v["frac"] = v["achieved"] / v["peak"]
    return out


def oracle_leg(args, sc, r, ctx, survey0, rgba_cam0, mom_cam0, kept_rgba0):
    """Sampled parity (camera 0) and the oracle's throughput on the same sample."""
    import torch
    import oracle
    import synth
    from oracle.parity import moment_parity
    H, W, m = sc.view["height"], sc.view["width"], sc.m
    dev = rgba_cam0.device
    pix = np.sort(np.random.default_rng(11).choice(H * W, min(args.cpu_pixels, H * W), replace=False))
    threads = host_threads()
    log("oracle on %d sampled pixels with %d threads" % (len(pix), threads))
    t0 = time.perf_counter()
    ref = oracle.render(sc, pixels=pix, threads=threads)
    cpu_s = time.perf_counter() - t0
    rate = ref["n_pieces"] / cpu_s
    idx = torch.as_tensor(pix, device=dev)
    mom = mom_cam0.reshape(m + 1, -1)[:, idx].double().cpu().numpy()
    rgba = rgba_cam0.reshape(-1, 4)[idx].double().cpu().numpy()
    mp = moment_parity(sc, pix, mom, ref, tol=1e-5, floor=1e-3, threads=threads)
    d = rgba - ref["rgba"]
    parity = {"pixels": int(len(pix)), "camera": 0, "covered": mp["covered"],
              "background_exact": mp["background_exact"],
              "moments_rel_forward": {k: mp[k] for k in ("forward_max", "forward_p50", "forward_p99", "forward_p999")},
              "moments_backward_bar_pixels": mp["backward_bar_pixels"],
              "moments_outside_backward_band": mp["outside_backward_band"],
              "rgba_max_abs": float(np.abs(d).max()), "rgba_rmse": float(math.sqrt(np.mean(d ** 2)))}
    if kept_rgba0 is not None:
        dk = kept_rgba0.reshape(-1, 4)[idx].double().cpu().numpy() - ref["rgba"]
        parity["kept_pieces_rgba_max_abs"] = float(np.abs(dk).max())
        parity["kept_pieces_rgba_rmse"] = float(math.sqrt(np.mean(dk ** 2)))
    log("parity %s" % parity)
    # the tiny workload's full frame on one thread, and on the job's threads
    tiny = synth.scene_tiny()
    t0 = time.perf_counter()
    rt = oracle.render(tiny, threads=1)
    tiny_1 = time.perf_counter() - t0
    cpu = {"value": round(rate, 1), "unit": "samples/s", "cores": threads, "kind": "oracle",
           "sample": "%d seeded pixels of the same %dx%d frame, camera 0 (%d samples, both passes, %.1f s)" % (
               len(pix), W, H, ref["n_pieces"], cpu_s),
           "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
           "extrapolated_s_per_frame": round(survey0["pieces"] / rate, 1),
           "extrapolated_note": "camera 0's samples per frame / the sample's samples/s (extrapolated, not run)",
           "tiny_full_frame_1_thread_s": round(tiny_1, 3), "tiny_samples": int(rt["n_pieces"])}
    return ref, pix, parity, cpu


def apc_vs_exact(threads):
    """The method against exact sorted compositing of the same pieces (a report, not a bar): the tiny
    workload in full and the medium workload on a seeded pixel sample."""
    import oracle
    import synth
    out = {}
    for name, sc, pix in (("tiny_128", synth.scene_tiny(), None),
                          ("medium_1024_sampled", synth.scene_medium(), np.sort(
                              np.random.default_rng(5).choice(1024 * 1024, 16384, replace=False)))):
        ref = oracle.render(sc, pixels=pix, exact=True, threads=threads)
        d = ref["rgba"] - ref["exact"]
        mse = float(np.mean(d ** 2))
        out[name] = {"pixels": int(ref["rgba"].shape[0]), "max_abs": float(np.abs(d).max()),
                     "rmse": math.sqrt(mse), "psnr_db": 10 * math.log10(1.0 / mse) if mse > 0 else None,
                     "mean_alpha_apc": float(ref["rgba"][:, 3].mean()),
                     "mean_alpha_exact": float(ref["exact"][:, 3].mean())}
    return out


def variants_leg(args, sc, r, ctx, fr, survey, rgba0, mom0):
    """Labelled variants of the same frames: kept pieces (stage one keeps every piece, stage two evaluates
    them without walking again), the separate moment sum (per-subdomain images + apc_sum_moments, the form
    several GPUs would run), FP16 moment images, a HIP-graph replay of the frame, and the frame with the
    RGBA image copied to host memory."""
    import torch
    import paper_2501_12581_amd as apc
    out = {}
    n_cam = len(fr.views)
    # kept pieces, every camera: a sizing frame, then a timed one
    kf = Frames(r, ctx, fr.views, keep=True)
    kept_ms, kern = [], {"moments_ms": [], "eval_ms": []}
    kept0 = None
    for c in range(n_cam):
        kf.frame(c)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        kf.frame(c)
        tk = ctx.timings()
        torch.cuda.synchronize()
        kept_ms.append((time.perf_counter() - f0) * 1e3)
        kern["moments_ms"].append(tk["moments_ms"])
        kern["eval_ms"].append(tk["eval_ms"])
        if c == 0:
            kept0 = r.rgba.clone()
    kept_pieces = float(np.mean([s["pieces"] for s in survey]))
    out["kept_pieces"] = {
        "frame_ms_by_camera": [round(x, 2) for x in kept_ms], "median_frame_ms": round(float(np.median(kept_ms)), 3),
        "frames_per_s": round(1e3 / float(np.median(kept_ms)), 4),
        "kernels_ms_mean": {k: round(float(np.mean(v)), 3) for k, v in kern.items()},
        "piece_store_bytes_per_frame": kept_pieces * PIECE_BYTES,
        "rgba_max_abs_vs_plain_camera0": float((kept0 - rgba0).abs().max().item())}
    ctx.set_workspace_limit(1 << 20)  # gives the pool back
    ctx.set_workspace_limit(0)
    log("kept pieces %s" % out["kept_pieces"])
    # the separate moment sum (camera 0)
    sf = Frames(r, ctx, fr.views, global_sum=False)
    other = []
    for _ in range(2):
        f0 = time.perf_counter()
        sf.frame(0)
        tk = ctx.timings()
        torch.cuda.synchronize()
        other.append(((time.perf_counter() - f0) * 1e3, tk["moments_ms"], tk["sum_ms"]))
    out["separate_sum"] = {"frame_ms": round(other[-1][0], 2), "moments_ms": round(other[-1][1], 3),
                           "sum_ms": round(other[-1][2], 3),
                           "global_moments_bitwise_equal": bool(torch.equal(r.moments, mom0)),
                           "rgba_bitwise_equal": bool(torch.equal(r.rgba, rgba0))}
    dense_bytes = int(r.per_sub.numel() * 4)
    out["separate_sum"]["per_subdomain_image_bytes"] = dense_bytes
    r._per_sub = None
    torch.cuda.empty_cache()
    log("separate sum %s" % out["separate_sum"])
    # the frames in the other form over every camera: one workgroup per tile (all its subdomains, stage
    # one's sum folded in), or by (tile, subdomain) pairs and ordered sums in both passes
    of = Frames(r, ctx, fr.views, by_pair=not fr.by_pair)
    of_ms, of_mom, of_sum, of_rw = [], [], [], []
    for c in range(n_cam):
        of.frame(c)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        of.frame(c)
        tk = ctx.timings()
        torch.cuda.synchronize()
        of_ms.append((time.perf_counter() - f0) * 1e3)
        of_mom.append(tk["moments_ms"])
        of_sum.append(tk["sum_ms"])
        of_rw.append(tk["rewalk_ms"])
        if c == 0:
            same_mom = bool(torch.equal(r.moments, mom0))
            rgba_diff = float((r.rgba - rgba0).abs().max().item())
    key = "frames_by_pair" if of.by_pair else "frames_by_tile"
    out[key] = {"frame_ms_by_camera": [round(x, 2) for x in of_ms], "median_frame_ms": round(float(np.median(of_ms)), 3),
                "moments_ms_mean": round(float(np.mean(of_mom)), 3), "sum_ms_mean": round(float(np.mean(of_sum)), 3),
                "rewalk_ms_mean": round(float(np.mean(of_rw)), 3),
                "global_moments_bitwise_equal_camera0": same_mom, "rgba_max_abs_diff_camera0": rgba_diff}
    log("%s %s" % (key, out[key]))
    # the same per-subdomain moments as tiles of the (tile, subdomain) pairs with binned faces, one
    # workgroup per tile walking all its subdomains (camera 0)
    r.view = fr.views[0]
    m1 = r.moments.shape[0]
    n = ctx.moments_pass_tiles(r.mesh, r.view, r.tf, m1 - 1, r.subs)
    tiles = torch.empty((n, m1, 64), dtype=torch.float32, device=r.moments.device)
    pair_bin = torch.empty((n,), dtype=torch.int32, device=r.moments.device)
    glob = torch.empty_like(r.moments)
    for _ in range(2):
        f0 = time.perf_counter()
        ctx.moments_pass_tiles(r.mesh, r.view, r.tf, m1 - 1, r.subs, tiles, pair_bin)
        ctx.sum_moment_tiles(tiles, pair_bin, n, len(r.subs), m1 - 1, r.view.height, r.view.width, glob)
        tk = ctx.timings()
        torch.cuda.synchronize()
        t_ms = (time.perf_counter() - f0) * 1e3
    out["moment_tiles"] = {"pairs": int(n), "tile_bytes": int(tiles.numel() * 4 + pair_bin.numel() * 4),
                           "dense_bytes": dense_bytes, "moments_and_sum_ms": round(t_ms, 2),
                           "moments_ms": round(tk["moments_ms"], 3), "sum_ms": round(tk["sum_ms"], 3),
                           "global_moments_bitwise_equal": bool(torch.equal(glob, mom0))}
    del tiles, pair_bin, glob
    torch.cuda.empty_cache()
    log("moment tiles %s" % out["moment_tiles"])
    # FP16 moment images (camera 0); their error against the oracle is added by the oracle leg
    fr.frame(0, moments_f16=True)
    torch.cuda.synchronize()
    out["fp16_moments"] = {"moment_image_bytes": int(r.moments_h.numel() * 2),
                           "fp32_moment_image_bytes": int(r.moments.numel() * 4)}
    rgba16 = r.rgba.clone()
    # HIP graph of the plain frame (camera 0): replays timed with events on the current stream
    r.view = fr.views[0]
    g = apc.FrameGraph(r, global_sum=True)
    try:
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g.launch()
        torch.cuda.synchronize()
        reps = 3
        e0.record(stream)
        for _ in range(reps):
            g.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        out["graph_replay"] = {"ms_per_frame": round(e0.elapsed_time(e1) / reps, 3),
                               "rgba_bitwise_equal_to_eager": bool(torch.equal(r.rgba, rgba0))}
    finally:
        g.close()
    # the frame with its image copied to pinned host memory (camera 0)
    host = torch.empty(r.rgba.shape, dtype=torch.float32, pin_memory=True)
    d2h = []
    for _ in range(3):
        f0 = time.perf_counter()
        fr.frame(0)
        host.copy_(r.rgba, non_blocking=True)
        torch.cuda.synchronize()
        d2h.append((time.perf_counter() - f0) * 1e3)
    out["with_rgba_d2h"] = {"frame_ms": round(float(np.median(d2h)), 3), "rgba_bytes": int(r.rgba.numel() * 4)}
    log("variants %s" % {k: out[k] for k in ("fp16_moments", "graph_replay", "with_rgba_d2h")})
    return out, kept0, rgba16


def passes_by_size(ctx, r, seed, sizes=(256, 512, 1024, 2048, 2560)):
    """Both passes of orbit camera 0 at several image sizes on the renderer's mesh: one workgroup per tile
    against one per (tile, subdomain) pair plus the ordered sum of the pairs, each the best of 3 by the
    library's HIP events; stage one's global moments compared bit for bit, stage two's images by their
    largest difference."""
    import torch
    import paper_2501_12581_amd as apc
    import synth
    m, S, out = r.scene.m, len(r.subs), {}
    dev = r.moments.device
    for size in sizes:
        v = apc.make_view(synth.orbit_view(seed, 0, size), r.scene.step)
        mom = torch.empty((m + 1, size, size), dtype=torch.float32, device=dev)
        glob = torch.empty_like(mom)
        rgba = torch.empty((size, size, 4), dtype=torch.float32, device=dev)
        n = ctx.moments_pass_tiles(r.mesh, v, r.tf, m, r.subs)
        tiles = torch.empty((max(n, 1), m + 1, 64), dtype=torch.float32, device=dev)
        pb = torch.empty((max(n, 1),), dtype=torch.int32, device=dev)
        res = {"pairs": int(n), "tiles": -(-size // ctx.tile_shape()[0]) * -(-size // ctx.tile_shape()[1])}
        for form in ("by_tile", "by_pair"):
            best = None
            for _ in range(3):
                if form == "by_tile":
                    ctx.moments_pass(r.mesh, v, r.tf, m, r.subs, mom, None, global_sum=True)
                else:
                    ctx.moments_pass_tiles(r.mesh, v, r.tf, m, r.subs, tiles, pb, by_pair=True)
                    ctx.sum_moment_tiles(tiles, pb, n, S, m, size, size, glob)
                tk = ctx.timings()
                torch.cuda.synchronize()
                t = tk["moments_ms"] + (tk["sum_ms"] if form == "by_pair" else 0.0)
                best = t if best is None else min(best, t)
            res[form + "_ms"] = round(best, 3)
        res["global_moments_bitwise_equal"] = bool(torch.equal(glob, mom))
        rgba2 = torch.empty_like(rgba)
        for form in ("by_tile", "by_pair"):
            best = None
            for _ in range(3):
                ctx.resolve_pass(r.mesh, v, r.tf, r.mboit, mom, r.subs, rgba2 if form == "by_pair" else rgba,
                                 finalize=True, by_pair=form == "by_pair")
                t = ctx.timings()["rewalk_ms"]
                torch.cuda.synchronize()
                best = t if best is None else min(best, t)
            res["rewalk_" + form + "_ms"] = round(best, 3)
        res["rgba_max_abs_diff"] = float((rgba2 - rgba).abs().max().item())
        out[str(size)] = res
        log("both passes at %d^2: %s" % (size, res))
        del mom, glob, rgba, rgba2, tiles, pb
    torch.cuda.empty_cache()
    return out


def batching_leg(bsc, steps=5):
    """The batching configuration (adaptive mesh, 72 uneven subdomains, 2560^2, m = 8): the autotuned tile
    shape, plain frames over the 5 orbit cameras, the kept-piece variant, and a HIP-graph replay of the
    plain frame against the eager one."""
    import torch
    import paper_2501_12581_amd as apc
    import synth
    ctx = apc.Context(0)
    r = apc.Renderer(ctx, bsc)
    best, mode, table = ctx.autotune_launch(r.mesh, r.view, r.tf, r.mboit, r.subs, r.moments, r.rgba, repeats=1)
    ms = {w: v for (d, w), v in table.items() if d == apc.APC_DISPATCH_GRID}
    views = [synth.orbit_view(synth.BATCHING_SEED, c, bsc.view["width"]) for c in range(N_CAMERAS)]
    fr = Frames(r, ctx, views)
    survey = fr.survey()
    run = fr.timed(steps)
    pieces = [survey[c]["pieces"] for c in run["cameras"]]
    out = {"workload": "batching: %d tets (32^3 base refined 0-3 levels, cone decomposition), 72 Morton subdomains "
                       "of tet-count ratio 12, %dx%d perspective views (5 orbit cameras), m=%d" % (
                           bsc.mesh.n_tets, bsc.view["width"], bsc.view["height"], bsc.m),
           "autotune": {"best_width": best, "best_dispatch": "queue" if mode == apc.APC_DISPATCH_QUEUE else "grid",
                        "frame_ms_by_width": {str(k): round(v, 3) for k, v in ms.items()},
                        "queue_frame_ms_by_width": {str(w): round(v, 3) for (d, w), v in table.items()
                                                    if d == apc.APC_DISPATCH_QUEUE}},
           "steps": steps, "ms_per_step": round(run["elapsed_s"] * 1e3 / steps, 3),
           "median_camera_frame_ms": round(run["median_camera_ms"], 3),
           "frames_per_s": round(1e3 / run["median_camera_ms"], 3),
           "samples_per_s": round(sum(pieces) / run["elapsed_s"], 1),
           "kernels_ms_mean": {k: round(float(np.mean(v)), 3) for k, v in run["kernels"].items()}}
    # kept pieces (camera 0) and the graph of the plain frame (camera 0)
    kf = Frames(r, ctx, views, keep=True)
    for _ in range(2):
        f0 = time.perf_counter()
        kf.frame(0)
        torch.cuda.synchronize()
    out["kept_pieces_frame_ms_camera0"] = round((time.perf_counter() - f0) * 1e3, 3)
    ctx.set_workspace_limit(1 << 20)
    ctx.set_workspace_limit(0)
    eager = []
    for _ in range(3):
        f0 = time.perf_counter()
        fr.frame(0)
        torch.cuda.synchronize()
        eager.append((time.perf_counter() - f0) * 1e3)
    rgba0 = r.rgba.clone()
    r.view = fr.views[0]
    g = apc.FrameGraph(r, global_sum=True)
    try:
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g.launch()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(3):
            g.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        out["camera0_eager_frame_ms"] = round(float(np.median(eager)), 3)
        out["camera0_graph_replay_ms"] = round(e0.elapsed_time(e1) / 3, 3)
        out["graph_rgba_bitwise_equal"] = bool(torch.equal(r.rgba, rgba0))
    finally:
        g.close()
    # the same plain frames in the other dispatch mode than the autotuned one (a persistent launch taking
    # tiles from a work queue, or one workgroup per tile): all 5 cameras, each pass's kernel time
    other = apc.APC_DISPATCH_GRID if mode == apc.APC_DISPATCH_QUEUE else apc.APC_DISPATCH_QUEUE
    ctx.set_dispatch(other)
    try:
        fr.frame(0)
        torch.cuda.synchronize()
        same = bool(torch.equal(r.rgba, rgba0))
        qrun = fr.timed(steps)
        out["other_dispatch"] = {
            "dispatch": "queue" if other == apc.APC_DISPATCH_QUEUE else "grid",
            "median_camera_frame_ms": round(qrun["median_camera_ms"], 3),
            "kernels_ms_mean": {k: round(float(np.mean(v)), 3) for k, v in qrun["kernels"].items()},
            "rgba_bitwise_equal_camera0": same}
    finally:
        ctx.set_dispatch(mode)
    out["passes_by_size_camera0"] = passes_by_size(ctx, r, synth.BATCHING_SEED)
    del fr, kf, r
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("batching %s" % out)
    return out


def serve_leg(n_requests, n_requests_30, sc):
    """p50/p99 frame latency of a served request stream on the batching configuration's mesh: batched
    (continuous batching over slots) against one request at a time, both in the plain form with both passes by
    (tile, subdomain) pairs; at 30 requests/s also with both passes by tiles."""
    import synth
    from paper_2501_12581_amd.serve import Server
    t0 = time.time()
    m = sc.mesh
    tfs = [synth.make_tf(s) for s in (21, 22, 23)]
    srv = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=4,
                 hbm_budget=16 << 30, by_pair=True)
    srv.warm()
    log("serving: %d tets, resident and warm in %.1fs" % (m.n_tets, time.time() - t0))
    warm = synth.request_stream(8, rate=1000.0, seed=99)
    srv.run(warm, "batched")
    srv.run(warm, "fifo")
    res = {}
    for rate, n in ((50.0, n_requests), (30.0, n_requests_30)):
        if n <= 0:
            continue
        reqs = synth.request_stream(n, rate=rate, seed=12)
        for mode in ("batched", "fifo"):
            st = srv.run(reqs, mode)
            st.pop("records")
            res["%s_%g" % (mode, rate)] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            log("serving %g/s %s: %s" % (rate, mode, res["%s_%g" % (mode, rate)]))
    if n_requests_30 > 0:
        srv.by_pair = False
        reqs = synth.request_stream(n_requests_30, rate=30.0, seed=12)
        for mode in ("batched", "fifo"):
            st = srv.run(reqs, mode)
            st.pop("records")
            res["%s_by_tile_30" % mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            log("serving 30/s %s, by tiles: %s" % (mode, res["%s_by_tile_30" % mode]))
    srv.close()
    out = {"workload": "batching mesh: %d tets, 72 Morton subdomains of tet-count ratio 12; Poisson arrivals, sizes "
                       "{256,512,1024,2048}^2, m in {4,6,8}, 3 transfer functions, cameras on the radius-2 sphere; "
                       "plain form (stage two walks again), both passes by (tile, subdomain) pairs" % m.n_tets}
    for rate in (50, 30):
        if "batched_%d" % rate in res:
            out["rate_%d_per_s" % rate] = {"batched": res["batched_%d" % rate], "one_at_a_time": res["fifo_%d" % rate]}
    if "batched_by_tile_30" in res:
        out["rate_30_per_s_by_tiles"] = {"batched": res["batched_by_tile_30"],
                                                   "one_at_a_time": res["fifo_by_tile_30"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["large", "batching", "medium", "tiny", "slabs"])
    ap.add_argument("--ranks", type=int, default=16, help="slabs workload: subdomains (4 slabs each)")
    ap.add_argument("--m", type=int, default=None, help="override the number of moments (4, 6, 8)")
    ap.add_argument("--tile-width", type=int, default=None, help="pixels per tile row (tile = w x 64/w)")
    ap.add_argument("--autotune", action="store_true", help="pick the tile shape with the autotuner first")
    ap.add_argument("--size", type=int, default=None, help="override the image size (square)")
    ap.add_argument("--grid", type=int, default=None, help="override cubes per axis (large workload)")
    ap.add_argument("--by-pair", action="store_true",
                    help="both passes by (tile, subdomain) pairs, each followed by the pairs' ordered sum "
                         "(default: one workgroup per tile walks all its subdomains)")
    ap.add_argument("--keep", action="store_true",
                    help="time the kept-piece variant (stage one keeps every piece for stage two) instead of the "
                         "plain form")
    ap.add_argument("--cpu-pixels", type=int, default=65536, help="oracle sample size (0 = skip)")
    ap.add_argument("--profile-steps", action="store_true",
                    help="only the timed frames (no variants, oracle, batching or serving legs; for profiler runs)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per mode of the 50/s serving run (batching mesh); 0 = no serving")
    ap.add_argument("--serve-requests-30", type=int, default=600, help="requests per mode at 30/s")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (every subdomain of the frame on one device); a run on %d GPUs "
              "is not available" % args.gpus, file=sys.stderr)
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
    if args.autotune:
        best, mode, table = ctx.autotune_launch(r.mesh, r.view, r.tf, r.mboit, r.subs, r.moments, r.rgba, repeats=1)
        tuned = {"best_width": best, "best_dispatch": "queue" if mode == apc.APC_DISPATCH_QUEUE else "grid",
                 "frame_ms": {"%s/%d" % ("queue" if d else "grid", w): round(v, 3) for (d, w), v in table.items()}}
        log("autotuned launch: %s" % tuned)

    views = camera_views(args, sc)
    fr = Frames(r, ctx, views, keep=args.keep, by_pair=args.by_pair)
    by_pair = fr.by_pair
    survey = fr.survey()  # one untimed frame per camera
    rgba0, mom0 = None, None
    for k in range(args.warmup):
        fr.frame(k % len(views))
    torch.cuda.synchronize()
    log("survey + %d warm-up frames done" % args.warmup)
    ctx.counters(reset=True)
    run = fr.timed(args.steps)
    cnt = ctx.counters()
    tile_shape = list(ctx.tile_shape())
    H, W, m = r.view.height, r.view.width, sc.m
    samples = sum(survey[c]["pieces"] for c in run["cameras"])
    samples_per_s = samples / run["elapsed_s"]
    ms_per_step = run["elapsed_s"] * 1e3 / args.steps
    for k in range(args.steps):
        log("step %d (camera %d): %.1f ms (moments %.1f, re-walk %.1f, evaluation %.1f)" % (
            k, run["cameras"][k], run["frame_ms"][k], run["kernels"]["moments_ms"][k], run["kernels"]["rewalk_ms"][k],
            run["kernels"]["eval_ms"][k]))
    kern_mean = {k: round(float(np.mean(v)), 3) for k, v in run["kernels"].items()}

    rooflines = roofline_figures(mesh, m, H, W, survey, run, by_pair=by_pair)
    timed = {k: v["kernel_ms"] for k, v in rooflines.items()}
    dom = max(timed, key=timed.get)
    rf = rooflines[dom]
    traffic, traffic_note = measured_traffic(args, dom)
    algo_bytes = None
    if rf["bound"] == "hbm":
        algo_bytes = rf["achieved"] * 1e9 * rf["kernel_ms"] / 1e3
    roofline = {"kernel": dom, "kernel_ms": round(rf["kernel_ms"], 3), "bound": rf["bound"],
                "achieved": round(rf["achieved"], 4), "peak": rf["peak"], "unit": rf["unit"],
                "frac": round(rf["frac"], 5), "traffic": traffic, "traffic_source": traffic_note,
                "traffic_over_algorithmic": round(traffic / algo_bytes, 2) if (traffic and algo_bytes) else None,
                "work_per_launch": rf["work_per_launch"],
                "other": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                          for k, v in rooflines.items() if k != dom}}

    seg_stats = {k: round(float(np.mean([s[k] for s in survey])), 4)
                 for k in ("covered_pixels", "segments_mean", "subdomains_met_mean")}
    seg_stats["segments_max"] = int(max(s["segments_max"] for s in survey))
    seg_stats["apc_exchanged_per_pixel_mean"] = round(2.0 * seg_stats["subdomains_met_mean"], 4)
    seg_stats["apc_exchanged_upper_bound"] = 2 * mesh.n_sub

    cpu = parity = variants = None
    exact_report = None
    if not args.profile_steps:
        fr.frame(0)
        torch.cuda.synchronize()
        rgba0, mom0 = r.rgba.clone(), r.moments.clone()
        kept0 = rgba16 = None
        if not args.keep:
            variants, kept0, rgba16 = variants_leg(args, sc, r, ctx, fr, survey, rgba0, mom0)
        if args.cpu_pixels > 0:
            sc0 = synth.Scene(**{**sc.__dict__, "view": views[0]})
            ref, pix, parity, cpu = oracle_leg(args, sc0, r, ctx, survey[0], rgba0, mom0, kept0)
            if rgba16 is not None:
                d16 = rgba16.reshape(-1, 4)[torch.as_tensor(pix, device=dev)].double().cpu().numpy() - ref["rgba"]
                variants["fp16_moments"].update(rgba_max_abs=float(np.abs(d16).max()),
                                                rgba_rmse=float(math.sqrt(np.mean(d16 ** 2))))
            exact_report = apc_vs_exact(host_threads())
            log("APC vs exact compositing %s" % exact_report)

    batching = serving = None
    if not args.profile_steps and (args.serve_requests > 0 or args.workload != "batching"):
        del r, fr
        import gc
        gc.collect()
        ctx.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        t0 = time.time()
        bsc = synth.scene_batching() if args.workload != "batching" else sc
        log("batching mesh: %d tets in %.1fs" % (bsc.mesh.n_tets, time.time() - t0))
        if args.workload != "batching":
            batching = batching_leg(bsc)
        if args.serve_requests > 0:
            serving = serve_leg(args.serve_requests, args.serve_requests_30, bsc)

    out = {
        "metric": METRIC, "value": round(samples_per_s, 1), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d tets (%s), %d %s subdomains, %dx%d %s view%s, m=%d, %s" % (
            sc.name, mesh.n_tets, "adaptive: 32^3 base refined 0-3 levels, cone decomposition"
            if args.workload == "batching" else "jittered Kuhn grid", mesh.n_sub,
            {"slabs": "interleaved-slab (4 slabs each)", "batching": "Morton (tet-count ratio 12)"}.get(
                args.workload, "Morton"),
            W, H, "perspective" if sc.view["projection"] else "orthographic",
            "s (%d orbit cameras)" % len(views) if len(views) > 1 else "", m,
            "kept-piece variant" if args.keep else "plain form: stage two walks the rays again" + (
                ", both passes by (tile, subdomain) pairs" if by_pair else ", both passes by tiles")),
            "global_batch": 1, "seq_len": None, "parallelism": "single GPU, all subdomains on device"},
        "frames_per_s": round(1e3 / run["median_camera_ms"], 4),
        "frames_per_s_definition": "1 / median over the cameras of their mean frame time (RGBA stays on the device)",
        "camera_mean_frame_ms": {str(c): round(v, 3) for c, v in sorted(run["camera_mean_ms"].items())},
        "samples_per_frame_by_camera": [int(s["pieces"]) for s in survey],
        "tet_steps_per_frame_by_camera": [int(s["tet_steps"]) for s in survey],
        "kernels_ms": kern_mean,
        "frame_ms_each": [round(x, 2) for x in run["frame_ms"]],
        "tile_shape": tile_shape, "autotune": tuned,
        "segments": seg_stats, "counters": cnt, "roofline": roofline, "cpu_baseline": cpu, "parity": parity,
        "apc_vs_exact_compositing": exact_report, "variants": variants, "batching": batching, "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
