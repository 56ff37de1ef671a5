"""Render-request serving over the library: a resident mesh, continuous batching, admission by HBM footprint.

A `Server` keeps one mesh resident and runs frames for a stream of requests (image size, camera, number of
moments, transfer function).  It has `slots`: each slot is a library context (its own workspace) with its own
HIP stream, driven by one worker thread.  In "batched" mode a request is admitted as soon as it has arrived, a
slot that can hold its size is free and its HBM footprint (its images and the library workspace a frame of its
size needs, see Server.footprint) fits the budget beside the requests already in flight, so frames of
different requests overlap on the device; each frame's interval on the device is taken from HIP events on its
slot's stream.  Slots come in two sizes: large ones take any request, small ones only requests up to a smaller
image size.  In "fifo" mode one request runs at a time in arrival order.  A frame is stage one summing every
subdomain itself (`APC_MOMENTS_GLOBAL`: the server holds the whole mesh) and the resolve pass, in the plain
form (stage two walks again) unless the server keeps pieces.  With by_pair, stage one of a frame of at most
moments_pair_max_tiles tiles and stage two of one of at most pair_max_tiles tiles walk the (tile, subdomain)
pairs in parallel (such a frame has too few tiles to fill the device one workgroup per tile; a larger one
is faster per tile):
stage one into buffers the slot sized when it was warmed, whose ordered sum gives the same global moments
(a frame with more pairs than the buffers hold takes the per-tile form instead, counted, never an
allocation), and stage two (APC_BY_PAIR) into the library's pair buffers, the image to FP32 rounding.  Every step of a frame runs in the library's
kernels; this module only schedules, allocates buffers and times.
"""
from __future__ import annotations

import math
import queue
import threading
import time

import numpy as np

from . import Context, make_mboit, make_tf, make_view


def look_at_view(eye, target, width: int, height: int, fovy_deg: float = 45.0) -> dict:
    """Pinhole camera frame for apc_view: un-normalised pixel direction dir + (j+1/2-W/2) right + (i+1/2-H/2) down."""
    e = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - e
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) <= 0.99 else np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    t = math.tan(math.radians(fovy_deg) / 2.0)
    return dict(width=width, height=height, projection=1, eye=tuple(e), dir=tuple(f),
                right=tuple(r * (2.0 * t / width)), down=tuple(-u * (2.0 * t / height)))


class Server:
    def __init__(self, mesh, step, tfs, s_range, kappa=4.0, absorbance_max=10.0, alpha=5e-5, eta=0.3,
                 slots=4, workspace_limit=8 << 30, hbm_budget=64 << 30, max_size=2048, max_m=8, device=0,
                 small_slots=0, small_size=1024, small_workspace_limit=None, keep=False, by_pair=False,
                 pair_slack=2.0, pair_max_tiles=4096, moments_pair_max_tiles=16384):
        """mesh: arrays (xyz, scalar, tets, tet_sub, n_sub); tfs: list of [n][4] float32 tables;
        s_range: (s_min, s_max) of the transfer functions' domain; workspace_limit: bytes per slot for the
        kept-piece pool; hbm_budget: bytes of the requests' footprints (see footprint) allowed in flight;
        max_size, max_m: the largest request, for which every slot's buffers are allocated once (no
        allocation while serving: device allocations would synchronise the other slots' work).
        small_slots more slots take only requests up to small_size^2, with small_workspace_limit bytes each
        (default: workspace_limit scaled by the pixel ratio): a slot's workspace must hold the kept pieces
        of its largest frame, so HBM allows more small slots than large ones.  keep: frames keep their pieces
        in stage one for stage two (APC_KEEP_PIECES) instead of walking twice (the plain form).  by_pair
        (plain form only): stage one by (tile, subdomain) pairs for frames of at most moments_pair_max_tiles
        tiles (16384: 1024^2 in 8 x 8 tiles), stage two for frames of at most pair_max_tiles (4096: 512^2);
        measured on the batching mesh, stage one is faster by pairs up to 1024^2 and stage two up to 512^2,
        both per tile beyond.  Stage one writes into per-slot buffers of pair_slack times the pairs of the
        slot's largest such frame at warm-up (allocated by warm())."""
        if by_pair and keep:
            raise ValueError("stage one by pairs keeps no pieces")
        import torch
        self.torch = torch
        self.device = device
        self.dev = torch.device("cuda:%d" % device)
        self.owner = Context(device)
        xyz, scalar, tets, tet_sub, n_sub = mesh
        self.mesh = self.owner.load_mesh(xyz, scalar, tets, tet_sub, n_sub)
        self.n_boundary_faces = self.mesh.info()["n_boundary_faces"]
        self.slot_ws = None  # measured by warm()
        self.n_sub = n_sub
        self.subs = np.arange(n_sub, dtype=np.int32)
        self.step = step
        self.tf_dev = [torch.as_tensor(np.ascontiguousarray(t, dtype=np.float32), device=self.dev) for t in tfs]
        self.s_range = s_range
        self.kappa, self.absorbance_max = kappa, absorbance_max
        self.alpha, self.eta = alpha, eta
        self.slots = []
        self.bufs = []
        self.max_size, self.max_m = max_size, max_m
        if small_slots and not 0 < small_size < max_size:
            raise ValueError("small_size must lie below max_size")
        if small_workspace_limit is None:
            small_workspace_limit = workspace_limit * small_size * small_size // (max_size * max_size)
        self.slot_size = [max_size] * slots + [small_size] * small_slots
        for k, size in enumerate(self.slot_size):
            c = Context(device)
            c.set_workspace_limit(workspace_limit if k < slots else small_workspace_limit)
            self.slots.append((c, torch.cuda.Stream(device=self.dev)))
            px = size * size
            self.bufs.append((torch.empty((max_m + 1) * px, dtype=torch.float32, device=self.dev),
                              torch.empty(4 * px, dtype=torch.float32, device=self.dev)))
        self.workspace_limit = workspace_limit
        self.hbm_budget = hbm_budget
        self.keep = keep
        self.by_pair, self.pair_slack, self.pair_max_tiles = by_pair, pair_slack, pair_max_tiles
        self.moments_pair_max_tiles = moments_pair_max_tiles
        self.pair_bufs = [None] * len(self.slot_size)  # (flat FP32 tiles, int32 pair bins) per slot
        # per slot (each has one worker thread): frames with more pairs than the slot's buffers, run per tile
        self.pair_overflow = [0] * len(self.slot_size)
        self.events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in self.slot_size]
        self.t_ref = None
        self.last_device = [None] * len(self.slot_size)

    def warm(self, eye=(2.0, 0.9, 0.7), tf=0):
        """One frame of each slot's largest request (its size, max_m) on every slot, one slot at a time: the
        library grows a context's buffers (bins, piece pool, staging) to what a frame needs, and a device
        allocation or release while other slots' frames run waits for all of them."""
        torch = self.torch
        for k in range(len(self.slots)):
            req = {"id": -1, "arrival": 0.0, "size": self.slot_size[k], "eye": eye, "m": self.max_m, "tf": tf}
            ps = self._pair_size(k, self.moments_pair_max_tiles)
            if self.by_pair and ps > 0 and self.pair_bufs[k] is None:
                ctx, stream = self.slots[k]
                view, tfd, _ = self._frame_args({**req, "size": ps})
                n = ctx.moments_pass_tiles(self.mesh, view, tfd, self.max_m, self.subs, stream=stream.cuda_stream)
                cap = max(256, int(math.ceil(n * self.pair_slack)))
                self.pair_bufs[k] = (
                    torch.empty(cap * (self.max_m + 1) * 64, dtype=torch.float32, device=self.dev),
                    # as many bins as the FP32 buffer holds tiles of the smallest m (4)
                    torch.empty(cap * (self.max_m + 1) // 5, dtype=torch.int32, device=self.dev))
            sizes = sorted({ps, self._pair_size(k, self.pair_max_tiles)} - {0, req["size"]}) if self.by_pair else []
            for _ in range(2):  # the second frame runs at the grown size
                self.render(k, req)
                for size in sizes:  # the largest frames by pairs of each pass size their buffers
                    self.render(k, {**req, "size": size})
        self.slot_ws = [c.workspace_bytes() + (0 if b is None else b[0].numel() * 4 + b[1].numel() * 4)
                        for (c, _), b in zip(self.slots, self.pair_bufs)]

    def footprint(self, req) -> int:
        """HBM bytes a request occupies while it runs: its moment image and RGBA image, and the workspace of
        the slot it runs on (with its stage-one pair buffers).  A library context keeps the buffers its largest frame needed (FP64 moment
        partials, segment statistics, piece counts, binning state, and the piece pool when frames keep their
        pieces), so after warm() the workspace of every slot that could take the request is measured with
        apc_get_workspace_bytes and the largest is counted; before it, an estimate from the request's size
        (8 (m+1) + 12 bytes per pixel, 12 bytes per (tile, subdomain) pair, 4 per binned face record -- two
        per boundary face, since a face's conservative pixel box can reach into a neighbouring tile -- with the
        library's growth slack, plus the pool limit when frames keep their pieces)."""
        size, m = req["size"], req["m"]
        px = size * size
        own = px * (4 * (m + 1) + 16)
        eligible = [k for k, s in enumerate(self.slot_size) if s >= size]
        if self.slot_ws is not None and eligible:
            return own + max(self.slot_ws[k] for k in eligible)
        tiles = -(-size // 8) ** 2
        ws = px * (8 * (m + 1) + 12) + tiles * 12 * self.n_sub + 4 * 2 * max(self.n_boundary_faces, 16 * tiles)
        ws = ws * 5 // 4 + (64 << 10)  # the library's buffers grow with a quarter of slack, 4 KiB at least
        if self.keep:
            ws += self.workspace_limit
        return own + ws
    def _bias(self, m):
        j = np.arange(1, m + 1)
        return np.where(j % 2 == 0, 1.0 / (j + 1.0), 0.0)

    def _pair_tiles(self, slot, size) -> int:
        tw, th = self.slots[slot][0].tile_shape()
        return -(-size // tw) * -(-size // th)

    def _pair_size(self, slot, max_tiles) -> int:
        """The largest square frame of the slot with at most max_tiles tiles (0: none)."""
        size = self.slot_size[slot]
        while size > 0 and self._pair_tiles(slot, size) > max_tiles:
            size -= 1
        return size

    def _frame_args(self, req):
        W = H = req["size"]
        m = req["m"]
        view = make_view(look_at_view(req["eye"], (0.5, 0.5, 0.5), W, H), self.step)
        tf = make_tf(self.tf_dev[req["tf"]], self.s_range[0], self.s_range[1], self.kappa, self.absorbance_max)
        return view, tf, make_mboit(m, self.alpha, self._bias(m), self.eta, 1)

    def _moments_by_pair(self, slot, view, tf, m, mom, s) -> bool:
        """Stage one by pairs into the slot's buffers and their ordered sum into mom; False (nothing written)
        when the frame has more pairs than the buffers hold."""
        from . import ApcError
        ctx, _ = self.slots[slot]
        flat, bins = self.pair_bufs[slot]
        cap = min(flat.numel() // ((m + 1) * 64), bins.numel())
        tiles = flat[: cap * (m + 1) * 64].view(cap, m + 1, 64)
        try:
            n = ctx.moments_pass_tiles(self.mesh, view, tf, m, self.subs, tiles, bins[:cap], s, by_pair=True)
        except ApcError as e:
            if e.status != 3:  # APC_E_NOMEM: the buffers stay untouched
                raise
            return False
        ctx.sum_moment_tiles(tiles, bins, n, len(self.subs), m, view.height, view.width, mom, s)
        return True

    def render(self, slot: int, req) -> "object":
        """One frame for `req` on slot `slot` (stage one, moment sum, resolve); returns the RGBA image (a view
        of the slot's buffer, valid until the slot's next request) after the slot's stream has finished it."""
        torch = self.torch
        ctx, stream = self.slots[slot]
        W = H = req["size"]
        m = req["m"]
        view, tf, mb = self._frame_args(req)
        if W > self.slot_size[slot] or m > self.max_m:
            raise ValueError("request larger than slot %d (%d^2, m=%d)" % (slot, self.slot_size[slot], self.max_m))
        b_mom, b_rgba = self.bufs[slot]
        mom = b_mom[: (m + 1) * H * W].view(m + 1, H, W)
        rgba = b_rgba[: 4 * H * W].view(H, W, 4)
        s = stream.cuda_stream
        ev0, ev1 = self.events[slot]
        ev0.record(stream)
        tiles = self._pair_tiles(slot, W)
        pairs = self.by_pair and not self.keep
        one_by_pair = pairs and self.pair_bufs[slot] is not None and tiles <= self.moments_pair_max_tiles
        if not (one_by_pair and self._moments_by_pair(slot, view, tf, m, mom, s)):
            if one_by_pair:
                self.pair_overflow[slot] += 1
            ctx.moments_pass(self.mesh, view, tf, m, self.subs, mom, s, global_sum=True, keep=self.keep)
        ctx.resolve_pass(self.mesh, view, tf, mb, mom, self.subs, rgba, finalize=True, stream=s,
                         by_pair=pairs and tiles <= self.pair_max_tiles)
        ev1.record(stream)
        stream.synchronize()
        if self.t_ref is not None:  # the frame's interval on the device, in ms after the run's reference event
            self.last_device[slot] = (self.t_ref.elapsed_time(ev0), self.t_ref.elapsed_time(ev1))
        return rgba

    def run(self, requests, mode="batched", keep_images=False) -> dict:
        """Serve `requests` (dicts with arrival [s], size, eye, m, tf) open loop: request k is released at
        its arrival time after the start.  Returns per-request records and latency statistics."""
        if mode not in ("batched", "fifo"):
            raise ValueError(mode)
        n_slots = len(self.slots) if mode == "batched" else 1

        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self.t_ref = torch.cuda.Event(enable_timing=True)
        self.t_ref.record(torch.cuda.current_stream(self.dev))
        self.pair_overflow = [0] * len(self.slot_size)
        device = {}

        def render(slot, req):
            rgba = self.render(slot, req)
            device[req["id"]] = self.last_device[slot]
            return rgba.cpu() if keep_images else None

        st = schedule(requests, n_slots, self.footprint, self.hbm_budget, render, mode, slot_size=self.slot_size)
        for rec in st["records"]:
            rec["device_start_ms"], rec["device_end_ms"] = device[rec["id"]]
        st["device_overlap_frac"] = device_overlap(st["records"])
        st["passes"] = ("by (tile, subdomain) pairs up to %d (stage one) and %d (stage two) tiles per frame, else "
                        "by tiles" % (self.moments_pair_max_tiles, self.pair_max_tiles) if self.by_pair else "by tiles")
        if self.by_pair:
            st["pair_buffer_overflows"] = int(sum(self.pair_overflow))
        self.t_ref = None
        return st

    def close(self):
        self.torch.cuda.synchronize(self.dev)
        for c, _ in self.slots:
            c.close()
        self.mesh.free()
        self.owner.close()


def device_overlap(records) -> float:
    """Fraction of the requests whose frame ran on the device (HIP event interval) while another request's
    frame did."""
    iv = sorted((r["device_start_ms"], r["device_end_ms"]) for r in records)
    n = len(iv)
    hit = [False] * n
    for i in range(n):
        for j in range(i + 1, n):
            if iv[j][0] >= iv[i][1]:
                break
            hit[i] = hit[j] = True
    return sum(hit) / max(n, 1)


def schedule(requests, n_slots, footprint, hbm_budget, render, mode="batched", slot_size=None) -> dict:
    """Open-loop continuous batching.  Request k is released at requests[k]["arrival"] seconds after the
    start and admitted, in arrival order, as soon as a slot that can hold it is free (slot_size[s] >= its
    "size"; every slot when slot_size is None) and the footprints of the requests in flight plus its own fit
    `hbm_budget` (a request alone is always admitted).  Of the free slots that can hold it, it takes the
    smallest (then the lowest index), so that large slots stay free for large requests.  `render(slot, req)`
    then runs it on a worker thread (its return value, if not None, is kept as the record's "rgba").
    Returns the records (arrival, start, end, latency in seconds) and p50/p99/mean latency in ms and
    frames/s."""
    reqs = sorted(requests, key=lambda r: r["arrival"])
    if slot_size is not None:
        if len(slot_size) < n_slots:
            raise ValueError("slot_size lists %d slots, %d are used" % (len(slot_size), n_slots))
        biggest = max(slot_size[:n_slots])
        too_big = [r["id"] for r in reqs if r.get("size", 0) > biggest]
        if too_big:
            raise ValueError("requests %s are larger than every slot (%d)" % (too_big[:3], biggest))
    cv = threading.Condition()
    free = set(range(n_slots))
    inflight = [0]
    done = {}
    errors = []
    t0 = time.perf_counter()

    def work(slot, req):
        start = time.perf_counter() - t0
        try:
            img = render(slot, req)
            end = time.perf_counter() - t0
            rec = {"id": req["id"], "arrival": req["arrival"], "start": start, "end": end, "slot": slot,
                   "latency": end - req["arrival"], "size": req.get("size"), "m": req.get("m")}
            if img is not None:
                rec["rgba"] = img
            done[req["id"]] = rec
        except Exception as e:  # reported after the run
            errors.append((req["id"], repr(e)))
        finally:
            with cv:
                inflight[0] -= footprint(req)
                free.add(slot)
                cv.notify_all()

    threads = []
    for req in reqs:
        wait = req["arrival"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        fp = footprint(req)
        size = req.get("size", 0)
        with cv:
            while True:  # admission: a free slot that holds the request and room in the HBM budget
                cands = [k for k in free if slot_size is None or slot_size[k] >= size]
                if cands and (inflight[0] == 0 or inflight[0] + fp <= hbm_budget):
                    slot = min(cands, key=lambda k: (0 if slot_size is None else slot_size[k], k))
                    free.discard(slot)
                    inflight[0] += fp
                    break
                cv.wait(0.05)
        th = threading.Thread(target=work, args=(slot, req))
        th.start()
        threads.append(th)
    for th in threads:
        th.join()
    if errors:
        raise RuntimeError("requests failed: %s" % errors[:3])
    recs = [done[r["id"]] for r in reqs]
    lat = np.array([r["latency"] for r in recs]) * 1e3
    span = max(r["end"] for r in recs) - min(r["arrival"] for r in recs)
    return {"mode": mode, "slots": n_slots, "requests": len(recs),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "frames_per_s": len(recs) / span, "records": recs}
