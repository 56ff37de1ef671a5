"""Serving (continuous batching over the C ABI): every request's image is the
same alone and in the mix, requests overlap on the device, and a served frame
matches the oracle."""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def server():
    import paper_2501_12581_amd as P
    from paper_2501_12581_amd.serve import Server
    P.lib()
    sc = synth.scene_medium(size=128)
    m = sc.mesh
    tfs = [synth.make_tf(s) for s in (13, 14, 15)]
    srv = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=3,
                 workspace_limit=1 << 30, hbm_budget=1 << 30)
    yield srv, sc, tfs
    srv.close()


def test_each_result_is_the_same_alone_and_in_the_mix(server):
    srv, sc, tfs = server
    reqs = synth.request_stream(18, rate=400.0, seed=3, sizes=(96, 128, 192), ms=(4, 6, 8))
    mix = srv.run(reqs, "batched", keep_images=True)
    alone = srv.run(reqs, "fifo", keep_images=True)
    for a, b in zip(mix["records"], alone["records"]):
        assert a["id"] == b["id"]
        assert torch.equal(a["rgba"], b["rgba"]), a["id"]
    # frames of different requests ran on the device at the same time (HIP event intervals on the slots'
    # streams), and never one at a time
    print("device overlap: batched %.2f, one at a time %.2f" % (mix["device_overlap_frac"],
                                                                 alone["device_overlap_frac"]))
    assert mix["device_overlap_frac"] > 0.2
    assert alone["device_overlap_frac"] == 0.0
    assert mix["p50_ms"] <= mix["p99_ms"] and alone["p50_ms"] <= alone["p99_ms"]
    print("batched p50 %.2f p99 %.2f ms, %.1f frames/s; fifo p50 %.2f p99 %.2f ms, %.1f frames/s" % (
        mix["p50_ms"], mix["p99_ms"], mix["frames_per_s"], alone["p50_ms"], alone["p99_ms"], alone["frames_per_s"]))


def test_served_frame_matches_oracle(server):
    srv, sc, tfs = server
    req = {"id": 0, "arrival": 0.0, "size": 96, "eye": (2.1, 1.3, -0.4), "m": 8, "tf": 2}
    got = srv.render(0, req).cpu().numpy().astype(np.float64).reshape(-1, 4)
    sc2 = synth.Scene(**{**sc.__dict__, "view": synth.perspective_view(req["eye"], (0.5, 0.5, 0.5), 96, 96),
                         "m": 8, "bias": synth.default_bias(8), "tf": tfs[2]})
    ref = oracle.render(sc2)
    d = got - ref["rgba"]
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


def test_served_frames_keep_their_pieces():
    """Slots that keep their pieces (APC_KEEP_PIECES): a slot's workspace limit gives its pool no slack
    beyond the size it asks for, yet the pool must hold a repeated request's pieces, including the chunks
    each wavefront's last block leaves unused, so from the second frame on stage two reads kept pieces (one
    walk per frame); the image equals the plain form's to rounding."""
    from paper_2501_12581_amd.serve import Server
    sc = synth.scene_medium(size=128)
    m = sc.mesh
    tfs = [synth.make_tf(s) for s in (13, 14)]
    srv = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=1,
                 workspace_limit=1 << 30, hbm_budget=1 << 30, max_size=192, keep=True)
    plain = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=1,
                   workspace_limit=1 << 30, hbm_budget=1 << 30, max_size=192)
    try:
        ctx = srv.slots[0][0]
        req = {"id": 0, "arrival": 0.0, "size": 192, "eye": (0.3, 2.4, 0.9), "m": 6, "tf": 1}
        srv.render(0, req)  # the first frame sizes the slot's pool (its stage two may walk again)
        first = srv.render(0, req).clone()
        for _ in range(2):
            ctx.counters(reset=True)
            again = srv.render(0, req)
            t, c = ctx.timings(), ctx.counters()
            assert t["rewalk_ms"] == 0.0 and t["eval_ms"] > 0, t
            assert torch.equal(first, again)
        assert c["pieces"] > 0
        ref = plain.render(0, req)
        assert (ref - first).abs().max().item() <= 2e-5
    finally:
        srv.close()
        plain.close()


def test_serving_by_pair_gives_the_same_images():
    """Slots that walk both passes by (tile, subdomain) pairs (stage one into buffers sized when they were
    warmed) give every request the image of the per-tile form to FP32 rounding (stage two's colour sums are
    grouped by subdomain: the bar of the kept-piece form, 2e-5), batched or one at a time; a frame with more
    pairs than its slot's buffers hold (a tiny pair_slack) takes the per-tile stage one, with bitwise the
    same image (the same moments), and is counted.  With pair_max_tiles = 256 the 192^2 frames (576 tiles)
    run stage two per tile, bitwise the per-tile image (stage one by pairs gives the same moments), and the
    smaller ones both passes by pairs; with moments_pair_max_tiles = 256 as well, stage one of the 192^2
    frames runs per tile too, the same image."""
    from paper_2501_12581_amd.serve import Server
    sc = synth.scene_medium(size=128)
    m = sc.mesh
    tfs = [synth.make_tf(s) for s in (13, 14)]
    args = ((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max))
    kw = dict(workspace_limit=1 << 30, hbm_budget=1 << 30, max_size=192)
    ref = Server(*args, slots=1, **kw)
    pair = Server(*args, slots=2, by_pair=True, **kw)
    tight = Server(*args, slots=1, by_pair=True, pair_slack=1e-3, **kw)
    mixed = Server(*args, slots=1, by_pair=True, pair_max_tiles=256, **kw)
    mixed1 = Server(*args, slots=1, by_pair=True, pair_max_tiles=256, moments_pair_max_tiles=256, **kw)
    try:
        with pytest.raises(ValueError):
            Server(*args, slots=1, by_pair=True, keep=True, **kw)
        for s in (ref, pair, tight, mixed, mixed1):
            s.warm()
        reqs = synth.request_stream(12, rate=400.0, seed=7, sizes=(96, 128, 192), ms=(4, 6, 8), n_tf=2)
        want = ref.run(reqs, "fifo", keep_images=True)
        got = pair.run(reqs, "batched", keep_images=True)
        low = tight.run(reqs, "fifo", keep_images=True)
        mix = mixed.run(reqs, "fifo", keep_images=True)
        mix1 = mixed1.run(reqs, "fifo", keep_images=True)
        for a, b, c, d, e in zip(want["records"], got["records"], low["records"], mix["records"], mix1["records"]):
            assert a["id"] == b["id"] == c["id"] == d["id"] == e["id"]
            assert torch.equal(d["rgba"], a["rgba"] if a["size"] == 192 else b["rgba"]), a["id"]
            assert torch.equal(e["rgba"], d["rgba"]), a["id"]
            assert torch.equal(b["rgba"], c["rgba"]), a["id"]
            assert (a["rgba"] - b["rgba"]).abs().max().item() <= 2e-5, a["id"]
        print("overflows: slack 2 %d, slack 1e-3 %d of %d" % (got["pair_buffer_overflows"],
                                                             low["pair_buffer_overflows"], len(reqs)))
        assert want["passes"] == "by tiles" and got["passes"].startswith("by (tile, subdomain) pairs")
        assert got["pair_buffer_overflows"] < len(reqs) and low["pair_buffer_overflows"] > 0
    finally:
        for s in (ref, pair, tight, mixed, mixed1):
            s.close()


def test_small_slots_take_small_requests_with_the_same_results():
    """Slots of two sizes: 2 that take any request and 2 that take requests up to 128^2 (with a smaller
    workspace).  Every request runs on a slot that holds it, the small slots are used, and each image is
    bitwise the one-at-a-time image."""
    from paper_2501_12581_amd.serve import Server
    sc = synth.scene_medium(size=128)
    m = sc.mesh
    tfs = [synth.make_tf(s) for s in (13, 14)]
    srv = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=2,
                 workspace_limit=1 << 30, hbm_budget=1 << 30, max_size=192, small_slots=2, small_size=128,
                 small_workspace_limit=512 << 20)
    try:
        srv.warm()
        reqs = synth.request_stream(16, rate=400.0, seed=5, sizes=(96, 128, 192), ms=(4, 8), n_tf=2)
        mix = srv.run(reqs, "batched", keep_images=True)
        alone = srv.run(reqs, "fifo", keep_images=True)
        for a, b in zip(mix["records"], alone["records"]):
            assert a["id"] == b["id"]
            assert srv.slot_size[a["slot"]] >= a["size"]
            assert torch.equal(a["rgba"], b["rgba"]), a["id"]
        assert any(r["slot"] >= 2 for r in mix["records"])  # the small slots served requests
    finally:
        srv.close()


def test_footprint_counts_the_slot_workspace(server):
    """The footprint a request is admitted with holds its own images and the device memory its slot's library
    context keeps (measured after the warm-up); before the warm-up an estimate from the request's size
    bounds what a fresh context holds after one frame of that size."""
    import paper_2501_12581_amd as P
    srv, sc, tfs = server
    srv.warm()
    for size, m in ((96, 4), (128, 8)):
        req = {"id": 0, "arrival": 0.0, "size": size, "eye": (2.2, 0.4, 1.1), "m": m, "tf": 0}
        own = size * size * (4 * (m + 1) + 16)
        held = max(c.workspace_bytes() for c, _ in srv.slots)
        assert srv.footprint(req) == own + held
    ws, srv.slot_ws = srv.slot_ws, None
    try:
        for size, m in ((96, 4), (128, 8), (192, 6)):
            ctx = P.Context(0)
            try:
                req = {"id": 0, "arrival": 0.0, "size": size, "eye": (2.2, 0.4, 1.1), "m": m, "tf": 0}
                saved = srv.slots[0]
                srv.slots[0] = (ctx, saved[1])
                try:
                    srv.render(0, req)
                finally:
                    srv.slots[0] = saved
                held = ctx.workspace_bytes()
                est = srv.footprint(req) - size * size * (4 * (m + 1) + 16)
                print("size %d m %d: workspace %d B, estimate %d B" % (size, m, held, est))
                assert held <= est
            finally:
                ctx.close()
    finally:
        srv.slot_ws = ws


def test_a_request_over_the_budget_waits():
    """Admission by HBM footprint: with a budget that holds one 192^2 frame but not two, two such requests
    that arrive together run one after the other on the device although two slots are free; with a budget
    for both, they run at the same time."""
    from paper_2501_12581_amd.serve import Server
    sc = synth.scene_medium(size=128)
    m = sc.mesh
    tfs = [synth.make_tf(13)]
    probe = {"id": 0, "arrival": 0.0, "size": 192, "eye": (0.3, 2.4, 0.9), "m": 8, "tf": 0}
    srv = Server((m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub), sc.step, tfs, (sc.s_min, sc.s_max), slots=2,
                 hbm_budget=1 << 40, max_size=192)
    try:
        srv.warm()
        big = srv.footprint(probe)
        srv.hbm_budget = int(1.5 * big)
        reqs = [dict(probe, id=0), dict(probe, id=1, eye=(2.1, 1.3, -0.4))]
        st = srv.run(reqs, "batched")
        a, b = sorted(st["records"], key=lambda r: r["device_start_ms"])
        assert b["device_start_ms"] >= a["device_end_ms"]  # the second waited for the first
        # with room for two at a time, six such requests overlap on the device
        srv.hbm_budget = 3 * big
        eyes = ((2.1, 1.3, -0.4), (0.3, 2.4, 0.9), (2.0, -1.0, 0.5), (-1.2, 0.4, 2.0), (0.5, -1.5, -1.0),
                (2.4, 0.5, 0.5))
        st = srv.run([dict(probe, id=k, eye=e) for k, e in enumerate(eyes)], "batched")
        assert st["device_overlap_frac"] > 0
    finally:
        srv.close()
