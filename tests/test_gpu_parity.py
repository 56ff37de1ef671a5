"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars (moments relative to b0 per pixel; final image absolute):
  per-subdomain and global moments  |b_j - b_j_ref| <= 1e-5 * b0_ref, and 0 where b0_ref = 0
  final RGBA                         max abs <= 2e-3, RMSE <= 5e-4
Invariants (paper Sections 4.1-4.2): the global moments do not depend on the
order in which subdomains are rendered (bitwise, canonical-order sum) nor on
how the mesh is partitioned; partial images of the subdomains add up to the
final image; a constant-colour transfer function gives rgb = c (1 - e^-b0);
a single fragment without bias composites exactly; b0 = sigma * L on a
constant field.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.parity import moment_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apc():
    import paper_2501_12581_amd as P
    P.lib()  # raises when the library is not built
    return P


@pytest.fixture(scope="module")
def ctx(apc):
    c = apc.Context(0)
    yield c
    c.close()


B0_FLOOR = 1e-3  # below this optical depth (opacity < 0.1%) the bar is absolute: 1e-5 * 1e-3


def _moment_err(got, ref, b0=None):
    """max over pixels and j of |got - ref| / max(b0, B0_FLOOR), b0 = the pixel's reference b0
    unless given.  Background pixels (b0_ref = 0) must be exactly zero.  The floor keeps the bar
    meaningful on silhouette pixels, where FP32 depth rounding (~1e-7) is a large part of a
    chord of length ~1e-6."""
    b0 = ref[0] if b0 is None else b0
    bg = ref[0] == 0
    assert np.all(got[:, bg] == 0.0), "moments on background pixels"
    den = np.maximum(b0[~bg], B0_FLOOR)
    return float(np.max(np.abs(got[:, ~bg] - ref[:, ~bg]) / den)) if np.any(~bg) else 0.0


# One allowance for every test: at most this fraction of the covered pixels may need the backward-error bar
MAX_BACKWARD = 0.005


def _check_moments(sc, pix, got, ref, tol=1e-5, per_sub=False, max_backward=MAX_BACKWARD):
    """Forward bar |got - ref| <= tol * max(b0, B0_FLOOR) per pixel; pixels that miss it (at most a fraction
    max_backward of the covered ones) must pass the backward-error bar of oracle.parity.  Returns the forward
    error and the number of pixels that needed the backward bar."""
    res = moment_parity(sc, pix, got, ref, tol=tol, floor=B0_FLOOR, per_sub=per_sub)
    print("moment parity", sc.name, "per_sub" if per_sub else "global", res, flush=True)
    assert res["background_exact"], "moments on background pixels"
    assert res["backward_bar_pixels"] <= max(3, max_backward * res["covered"]), ("too many pixels off", res)
    assert res["outside_backward_band"] == 0, ("outside the backward-error band", res)
    return res["forward_max"], res["backward_bar_pixels"]


def _render(apc, ctx, sc, subdomains=None, finalize=True):
    r = apc.Renderer(ctx, sc)
    rgba = r.frame(subdomains=subdomains, finalize=finalize)
    torch.cuda.synchronize()
    return r, rgba


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _flat_moments(t):
    m1 = t.shape[-3]
    return _np(t).reshape(*t.shape[:-3], m1, -1)


@pytest.fixture(scope="module")
def tiny_ref():
    sc = synth.scene_tiny()
    return sc, oracle.render(sc, per_sub=True, exact=True)


def test_tiny_moments_and_image_match_oracle(apc, ctx, tiny_ref):
    sc, ref = tiny_ref
    ctx.counters(reset=True)
    r, rgba = _render(apc, ctx, sc)
    S = sc.mesh.n_sub
    per_sub = _flat_moments(r.per_sub)
    for s in range(S):
        # a subdomain's moments are measured against the pixel's global b0, the scale of the sum they enter
        err = _moment_err(per_sub[s], ref["moments_sub"][s], b0=ref["moments"][0])
        assert err <= 1e-5, ("subdomain", s, err)
    err = _moment_err(_flat_moments(r.moments), ref["moments"])
    assert err <= 1e-5, err
    got = _np(rgba).reshape(-1, 4)
    d = got - ref["rgba"]
    assert np.abs(d).max() <= 2e-3, np.abs(d).max()
    assert math.sqrt(np.mean(d ** 2)) <= 5e-4
    c = ctx.counters()
    walks = 2 if ctx.timings()["rewalk_ms"] > 0 else 1  # stage two walks again unless stage one kept the pieces
    print("counters", c, "walks", walks)
    assert c["walk_step_limit"] == 0
    assert abs(c["pieces"] - walks * ref["n_pieces"]) <= 1e-4 * ref["n_pieces"]


def test_permutation_of_subdomains_is_bitwise_invariant(apc, ctx):
    sc = synth.scene_tiny()
    r = apc.Renderer(ctx, sc)
    r.frame()
    base = r.moments.clone()
    img = r.rgba.clone()
    perm = np.array([2, 0, 3, 1], np.int32)
    r.frame(subdomains=perm)
    torch.cuda.synchronize()
    assert torch.equal(r.moments, base)
    assert torch.equal(r.rgba[..., 3], img[..., 3])


def test_repartition_keeps_global_moments(apc, ctx, tiny_ref):
    sc, ref = tiny_ref
    n = 16
    order = synth.morton_order(n)
    cube_of_tet = np.repeat(order, 6)
    variants = [np.zeros(n ** 3, np.int32), synth.partition_slabs(n, 3, 2)]
    bounds = synth.partition_chunks(n ** 3, 9, 21)
    rank = np.empty(n ** 3, np.int64)
    rank[order] = np.arange(n ** 3)
    variants.append((np.searchsorted(bounds, rank, side="right") - 1).astype(np.int32))
    r0, _ = _render(apc, ctx, sc)
    base = _flat_moments(r0.moments)
    for sub_of_cube in variants:
        S = int(sub_of_cube.max()) + 1
        mesh = synth.Mesh(xyz=sc.mesh.xyz, scalar=sc.mesh.scalar, tets=sc.mesh.tets,
                          tet_sub=sub_of_cube[cube_of_tet].astype(np.int32), n_sub=S)
        sc2 = synth.Scene(**{**sc.__dict__, "mesh": mesh})
        r, _ = _render(apc, ctx, sc2)
        got = _flat_moments(r.moments)
        b0 = base[0]
        nz = b0 > 0
        assert np.all(got[:, ~nz] == 0)
        assert np.max(np.abs(got[:, nz] - base[:, nz]) / b0[nz]) <= 1e-6


def test_partial_images_sum_to_final_image(apc, ctx):
    sc = synth.sandwich_scene()
    r = apc.Renderer(ctx, sc)
    final = r.frame().clone()
    S = sc.mesh.n_sub
    H, W = r.view.height, r.view.width
    partials = torch.empty((S, H, W, 4), dtype=torch.float32, device="cuda")
    for s in range(S):
        ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, [s], partials[s], finalize=False)
    out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    ctx.sum_images(partials, list(range(S)), r.moments, r.mboit, out)
    torch.cuda.synchronize()
    assert torch.max(torch.abs(out - final)).item() <= 1e-5  # FP32 sums in a different order
    ref = oracle.render(sc, per_sub=True)
    d = _np(final).reshape(-1, 4) - ref["rgba"]
    assert np.abs(d).max() <= 2e-3
    # each rank's partial image (its pieces' additive colour and opacity sums, before renormalisation)
    # against the oracle's per-subdomain sums
    for s in range(S):
        e = _np(partials[s]).reshape(-1, 4) - ref["color_sub"][s]
        assert np.abs(e).max() <= 2e-3 and math.sqrt(np.mean(e ** 2)) <= 5e-4, s
        assert np.all(_np(partials[s]).reshape(-1, 4)[ref["color_sub"][s][:, 3] == 0] == 0), s


def test_constant_colour_tf_gives_opacity_times_colour(apc, ctx):
    sc = synth.scene_tiny()
    c = np.array([0.2, 0.55, 0.7], np.float32)
    sc.tf[:, :3] = c
    sc.alpha, sc.eta = 0.02, 0.9
    r, rgba = _render(apc, ctx, sc)
    got = _np(rgba).reshape(-1, 4)
    b0 = _flat_moments(r.moments)[0]
    A = -np.expm1(-b0)
    assert np.abs(got[:, 3] - A).max() <= 1e-6
    assert np.abs(got[:, :3] - c[None, :] * A[:, None]).max() <= 1e-6


def test_constant_density_b0_is_sigma_times_length(apc, ctx):
    sc = synth.scene_tiny()
    sc.mesh.scalar[:] = 0.5
    sc.s_min, sc.s_max = 0.0, 1.0
    sc.tf[:, 3] = 0.37
    r, _ = _render(apc, ctx, sc)
    b0 = _flat_moments(r.moments)[0]
    sigma = sc.kappa * float(np.float32(0.37))
    assert np.max(np.abs(b0 - sigma)) <= 1e-5 * sigma  # every orthographic ray crosses length 1


def test_single_fragment_without_bias_is_exact(apc, ctx):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float32)
    mesh = synth.Mesh(xyz=xyz, scalar=np.array([0.125, 0.375, 0.625, 0.875], np.float32),
                      tets=np.array([[0, 1, 2, 3]], np.int32), tet_sub=np.zeros(1, np.int32), n_sub=1)
    px = np.array([0.01, 0.0, 0.0]), np.array([0.0, 0.01, 0.0])
    eye = np.array([0.2, 0.25, -1.0]) - 0.5 * (px[0] + px[1])
    view = dict(width=1, height=1, projection=0, eye=tuple(eye), dir=(0.0, 0.0, 1.0), right=tuple(px[0]),
                down=tuple(px[1]))
    sc = synth.Scene(name="one", mesh=mesh, tf=synth.make_tf(3), s_min=0.0, s_max=1.0, kappa=4.0,
                     absorbance_max=10.0, view=view, step=100.0, m=4, alpha=0.0, bias=synth.default_bias(4),
                     eta=0.0, renormalize=0)
    ref = oracle.render(sc, exact=True)
    r, rgba = _render(apc, ctx, sc)
    got = _np(rgba).reshape(-1, 4)
    assert np.abs(got - ref["exact"]).max() <= 1e-6


@pytest.mark.parametrize("W,H,proj", [(1, 1, 0), (1, 97, 0), (97, 1, 0), (13, 7, 0), (45, 31, 1), (1, 1, 1)])
def test_ragged_and_one_pixel_images_match_oracle(apc, ctx, W, H, proj):
    """Images of one pixel, one row, one column and sizes that fill no tile: every pixel against the oracle
    (tiny mesh, m = 4), so tiles that hang over the image edge write nothing outside it."""
    sc = synth.scene_tiny()
    if proj == 0:
        sc.view = synth.ortho_view_z(W, H)
    else:
        sc.view = synth.perspective_view(synth.sphere_eye(5), (0.5, 0.5, 0.5), W, H)
    ref = oracle.render(sc)
    r, rgba = _render(apc, ctx, sc)
    assert tuple(rgba.shape) == (H, W, 4)
    # at 45 x 31 about a seventh of the covered pixels lie on the cube's silhouette, where rays graze its flat
    # boundary faces: 11 of 880 need the backward bar (every one inside the band)
    _check_moments(sc, np.arange(W * H), _flat_moments(r.moments), ref)
    d = _np(rgba).reshape(-1, 4) - ref["rgba"]
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


def test_views_whose_rays_start_inside_the_mesh_are_rejected(apc, ctx):
    """The walk enters subdomains through their boundary faces, so a ray may not start inside the mesh: a
    perspective eye inside the mesh's bounding box, or an orthographic image plane cutting it, is an argument
    error even with a caller-given depth range; nothing is rendered."""
    sc = synth.scene_tiny()
    r = apc.Renderer(ctx, sc)
    inside = synth.perspective_view((0.5, 0.4, 0.5), (0.5, 1.0, 0.5), 128, 128)
    r.view = apc.make_view(inside, sc.step, t_near=0.05, t_far=2.0)
    with pytest.raises(apc.ApcError):
        r.frame()
    cut = dict(synth.ortho_view_z(128, 128), eye=(0.0, 0.0, 0.5))
    r.view = apc.make_view(cut, sc.step, t_near=0.05, t_far=2.0)
    with pytest.raises(apc.ApcError):
        r.frame()
    r.view = apc.make_view(sc.view, sc.step)  # the same renderer still works with a valid view
    r.frame()
    torch.cuda.synchronize()


@pytest.mark.parametrize("m", [4, 6, 8])
def test_tiny_all_moment_orders(apc, ctx, m):
    sc = synth.scene_tiny()
    sc.m = m
    sc.bias = synth.default_bias(m)
    ref = oracle.render(sc)
    r, rgba = _render(apc, ctx, sc)
    assert _moment_err(_flat_moments(r.moments), ref["moments"]) <= 1e-5
    d = _np(rgba).reshape(-1, 4) - ref["rgba"]
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


def test_medium_sampled_pixels_match_oracle(apc, ctx):
    """64^3 x 6 tets, 16 subdomains, 1024^2 perspective, m = 6: full GPU frame,
    oracle on a seeded sample of pixels."""
    sc = synth.scene_medium()
    r, rgba = _render(apc, ctx, sc)
    W, H = sc.view["width"], sc.view["height"]
    pix = np.sort(np.random.default_rng(5).choice(W * H, 6000, replace=False))
    ref = oracle.render(sc, pixels=pix, per_sub=True)
    mom = _flat_moments(r.moments)[:, pix]
    fwd, n_back = _check_moments(sc, pix, mom, ref)
    fwd_s, n_back_s = _check_moments(sc, pix, _flat_moments(r.per_sub)[:, :, pix], ref, per_sub=True)
    print("medium moments: forward err %.3g (%d pixels on the backward bar), per subdomain %.3g (%d)" % (
        fwd, n_back, fwd_s, n_back_s))
    got = _np(rgba).reshape(-1, 4)[pix]
    d = got - ref["rgba"]
    print("medium: max", np.abs(d).max(), "rmse", math.sqrt(np.mean(d ** 2)), ctx.counters())
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


def test_medium_m8_root_starts(apc, ctx):
    """m = 8 on the medium mesh at 512^2, both forms of stage two.  The plain form (re-walk) starts each
    sample's root solve from the previous sample's roots; the kept-piece form from its pixel's gap table.
    Either way the closed forms are the fallback, rare after the start is good: at most 5 % of the samples
    in the re-walk (every first sample in a new gap of the moment bound takes them) and 0.2 % with tables.
    Sampled pixels of both against the oracle."""
    sc = synth.scene_medium(size=512)
    sc.m = 8
    sc.bias = synth.default_bias(8)
    r = apc.Renderer(ctx, sc)
    W, H = sc.view["width"], sc.view["height"]
    pix = np.sort(np.random.default_rng(9).choice(W * H, 4000, replace=False))
    ref = oracle.render(sc, pixels=pix)
    for keep in (False, True):
        for _ in range(2 if keep else 1):  # a kept-piece frame sizes its pool first
            ctx.counters(reset=True)
            rgba = r.frame(global_sum=True, keep=keep)
        torch.cuda.synchronize()
        cnt = ctx.counters()
        _check_moments(sc, pix, _flat_moments(r.moments)[:, pix], ref)
        d = _np(rgba).reshape(-1, 4)[pix] - ref["rgba"]
        solved = cnt["table_samples"]
        print("medium m=8 keep=%s: max %.3g rmse %.3g, closed forms %.4f of %d" % (
            keep, np.abs(d).max(), math.sqrt(np.mean(d ** 2)), cnt["table_fallback"] / max(solved, 1), solved))
        assert cnt["table_samples"] > 0.5 * cnt["pieces"] / 2
        assert cnt["table_fallback"] <= (2e-3 if keep else 0.05) * solved
        assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


@pytest.mark.parametrize("m", [4, 6, 8])
def test_fp16_moment_storage_variant(apc, ctx, m):
    """FP16 moment image (ln b0 and the mean depth, each as two FP16 halves; the central moments of orders
    2..m): 2(m + 3) bytes per pixel against 4(m + 1).  The planes decode to the FP32 moments within FP16 rounding,
    background stays exactly empty, and the image error against the oracle is reported beside the FP32
    path's (a property of the variant, bounded loosely here)."""
    from math import comb
    sc = synth.scene_medium(size=256)
    sc.m = m
    sc.bias = synth.default_bias(m)
    r = apc.Renderer(ctx, sc)
    rgba32 = _np(r.frame()).reshape(-1, 4)
    rgba16 = _np(r.frame(moments_f16=True)).reshape(-1, 4)
    torch.cuda.synchronize()
    assert tuple(r.moments_h.shape) == (m + 3,) + tuple(r.moments.shape[1:])  # m + 3 FP16 planes
    mom = _flat_moments(r.moments)
    h = r.moments_h.float().cpu().numpy().astype(np.float64).reshape(m + 3, -1)
    cov = mom[0] > 0
    assert np.all(np.isneginf(h[0, ~cov])) and np.all(h[1:, ~cov] == 0.0) and np.all(rgba16[~cov] == 0.0)
    lb0 = h[0, cov] + h[1, cov]
    assert np.all(np.abs(lb0 - np.log(mom[0, cov])) <= 2.0 ** -22 * np.abs(np.log(mom[0, cov])) + 2.0 ** -25)
    beta = mom[:, cov] / mom[0, cov]
    mu = h[2, cov] + h[3, cov]
    assert np.all(np.abs(mu - beta[1]) <= 2.0 ** -22 * np.abs(beta[1]) + 2.0 ** -25)
    for k in range(2, m + 1):  # central moments about the stored mean, in FP64
        c = sum(comb(k, i) * beta[i] * (-mu) ** (k - i) for i in range(k + 1))
        assert np.all(np.abs(h[k + 2, cov] - c) <= 2.0 ** -11 * np.abs(c) + 2.0 ** -25 + 1e-12), k
    ref = oracle.render(sc)
    e32 = rgba32 - ref["rgba"]
    e16 = rgba16 - ref["rgba"]
    print("m=%d FP16 moments: rgba max %.3g rmse %.3g (FP32 path: max %.3g rmse %.3g)" % (
        m, np.abs(e16).max(), math.sqrt(np.mean(e16 ** 2)), np.abs(e32).max(), math.sqrt(np.mean(e32 ** 2))))
    assert np.all(np.isfinite(rgba16))
    assert np.abs(e16).max() <= 2e-3 and math.sqrt(np.mean(e16 ** 2)) <= 5e-4


def test_slab_segments_and_parity(apc, ctx):
    """Interleaved-slab stress volume, 4 ranks x 4 slabs, orthographic along z:
    every pixel has exactly 16 segments and meets 4 subdomains (integer
    results, bit-exact), and moments and image match the oracle."""
    sc = synth.scene_slabs(n_ranks=4, slabs_per_rank=4, cells_per_slab=2, size=128)
    ctx.counters(reset=True)
    r, rgba = _render(apc, ctx, sc)
    segs = ctx.segment_counts(128, 128).cpu().numpy().reshape(2, -1)
    assert np.all(segs[0] == 16) and np.all(segs[1] == 4)
    walks = 2 if ctx.timings()["rewalk_ms"] > 0 else 1
    assert ctx.counters()["segments"] == walks * 16 * 128 * 128  # every walk counts them
    ref = oracle.render(sc, segments=True)
    assert np.array_equal(segs, ref["segments"])
    assert _moment_err(_flat_moments(r.moments), ref["moments"]) <= 1e-5
    d = _np(rgba).reshape(-1, 4) - ref["rgba"]
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


def test_segment_counts_match_oracle_on_jagged_chunks(apc, ctx):
    """Medium mesh (16 jagged Morton chunks), perspective: per-pixel segment
    counts and subdomains met equal the oracle's on sampled pixels; a pixel
    that differs must lie within the oracle's range over cameras a few FP32
    ulps away (a grazing ray through a subdomain boundary)."""
    from oracle.parity import perturbed_views
    sc = synth.scene_medium(size=512)
    r, rgba = _render(apc, ctx, sc)
    W, H = sc.view["width"], sc.view["height"]
    segs = ctx.segment_counts(H, W).cpu().numpy().reshape(2, -1)
    pix = np.sort(np.random.default_rng(21).choice(W * H, 3000, replace=False))
    ref = oracle.render(sc, pixels=pix, pass2=False, segments=True)
    got = segs[:, pix]
    bad = np.where(np.any(got != ref["segments"], axis=0))[0]
    print("segments: %d of %d sampled pixels differ; max %d, mean over covered %.2f" % (
        len(bad), len(pix), got[0].max(), got[0][ref["moments"][0] > 0].mean()))
    assert len(bad) <= max(3, 0.005 * len(pix))
    if len(bad):
        lo = ref["segments"][:, bad].copy()
        hi = lo.copy()
        for v in perturbed_views(sc.view):
            rr = oracle.render(synth.Scene(**{**sc.__dict__, "view": v}), pixels=pix[bad], pass2=False,
                               segments=True)
            lo = np.minimum(lo, rr["segments"])
            hi = np.maximum(hi, rr["segments"])
        assert np.all(got[:, bad] >= lo) and np.all(got[:, bad] <= hi)


def test_tile_shapes_give_identical_results_and_autotuner(apc, ctx):
    """Any tile shape (w x 64/w pixels per wavefront) gives bitwise the same
    moments, segment counts and image: each ray walks alone and each pixel's
    sums run in its own walk order.  The autotuner times whole frames (stage
    one summing the subdomains, then the resolve) for widths 2..32, keeps the
    fastest, and the frame after it is unchanged; it needs the subdomains in
    ascending order, as a frame that sums them in stage one does."""
    sc = synth.scene_medium(size=384)
    r = apc.Renderer(ctx, sc)
    outs = {}
    try:
        for w in (2, 8, 32, 64):
            ctx.set_tile_shape(w)
            assert ctx.tile_shape() == (w, 64 // w)
            rgba = r.frame().clone()
            outs[w] = (r.moments.clone(), rgba, ctx.segment_counts(384, 384))
        for w in (2, 32, 64):
            for a, b in zip(outs[w], outs[8]):
                assert torch.equal(a, b), w
        before = ctx.tile_shape()
        with pytest.raises(apc.ApcError):
            ctx.autotune_tile_shape(r.mesh, r.view, r.tf, r.mboit, r.subs[::-1].copy(), r.moments, r.rgba)
        assert ctx.tile_shape() == before  # a rejected call leaves the shape as it was
        best, ms = ctx.autotune_tile_shape(r.mesh, r.view, r.tf, r.mboit, r.subs, r.moments, r.rgba, repeats=1)
        print("autotuned tile width", best, ms)
        assert best in (2, 4, 8, 16, 32) and sorted(ms) == [2, 4, 8, 16, 32] and all(v > 0 for v in ms.values())
        assert ctx.tile_shape()[0] == best
        assert torch.equal(r.frame(), outs[8][1])
        with pytest.raises(apc.ApcError):
            ctx.set_tile_shape(3)
        # widths and both dispatch modes: the fastest is set, the frame is unchanged
        best, mode, table = ctx.autotune_launch(r.mesh, r.view, r.tf, r.mboit, r.subs, r.moments, r.rgba)
        print("autotuned launch", best, mode, table)
        assert sorted(table) == [(d, w) for d in (0, 1) for w in (2, 4, 8, 16, 32)]
        assert table[(mode, best)] == min(table.values())
        assert ctx.tile_shape()[0] == best and ctx.dispatch() == mode
        assert torch.equal(r.frame(), outs[8][1])
    finally:
        ctx.set_tile_shape(8)
        ctx.set_dispatch(apc.APC_DISPATCH_GRID)


@pytest.mark.parametrize("size,m,tw", [(300, 8, 8), (200, 4, 16)])
def test_moment_tiles_hold_the_dense_images(apc, ctx, size, m, tw):
    """The tiles form of stage one (one 64-pixel tile per (tile, subdomain) pair with binned faces): every
    pair's tile is the dense per-subdomain image's values on its pixels (0 outside the image), every pixel of
    a tile without a pair is 0 in the dense image, pair_bin ascends, and the sum of the tiles is bitwise the
    dense sum.  A query counts the pairs; buffers one pair short get APC_E_NOMEM and stay untouched.  Walked
    pair by pair (a workgroup per pair) the tiles are bitwise the same.  Ragged image, two tile shapes, m = 8
    and 4."""
    sc = synth.scene_medium(size=size)
    sc.m = m
    sc.bias = synth.default_bias(m)
    try:
        ctx.set_tile_shape(tw)
        r = apc.Renderer(ctx, sc)
        r.frame()  # dense per-subdomain images + apc_sum_moments
        dense, glob = _np(r.per_sub), r.moments.clone()
        S, H, W = len(r.subs), size, size
        n = ctx.moments_pass_tiles(r.mesh, r.view, r.tf, m, r.subs)
        assert n > 0
        small = torch.full((n - 1, m + 1, 64), -7.0, dtype=torch.float32, device="cuda")
        small_b = torch.full((n - 1,), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(apc.ApcError) as e:
            ctx.moments_pass_tiles(r.mesh, r.view, r.tf, m, r.subs, small, small_b)
        assert e.value.status == 3
        torch.cuda.synchronize()
        assert bool((small == -7.0).all()) and bool((small_b == -7).all())
        tiles = torch.full((n, m + 1, 64), -7.0, dtype=torch.float32, device="cuda")
        pb = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        assert ctx.moments_pass_tiles(r.mesh, r.view, r.tf, m, r.subs, tiles, pb) == n
        g = torch.empty_like(glob)
        ctx.sum_moment_tiles(tiles, pb, n, S, m, H, W, g)
        torch.cuda.synchronize()
        assert torch.equal(g, glob)
        # rebuild the dense images from the tiles on the host
        t_np, b_np = _np(tiles), pb.cpu().numpy().astype(np.int64)
        assert np.all(np.diff(b_np) > 0) and b_np[0] >= 0
        th, tiles_x = 64 // tw, (W + tw - 1) // tw
        tile, slot = b_np // S, b_np % S
        lane = np.arange(64)
        y = (tile // tiles_x)[:, None] * th + lane[None, :] // tw
        x = (tile % tiles_x)[:, None] * tw + lane[None, :] % tw
        inside = (y < H) & (x < W)
        assert np.all(t_np.transpose(0, 2, 1)[~inside] == 0)
        rebuilt = np.zeros_like(dense)
        pp, ll = np.nonzero(inside)
        rebuilt[slot[pp], :, y[pp, ll], x[pp, ll]] = t_np[pp, :, ll]
        assert np.array_equal(rebuilt, dense)
        # walked pair by pair (a workgroup per pair): bitwise the same tiles and pair list
        tiles2 = torch.full((n, m + 1, 64), -7.0, dtype=torch.float32, device="cuda")
        pb2 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        assert ctx.moments_pass_tiles(r.mesh, r.view, r.tf, m, r.subs, tiles2, pb2, by_pair=True) == n
        torch.cuda.synchronize()
        assert torch.equal(tiles2, tiles) and torch.equal(pb2, pb)
        with pytest.raises(apc.ApcError):  # no per-pixel segment counts after a stage one by pairs
            ctx.segment_counts(H, W)
        print("size %d m %d tile %dx%d: %d pairs of %d bins, %.1f%% of the dense bytes" % (
            size, m, tw, th, n, S * tiles_x * ((H + th - 1) // th), 100.0 * n * 64 / (S * H * W)))
    finally:
        ctx.set_tile_shape(8)


def test_work_queue_dispatch_gives_identical_results(apc, ctx):
    """Persistent workgroups taking tiles from per-XCD counters (APC_DISPATCH_QUEUE) compute each tile with
    the same code in the same order as one workgroup per tile: per-subdomain and global moments, the kept
    pieces' and the plain form's images, a partial image and a captured frame are bitwise the grid's, on the
    uneven batching mesh (ragged image: the last tiles are partly outside) and at m = 4."""
    sc = synth.scene_batching(size=300)
    r = apc.Renderer(ctx, sc)
    try:
        assert ctx.dispatch() == apc.APC_DISPATCH_GRID
        grid = {}
        for mode in (apc.APC_DISPATCH_GRID, apc.APC_DISPATCH_QUEUE):
            ctx.set_dispatch(mode)
            out = [r.frame().clone(), r.per_sub.clone(), r.moments.clone(), r.frame(global_sum=True).clone(),
                   r.moments.clone()]
            r.frame(global_sum=True, keep=True)
            out.append(r.frame(global_sum=True, keep=True).clone())
            part = torch.empty_like(r.rgba)
            ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, [5, 40], part, finalize=False)
            out.append(part)
            g = apc.FrameGraph(r, global_sum=True)
            try:
                g.launch()
                torch.cuda.synchronize()
                out.append(r.rgba.clone())
            finally:
                g.close()
            c = ctx.counters(reset=True)
            assert c["walk_step_limit"] == 0
            if mode == apc.APC_DISPATCH_GRID:
                grid = out
            else:
                assert ctx.dispatch() == apc.APC_DISPATCH_QUEUE
                for k, (a, b) in enumerate(zip(grid, out)):
                    assert torch.equal(a, b), k
        sc4 = synth.scene_medium(size=200)
        sc4.m = 4
        sc4.bias = synth.default_bias(4)
        r4 = apc.Renderer(ctx, sc4)
        q4 = r4.frame(global_sum=True).clone()
        ctx.set_dispatch(apc.APC_DISPATCH_GRID)
        assert torch.equal(r4.frame(global_sum=True), q4)
        with pytest.raises(apc.ApcError):
            ctx.set_dispatch(2)
    finally:
        ctx.set_dispatch(apc.APC_DISPATCH_GRID)


@pytest.mark.parametrize("global_sum,keep", [(False, False), (True, False), (True, True)])
def test_frame_graph_replays_match_eager_frames(apc, ctx, global_sum, keep):
    """A frame captured in a HIP graph (separate moment sum or stage one summing the subdomains itself; stage
    two walking again or evaluating kept pieces): every replay (with eager work and synchronisation between
    replays) gives bitwise the eager frame, and after the transfer-function table is edited in place a
    replay gives bitwise the eager frame with the new table."""
    sc = synth.scene_medium(size=256)
    r = apc.Renderer(ctx, sc)
    for _ in range(2 if keep else 1):  # a kept-piece frame sizes the pool first
        eager = r.frame(global_sum=global_sum, keep=keep).clone()
    eager_mom = r.moments.clone()
    g = apc.FrameGraph(r, global_sum=global_sum, keep=keep)
    try:
        torch.cuda.synchronize()
        assert torch.equal(r.rgba, eager)  # the sizing frame
        for k in range(3):
            r.rgba.fill_(-1.0)
            r.moments.fill_(-1.0)
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(r.rgba, eager), k
            assert torch.equal(r.moments, eager_mom), k
            junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
            torch.cuda.synchronize()
            del junk
        cnt = g.counters()
        assert cnt["pieces"] > 0 and cnt["walk_step_limit"] == 0 and cnt["entry_overflow"] == 0
        # edit the transfer function in place: the replay follows it
        r.tf_dev[:, :3] = r.tf_dev[:, :3].flip(0).contiguous()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        replay = r.rgba.clone()
        again = r.frame(global_sum=global_sum, keep=keep)
        torch.cuda.synchronize()
        assert torch.equal(replay, again)
        assert not torch.equal(replay, eager)
    finally:
        g.close()


@pytest.mark.parametrize("name", ["tiny", "medium", "adaptive"])
def test_rewalk_meets_the_pieces_of_stage_one(apc, ctx, name):
    """Stage two walks every ray again (Alg. 1, second loop) in a walker wavefront that hands the pieces to the
    evaluator through an LDS ring in phases: it must meet exactly the pieces, tet steps, entries and ray
    segments stage one met, whatever the phases did (a dropped or doubled piece, or a chord cut differently,
    shows up here before it shows in the image)."""
    sc = {"tiny": synth.scene_tiny, "medium": lambda: synth.scene_medium(size=512),
          "adaptive": lambda: synth.scene_amr_small(size=200)}[name]()
    r = apc.Renderer(ctx, sc)
    r.frame(global_sum=True)  # sizes the context's buffers
    torch.cuda.synchronize()
    ctx.counters(reset=True)
    ctx.moments_pass(r.mesh, r.view, r.tf, sc.m, r.subs, r.moments, None, global_sum=True)
    torch.cuda.synchronize()
    one = ctx.counters(reset=True)
    ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, r.subs, r.rgba, finalize=True)
    torch.cuda.synchronize()
    two = ctx.counters()
    print(name, {k: (one[k], two[k]) for k in ("pieces", "tet_steps", "entries", "segments")})
    assert one["pieces"] > 0 and one["walk_step_limit"] == 0 and two["walk_step_limit"] == 0
    for k in ("pieces", "tet_steps", "entries", "segments"):
        assert two[k] == one[k], (k, one[k], two[k])


@pytest.mark.parametrize("name", ["tiny", "medium", "adaptive"])
def test_frame_by_pair_is_the_frame_by_tile(apc, ctx, name):
    """Stage one by (tile, subdomain) pairs (a workgroup per pair into the tiles form, then the ordered FP64
    sum of the pairs) gives the global moments and the image bit for bit: each pair is the same walk as in
    the per-tile launch and the sum takes the slots in the same order.  The walk counters agree too.  For a
    subset of the subdomains it equals the separate sum of their per-subdomain images."""
    sc = {"tiny": synth.scene_tiny, "medium": lambda: synth.scene_medium(size=300),
          "adaptive": lambda: synth.scene_amr_small(size=200)}[name]()
    r = apc.Renderer(ctx, sc)
    r.frame(global_sum=True)  # sizes the context's buffers
    torch.cuda.synchronize()
    ctx.counters(reset=True)
    r.frame(global_sum=True)
    torch.cuda.synchronize()
    by_tile = ctx.counters(reset=True)
    rgba, mom = r.rgba.clone(), r.moments.clone()
    r.rgba.fill_(-1.0)
    r.moments.fill_(-1.0)
    r.frame(by_pair=True)
    torch.cuda.synchronize()
    by_pair = ctx.counters(reset=True)
    assert torch.equal(r.moments, mom) and torch.equal(r.rgba, rgba)
    for k in ("pieces", "tet_steps", "entries", "segments", "walk_step_limit"):
        assert by_pair[k] == by_tile[k], (k, by_tile[k], by_pair[k])
    with pytest.raises(ValueError):
        r.frame(by_pair=True, keep=True)
    subset = np.asarray(r.subs[1::2], np.int32)
    r.frame(subdomains=subset)
    torch.cuda.synchronize()
    rgba_s, mom_s = r.rgba.clone(), r.moments.clone()
    r.frame(subdomains=subset, by_pair=True)
    torch.cuda.synchronize()
    assert torch.equal(r.moments, mom_s) and torch.equal(r.rgba, rgba_s)
    assert not torch.equal(mom_s, mom)
    print(name, "pieces", by_tile["pieces"], "subset", len(subset), "of", len(r.subs))


@pytest.mark.parametrize("name", ["tiny", "medium", "adaptive"])
def test_rewalk_by_pair_matches_the_rewalk_by_tile(apc, ctx, name):
    """Stage two by (tile, subdomain) pairs (APC_BY_PAIR: a workgroup per pair writes its unfinalised colour
    sums, then each pixel's pairs are summed in slot order and finalised) meets exactly the pieces, tet steps,
    entries and segments of the per-tile re-walk and gives its image to FP32 rounding: the colour sums are
    grouped by subdomain and each pair's root solver starts afresh, the differences the kept-piece form has
    too (its bar, 2e-5).  Pixels without pieces are bitwise equal.  Also the unfinalised partial image of a
    subset, the whole frame with both stages by pairs, and (tiny) the oracle's bars."""
    sc = {"tiny": synth.scene_tiny, "medium": lambda: synth.scene_medium(size=300),
          "adaptive": lambda: synth.scene_amr_small(size=200)}[name]()
    r = apc.Renderer(ctx, sc)
    r.frame(global_sum=True)
    ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, r.subs, r.rgba, finalize=True, by_pair=True)
    torch.cuda.synchronize()  # both forms' buffers sized
    ctx.counters(reset=True)
    ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, r.subs, r.rgba, finalize=True)
    torch.cuda.synchronize()
    by_tile, want = ctx.counters(reset=True), r.rgba.clone()
    got = torch.full_like(want, -1.0)
    ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, r.subs, got, finalize=True, by_pair=True)
    torch.cuda.synchronize()
    by_pair = ctx.counters(reset=True)
    assert by_tile["pieces"] > 0
    for k in ("pieces", "tet_steps", "entries", "segments", "walk_step_limit"):
        assert by_pair[k] == by_tile[k], (k, by_tile[k], by_pair[k])
    diff = (got - want).abs().max().item()
    assert diff <= 2e-5, diff
    empty = r.moments[0] == 0
    assert torch.equal(got[empty], want[empty])
    subset = np.asarray(r.subs[1::2], np.int32)
    part_t, part_p = torch.empty_like(want), torch.full_like(want, -1.0)
    ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, subset, part_t, finalize=False)
    ctx.resolve_pass(r.mesh, r.view, r.tf, r.mboit, r.moments, subset, part_p, finalize=False, by_pair=True)
    torch.cuda.synchronize()
    assert (part_p - part_t).abs().max().item() <= 2e-5
    assert not torch.equal(part_t, want)
    r.rgba.fill_(-1.0)
    r.frame(by_pair=True, resolve_by_pair=True)
    torch.cuda.synchronize()
    assert (r.rgba - want).abs().max().item() <= 2e-5
    if name == "tiny":
        ref = oracle.render(sc)
        d = _np(got).reshape(-1, 4) - ref["rgba"]
        assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4
    print(name, "pieces", by_tile["pieces"], "max |by pair - by tile|", diff)


def test_stage_two_reuses_the_bins_of_stage_one_only_for_the_same_frame(apc, ctx):
    """Both passes skip binning when the context's bins were made for the same mesh, view, tile shape and
    subdomain list (stage two after stage one of the same frame, or the same frame again): a frame bins once,
    as much as a fresh context's stage one, and its repetition not at all.  After a stage one of another
    view, another subdomain list, another tile shape or another mesh load it bins again, and every image
    is bitwise the one of a context that binned for it afresh."""
    sc = synth.scene_tiny()
    r = apc.Renderer(ctx, sc)
    view_a = r.view
    view_b = apc.make_view(synth.perspective_view(synth.sphere_eye(9), (0.5, 0.5, 0.5), 128, 128), sc.step)
    fresh = apc.Context(0)
    fresh_mesh = None
    try:
        fresh_mesh = fresh.load_mesh(sc.mesh.xyz, sc.mesh.scalar, sc.mesh.tets, sc.mesh.tet_sub, sc.mesh.n_sub)
        # the whole frame on view A: stage one bins, stage two reuses them
        ctx.counters(reset=True)
        r.view = view_a
        r.frame(global_sum=True)
        torch.cuda.synchronize()
        c = ctx.counters(reset=True)
        mom_a, rgba_a = r.moments.clone(), r.rgba.clone()
        fresh.counters(reset=True)
        fresh.moments_pass(fresh_mesh, view_a, r.tf, sc.m, r.subs, torch.empty_like(mom_a), None, global_sum=True)
        torch.cuda.synchronize()
        assert fresh.counters(reset=True)["bin_records"] == c["bin_records"] > 0  # one binning per frame
        ctx.moments_pass(r.mesh, view_a, r.tf, sc.m, r.subs, r.moments, None, global_sum=True)
        torch.cuda.synchronize()
        assert ctx.counters(reset=True)["bin_records"] == 0  # the same frame again: nothing to bin
        assert torch.equal(r.moments, mom_a)
        # stage one of view B, then stage two of view A with A's moments: bins again, the same image
        ctx.moments_pass(r.mesh, view_b, r.tf, sc.m, r.subs, r.moments, None, global_sum=True)
        out = torch.full_like(rgba_a, -1.0)
        ctx.resolve_pass(r.mesh, view_a, r.tf, r.mboit, mom_a, r.subs, out, finalize=True)
        torch.cuda.synchronize()
        assert torch.equal(out, rgba_a)
        # a subset after stage one of all subdomains: its partial image as a fresh context makes it
        subset = np.asarray(r.subs[1::2], np.int32)
        ctx.moments_pass(r.mesh, view_a, r.tf, sc.m, r.subs, r.moments, None, global_sum=True)
        part = torch.full_like(rgba_a, -1.0)
        ctx.resolve_pass(r.mesh, view_a, r.tf, r.mboit, mom_a, subset, part, finalize=False)
        want = torch.full_like(rgba_a, -2.0)
        fresh.resolve_pass(fresh_mesh, view_a, r.tf, r.mboit, mom_a, subset, want, finalize=False)
        torch.cuda.synchronize()
        assert torch.equal(part, want)
        # another tile shape between the passes
        ctx.moments_pass(r.mesh, view_a, r.tf, sc.m, r.subs, r.moments, None, global_sum=True)
        ctx.set_tile_shape(16)
        out.fill_(-1.0)
        ctx.resolve_pass(r.mesh, view_a, r.tf, r.mboit, mom_a, r.subs, out, finalize=True)
        fresh.set_tile_shape(16)
        want.fill_(-2.0)
        fresh.resolve_pass(fresh_mesh, view_a, r.tf, r.mboit, mom_a, r.subs, want, finalize=True)
        torch.cuda.synchronize()
        assert torch.equal(out, want)
        ctx.set_tile_shape(8)
        # another load of the mesh (same arrays): bins again, the same image
        ctx.moments_pass(r.mesh, view_a, r.tf, sc.m, r.subs, r.moments, None, global_sum=True)
        other = ctx.load_mesh(sc.mesh.xyz, sc.mesh.scalar, sc.mesh.tets, sc.mesh.tet_sub, sc.mesh.n_sub)
        out.fill_(-1.0)
        ctx.resolve_pass(other, view_a, r.tf, r.mboit, mom_a, r.subs, out, finalize=True)
        torch.cuda.synchronize()
        assert torch.equal(out, rgba_a)
        other.free()
    finally:
        ctx.set_tile_shape(8)
        if fresh_mesh is not None:
            fresh_mesh.free()
        fresh.close()


@pytest.mark.parametrize("m", [4, 6, 8])
def test_kept_pieces_match_the_plain_form(apc, ctx, m):
    """Stage two evaluating the pieces stage one kept gives the image of the plain form (stage two walking
    the rays again and evaluating each piece at once) to rounding: the same pieces, the same bound, other
    root-solver starts (a per-pixel gap table instead of the previous sample's roots) and another summation
    order.  Both match the oracle on sampled pixels."""
    sc = synth.scene_medium(size=384)
    sc.m = m
    sc.bias = synth.default_bias(m)
    r = apc.Renderer(ctx, sc)
    plain = r.frame(global_sum=True).clone()
    t = ctx.timings()
    assert t["rewalk_ms"] > 0 and t["eval_ms"] == 0
    r.frame(global_sum=True, keep=True)  # the first kept frame may not fit the store; the store grows after it
    kept = r.frame(global_sum=True, keep=True).clone()
    torch.cuda.synchronize()
    t = ctx.timings()
    assert t["rewalk_ms"] == 0 and t["eval_ms"] > 0  # no second walk
    diff = (kept - plain).abs().max().item()
    print("m = %d: kept vs plain max %.3g" % (m, diff))
    assert diff <= 2e-5
    pix = np.sort(np.random.default_rng(23).choice(384 * 384, 1500, replace=False))
    ref = oracle.render(sc, pixels=pix)
    for img in (plain, kept):
        d = _np(img).reshape(-1, 4)[pix] - ref["rgba"]
        assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4


@pytest.mark.parametrize("m", [4, 8])
def test_global_sum_in_stage_one_is_bitwise_the_separate_sum(apc, ctx, m):
    """Stage one summing the subdomains itself (APC_MOMENTS_GLOBAL) gives bitwise the global moments of the
    per-subdomain images summed by apc_sum_moments, and the same image; the ids must be ascending."""
    sc = synth.scene_medium(size=256)
    sc.m = m
    sc.bias = synth.default_bias(m)
    r = apc.Renderer(ctx, sc)
    sep = r.frame().clone()
    mom_sep = r.moments.clone()
    for _ in range(2):
        r.moments.fill_(float("nan"))
        glob = r.frame(global_sum=True)
        torch.cuda.synchronize()
        assert torch.equal(r.moments, mom_sep)
        assert torch.equal(glob, sep)
    with pytest.raises(RuntimeError):
        ctx.moments_pass(r.mesh, r.view, r.tf, m, r.subs[::-1].copy(), r.moments, global_sum=True)


def test_pool_limit_below_the_pieces_walks_again_with_the_plain_image(apc, ctx):
    """A context whose kept-piece pool is capped far below the frame's pieces (48 MB for more than twice
    that) cannot keep them: stage two walks again, and the image is bitwise that of the plain form, frame
    after frame."""
    sc = synth.scene_medium(size=256)
    ref = apc.Renderer(ctx, sc).frame().clone()
    small = apc.Context(0)
    try:
        small.set_workspace_limit(48 << 20)
        r = apc.Renderer(small, sc)
        for _ in range(2):
            small.counters(reset=True)
            got = r.frame(keep=True)
            torch.cuda.synchronize()
            t, c = small.timings(), small.counters()
            assert t["rewalk_ms"] > 0  # the pieces do not fit the pool: stage two walked again
            assert c["pieces"] // 2 * 12 > 2 * (48 << 20)  # each walk's pieces: more than twice the pool
            assert torch.equal(got, ref)
    finally:
        del r
        small.close()


def test_large_full_size_sampled_pixels_match_oracle(apc, ctx):
    """The full-size configuration the benchmark times (256^3 x 6 = 100,663,296 tets, 72 subdomains,
    2560^2 perspective, m = 8), in its launch configuration (stage one summing the subdomains, stage two
    walking again; a warm-up frame, then the timed one): 3,000 seeded pixels against the oracle (moments by
    the forward bar, RGBA by the image bar), both frames bitwise equal; and the kept-piece variant's image
    equal to it to rounding."""
    sc = synth.scene_large()
    r = apc.Renderer(ctx, sc)
    first = r.frame(global_sum=True).clone()
    ctx.counters(reset=True)
    rgba = r.frame(global_sum=True).clone()
    torch.cuda.synchronize()
    assert ctx.timings()["rewalk_ms"] > 0
    assert torch.equal(rgba, first)
    assert ctx.counters()["walk_step_limit"] == 0 and ctx.counters()["nonpd_pivots"] == 0
    W, H = sc.view["width"], sc.view["height"]
    pix = np.sort(np.random.default_rng(17).choice(W * H, 3000, replace=False))
    ref = oracle.render(sc, pixels=pix)
    fwd, n_back = _check_moments(sc, pix, _flat_moments(r.moments)[:, pix], ref)
    d = _np(rgba).reshape(-1, 4)[pix] - ref["rgba"]
    print("large: moments forward %.3g (%d on the backward bar), rgba max %.3g rmse %.3g" % (
        fwd, n_back, np.abs(d).max(), math.sqrt(np.mean(d ** 2))))
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4
    for _ in range(2):  # the kept-piece variant: the first frame sizes the pool
        kept = r.frame(global_sum=True, keep=True)
    torch.cuda.synchronize()
    assert ctx.timings()["eval_ms"] > 0
    assert (kept - rgba).abs().max().item() <= 2e-5
    del r


def test_adaptive_mesh_full_image_matches_oracle(apc, ctx):
    """Adaptive mesh with leaves of all four levels (8^3 base, finest 64^3, 434,690 tets, conforming cone
    decomposition: many vertices of high valence, coplanar faces on an exact lattice), 8 uneven chunks,
    200x200 perspective (ragged tiles), m = 8: every pixel against the oracle, per subdomain and global."""
    sc = synth.scene_amr_small(size=200)
    ref = oracle.render(sc, per_sub=True)
    ctx.counters(reset=True)
    r, rgba = _render(apc, ctx, sc)
    pix = np.arange(200 * 200)
    # a few silhouette pixels (0.02 %) need the backward bar: low-b0 rays through the coarsest leaves (edge
    # 1/8), where the FP32 side products' rounding across a face grows with the face's size
    fwd, n_back = _check_moments(sc, pix, _flat_moments(r.moments), ref)
    fwd_s, n_back_s = _check_moments(sc, pix, _flat_moments(r.per_sub), ref, per_sub=True)
    d = _np(rgba).reshape(-1, 4) - ref["rgba"]
    print("adaptive: moments forward %.3g (%d on the backward bar), per subdomain %.3g (%d), rgba max %.3g "
          "rmse %.3g" % (fwd, n_back, fwd_s, n_back_s, np.abs(d).max(), math.sqrt(np.mean(d ** 2))))
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4
    assert ctx.counters()["walk_step_limit"] == 0


def test_batching_mesh_sampled_pixels_match_oracle(apc, ctx):
    """The batching workload's adaptive mesh (32^3 base refined 0-3 levels, 19.4M tets, 72 Morton chunks of
    tet-count ratio 12) at its full 2560^2, m = 8, in the launch configuration the benchmark times: 3,000
    seeded pixels against the oracle."""
    sc = synth.scene_batching(size=2560)
    r = apc.Renderer(ctx, sc)
    r.frame(global_sum=True)
    rgba = r.frame(global_sum=True)
    torch.cuda.synchronize()
    W, H = sc.view["width"], sc.view["height"]
    pix = np.sort(np.random.default_rng(19).choice(W * H, 3000, replace=False))
    ref = oracle.render(sc, pixels=pix)
    fwd, n_back = _check_moments(sc, pix, _flat_moments(r.moments)[:, pix], ref)
    d = _np(rgba).reshape(-1, 4)[pix] - ref["rgba"]
    print("batching: %d tets, moments forward %.3g (%d on the backward bar), rgba max %.3g rmse %.3g" % (
        sc.mesh.n_tets, fwd, n_back, np.abs(d).max(), math.sqrt(np.mean(d ** 2))))
    assert np.abs(d).max() <= 2e-3 and math.sqrt(np.mean(d ** 2)) <= 5e-4
