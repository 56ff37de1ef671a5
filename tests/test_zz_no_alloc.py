"""apc_resolve_pass_noalloc through the C ABI: the allocation-free variant of
apc_resolve_pass (its binning state in the library's static device workspace)
gives bitwise the image of apc_resolve_pass in the plain form, on two calls in
a row, the second with a smaller frame (the workspace keeps the first call's
contents, which the second must not depend on); a frame beyond the workspace
is rejected with APC_E_NOMEM and leaves the output untouched."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apc():
    import paper_2501_12581_amd as P
    P.lib()
    return P


def _frame(apc, ctx, r, view_dict, noalloc, m):
    view = apc.make_view(view_dict, r.scene.step)
    H, W = view.height, view.width
    mom = torch.empty((m + 1, H, W), dtype=torch.float32, device="cuda")
    rgba = torch.full((H, W, 4), -7.0, dtype=torch.float32, device="cuda")
    ctx.moments_pass(r.mesh, view, r.tf, m, r.subs, mom, global_sum=True)
    call = ctx.resolve_pass_noalloc if noalloc else ctx.resolve_pass
    call(r.mesh, view, r.tf, r.mboit, mom, r.subs, rgba)
    torch.cuda.synchronize()
    return rgba


@pytest.mark.parametrize("m", [4, 8])
def test_noalloc_resolve_matches_the_plain_resolve(apc, m):
    ctx = apc.Context(0)
    try:
        sc = synth.scene_medium(size=512)
        sc.m = m
        sc.bias = synth.default_bias(m)
        r = apc.Renderer(ctx, sc)
        for size in (512, 200):  # two calls in a row, the second smaller (ragged tiles)
            v = synth.perspective_view(synth.sphere_eye(5), (0.5, 0.5, 0.5), size, size)
            ref = _frame(apc, ctx, r, v, False, m)
            ctx.counters(reset=True)
            got = _frame(apc, ctx, r, v, True, m)
            c = ctx.counters()
            assert c["entry_overflow"] == 0 and c["pieces"] > 0
            assert torch.equal(got, ref), (size, (got - ref).abs().max().item())
            assert ctx.timings()["rewalk_ms"] > 0
        # the partial image of one subdomain (no finalisation) as well
        view = apc.make_view(synth.perspective_view(synth.sphere_eye(5), (0.5, 0.5, 0.5), 200, 200), sc.step)
        mom = torch.empty((m + 1, 200, 200), dtype=torch.float32, device="cuda")
        ctx.moments_pass(r.mesh, view, r.tf, m, r.subs, mom, global_sum=True)
        a = torch.empty((200, 200, 4), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        ctx.resolve_pass(r.mesh, view, r.tf, r.mboit, mom, [3], a, finalize=False)
        ctx.resolve_pass_noalloc(r.mesh, view, r.tf, r.mboit, mom, [3], b, finalize=False)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        del r
    finally:
        ctx.close()


def test_noalloc_rejects_a_frame_beyond_its_workspace(apc):
    ctx = apc.Context(0)
    try:
        sc = synth.scene_medium(size=64)
        r = apc.Renderer(ctx, sc)
        size = 6144  # 589,824 tiles x 16 subdomains x 12 bytes of counts alone exceed 64 MiB
        view = apc.make_view(synth.perspective_view(synth.sphere_eye(5), (0.5, 0.5, 0.5), size, size), sc.step)
        mom = torch.zeros((sc.m + 1, size, size), dtype=torch.float32, device="cuda")
        rgba = torch.full((size, size, 4), -7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(apc.ApcError) as e:
            ctx.resolve_pass_noalloc(r.mesh, view, r.tf, r.mboit, mom, r.subs, rgba)
        assert e.value.status == 3 and "static workspace" in str(e.value)
        torch.cuda.synchronize()
        assert bool((rgba == -7.0).all())
        del r
    finally:
        ctx.close()
