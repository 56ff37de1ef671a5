"""The C ABI's failure contract, on the CPU, through a host-only context.

apc_create(APC_DEVICE_NONE) makes no HIP call: every entry point validates its
arguments exactly as on a device and then returns APC_E_DEVICE ("nothing was
launched").  So each status path is reachable here: a bad argument gives its
own status and message, a good one reaches APC_E_DEVICE, and no call writes
through an output pointer (the output buffers below are host arrays holding a
sentinel, which must survive every call).  The mesh contract follows the
paper's statement of the problem: disjoint subdomains of positively oriented
tets meeting face to face (Section 4; Section 6 rules out overlapping
volumes).
"""
import ctypes as C

import numpy as np
import pytest

import synth

SENTINEL = np.float32(-12345.0)


@pytest.fixture(scope="module")
def P():
    import paper_2501_12581_amd as P
    import os
    if not os.path.exists(P.LIB_PATH):
        from paper_2501_12581_amd import build
        build.build()
    P.lib()
    return P


@pytest.fixture()
def ctx(P):
    h = C.c_void_p()
    assert P.lib().apc_create(P.APC_DEVICE_NONE, C.byref(h)) == 0
    yield h
    assert P.lib().apc_destroy(h) == 0


def small_mesh():
    """4^3 cubes x 6 Kuhn tets, 3 Morton chunks."""
    return synth.grid_mesh(4, 3, seed=3, n_gauss=2, jagged_seed=5)


def desc(P, xyz, scal, tets, sub, n_sub, flags=0):
    keep = [np.ascontiguousarray(xyz, np.float32), np.ascontiguousarray(scal, np.float32),
            np.ascontiguousarray(tets, np.int32), np.ascontiguousarray(sub, np.int32)]
    d = P.MeshDesc(n_vertices=keep[0].shape[0], n_tets=keep[2].shape[0], n_subdomains=n_sub, flags=flags,
                   xyz=keep[0].ctypes.data, scalar=keep[1].ctypes.data, tet_vertices=keep[2].ctypes.data,
                   tet_subdomain=keep[3].ctypes.data)
    return d, keep


def load(P, ctx, d):
    h = C.c_void_p(12345)  # must be reset to NULL on failure
    st = P.lib().apc_load_mesh(ctx, C.byref(d), C.byref(h), None)
    return st, h


def err(P, ctx):
    return P.lib().apc_last_error(ctx).decode()


def test_host_only_context_loads_a_valid_mesh(P, ctx):
    m = small_mesh()
    d, keep = desc(P, m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub)
    st, h = load(P, ctx, d)
    assert st == 0, err(P, ctx)
    info = P.MeshInfo()
    assert P.lib().apc_mesh_get_info(h, C.byref(info)) == 0
    assert info.n_tets == m.n_tets and info.n_subdomains == 3 and info.device_bytes == 0
    assert info.n_boundary_faces >= 6 * 2 * 16  # at least the hull (6 sides x 16 squares x 2 triangles)
    assert tuple(info.bbox_lo) == (0.0, 0.0, 0.0) and tuple(info.bbox_hi) == (1.0, 1.0, 1.0)
    total = 0
    for s in range(3):
        nt, nf = C.c_int64(), C.c_int64()
        assert P.lib().apc_mesh_subdomain_info(h, s, C.byref(nt), C.byref(nf)) == 0
        total += nt.value
    assert total == m.n_tets
    assert P.lib().apc_mesh_subdomain_info(h, 3, None, None) == 1  # APC_E_ARG: id out of range
    assert P.lib().apc_free_mesh(ctx, h) == 0


def _mesh_case(P, ctx, mutate, status, words):
    m = small_mesh()
    xyz, scal, tets, sub = m.xyz.copy(), m.scalar.copy(), m.tets.copy(), m.tet_sub.copy()
    n_sub, flags = mutate(xyz, scal, tets, sub)
    d, keep = desc(P, xyz, scal, tets, sub, n_sub, flags)
    st, h = load(P, ctx, d)
    msg = err(P, ctx)
    assert st == status, (st, msg)
    assert h.value is None, "a failed load must not return a mesh"
    assert all(w in msg for w in words), msg


def test_inverted_tet(P, ctx):
    def f(xyz, scal, tets, sub):
        tets[5, [1, 2]] = tets[5, [2, 1]]  # swapping two vertices flips the orientation
        return 3, 0
    _mesh_case(P, ctx, f, 2, ["tet 5", "non-positive signed volume"])


def test_repeated_vertex(P, ctx):
    def f(xyz, scal, tets, sub):
        tets[7, 3] = tets[7, 0]
        return 3, 0
    _mesh_case(P, ctx, f, 2, ["tet 7", "repeated vertex"])


def test_vertex_id_out_of_range(P, ctx):
    def f(xyz, scal, tets, sub):
        tets[2, 1] = xyz.shape[0]
        return 3, 0
    _mesh_case(P, ctx, f, 2, ["tet 2", "vertex id out of range"])
    def g(xyz, scal, tets, sub):
        tets[4, 0] = -1
        return 3, 0
    _mesh_case(P, ctx, g, 2, ["tet 4", "vertex id out of range"])


def test_subdomain_id_out_of_range(P, ctx):
    def f(xyz, scal, tets, sub):
        sub[11] = 3
        return 3, 0
    _mesh_case(P, ctx, f, 2, ["tet 11", "subdomain id out of range"])


def test_non_finite_vertex(P, ctx):
    def f(xyz, scal, tets, sub):
        xyz[tets[0, 0], 1] = np.nan
        return 3, 0
    _mesh_case(P, ctx, f, 2, ["not finite"])


def test_sizes_and_flags(P, ctx):
    _mesh_case(P, ctx, lambda *a: (0, 0), 1, ["n_subdomains"])
    _mesh_case(P, ctx, lambda *a: (3, 4), 1, ["unknown mesh flags"])
    # device arrays need a device: the host-only context stops before reading them
    _mesh_case(P, ctx, lambda *a: (3, P.APC_MESH_DEVICE), 4, ["host-only", "nothing was launched"])
    m = small_mesh()
    d, keep = desc(P, m.xyz, m.scalar, m.tets, m.tet_sub, 3)
    d.n_tets = 0
    assert load(P, ctx, d)[0] == 1 and "n_tets" in err(P, ctx)
    d, keep = desc(P, m.xyz, m.scalar, m.tets, m.tet_sub, 3)
    d.xyz = None
    assert load(P, ctx, d)[0] == 1 and "NULL" in err(P, ctx)
    h = C.c_void_p()
    assert P.lib().apc_load_mesh(ctx, None, C.byref(h), None) == 1


def test_face_shared_by_three_tets(P, ctx):
    # a triangle (0, 1, 2) in z = 0 with apexes above and below: three positively oriented tets share it
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.2, 1], [0.2, 0.2, -1], [0.3, 0.3, 2]], np.float32)
    tets = []
    for apex in (3, 4, 5):
        t = [0, 1, 2, apex]
        p = xyz[t].astype(np.float64)
        if np.linalg.det(np.stack([p[1] - p[0], p[2] - p[0], p[3] - p[0]])) < 0:
            t[1], t[2] = t[2], t[1]
        tets.append(t)
    tets = np.array(tets, np.int32)
    d, keep = desc(P, xyz, np.zeros(6, np.float32), tets, np.zeros(3, np.int32), 1)
    st, h = load(P, ctx, d)
    assert st == 2 and "non-manifold" in err(P, ctx), err(P, ctx)
    assert h.value is None
    # two of them are a valid mesh
    d, keep = desc(P, xyz, np.zeros(6, np.float32), tets[:2], np.zeros(2, np.int32), 1)
    st, h = load(P, ctx, d)
    assert st == 0, err(P, ctx)
    P.lib().apc_free_mesh(ctx, h)


# ------------------------------------------------------------------ the passes

@pytest.fixture()
def scene(P, ctx):
    m = small_mesh()
    d, keep = desc(P, m.xyz, m.scalar, m.tets, m.tet_sub, m.n_sub)
    st, mesh = load(P, ctx, d)
    assert st == 0
    view = synth.perspective_view(synth.sphere_eye(4), (0.5, 0.5, 0.5), 32, 24)
    v = P.make_view(view, 1.0 / 16)
    tf_host = np.full((256, 4), 0.5, np.float32)
    tf = P.TF(n_entries=256, pad=0, rgba=tf_host.ctypes.data, s_min=0.0, s_max=1.0, kappa=4.0, absorbance_max=10.0)
    mb = P.make_mboit(8, 5e-5, synth.default_bias(8), 0.3)
    subs = np.arange(3, dtype=np.int32)
    out = {"mom_sub": np.full((3, 9, 24, 32), SENTINEL, np.float32), "mom": np.full((9, 24, 32), SENTINEL, np.float32),
           "rgba": np.full((24, 32, 4), SENTINEL, np.float32), "f16": np.full((11, 24, 32), 7, np.uint16),
           "segs": np.full((2, 24, 32), 99, np.int32)}
    yield dict(mesh=mesh, view=v, tf=tf, tf_host=tf_host, mb=mb, subs=subs, out=out)
    for name, a in out.items():
        untouched = np.all(a == (SENTINEL if a.dtype == np.float32 else a.flat[0]))
        assert untouched, "a call wrote into %s" % name
    P.lib().apc_free_mesh(ctx, mesh)


def ptr(a):
    return C.c_void_p(a.ctypes.data)


def moments(P, ctx, sc, m=8, subs=None, out="mom", flags=None, view=None, tf=None):
    subs = sc["subs"] if subs is None else np.ascontiguousarray(subs, np.int32)
    flags = P.APC_MOMENTS_GLOBAL if flags is None else flags
    o = None if out is None else ptr(sc["out"][out])
    return P.lib().apc_moments_pass(ctx, sc["mesh"], C.byref(view or sc["view"]), C.byref(tf or sc["tf"]), m,
                                    ptr(subs), len(subs), o, flags, None)


def test_moments_pass_statuses(P, ctx, scene):
    sc = scene
    assert moments(P, ctx, sc) == 4 and "nothing was launched" in err(P, ctx)
    assert moments(P, ctx, sc, out="mom_sub", flags=0) == 4
    assert moments(P, ctx, sc, m=5) == 1 and "m = 5" in err(P, ctx)
    assert moments(P, ctx, sc, out=None) == 1 and "NULL" in err(P, ctx)
    assert moments(P, ctx, sc, subs=[0, 2, 1]) == 1 and "ascending" in err(P, ctx)
    assert moments(P, ctx, sc, subs=[0, 2, 1], out="mom_sub", flags=0) == 4  # any order without the global sum
    assert moments(P, ctx, sc, subs=[0, 3]) == 1 and "out of range" in err(P, ctx)
    assert moments(P, ctx, sc, subs=[1, 1]) == 1 and "twice" in err(P, ctx)
    assert moments(P, ctx, sc, flags=64) == 1 and "unknown flags" in err(P, ctx)
    assert P.lib().apc_moments_pass(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), 8, None, 3,
                                    ptr(sc["out"]["mom"]), 0, None) == 1
    assert P.lib().apc_moments_pass(ctx, None, C.byref(sc["view"]), C.byref(sc["tf"]), 8, ptr(sc["subs"]), 3,
                                    ptr(sc["out"]["mom"]), 0, None) == 1


def test_perspective_views_need_the_mesh_in_front_of_the_eye(P, ctx, scene):
    """The walk's entry test sees the whole line of a ray, so a perspective view must have the mesh's
    bounding box in front of the eye: a camera outside the box looking away from it, or looking sideways
    past it with part of the box behind, is an argument error; looking at it is valid (a host-only context
    then reports that nothing was launched)."""
    sc = scene
    eye = np.asarray(synth.sphere_eye(4))
    c = np.array([0.5, 0.5, 0.5])
    side = np.cross(c - eye, [0.0, 0.0, 1.0])
    for target, status in ((tuple(c), 4), (tuple(eye + (eye - c)), 1), (tuple(eye + side), 1)):
        v = P.make_view(synth.perspective_view(tuple(eye), target, 32, 24), 1.0 / 16)
        assert moments(P, ctx, sc, view=v) == status, (target, err(P, ctx))
        if status == 1:
            assert "in front of the camera" in err(P, ctx)
    # a camera beside the box, looking along it, outside the box but with its corners on both sides
    v = P.make_view(synth.perspective_view((0.5, -0.2, 0.5), (0.5, 1.5, 1.2), 32, 24), 1.0 / 16)
    assert moments(P, ctx, sc, view=v) == 1


def test_view_and_transfer_function_statuses(P, ctx, scene):
    sc = scene
    def copy_struct(x):
        return type(x).from_buffer_copy(x)

    def v_with(**kw):
        v = copy_struct(sc["view"])
        for k, val in kw.items():
            setattr(v, k, val)
        return v
    assert moments(P, ctx, sc, view=v_with(width=0)) == 1 and "image size" in err(P, ctx)
    assert moments(P, ctx, sc, view=v_with(step=0.0)) == 1 and "step" in err(P, ctx)
    assert moments(P, ctx, sc, view=v_with(projection=7)) == 1 and "projection" in err(P, ctx)
    inside = v_with()
    inside.eye = (C.c_double * 3)(0.5, 0.5, 0.5)
    assert moments(P, ctx, sc, view=inside) == 1 and "inside" in err(P, ctx)
    nan = v_with()
    nan.dir = (C.c_double * 3)(np.nan, 0.0, 1.0)
    assert moments(P, ctx, sc, view=nan) == 1 and "finite" in err(P, ctx)
    tf = copy_struct(sc["tf"])
    tf.n_entries = 1
    assert moments(P, ctx, sc, tf=tf) == 1 and "entries" in err(P, ctx)
    tf = copy_struct(sc["tf"])
    tf.s_max = tf.s_min
    assert moments(P, ctx, sc, tf=tf) == 1 and "domain" in err(P, ctx)
    tf = copy_struct(sc["tf"])
    tf.rgba = None
    assert moments(P, ctx, sc, tf=tf) == 1 and "NULL" in err(P, ctx)


def resolve(P, ctx, sc, mb=None, flags=None, rgba=None, moments_buf=None):
    flags = P.APC_FINALIZE if flags is None else flags
    mom = ptr(sc["out"]["mom"]) if moments_buf is None else moments_buf
    out = ptr(sc["out"]["rgba"]) if rgba is None else rgba
    return P.lib().apc_resolve_pass(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), C.byref(mb or sc["mb"]),
                                    mom, ptr(sc["subs"]), 3, out, flags, None)


def test_resolve_pass_statuses(P, ctx, scene):
    sc = scene
    assert resolve(P, ctx, sc) == 4 and "nothing was launched" in err(P, ctx)
    assert resolve(P, ctx, sc, mb=P.make_mboit(5, 5e-5, np.zeros(5), 0.3)) == 1 and "m = 5" in err(P, ctx)
    assert resolve(P, ctx, sc, mb=P.make_mboit(8, 1.0, synth.default_bias(8), 0.3)) == 1 and "alpha" in err(P, ctx)
    assert resolve(P, ctx, sc, mb=P.make_mboit(8, 5e-5, synth.default_bias(8), 1.5)) == 1 and "eta" in err(P, ctx)
    misaligned = C.c_void_p(sc["out"]["rgba"].ctypes.data + 4)
    assert resolve(P, ctx, sc, rgba=misaligned) == 1 and "aligned" in err(P, ctx)
    odd = C.c_void_p(sc["out"]["f16"].ctypes.data + 1)
    assert resolve(P, ctx, sc, flags=P.APC_FINALIZE | P.APC_MOMENTS_F16, moments_buf=odd) == 1
    assert resolve(P, ctx, sc, flags=P.APC_MOMENTS_F16, moments_buf=ptr(sc["out"]["f16"])) == 4
    assert resolve(P, ctx, sc, flags=P.APC_KEEP_PIECES) == 1 and "unknown flags" in err(P, ctx)
    assert resolve(P, ctx, sc, rgba=C.c_void_p()) == 1 and "NULL" in err(P, ctx)
    # the allocation-free variant validates the same way
    L = P.lib()
    args = (ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]))
    ok = L.apc_resolve_pass_noalloc(*args, C.byref(sc["mb"]), ptr(sc["out"]["mom"]), ptr(sc["subs"]), 3,
                                    ptr(sc["out"]["rgba"]), P.APC_FINALIZE, None)
    assert ok == 4 and "apc_resolve_pass_noalloc" in err(P, ctx) and "nothing was launched" in err(P, ctx)
    bad = L.apc_resolve_pass_noalloc(*args, C.byref(P.make_mboit(5, 5e-5, np.zeros(5), 0.3)),
                                     ptr(sc["out"]["mom"]), ptr(sc["subs"]), 3, ptr(sc["out"]["rgba"]), 0, None)
    assert bad == 1 and "m = 5" in err(P, ctx)
    # stage two by pairs: a valid call reaches the device check; not with the FP16 moments; not allocation-free
    assert resolve(P, ctx, sc, flags=P.APC_FINALIZE | P.APC_BY_PAIR) == 4 and "nothing was launched" in err(P, ctx)
    assert resolve(P, ctx, sc, flags=P.APC_BY_PAIR | P.APC_MOMENTS_F16, moments_buf=ptr(sc["out"]["f16"])) == 1
    assert "FP32 moments" in err(P, ctx)
    by_pair = L.apc_resolve_pass_noalloc(*args, C.byref(sc["mb"]), ptr(sc["out"]["mom"]), ptr(sc["subs"]), 3,
                                         ptr(sc["out"]["rgba"]), P.APC_FINALIZE | P.APC_BY_PAIR, None)
    assert by_pair == 1 and "unknown flags" in err(P, ctx) and "apc_resolve_pass_noalloc" in err(P, ctx)


def test_sums_pack_and_settings_statuses(P, ctx, scene):
    sc = scene
    L = P.lib()
    ms, mg = ptr(sc["out"]["mom_sub"]), ptr(sc["out"]["mom"])
    assert L.apc_sum_moments(ctx, ms, 3, 8, 24, 32, ptr(sc["subs"]), mg, None) == 4
    assert L.apc_sum_moments(ctx, ms, 3, 5, 24, 32, None, mg, None) == 1
    assert L.apc_sum_moments(ctx, ms, 0, 8, 24, 32, None, mg, None) == 1
    assert L.apc_sum_moments(ctx, ms, 2, 8, 24, 32, ptr(np.array([1, 1], np.int32)), mg, None) == 1
    assert L.apc_sum_moments(ctx, None, 3, 8, 24, 32, None, mg, None) == 1
    f16 = ptr(sc["out"]["f16"])
    assert L.apc_pack_moments_f16(ctx, mg, 8, 24, 32, f16, None) == 4
    assert L.apc_pack_moments_f16(ctx, mg, 7, 24, 32, f16, None) == 1
    assert L.apc_pack_moments_f16(ctx, mg, 8, 24, 32, C.c_void_p(sc["out"]["f16"].ctypes.data + 1), None) == 1
    rgba = ptr(sc["out"]["rgba"])
    assert L.apc_sum_images(ctx, rgba, 1, 24, 32, None, mg, C.byref(sc["mb"]), rgba, None) == 4
    assert L.apc_sum_images(ctx, rgba, 0, 24, 32, None, mg, C.byref(sc["mb"]), rgba, None) == 1
    assert L.apc_segment_counts(ctx, ptr(sc["out"]["segs"]), 24, 32, None) == 1  # no stage one has run
    assert L.apc_set_tile_shape(ctx, 3) == 1 and "power of two" in err(P, ctx)
    assert L.apc_set_tile_shape(ctx, 16) == 0
    w, h = C.c_int32(), C.c_int32()
    assert L.apc_get_tile_shape(ctx, C.byref(w), C.byref(h)) == 0 and (w.value, h.value) == (16, 4)
    assert L.apc_set_workspace_limit(ctx, -1) == 1
    assert L.apc_set_workspace_limit(ctx, 1 << 30) == 0
    mode = C.c_int32(-5)
    assert L.apc_get_dispatch(ctx, C.byref(mode)) == 0 and mode.value == P.APC_DISPATCH_GRID
    assert L.apc_set_dispatch(ctx, 2) == 1 and "dispatch mode" in err(P, ctx)
    assert L.apc_set_dispatch(ctx, P.APC_DISPATCH_QUEUE) == 0  # a host-only context allocates nothing
    assert L.apc_get_dispatch(ctx, C.byref(mode)) == 0 and mode.value == P.APC_DISPATCH_QUEUE
    assert L.apc_get_dispatch(ctx, None) == 1
    n = C.c_int64(-1)
    args = (ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), 8)
    assert L.apc_moments_pass_tiles(*args, ptr(np.array([2, 0, 1], np.int32)), 3, None, None, 0, C.byref(n),
                                    None) == 1 and "ascending" in err(P, ctx)
    assert L.apc_moments_pass_tiles(*args, ptr(sc["subs"]), 3, None, None, 0, None, None) == 1
    assert L.apc_moments_pass_tiles(*args, ptr(sc["subs"]), 3, None, None, -1, C.byref(n), None) == 1
    assert L.apc_moments_pass_tiles(*args, ptr(sc["subs"]), 3, None, None, 5, C.byref(n), None) == 1
    assert L.apc_moments_pass_tiles(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), 5, ptr(sc["subs"]), 3,
                                    None, None, 0, C.byref(n), None) == 1
    assert L.apc_moments_pass_tiles(*args, ptr(sc["subs"]), 3, None, None, 0, C.byref(n), None) == 4
    assert n.value == -1  # nothing written by a call that failed
    assert L.apc_moments_pass_pairs(*args, ptr(np.array([2, 0, 1], np.int32)), 3, None, None, 0, C.byref(n),
                                    None) == 1 and "ascending" in err(P, ctx)
    assert L.apc_moments_pass_pairs(*args, ptr(sc["subs"]), 3, None, None, 5, C.byref(n), None) == 1
    assert L.apc_moments_pass_pairs(*args, ptr(sc["subs"]), 3, None, None, 0, C.byref(n), None) == 4
    assert "apc_moments_pass_pairs" in err(P, ctx) and n.value == -1
    tl, pb = ptr(sc["out"]["mom"]), ptr(np.zeros(4, np.int32))
    assert L.apc_sum_moment_tiles(ctx, tl, pb, 4, 3, 8, 24, 32, 3, mg, None) == 1 and "power of two" in err(P, ctx)
    assert L.apc_sum_moment_tiles(ctx, tl, pb, 10 ** 6, 3, 8, 24, 32, 8, mg, None) == 1  # more pairs than bins
    assert L.apc_sum_moment_tiles(ctx, None, None, 4, 3, 8, 24, 32, 8, mg, None) == 1
    assert L.apc_sum_moment_tiles(ctx, tl, pb, 4, 3, 8, 24, 32, 8, None, None) == 1
    assert L.apc_sum_moment_tiles(ctx, tl, pb, 4, 3, 8, 24, 32, 8, mg, None) == 4
    best = C.c_int32()
    assert L.apc_autotune_tile_shape(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), C.byref(sc["mb"]),
                                     ptr(sc["subs"]), 3, mg, rgba, 0, C.byref(best), None, None) == 1
    assert L.apc_autotune_tile_shape(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), C.byref(sc["mb"]),
                                     ptr(sc["subs"]), 3, mg, rgba, 1, C.byref(best), None, None) == 4
    mode = C.c_int32()
    assert L.apc_autotune_launch(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), C.byref(sc["mb"]),
                                 ptr(sc["subs"]), 3, mg, rgba, 0, C.byref(best), C.byref(mode), None, None) == 1
    assert L.apc_autotune_launch(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), None,
                                 ptr(sc["subs"]), 3, mg, rgba, 1, C.byref(best), C.byref(mode), None, None) == 1
    assert L.apc_autotune_launch(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), C.byref(sc["mb"]),
                                 ptr(sc["subs"]), 3, mg, rgba, 1, C.byref(best), C.byref(mode), None, None) == 4
    cnt = P.Counters()
    assert L.apc_get_counters(ctx, C.byref(cnt), 0) == 4
    g = C.c_void_p()
    assert L.apc_frame_graph_create(ctx, sc["mesh"], C.byref(sc["view"]), C.byref(sc["tf"]), C.byref(sc["mb"]),
                                    ptr(sc["subs"]), 3, None, mg, rgba, P.APC_MOMENTS_GLOBAL, C.byref(g)) == 4
    assert g.value is None


def test_null_context_and_errors_are_per_call(P):
    L = P.lib()
    cnt = P.Counters()
    assert L.apc_get_counters(None, C.byref(cnt), 0) == 1
    assert "context is NULL" in L.apc_last_error(None).decode()
    assert L.apc_create(-1, None) == 1
    assert L.apc_destroy(None) == 0
