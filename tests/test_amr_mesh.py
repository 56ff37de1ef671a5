"""The adaptive mesh generator of the batching workload (CPU): the cone decomposition tiles the unit cube
with positively oriented tets that meet face to face, the octree is 2:1 balanced, unrefined leaves satisfy
the refinement criterion, the threshold search lands in its tet-count window, and the chunks are runs of
whole leaves in Morton order with tet counts in the asked ratio."""
import numpy as np
import pytest

import synth
from synth import amr


def _faces(tets):
    f = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 3, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 1]]])
    return f  # outward-oriented faces of positively oriented tets


def _check_tiling(mesh):
    xyz = mesh.xyz.astype(np.float64)
    vol6 = synth.signed_volumes(mesh.xyz, mesh.tets)
    assert vol6.min() > 0
    assert abs(vol6.sum() / 6.0 - 1.0) < 1e-9
    f = _faces(mesh.tets)
    key = np.sort(f, axis=1)
    u, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    assert set(np.unique(cnt)) <= {1, 2}
    # an interior face is seen from its two tets with opposite orientations: their outward normals cancel
    n = np.cross(xyz[f[:, 1]] - xyz[f[:, 0]], xyz[f[:, 2]] - xyz[f[:, 0]])
    acc = np.zeros((len(u), 3))
    np.add.at(acc, inv.ravel(), n)
    interior = cnt == 2
    assert np.abs(acc[interior]).max() < 1e-12
    # boundary faces lie in the cube's surface and their outward areas give the six unit faces
    bx = xyz[u[~interior]]
    on_plane = np.zeros(len(bx), dtype=bool)
    for a in range(3):
        for v in (0.0, 1.0):
            on_plane |= np.all(bx[:, :, a] == v, axis=1)
    assert on_plane.all()
    area = acc[~interior]
    for a in range(3):
        assert abs(area[area[:, a] > 0, a].sum() / 2.0 - 1.0) < 1e-12
        assert abs(area[area[:, a] < 0, a].sum() / 2.0 + 1.0) < 1e-12
    return int(interior.sum()), int((~interior).sum())


@pytest.mark.parametrize("base,levels,threshold", [(8, 3, 0.3), (8, 3, 0.6), (4, 3, 0.05), (6, 2, 0.08)])
def test_cone_decomposition_tiles_the_cube_face_to_face(base, levels, threshold):
    mesh, leaves, _ = amr.amr_mesh(base, levels, 4, seed=11, threshold=threshold)
    _check_tiling(mesh)
    lf = amr._Leaves(leaves, levels, base)
    assert lf.n_tets() == mesh.n_tets
    # every tet lies in its own leaf's cube, and every leaf has at least its 12 unfanned-face tets
    points, tets, tet_leaf, n_leaf = amr.amr_tets(leaves, levels, base)
    p = points[tets]
    assert (p >= lf.org[tet_leaf][:, None, :]).all()
    assert (p <= (lf.org + lf.size[:, None])[tet_leaf][:, None, :]).all()
    assert np.bincount(tet_leaf, minlength=n_leaf).min() >= 12


def test_mixed_levels_including_unrefined_base_cells():
    _, leaves, _ = amr.amr_mesh(8, 3, 4, seed=11, threshold=0.3)
    counts = [int(g.sum()) for g in leaves]
    assert all(c > 0 for c in counts), counts  # all four levels are present, so every face rule is exercised


def test_octree_is_two_to_one_balanced_and_unrefined_leaves_pass_the_criterion():
    rng = np.random.default_rng(12)
    centres = rng.uniform(0.2, 0.8, size=(16, 3))
    base, levels, thr = 8, 3, 0.3
    leaves = amr.refine(base, levels, centres, thr)
    N = base << levels
    lev = np.full((N,) * 3, -1, dtype=np.int8)
    for L, g in enumerate(leaves):
        r = 1 << (levels - L)
        blk = np.kron(g, np.ones((r, r, r), dtype=bool))
        assert not (blk & (lev >= 0)).any()  # leaves do not overlap
        lev[blk] = L
    assert (lev >= 0).all()  # and cover the cube
    # touching finest cells (26 neighbours) belong to leaves whose levels differ by at most one
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                a = lev[max(dk, 0):N + min(dk, 0), max(dj, 0):N + min(dj, 0), max(di, 0):N + min(di, 0)]
                b = lev[max(-dk, 0):N + min(-dk, 0), max(-dj, 0):N + min(-dj, 0), max(-di, 0):N + min(-di, 0)]
                assert np.abs(a.astype(int) - b).max() <= 1
    # a leaf above the finest level was not marked for refinement: |grad f| h <= threshold at its centre,
    # with the gradient of the Gaussian sum written out here
    for L, g in enumerate(leaves[:-1]):
        n = base << L
        c = (np.argwhere(g)[:, ::-1] + 0.5) / n
        grad = np.zeros_like(c)
        for q in centres:
            d = c - q
            grad += -d / 0.15 ** 2 * np.exp(-(d * d).sum(axis=1) / (2 * 0.15 ** 2))[:, None]
        assert (np.linalg.norm(grad, axis=1) / n <= thr).all()


def test_threshold_search_lands_in_the_window():
    for lo, hi in [(400_000, 440_000), (1_000_000, 1_100_000)]:
        mesh, _, thr = amr.amr_mesh(8, 3, 4, seed=3, tet_range=(lo, hi))
        assert lo <= mesh.n_tets <= hi
        again, _, _ = amr.amr_mesh(8, 3, 4, seed=3, threshold=thr)
        assert again.n_tets == mesh.n_tets


def test_chunks_are_morton_runs_of_whole_leaves_with_weighted_tet_counts():
    w = synth.uneven_weights(6, 12.0, seed=5)
    mesh, leaves, _ = amr.amr_mesh(8, 3, 6, seed=11, threshold=0.3, chunk_weights=w)
    sub = mesh.tet_sub
    assert (np.diff(sub) != 0).sum() == 5  # tets come leaf by leaf, chunk by chunk
    cnt = np.bincount(sub, minlength=6)
    assert np.abs(cnt / cnt.sum() - w / w.sum()).max() < 48.0 / cnt.sum() + 1e-12  # one leaf holds at most 48 tets
    # the leaves' anchors come in Morton order
    lf = amr._Leaves(leaves, 3, 8)
    code = amr._morton(lf.org)
    assert (np.diff(code.astype(np.int64)) > 0).all()
