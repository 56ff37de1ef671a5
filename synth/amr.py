"""Adaptive (octree) conforming tetrahedral meshes for the batching workload.

A base grid of B^3 cubes is refined, level by level up to `max_level`, where the
Gaussian-sum field changes fast across a cell (|grad f| * h above a threshold),
then 2:1 balanced over all 26 neighbours (no two touching leaves differ by more
than one level, so an edge or face of a leaf is split at most once).  Each leaf
is cut into tets by cone decomposition: every face of the leaf is triangulated
to match its neighbours, and each triangle is joined to the leaf's centre.

Face triangulation (the same rule on both sides of every face, so the mesh is
conforming):
  * a face whose centre is a corner of a finer leaf (split face), or with any
    edge whose midpoint is a corner of a finer leaf, gets a vertex at its
    centre and is fanned around it over its boundary polygon (corners and the
    edge midpoints that exist);
  * any other face of a leaf of level >= 1 is cut by the diagonal through its
    corner nearest the centre of the leaf's parent cube (that corner is the
    centre of the coarser neighbour's split face, or the shared parent centre
    between siblings, or the same parent-face centre seen from a same-level
    neighbour);
  * any other face of a level-0 leaf (its neighbour is then level 0 too) is cut
    by the diagonal through its corner of smallest key.
Points are kept on the integer lattice of spacing 1 / (2 B 2^max_level), so
keys identify shared vertices exactly.  The module holds no arithmetic of the
rendering method.
"""
from __future__ import annotations

import numpy as np

from scipy.ndimage import maximum_filter


def _grad_norm(p: np.ndarray, centres: np.ndarray, sigma: float) -> np.ndarray:
    g = np.zeros_like(p)
    for c in centres:
        d = p - c
        w = np.exp(-np.sum(d * d, axis=1) / (2.0 * sigma * sigma)) / (sigma * sigma)
        g -= d * w[:, None]
    return np.sqrt(np.sum(g * g, axis=1))


def refine(base: int, max_level: int, centres: np.ndarray, threshold: float, sigma: float = 0.15) -> list:
    """Leaf grids per level (boolean [n_L]^3, n_L = base * 2^L) after refinement and 2:1 balance."""
    leaves = [np.ones((base,) * 3, dtype=bool)]
    for L in range(max_level):
        n = base << L
        idx = np.argwhere(leaves[L])
        pc = (idx[:, ::-1] + 0.5) / n  # (x, y, z) of the cell centres; arrays are indexed [k, j, i]
        split = _grad_norm(pc, centres, sigma) * (1.0 / n) > threshold
        s = idx[split]
        leaves[L][s[:, 0], s[:, 1], s[:, 2]] = False
        child = np.zeros((2 * n,) * 3, dtype=bool)
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    child[2 * s[:, 0] + dk, 2 * s[:, 1] + dj, 2 * s[:, 2] + di] = True
        leaves.append(child)
    # 2:1 balance over face, edge and corner neighbours
    N = base << max_level
    while True:
        levmap = np.zeros((N,) * 3, dtype=np.int8)
        for L, g in enumerate(leaves):
            r = 1 << (max_level - L)
            levmap = np.maximum(levmap, np.kron(g, np.ones((r, r, r), dtype=bool)).astype(np.int8) * L)
        changed = False
        for L in range(max_level - 1):
            n = base << L
            r = 1 << (max_level - L)
            lev = levmap.reshape(n, r, n, r, n, r).max(axis=(1, 3, 5))
            nb = maximum_filter(lev, size=3, mode="constant", cval=0)
            bad = leaves[L] & (nb >= L + 2)
            if bad.any():
                s = np.argwhere(bad)
                leaves[L][bad] = False
                for dk in (0, 1):
                    for dj in (0, 1):
                        for di in (0, 1):
                            leaves[L + 1][2 * s[:, 0] + dk, 2 * s[:, 1] + dj, 2 * s[:, 2] + di] = True
                changed = True
        if not changed:
            return leaves


def _leaf_arrays(leaves: list, max_level: int):
    """Per leaf: level, integer origin (x, y, z) and size on the lattice of spacing 1/(2N)."""
    lv, org, size = [], [], []
    for L, g in enumerate(leaves):
        idx = np.argwhere(g)[:, ::-1]  # (i, j, k)
        s = 2 << (max_level - L)
        lv.append(np.full(len(idx), L, dtype=np.int64))
        org.append(idx.astype(np.int64) * s)
        size.append(np.full(len(idx), s, dtype=np.int64))
    return np.concatenate(lv), np.concatenate(org), np.concatenate(size)


def _morton(x: np.ndarray) -> np.ndarray:
    from . import _part1by2
    return _part1by2(x[:, 0]) | (_part1by2(x[:, 1]) << np.uint64(1)) | (_part1by2(x[:, 2]) << np.uint64(2))


# the 6 faces of a cube: (normal axis, side); the face's two in-plane axes (u, v) in cyclic order
_FACES = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]


class _Leaves:
    """Balanced leaves in Morton order of their anchors, with the face data both the tet count and the cone
    decomposition need."""

    def __init__(self, leaves: list, max_level: int, base: int):
        N = base << max_level
        self.M = 2 * N + 1
        lv, org, size = _leaf_arrays(leaves, max_level)
        order = np.argsort(_morton(org), kind="stable")
        self.lv, self.org, self.size = lv[order], org[order], size[order]
        self.n = len(self.lv)
        off = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)
        corners = self.org[:, None, :] + off[None] * self.size[:, None, None]
        self.is_leaf_corner = np.zeros(self.M ** 3, dtype=bool)  # dense lattice: O(1) membership
        self.is_leaf_corner[self.key(corners).ravel()] = True
        self.centre = self.org + (self.size // 2)[:, None]
        s2 = 2 * self.size[:, None]
        self.parent_centre = np.where(self.lv[:, None] > 0, (self.org // s2) * s2 + self.size[:, None], -1)

    def key(self, p):
        return p[..., 0] + self.M * (p[..., 1] + self.M * p[..., 2])

    def is_corner(self, p):
        return self.is_leaf_corner[self.key(p)]

    def face_status(self, axis: int, side: int):
        """Which of the boundary polygon's vertices (corner, edge midpoint, corner, ...: (u, v) = (0,0)
        (1/2,0) (1,0) (1,1/2) (1,1) (1/2,1) (0,1) (0,1/2)) are used [n, 8], and whether the face is fanned
        around its centre [n].  Keys are linear in the point, so each is an offset from the face's origin."""
        ua, va = (axis + 1) % 3, (axis + 2) % 3
        stride = (1, self.M, self.M * self.M)
        k0 = self.key(self.org) + side * self.size * stride[axis]
        hu, hv = (self.size // 2) * stride[ua], (self.size // 2) * stride[va]
        mids = np.stack([self.is_leaf_corner[k0 + hu], self.is_leaf_corner[k0 + 2 * hu + hv],
                         self.is_leaf_corner[k0 + hu + 2 * hv], self.is_leaf_corner[k0 + hv]], axis=1)
        split = self.is_leaf_corner[k0 + hu + hv]
        present = np.ones((self.n, 8), dtype=bool)
        present[:, [1, 3, 5, 7]] = mids | split[:, None]
        return present, split | mids.any(axis=1)

    def face(self, axis: int, side: int):
        """Boundary polygon [n, 8, 3] in the order of face_status, the face centre, and face_status."""
        ua, va = (axis + 1) % 3, (axis + 2) % 3
        base_pt = self.org.copy()
        base_pt[:, axis] += self.size * side
        U = np.zeros((self.n, 3), dtype=np.int64)
        V = np.zeros((self.n, 3), dtype=np.int64)
        U[:, ua] = self.size
        V[:, va] = self.size
        uv = [(0, 0), (1, 0), (2, 0), (2, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
        poly = np.stack([base_pt + (U * a + V * b) // 2 for a, b in uv], axis=1)
        fc = base_pt + (U + V) // 2
        return (poly, fc) + self.face_status(axis, side)

    def n_tets(self) -> int:
        t = 0
        for axis, side in _FACES:
            present, fan = self.face_status(axis, side)
            t += int(np.where(fan, present.sum(axis=1), 2).sum())
        return t


def amr_tets(leaves: list, max_level: int, base: int):
    """Cone decomposition of the balanced leaves.  Returns (points [P,3] int64 lattice coordinates,
    tets [T,4] int64 point ids, leaf of each tet in Morton order, number of leaves)."""
    lf = _Leaves(leaves, max_level, base)
    tet_pts, tet_leaf = [], []
    for axis, side in _FACES:
        poly, fc, present, fan = lf.face(axis, side)
        # fanned faces: a triangle (face centre, vertex, next used vertex) per used polygon vertex
        for t in range(8):
            nxt = (t + 1) % 8
            sel = np.nonzero(fan & present[:, t])[0]
            if len(sel):
                nxt_pt = np.where(present[sel, nxt][:, None], poly[sel, nxt], poly[sel, (t + 2) % 8])
                tet_pts.append(np.stack([fc[sel], poly[sel, t], nxt_pt, lf.centre[sel]], axis=1))
                tet_leaf.append(sel)
        # the other faces: two triangles split by the diagonal through corner q of c0..c3
        cs = poly[:, [0, 2, 4, 6]]
        q_par = np.argmin(np.abs(cs - lf.parent_centre[:, None, :]).sum(axis=2), axis=1)
        q_key = np.argmin(lf.key(cs), axis=1)
        q = np.where(lf.lv > 0, q_par, q_key)
        sel = np.nonzero(~fan)[0]
        if len(sel):
            qq, c, r = q[sel], cs[sel], np.arange(len(sel))
            a0, a1, a2, a3 = c[r, qq], c[r, (qq + 1) % 4], c[r, (qq + 2) % 4], c[r, (qq + 3) % 4]
            tet_pts.append(np.stack([a0, a1, a2, lf.centre[sel]], axis=1))
            tet_leaf.append(sel)
            tet_pts.append(np.stack([a0, a2, a3, lf.centre[sel]], axis=1))
            tet_leaf.append(sel)
    pts = np.concatenate(tet_pts)
    del tet_pts
    tl = np.concatenate(tet_leaf)
    o = np.argsort(tl, kind="stable")  # tets grouped by leaf, leaves in Morton order
    pts, tl = pts[o], tl[o]
    k = lf.key(pts).ravel()
    del pts
    used = np.zeros(lf.M ** 3, dtype=bool)
    used[k] = True
    uk = np.flatnonzero(used)  # point ids in key order
    pid = np.zeros(lf.M ** 3, dtype=np.int64)
    pid[uk] = np.arange(len(uk))
    M = lf.M
    points = np.stack([uk % M, (uk // M) % M, uk // (M * M)], axis=1)
    return points, pid[k].reshape(-1, 4), tl, lf.n


def find_threshold(base: int, max_level: int, centres: np.ndarray, t_lo: int, t_hi: int, iters: int = 30):
    """Refinement threshold whose mesh has between t_lo and t_hi tets; returns (threshold, leaves).

    The tet count falls as the threshold grows.  Above the largest |grad f| * h over the base cells nothing is
    refined; the search steps down from there by factors of 8 until the count passes t_hi, then narrows that
    bracket by false position on (log threshold, log count), halving the retained end's weight when the same
    end is kept twice (the Illinois rule), which is deterministic for a given field."""
    def count(x):
        lv = refine(base, max_level, centres, float(np.exp(x)))
        return np.log(_Leaves(lv, max_level, base).n_tets()), lv

    g = np.arange(base) + 0.5
    pc = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3) / base
    target = 0.5 * (np.log(t_lo) + np.log(t_hi))
    xa = np.log(_grad_norm(pc, centres, 0.15).max() / base * 1.001)
    fa, lv = count(xa)
    xb, fb = xa, fa
    while fb <= np.log(t_hi):
        if np.log(t_lo) <= fb:
            return float(np.exp(xb)), lv
        xa, fa = xb, fb
        xb -= np.log(8.0)
        fb, lv = count(xb)
    fa, fb = fa - target, fb - target  # fa < 0 < fb
    side = 0
    for _ in range(iters):
        x = (xa * fb - xb * fa) / (fb - fa)
        f, lv = count(x)
        if abs(f - target) <= 0.5 * (np.log(t_hi) - np.log(t_lo)):
            return float(np.exp(x)), lv
        f -= target
        if f < 0:
            xa, fa = x, f
            if side == -1:
                fb *= 0.5
            side = -1
        else:
            xb, fb = x, f
            if side == 1:
                fa *= 0.5
            side = 1
    raise ValueError("no threshold gives a tet count in [%d, %d]" % (t_lo, t_hi))


def amr_mesh(base: int, max_level: int, n_sub: int, seed: int, threshold: float | None = None,
             tet_range: tuple | None = None, n_gauss: int = 16, chunk_weights: np.ndarray | None = None):
    """Conforming adaptive tet mesh on [0,1]^3 with the Gaussian-sum scalar, split into n_sub chunks of
    whole leaves in Morton order (tet counts in proportion to `chunk_weights`, else equal).  The refinement
    threshold is `threshold`, or is found by bisection so that the tet count falls in `tet_range`.
    Returns (mesh, leaf grids per level, threshold)."""
    from . import Mesh, gaussian_field
    rng = np.random.default_rng(seed + 1)
    centres = rng.uniform(0.2, 0.8, size=(n_gauss, 3))
    if threshold is None:
        threshold, leaves = find_threshold(base, max_level, centres, *tet_range)
    else:
        leaves = refine(base, max_level, centres, threshold)
    points, tets, tet_leaf, n_leaf = amr_tets(leaves, max_level, base)
    N = base << max_level
    xyz = (points.astype(np.float64) / (2.0 * N)).astype(np.float32)
    # positive orientation
    p = xyz.astype(np.float64)[tets]
    vol = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    neg = vol < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    scalar = gaussian_field(xyz, centres)
    # chunks of whole leaves, balanced by tet count
    tets_per_leaf = np.bincount(tet_leaf, minlength=n_leaf)
    cum = np.concatenate([[0], np.cumsum(tets_per_leaf)])
    w = np.ones(n_sub) if chunk_weights is None else np.asarray(chunk_weights, dtype=np.float64)
    targets = np.concatenate([[0.0], np.cumsum(w)]) / w.sum() * cum[-1]
    bounds = np.searchsorted(cum, targets[1:-1])  # leaf index where each chunk ends
    leaf_sub = np.searchsorted(bounds, np.arange(n_leaf), side="right").astype(np.int32)
    if len(np.unique(leaf_sub)) != n_sub:
        raise ValueError("empty chunk")
    return (Mesh(xyz=xyz, scalar=scalar, tets=tets.astype(np.int32), tet_sub=leaf_sub[tet_leaf], n_sub=n_sub),
            leaves, threshold)
