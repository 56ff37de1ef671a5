"""Seeded synthetic inputs for the APC hot path.

This module builds the inputs that both the FP64 oracle and the HIP library
consume: jittered-grid tetrahedral meshes (Kuhn split), Gaussian-sum vertex
scalars, Morton-order subdomain partitions, 256-entry transfer-function tables
and camera frames.  It holds none of the rendering method's arithmetic (no ray
setup, no depth range, no sampling, no moments, no reconstruction): every
number it produces is an input, drawn from numpy's seeded PCG64 generator.

Workloads (sizes follow the paper's evaluation set-up of Section 5 scaled to
one GPU; the paper's FUN3D and Exajet meshes are not available, these stand in):

  tiny      16^3 cubes x 6 = 24,576 tets, 4 subdomains, orthographic 128^2, m=4
  medium    64^3 cubes x 6 = 1,572,864 tets, 16 subdomains, perspective 1024^2, m=6
  large     256^3 cubes x 6 = 100,663,296 tets, 72 subdomains, perspective 2560^2, m=8
  batching  adaptive mesh (32^3 base refined 0-3 levels, 19M-21M tets, synth.amr), 72 subdomains of
            tet-count ratio 12, perspective 2560^2, m=8
  slabs     interleaved z-slabs (each subdomain owns 4 separated slabs)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Mesh", "Scene", "jittered_grid", "kuhn_tets", "morton_order", "partition_chunks",
    "partition_slabs", "gaussian_field", "make_tf", "ortho_view_z", "perspective_view",
    "sphere_eye", "default_bias", "scene_tiny", "scene_medium", "scene_large", "scene",
    "sandwich_scene", "scene_batching", "scene_amr_small", "scene_slabs", "orbit_view",
]


@dataclasses.dataclass
class Mesh:
    xyz: np.ndarray          # [V,3] float32 vertex positions
    scalar: np.ndarray       # [V]   float32 vertex scalars
    tets: np.ndarray         # [T,4] int32 vertex ids, positively oriented
    tet_sub: np.ndarray      # [T]   int32 subdomain id of each tet
    n_sub: int

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


@dataclasses.dataclass
class Scene:
    name: str
    mesh: Mesh
    tf: np.ndarray           # [256,4] float32 RGBA table
    s_min: float             # transfer-function domain (global min/max of vertex scalars)
    s_max: float
    kappa: float             # extinction per unit length per unit table alpha
    absorbance_max: float    # per-piece cap on optical depth
    view: dict               # camera frame, see ortho_view_z / perspective_view
    step: float              # world-space lattice spacing
    m: int                   # number of power moments (even)
    alpha: float             # mixing strength of the bias vector
    bias: np.ndarray         # [m] float64 bias moments b*_1..b*_m
    eta: float               # overestimation weight of the node at the sample depth
    renormalize: int = 1


# ----------------------------------------------------------------------------- mesh

def jittered_grid(n: int, seed: int, jitter: float = 0.15) -> np.ndarray:
    """(n+1)^3 vertices of the unit-cube grid, vertex id = i + (n+1)*(j + (n+1)*k).

    Interior coordinates move by U[-jitter*h, jitter*h]; a coordinate that lies on
    the domain boundary does not move, so boundary vertices slide only within
    their boundary face and the domain stays exactly [0,1]^3.
    """
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    g = np.arange(n + 1, dtype=np.float64) * h
    k, j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    idx = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    pos = g[idx]
    jit = rng.uniform(-jitter * h, jitter * h, size=pos.shape)
    on_boundary = (idx == 0) | (idx == n)
    jit[on_boundary] = 0.0
    return (pos + jit).astype(np.float32)


def _part1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_order(n: int) -> np.ndarray:
    """Cube ids c = i + n*(j + n*k) sorted by their Morton (z-order) code."""
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    code = _part1by2(i.ravel()) | (_part1by2(j.ravel()) << np.uint64(1)) | (_part1by2(k.ravel()) << np.uint64(2))
    return np.argsort(code, kind="stable").astype(np.int64)


# the six monotone lattice paths 000 -> 111 of the Kuhn (Freudenthal) split; the
# odd permutations get their middle vertices swapped so every tet is positive
_KUHN_PATHS = [(0, 1, 2), (1, 2, 0), (2, 0, 1), (1, 0, 2), (0, 2, 1), (2, 1, 0)]


def kuhn_tets(n: int, cube_order: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Split every cube into 6 tets sharing the main diagonal.

    Returns (tets [6*n^3, 4] int32, cube id of each tet).  Tets are emitted cube
    by cube in `cube_order` (default: Morton order).  All cubes use the same
    diagonal, so the triangulation is conforming.
    """
    if cube_order is None:
        cube_order = morton_order(n)
    ci = cube_order % n
    cj = (cube_order // n) % n
    ck = cube_order // (n * n)
    n1 = n + 1

    def vid(di, dj, dk):
        return (ci + di) + n1 * ((cj + dj) + n1 * (ck + dk))

    out = np.empty((cube_order.size, 6, 4), dtype=np.int64)
    for t, path in enumerate(_KUHN_PATHS):
        step = [0, 0, 0]
        verts = [vid(0, 0, 0)]
        for axis in path[:2]:
            step[axis] += 1
            verts.append(vid(*step))
        verts.append(vid(1, 1, 1))
        if t >= 3:  # odd permutation
            verts[1], verts[2] = verts[2], verts[1]
        out[:, t, :] = np.stack(verts, axis=1)
    tets = out.reshape(-1, 4).astype(np.int32)
    cube_of_tet = np.repeat(cube_order, 6)
    return tets, cube_of_tet


def signed_volumes(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Six times the signed volume of each tet (float64), for generator self-checks."""
    p = xyz.astype(np.float64)[tets]
    a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def partition_chunks(n_cells: int, n_sub: int, seed: int | None, jagged: float = 0.5,
                     weights: np.ndarray | None = None) -> np.ndarray:
    """Chunk boundaries [n_sub+1] of contiguous runs of Morton-ordered cells.

    Chunk weights are `weights` when given, else 1 + jagged*U(-1,1) (seeded)
    or equal when seed is None.
    """
    if weights is not None:
        w = np.asarray(weights, dtype=np.float64)
    elif seed is None:
        w = np.ones(n_sub)
    else:
        w = 1.0 + jagged * np.random.default_rng(seed).uniform(-1.0, 1.0, size=n_sub)
    cum = np.concatenate([[0.0], np.cumsum(w)]) / w.sum() * n_cells
    b = np.rint(cum).astype(np.int64)
    b[0], b[-1] = 0, n_cells
    if np.any(np.diff(b) <= 0):
        raise ValueError("empty chunk")
    return b


def partition_slabs(n: int, n_sub: int, slabs_per_sub: int) -> np.ndarray:
    """Subdomain of each cube (id i + n*(j + n*k)) for interleaved z-slabs.

    The z range is cut into n_sub*slabs_per_sub slabs; slab q belongs to
    subdomain q % n_sub, so every subdomain owns several separated slabs.
    """
    n_slabs = n_sub * slabs_per_sub
    if n_slabs > n:
        raise ValueError("more slabs than cube layers")
    k = np.arange(n * n * n) // (n * n)
    return (((k * n_slabs) // n) % n_sub).astype(np.int32)


def gaussian_field(xyz: np.ndarray, centres: np.ndarray, sigma: float = 0.15) -> np.ndarray:
    """Sum of isotropic unit-amplitude Gaussians evaluated at the vertices (float32)."""
    p = xyz.astype(np.float64)
    f = np.zeros(p.shape[0])
    for c in centres:
        f += np.exp(-np.sum((p - c) ** 2, axis=1) / (2.0 * sigma * sigma))
    return f.astype(np.float32)


def make_tf(seed: int, n_entries: int = 256, n_ctrl: int = 4) -> np.ndarray:
    """Piecewise-linear RGBA table through n_ctrl seeded control points.

    Control positions are sorted U(0,1), control RGBA are U(0,1)^4; the table
    is held constant outside the first and last control point.
    """
    rng = np.random.default_rng(seed)
    u = np.sort(rng.uniform(0.0, 1.0, size=n_ctrl))
    rgba = rng.uniform(0.0, 1.0, size=(n_ctrl, 4))
    x = np.arange(n_entries) / (n_entries - 1)
    tab = np.stack([np.interp(x, u, rgba[:, c]) for c in range(4)], axis=1)
    return tab.astype(np.float32)


# ----------------------------------------------------------------------------- cameras

def ortho_view_z(width: int, height: int) -> dict:
    """Orthographic view along +z over the window [0,1]^2, image plane z = -1.

    Pixel (row i, column j) has origin (j+1/2)/W, (i+1/2)/H, -1 and direction +z.
    """
    return dict(width=width, height=height, projection=0,
                eye=(0.0, 0.0, -1.0), dir=(0.0, 0.0, 1.0),
                right=(1.0 / width, 0.0, 0.0), down=(0.0, 1.0 / height, 0.0))


def perspective_view(eye, target, width: int, height: int, fovy_deg: float = 45.0, up=(0.0, 0.0, 1.0)) -> dict:
    """Pinhole camera frame.  The un-normalised direction of pixel (i, j) is
    dir + (j + 1/2 - W/2)*right + (i + 1/2 - H/2)*down."""
    e = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - e
    f /= np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    if abs(float(f @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    tan_h = math.tan(math.radians(fovy_deg) / 2.0)
    right = r * (2.0 * tan_h / width)
    down = -u * (2.0 * tan_h / height)
    return dict(width=width, height=height, projection=1, eye=tuple(e), dir=tuple(f),
                right=tuple(right), down=tuple(down))


def sphere_eye(seed: int, radius: float = 2.0, centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    v = np.random.default_rng(seed).normal(size=3)
    v /= np.linalg.norm(v)
    return np.asarray(centre) + radius * v


def default_bias(m: int) -> np.ndarray:
    """b*_j for j = 1..m: moments of the uniform distribution on [-1, 1]."""
    j = np.arange(1, m + 1)
    return np.where(j % 2 == 0, 1.0 / (j + 1.0), 0.0)


# ----------------------------------------------------------------------------- workloads

def grid_mesh(n: int, n_sub: int, seed: int, n_gauss: int, jagged_seed: int | None, jitter: float = 0.15,
              sub_of_cube: np.ndarray | None = None, chunk_weights: np.ndarray | None = None) -> Mesh:
    rng = np.random.default_rng(seed + 1)
    xyz = jittered_grid(n, seed, jitter)
    order = morton_order(n)
    tets, cube_of_tet = kuhn_tets(n, order)
    centres = rng.uniform(0.2, 0.8, size=(n_gauss, 3))
    scalar = gaussian_field(xyz, centres)
    if sub_of_cube is None:
        bounds = partition_chunks(n ** 3, n_sub, jagged_seed, weights=chunk_weights)
        rank = np.empty(n ** 3, dtype=np.int64)
        rank[order] = np.arange(n ** 3)
        sub_of_cube = (np.searchsorted(bounds, rank, side="right") - 1).astype(np.int32)
    tet_sub = sub_of_cube[cube_of_tet].astype(np.int32)
    return Mesh(xyz=xyz, scalar=scalar, tets=tets, tet_sub=tet_sub, n_sub=n_sub)


def _scene(name, mesh, view, n, m, tf_seed, kappa=4.0) -> Scene:
    return Scene(name=name, mesh=mesh, tf=make_tf(tf_seed),
                 s_min=float(mesh.scalar.min()), s_max=float(mesh.scalar.max()),
                 kappa=kappa, absorbance_max=10.0, view=view, step=0.25 / n, m=m,
                 alpha=5e-5, bias=default_bias(m), eta=0.3)


def scene_tiny(seed: int = 1) -> Scene:
    """16^3 x 6 tets, 4 jagged Morton subdomains, orthographic 128^2 along +z, m = 4."""
    n = 16
    mesh = grid_mesh(n, 4, seed, n_gauss=4, jagged_seed=seed + 7)
    return _scene("tiny", mesh, ortho_view_z(128, 128), n, 4, tf_seed=seed + 11)


def scene_medium(seed: int = 2, size: int = 1024) -> Scene:
    """64^3 x 6 tets, 16 jagged Morton subdomains, perspective 1024^2 (45 deg), m = 6."""
    n = 64
    mesh = grid_mesh(n, 16, seed, n_gauss=16, jagged_seed=seed + 7)
    view = perspective_view(sphere_eye(seed + 3), (0.5, 0.5, 0.5), size, size)
    return _scene("medium", mesh, view, n, 6, tf_seed=seed + 11)


def orbit_view(seed: int, camera: int, size: int) -> dict:
    """Camera `camera` of a workload's seeded orbit: a perspective view from a point of the radius-2 sphere
    around the cube's centre, looking at the centre (the analogue of the paper's camera paths)."""
    return perspective_view(sphere_eye(seed + 3 + 97 * camera), (0.5, 0.5, 0.5), size, size)


LARGE_SEED, BATCHING_SEED = 4, 7


def scene_large(seed: int = LARGE_SEED, size: int = 2560, camera: int = 0, n: int = 256) -> Scene:
    """256^3 x 6 = 100,663,296 tets, 72 equal Morton chunks, perspective 2560^2, m = 8."""
    mesh = grid_mesh(n, 72, seed, n_gauss=16, jagged_seed=None)
    return _scene("large", mesh, orbit_view(seed, camera, size), n, 8, tf_seed=seed + 11)


def sandwich_scene(n: int = 24, n_sub: int = 3, slabs_per_sub: int = 2, m: int = 4, seed: int = 5,
                   size: int = 96) -> Scene:
    """Interleaved z-slabs (each subdomain owns separated slabs), viewed along +z."""
    sub = partition_slabs(n, n_sub, slabs_per_sub)
    mesh = grid_mesh(n, n_sub, seed, n_gauss=4, jagged_seed=None, sub_of_cube=sub)
    return _scene("sandwich", mesh, ortho_view_z(size, size), n, m, tf_seed=seed + 11)


def scene(name: str, **kw) -> Scene:
    return {"tiny": scene_tiny, "medium": scene_medium, "large": scene_large,
            "sandwich": sandwich_scene}[name](**kw)


def scene_slabs(n_ranks: int = 16, slabs_per_rank: int = 4, cells_per_slab: int = 2, size: int = 1024,
                m: int = 4, seed: int = 6, camera: int | None = None) -> Scene:
    """Interleaved-slab stress volume: the cube is cut along z into
    n_ranks * slabs_per_rank slabs of cells_per_slab cube layers, and slab q
    belongs to subdomain q % n_ranks, so every subdomain's slabs are separated
    by the other n_ranks - 1 subdomains' slabs.  Grid n^3 with
    n = n_ranks * slabs_per_rank * cells_per_slab (16 ranks: 128^3 x 6 =
    12,582,912 tets).  camera None: orthographic along +z (each ray crosses
    every slab: n_ranks * slabs_per_rank segments); else a seeded perspective
    camera on the radius-2 sphere."""
    n = n_ranks * slabs_per_rank * cells_per_slab
    sub = partition_slabs(n, n_ranks, slabs_per_rank)
    mesh = grid_mesh(n, n_ranks, seed, n_gauss=8, jagged_seed=None, sub_of_cube=sub)
    if camera is None:
        view = ortho_view_z(size, size)
    else:
        view = perspective_view(sphere_eye(seed + 3 + 97 * camera), (0.5, 0.5, 0.5), size, size)
    return _scene("slabs", mesh, view, n, m, tf_seed=seed + 11)


def uneven_weights(n_sub: int, ratio: float, seed: int) -> np.ndarray:
    """Chunk weights ratio^(k/(n_sub-1)), k = 0..n_sub-1, in a seeded order: max/min = ratio."""
    w = ratio ** (np.arange(n_sub) / (n_sub - 1.0))
    return np.random.default_rng(seed).permutation(w)


def scene_batching(size: int = 2560, m: int = 8, seed: int = BATCHING_SEED, camera: int = 0, base: int = 32, levels: int = 3,
                   tet_range: tuple = (19_000_000, 21_000_000), n_sub: int = 72) -> Scene:
    """Uneven-subdomain workload on an adaptive mesh: a base^3 grid of cubes refined 0..levels times where
    |grad f| * h exceeds a threshold chosen so that the tet count falls in tet_range, 2:1 balanced and cut
    into conforming tets by cone decomposition (synth.amr; defaults: 32^3 base, finest 256^3, 19M-21M tets);
    n_sub chunks of whole leaves in Morton order with tet counts in ratio 12^(k/(n_sub-1)), seeded order
    (largest / smallest = 12); perspective camera on the radius-2 sphere; step a quarter of the finest
    cell (1/1024)."""
    from .amr import amr_mesh
    w = uneven_weights(n_sub, 12.0, seed + 5)
    mesh, _, _ = amr_mesh(base, levels, n_sub, seed, tet_range=tet_range, chunk_weights=w)
    return _scene("batching", mesh, orbit_view(seed, camera, size), base << levels, m, tf_seed=seed + 11)


def scene_amr_small(size: int = 256, m: int = 8, seed: int = 8, threshold: float = 0.3, n_sub: int = 8) -> Scene:
    """A small adaptive mesh with leaves of all four levels (8^3 base, finest 64^3, about 480K tets at the
    default threshold), n_sub uneven chunks (ratio 12), perspective camera."""
    from .amr import amr_mesh
    w = uneven_weights(n_sub, 12.0, seed + 5)
    mesh, _, _ = amr_mesh(8, 3, n_sub, seed, threshold=threshold, chunk_weights=w)
    view = perspective_view(sphere_eye(seed + 3), (0.5, 0.5, 0.5), size, size)
    return _scene("amr_small", mesh, view, 64, m, tf_seed=seed + 11)


def request_stream(n: int, rate: float = 50.0, seed: int = 12, sizes=(256, 512, 1024, 2048), ms=(4, 6, 8),
                   n_tf: int = 3) -> list:
    """Open-loop Poisson stream of render requests: exponential inter-arrival times (mean 1/rate seconds),
    each with an image size, a camera on the radius-2 sphere around the cube's centre, a moment count and
    one of n_tf transfer functions, all drawn from one seeded generator."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for k in range(n):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        out.append({"id": k, "arrival": float(t[k]), "size": int(rng.choice(sizes)),
                    "eye": tuple((np.array([0.5, 0.5, 0.5]) + 2.0 * v).tolist()),
                    "m": int(rng.choice(ms)), "tf": int(rng.integers(n_tf))})
    return out
