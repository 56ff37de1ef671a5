"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each checks it against a
closed form, an exact rational computation by a different route, an
invariant, a library routine or a brute-force optimisation.

Geometry and sampling (Section 3, Alg. 2; fixed-step sampling of Section 5):
  * warp end points, monotonicity and the geometric-mean midpoint;
  * depth range of the orthographic tiny view in closed form;
  * chords against exact rational barycentric clipping, and chords that tile
    the ray's slab interval through the unit box;
  * b0 = sigma * L on a constant field (orthographic and pinhole);
  * b0 = exact integral on a linear field with a linear alpha ramp (the
    midpoint rule is exact there, so barycentric and table interpolation are
    both pinned);
  * one piece: b_j = a z^j; uniform field: second-order convergence of b_j.
Compositing invariants (Section 4.1, 4.2):
  * global moments do not depend on the partition (S=1, jagged S=4, random
    Morton chunks, interleaved slabs).
Reconstruction (Alg. 3):
  * the canonical nodes and weights reproduce all 2n+1 biased moments;
  * nodes against numpy's companion-matrix roots;
  * m=4 against the closed-form quadratic case;
  * F(eta=0) and F(eta=1) against the lower/upper Chebyshev-Markov-Stieltjes
    bounds found by linear programming over measures on a fine grid;
  * F is monotone in the depth and lies in [0, 1];
  * a single fragment without bias composites exactly; two fragments with a
    vanishing bias composite to within 1e-3 of front-to-back blending;
  * a constant-colour transfer function gives rgb = c * (1 - exp(-b0)).
"""
import math
import warnings
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize

import oracle
import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _scene_from(mesh, view, m=4, step=1.0 / 64, tf=None, alpha=5e-5, eta=0.3, s_min=None, s_max=None,
                kappa=4.0, renormalize=1, bias=None):
    tf = synth.make_tf(3) if tf is None else tf
    return synth.Scene(name="custom", mesh=mesh, tf=tf,
                       s_min=float(mesh.scalar.min()) if s_min is None else s_min,
                       s_max=float(mesh.scalar.max()) if s_max is None else s_max,
                       kappa=kappa, absorbance_max=10.0, view=view, step=step, m=m, alpha=alpha,
                       bias=synth.default_bias(m) if bias is None else bias, eta=eta, renormalize=renormalize)


def _box_interval(o, d):
    """Slab-method interval of the ray o + t d inside [0,1]^3 (FP64)."""
    t0, t1 = -np.inf, np.inf
    for k in range(3):
        if d[k] == 0.0:
            if not 0.0 <= o[k] <= 1.0:
                return 1.0, 0.0
            continue
        a, b = (0.0 - o[k]) / d[k], (1.0 - o[k]) / d[k]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return t0, t1


def _pixel_rays(view):
    W, H = view["width"], view["height"]
    j, i = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    i, j = i.ravel(), j.ravel()
    if view["projection"] == 0:
        o = np.asarray(view["eye"]) + j[:, None] * np.asarray(view["right"]) + i[:, None] * np.asarray(view["down"])
        d = np.tile(np.asarray(view["dir"], dtype=np.float64), (W * H, 1))
    else:
        o = np.tile(np.asarray(view["eye"], dtype=np.float64), (W * H, 1))
        d = (np.asarray(view["dir"]) + (j - W / 2)[:, None] * np.asarray(view["right"])
             + (i - H / 2)[:, None] * np.asarray(view["down"]))
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


# ----------------------------------------------------------------------------- warp / depth range

def test_warp_closed_form():
    tn, tf = 0.6339, 2.366
    assert abs(oracle.warp(tn, tn, tf) + 1.0) <= 1e-15
    assert abs(oracle.warp(tf, tn, tf) - 1.0) <= 1e-15
    assert abs(oracle.warp(math.sqrt(tn * tf), tn, tf)) <= 1e-15  # log warp: geometric mean -> 0
    z = np.array([oracle.warp(t, tn, tf) for t in np.linspace(tn, tf, 2001)])
    assert np.all(np.diff(z) > 0)
    assert oracle.warp(0.5 * tn, tn, tf) == -1.0 and oracle.warp(2.0 * tf, tn, tf) == 1.0


def test_depth_range_orthographic_closed_form():
    sc = synth.scene_tiny()
    tn, tf = oracle.depth_range(sc)
    # unit box centred at (0.5,0.5,0.5), image plane z = -1: distance 1.5, radius sqrt(3)/2
    assert abs(tn - (1.5 - math.sqrt(3) / 2)) <= 1e-15
    assert abs(tf - (1.5 + math.sqrt(3) / 2)) <= 1e-15


# ----------------------------------------------------------------------------- chords

def _exact_bary_chord(P, o, d):
    """Chord of the ray through tet P from exact rational barycentric coordinates."""
    P = [[Fr(float(c)) for c in p] for p in P]
    o = [Fr(float(c)) for c in o]
    d = [Fr(float(c)) for c in d]
    e = [[P[k][r] - P[0][r] for k in (1, 2, 3)] for r in range(3)]  # columns P1-P0, P2-P0, P3-P0

    def solve(rhs):  # Cramer's rule
        def det(M):
            return (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                    - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                    + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]))
        D = det(e)
        out = []
        for c in range(3):
            M = [row[:] for row in e]
            for r in range(3):
                M[r][c] = rhs[r]
            out.append(det(M) / D)
        return out

    base = solve([o[r] - P[0][r] for r in range(3)])
    slope = solve(d)
    coeffs = [(1 - sum(base), -sum(slope))] + list(zip(base, slope))
    lo, hi = None, None
    for a, b in coeffs:  # a + b t >= 0
        if b == 0:
            if a < 0:
                return None
            continue
        t = -a / b
        if b > 0:
            lo = t if lo is None else max(lo, t)
        else:
            hi = t if hi is None else min(hi, t)
    if lo is None or hi is None or hi <= lo:
        return None
    return lo, hi


def test_chords_exact_rational_and_tiling():
    mesh = synth.grid_mesh(4, 1, seed=3, n_gauss=1, jagged_seed=None)
    rng = np.random.default_rng(0)
    rays = []
    for _ in range(24):
        target = rng.uniform(0.1, 0.9, 3)
        src = np.array([0.5, 0.5, 0.5]) + 2.0 * rng.normal(size=3)
        d = target - src
        rays.append((src, d / np.linalg.norm(d)))
    for _ in range(6):
        rays.append((np.array([rng.uniform(0, 1), rng.uniform(0, 1), -1.0]), np.array([0.0, 0.0, 1.0])))
    P_all = mesh.xyz.astype(np.float64)[mesh.tets]
    for o, d in rays:
        chords = []
        for t in range(mesh.n_tets):
            ex = _exact_bary_chord(P_all[t], o, d)
            got = oracle.chord(P_all[t], o, d)
            if ex is None:
                assert got is None or got[1] - got[0] <= 1e-12
                continue
            assert got is not None
            assert abs(got[0] - float(ex[0])) <= 1e-12 and abs(got[1] - float(ex[1])) <= 1e-12
            chords.append(ex)
        chords.sort()
        b0, b1 = _box_interval(o, d)
        if not b1 > b0:
            assert not chords
            continue
        # consecutive chords meet exactly and cover the slab interval
        for (a0, a1), (c0, c1) in zip(chords, chords[1:]):
            assert a1 == c0
        assert abs(float(chords[0][0]) - b0) <= 1e-12 and abs(float(chords[-1][1]) - b1) <= 1e-12


# ----------------------------------------------------------------------------- b0 and moments

def _constant_field_scene(view, n=16, m=4, step=1.0 / 64, alpha_tab=0.37):
    mesh = synth.grid_mesh(n, 4, seed=1, n_gauss=1, jagged_seed=8)
    mesh.scalar[:] = 0.5
    tf = synth.make_tf(5)
    tf[:, 3] = alpha_tab
    return _scene_from(mesh, view, m=m, step=step, tf=tf, s_min=0.0, s_max=1.0)


@pytest.mark.parametrize("proj", ["ortho", "persp"])
def test_b0_constant_density_is_sigma_times_length(proj):
    view = synth.ortho_view_z(32, 32) if proj == "ortho" else synth.perspective_view(
        synth.sphere_eye(9), (0.5, 0.5, 0.5), 32, 32)
    sc = _constant_field_scene(view)
    r = oracle.render(sc, pass2=False)
    sigma = sc.kappa * float(np.float32(0.37))  # the table holds FP32 values
    o, d = _pixel_rays(view)
    L = np.array([max(0.0, b - a) for a, b in (_box_interval(oo, dd) for oo, dd in zip(o, d))])
    assert np.all(np.abs(r["moments"][0] - sigma * L) <= 1e-12 * np.maximum(1.0, sigma * L))
    if proj == "ortho":
        assert np.allclose(L, 1.0)


def test_b0_linear_field_linear_alpha_is_exact_integral():
    # unjittered grid: vertex coordinates and the linear field are exact in FP32
    mesh = synth.grid_mesh(16, 3, seed=2, n_gauss=1, jagged_seed=4, jitter=0.0)
    c = np.array([1.0, 2.0, 3.0])
    mesh.scalar = (mesh.xyz.astype(np.float64) @ c).astype(np.float32)
    assert np.array_equal(mesh.scalar.astype(np.float64), mesh.xyz.astype(np.float64) @ c)
    tf = synth.make_tf(6)
    tf[:, 3] = np.arange(256) / 256.0  # exact FP32 ramp: A(s) = (255/256) * s / 6 on [0, 6]
    view = synth.perspective_view(synth.sphere_eye(12), (0.5, 0.5, 0.5), 24, 24)
    sc = _scene_from(mesh, view, tf=tf, s_min=0.0, s_max=6.0, step=1.0 / 40)
    assert sc.s_min == 0.0 and sc.s_max == 6.0
    r = oracle.render(sc, pass2=False)
    o, d = _pixel_rays(view)
    for q in range(o.shape[0]):
        t0, t1 = _box_interval(o[q], d[q])
        if not t1 > t0:
            assert r["moments"][0, q] == 0.0
            continue
        integral = (c @ o[q]) * (t1 - t0) + (c @ d[q]) * (t1 * t1 - t0 * t0) / 2.0
        expect = sc.kappa * integral * 255.0 / (256.0 * 6.0)
        assert abs(r["moments"][0, q] - expect) <= 1e-12 * max(1.0, expect)


def _one_ray_view(o, d):
    """1x1 orthographic view whose single pixel-centre ray is o + t d (d along +z)."""
    px = np.array([0.01, 0.0, 0.0]), np.array([0.0, 0.01, 0.0])
    eye = np.asarray(o, np.float64) - 0.5 * (px[0] + px[1])
    return dict(width=1, height=1, projection=0, eye=tuple(eye), dir=tuple(d), right=tuple(px[0]),
                down=tuple(px[1]))


def _single_tet_scene(o, d, step=100.0, m=4, scalar=(0.125, 0.375, 0.625, 0.875), alpha=5e-5, eta=0.3, renorm=1):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float32)
    mesh = synth.Mesh(xyz=xyz, scalar=np.array(scalar, np.float32), tets=np.array([[0, 1, 2, 3]], np.int32),
                      tet_sub=np.zeros(1, np.int32), n_sub=1)
    view = _one_ray_view(o, d)
    return _scene_from(mesh, view, m=m, step=step, s_min=0.0, s_max=1.0, alpha=alpha, eta=eta,
                       renormalize=renorm)


def test_piece_absorbance_is_capped():
    """Alg. 2 caps the absorbance of a piece: one piece (the step is longer than the chord) on the ray along z
    through (0.2, 0.25) of the unit tet, chord length 1 - 0.2 - 0.25 = 0.55, constant table alpha A: b0 =
    min(kappa A 0.55, cap), below and above the cap."""
    o = np.array([0.2, 0.25, -1.0])
    d = np.array([0.0, 0.0, 1.0])
    A = float(np.float32(0.37))
    for kappa, cap in ((4.0, 10.0), (4.0, 0.5), (40.0, 3.0), (40.0, 100.0)):
        sc = _single_tet_scene(o, d, step=100.0, m=4, scalar=(0.5, 0.5, 0.5, 0.5))
        sc.tf = sc.tf.copy()
        sc.tf[:, 3] = 0.37
        sc.kappa, sc.absorbance_max = kappa, cap
        b0 = oracle.render(sc, pass2=False)["moments"][0, 0]
        want = min(kappa * A * 0.55, cap)
        assert abs(b0 - want) <= 1e-12 * max(1.0, want), (kappa, cap, b0, want)


@pytest.mark.parametrize("m", [4, 6, 8])
def test_bound_of_a_single_depth_is_a_step(m):
    """All absorbance at one depth z1 (b_j = b0 z1^j) and no bias: the bound is exact, a step from 0 in
    front of z1 to 1 behind it, with the overestimation weight eta at z1 itself."""
    bias = synth.default_bias(m)
    eta = 0.3
    for z1 in (-0.6, 0.1, 0.75):
        b = 1.7 * z1 ** np.arange(m + 1)
        for zf, want in ((z1 - 0.3, 0.0), (z1 - 1e-3, 0.0), (z1, eta), (z1 + 1e-3, 1.0), (z1 + 0.2, 1.0)):
            F = oracle.bound(b, 0.0, bias, eta, zf)[0]
            assert F == want, (m, z1, zf, F)


def test_single_piece_moments_closed_form():
    o = np.array([0.2, 0.25, -1.0])
    d = np.array([0.0, 0.0, 1.0])
    sc = _single_tet_scene(o, d, m=8)
    r = oracle.render(sc, pass2=False)
    ex = _exact_bary_chord(sc.mesh.xyz.astype(np.float64), o, d)
    t0, t1 = float(ex[0]), float(ex[1])
    tm, ln = 0.5 * (t0 + t1), t1 - t0
    # scalar along +z at (0.2, 0.25): linear field s = 0.125 + 0.25x + 0.5y + 0.75z
    s = 0.125 + 0.25 * 0.2 + 0.5 * 0.25 + 0.75 * (tm - 1.0)
    u = s * 255.0
    i0 = int(math.floor(u))
    A = (1 - (u - i0)) * float(sc.tf[i0, 3]) + (u - i0) * float(sc.tf[i0 + 1, 3])
    a = sc.kappa * A * ln
    tn, tf = r["t_near"], r["t_far"]
    z = 2 * (math.log(tm) - math.log(tn)) / (math.log(tf) - math.log(tn)) - 1
    expect = a * z ** np.arange(9)
    assert np.all(np.abs(r["moments"][:, 0] - expect) <= 1e-14)
    assert r["n_pieces"] == 1


def test_uniform_density_moments_converge_second_order():
    # midpoint rule on the pieces: error ~ step^2 once the lattice is fine compared to the tets
    view = synth.ortho_view_z(4, 4)
    errs = []
    for step in (1 / 128, 1 / 256, 1 / 512):
        sc = _constant_field_scene(view, n=2, m=4, step=step)
        r = oracle.render(sc, pass2=False)
        tn, tf = r["t_near"], r["t_far"]
        sigma = sc.kappa * float(np.float32(0.37))

        def zf(t):
            return 2 * (math.log(t) - math.log(tn)) / (math.log(tf) - math.log(tn)) - 1

        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            exact = np.array([sigma * scipy.integrate.quad(lambda t: zf(t) ** j, 1.0, 2.0, epsabs=1e-15,
                                                           epsrel=1e-15, limit=200)[0] for j in range(5)])
        errs.append(np.abs(r["moments"] - exact[:, None]).sum(axis=1))
    errs = np.array(errs)
    for j in (1, 2, 3, 4):
        r1, r2 = errs[0, j] / errs[1, j], errs[1, j] / errs[2, j]
        assert 3.7 <= r1 <= 4.3 and 3.7 <= r2 <= 4.3, (j, r1, r2)
    assert np.all(errs[:, 0] <= 1e-12)


# ----------------------------------------------------------------------------- order independence

def test_global_moments_independent_of_partition():
    base = synth.scene_tiny()
    ref = oracle.render(base, pass2=False)["moments"]
    n = 16
    order = synth.morton_order(n)
    variants = []
    for S, seed in ((1, None), (7, 3), (11, 5)):
        bounds = synth.partition_chunks(n ** 3, S, seed)
        rank = np.empty(n ** 3, np.int64)
        rank[order] = np.arange(n ** 3)
        variants.append((S, (np.searchsorted(bounds, rank, side="right") - 1).astype(np.int32)))
    variants.append((3, synth.partition_slabs(n, 3, 2)))
    cube_of_tet = np.repeat(order, 6)
    for S, sub_of_cube in variants:
        mesh = synth.Mesh(xyz=base.mesh.xyz, scalar=base.mesh.scalar, tets=base.mesh.tets,
                          tet_sub=sub_of_cube[cube_of_tet].astype(np.int32), n_sub=S)
        sc = synth.Scene(**{**base.__dict__, "mesh": mesh})
        got = oracle.render(sc, pass2=False)["moments"]
        assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(ref[0], 1e-300))


# ----------------------------------------------------------------------------- reconstruction

def _random_moments(rng, m, n_atoms, alpha_spread=1.0):
    x = rng.uniform(-alpha_spread, alpha_spread, n_atoms)
    w = rng.uniform(0.05, 1.0, n_atoms)
    b0 = rng.uniform(0.2, 4.0)
    w = w / w.sum() * b0
    return np.array([np.sum(w * x ** j) for j in range(m + 1)]), x, w


def _biased(b, alpha, bias):
    m = len(b) - 1
    return np.concatenate([[1.0], (1 - alpha) * b[1:] / b[0] + alpha * np.asarray(bias)[:m]])


@pytest.mark.parametrize("m", [4, 6, 8])
def test_canonical_representation_reproduces_moments(m):
    rng = np.random.default_rng(m)
    n = m // 2
    bias = synth.default_bias(m)
    checked = 0
    for _ in range(800):
        b, _, _ = _random_moments(rng, m, rng.integers(n + 1, 12))
        zf = rng.uniform(-1, 1)
        F, nodes, wts, flags = oracle.bound(b, 5e-5, bias, 0.3, zf)
        assert flags == 0
        bp = _biased(b, 5e-5, bias)
        fin = np.isfinite(nodes)
        assert np.all(wts >= -1e-12)
        assert abs(wts.sum() - 1.0) <= 1e-10
        if np.any(np.abs(nodes[fin]) > 5.0):
            # a node far out carries a tiny weight whose relative error is large; its
            # product with x^(2n) makes the high moments ill-conditioned, so skip those
            continue
        checked += 1
        for k in range(2 * n + 1):
            assert abs(np.sum(wts[fin] * nodes[fin] ** k) - bp[k]) <= 1e-9 * max(1.0, abs(bp[k])), k
        assert nodes[0] == zf
    assert checked >= 300


@pytest.mark.parametrize("m", [4, 6, 8])
def test_nodes_match_numpy_companion_roots(m):
    rng = np.random.default_rng(100 + m)
    n = m // 2
    bias = synth.default_bias(m)
    for _ in range(3000):
        b, _, _ = _random_moments(rng, m, rng.integers(n + 1, 10))
        zf = rng.uniform(-1, 1)
        bp = _biased(b, 5e-5, bias)
        B = np.array([[bp[j + k] for k in range(n + 1)] for j in range(n + 1)])
        L = np.linalg.cholesky(B)
        q = np.linalg.solve(L.T, np.linalg.solve(L, zf ** np.arange(n + 1)))
        ref = np.sort(np.roots(q[::-1]).real)
        _, nodes, _, _ = oracle.bound(b, 5e-5, bias, 0.3, zf)
        got = np.sort(nodes[1:])
        assert np.all(np.abs(got - ref) <= 1e-9 * np.maximum(1.0, np.abs(ref))), (got, ref)


def test_m4_matches_closed_form_quadratic_case():
    rng = np.random.default_rng(7)
    bias = synth.default_bias(4)
    for _ in range(2000):
        b, _, _ = _random_moments(rng, 4, rng.integers(3, 9))
        zf, eta = rng.uniform(-1, 1), rng.uniform(0, 1)
        bp = _biased(b, 5e-5, bias)
        # kernel polynomial coefficients from the 3x3 Hankel system, written out by hand
        B = np.array([[bp[0], bp[1], bp[2]], [bp[1], bp[2], bp[3]], [bp[2], bp[3], bp[4]]])
        q = np.linalg.solve(B, np.array([1.0, zf, zf * zf]))
        disc = q[1] ** 2 - 4 * q[2] * q[0]
        s = -0.5 * (q[1] + math.copysign(math.sqrt(max(disc, 0.0)), q[1]))
        x1, x2 = s / q[2], q[0] / s
        nodes = [zf, x1, x2]
        F = 0.0
        for i in range(3):
            a_, b_ = [nodes[k] for k in range(3) if k != i]
            lam = (bp[2] - bp[1] * (a_ + b_) + a_ * b_) / ((nodes[i] - a_) * (nodes[i] - b_))
            F += (eta if i == 0 else float(nodes[i] < zf)) * lam
        got = oracle.bound(b, 5e-5, bias, eta, zf)[0]
        assert abs(got - F) <= 1e-12, (got, F)


def _lp_bounds(bp, zf, grid):
    """min mass on (-inf, zf) and max mass on (-inf, zf] over measures on `grid`
    that reproduce the moments bp[0..2n]."""
    K = len(bp)
    A = np.vstack([grid ** k for k in range(K)])
    below = (grid < zf).astype(float)
    upto = (grid <= zf).astype(float)
    lo = scipy.optimize.linprog(below, A_eq=A, b_eq=bp, bounds=(0, None), method="highs")
    hi = scipy.optimize.linprog(-upto, A_eq=A, b_eq=bp, bounds=(0, None), method="highs")
    assert lo.status == 0 and hi.status == 0
    return lo.fun, -hi.fun


@pytest.mark.parametrize("m", [4, 6])
def test_bounds_equal_chebyshev_markov_stieltjes_extremes(m):
    rng = np.random.default_rng(200 + m)
    n = m // 2
    grid = np.linspace(-1.5, 1.5, 3001)
    checked = 0
    while checked < 25:
        b, _, _ = _random_moments(rng, m, rng.integers(n + 2, 8), alpha_spread=0.9)
        zf = grid[rng.integers(600, 2400)]
        F0, nodes, _, flags = oracle.bound(b, 0.0, None, 0.0, zf)
        F1 = oracle.bound(b, 0.0, None, 1.0, zf)[0]
        if flags or not np.all(np.abs(nodes) < 1.45):
            continue  # the grid must contain the extremal measure's support
        bp = _biased(b, 0.0, np.zeros(m))
        lo, hi = _lp_bounds(bp, zf, grid)
        assert abs(F0 - lo) <= 2e-3 and abs(F1 - hi) <= 2e-3, (F0, lo, F1, hi)
        checked += 1


@pytest.mark.parametrize("m", [4, 6, 8])
def test_bound_brackets_true_mass_and_is_monotone(m):
    rng = np.random.default_rng(300 + m)
    n = m // 2
    for _ in range(40):
        b, x, w = _random_moments(rng, m, rng.integers(n + 1, 9))
        zs = np.linspace(-1.0, 1.0, 301)
        for eta in (0.0, 0.3, 1.0):
            F = np.array([oracle.bound(b, 0.0, None, eta, z)[0] for z in zs])
            # unbiased Hankel matrices are ill-conditioned (cond ~1e6-1e8): FP64 rounding ~1e-12
            assert np.all(F >= -1e-10) and np.all(F <= 1 + 1e-10)
            assert np.all(np.diff(F) >= -1e-10)
        for z in rng.uniform(-1, 1, 10):
            lo = oracle.bound(b, 0.0, None, 0.0, z)[0]
            hi = oracle.bound(b, 0.0, None, 1.0, z)[0]
            assert lo <= np.sum(w[x < z]) / b[0] + 1e-10
            assert np.sum(w[x <= z]) / b[0] <= hi + 1e-10


def test_single_fragment_without_bias_is_exact():
    o, d = np.array([0.2, 0.25, -1.0]), np.array([0.0, 0.0, 1.0])
    sc = _single_tet_scene(o, d, alpha=0.0, eta=0.0, renorm=0)
    r = oracle.render(sc, exact=True)
    assert r["n_rank1"] == 1
    assert np.all(np.abs(r["rgba"] - r["exact"]) <= 1e-12)
    assert r["exact"][0, 3] > 0.01


def test_two_fragments_with_vanishing_bias_composite_front_to_back():
    # two disjoint tets on one ray, each cut into a single piece
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                    [0, 0, 2], [1, 0, 2], [0, 1, 2], [0, 0, 3]], dtype=np.float32)
    tets = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    scal = np.array([0.9, 0.9, 0.9, 0.9, 0.2, 0.2, 0.2, 0.2], np.float32)
    for sub in ([0, 0], [1, 0]):
        mesh = synth.Mesh(xyz=xyz, scalar=scal, tets=tets, tet_sub=np.array(sub, np.int32), n_sub=2)
        view = _one_ray_view((0.2, 0.25, -1.0), (0.0, 0.0, 1.0))
        sc = _scene_from(mesh, view, m=4, step=100.0, s_min=0.0, s_max=1.0, alpha=1e-10, eta=0.0,
                         renormalize=0)
        r = oracle.render(sc, exact=True)
        assert r["n_pieces"] == 2
        assert np.all(np.abs(r["rgba"][0, :3] - r["exact"][0, :3]) <= 1e-3)


def test_constant_colour_tf_renormalises_to_opacity():
    sc = synth.scene_tiny()
    c = np.array([0.2, 0.55, 0.7], np.float32)
    sc.tf[:, :3] = c
    for alpha, eta in ((5e-5, 0.3), (0.02, 0.0), (0.3, 1.0)):
        sc.alpha, sc.eta = alpha, eta
        r = oracle.render(sc)
        A = -np.expm1(-r["moments"][0])
        assert np.all(np.abs(r["rgba"][:, 3] - A) <= 1e-14)
        assert np.all(np.abs(r["rgba"][:, :3] - c.astype(np.float64)[None, :] * A[:, None]) <= 1e-14)


def test_apc_vs_exact_compositing_report():
    """Report (not a bar): APC against exact sorted compositing on the tiny workload."""
    r = oracle.render(synth.scene_tiny(), exact=True)
    d = r["rgba"] - r["exact"]
    mse = float(np.mean(d[:, :3] ** 2))
    psnr = 10 * math.log10(1.0 / mse)
    print("APC vs exact (tiny): max abs %.3g rmse %.3g psnr %.2f dB" % (np.abs(d).max(), math.sqrt(mse), psnr))
    assert psnr > 30.0
    assert np.all(np.abs(d[:, 3]) <= 1e-14)  # opacity is 1 - exp(-b0) in both


def test_depth_range_perspective_touches_the_bounding_sphere():
    # the near/far depths are where the ray through the sphere centre meets the sphere
    sc = synth.scene_medium(size=8)
    lo = sc.mesh.xyz.min(axis=0).astype(np.float64)
    hi = sc.mesh.xyz.max(axis=0).astype(np.float64)
    c, R = 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo)
    for seed in range(5):
        eye = synth.sphere_eye(100 + seed, radius=2.0 + seed)
        sc.view = synth.perspective_view(eye, (0.5, 0.5, 0.5), 8, 8)
        tn, tf = oracle.depth_range(sc)
        u = (c - eye) / np.linalg.norm(c - eye)
        for t in (tn, tf):
            assert abs(np.linalg.norm(eye + t * u - c) - R) <= 1e-12
        assert 0 < tn < tf


def test_exact_compositing_of_two_constant_fragments():
    # two disjoint tets with constant scalars; each ray chord is one piece of known optical depth
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                    [0, 0, 2], [1, 0, 2], [0, 1, 2], [0, 0, 3]], dtype=np.float32)
    tets = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    scal = np.array([0.25] * 4 + [0.75] * 4, np.float32)
    mesh = synth.Mesh(xyz=xyz, scalar=scal, tets=tets, tet_sub=np.array([0, 1], np.int32), n_sub=2)
    o, d = (0.2, 0.25, -1.0), (0.0, 0.0, 1.0)
    tf = synth.make_tf(8)
    sc = _scene_from(mesh, _one_ray_view(o, d), m=4, step=100.0, tf=tf, s_min=0.0, s_max=1.0, renormalize=0)
    r = oracle.render(sc, exact=True)
    # chord lengths along +z at (0.2, 0.25): both tets are x + y + z' <= 1 slices, length 1 - 0.45
    ln = 1.0 - 0.45
    rgba = []
    for s in (0.25, 0.75):
        u = s * 255.0
        i0 = int(math.floor(u))
        fr = u - i0
        rgba.append([(1 - fr) * float(tf[i0, c]) + fr * float(tf[i0 + 1, c]) for c in range(4)])
    a = [sc.kappa * rgba[k][3] * ln for k in range(2)]
    al = [-math.expm1(-x) for x in a]
    expect = [al[0] * rgba[0][c] + math.exp(-a[0]) * al[1] * rgba[1][c] for c in range(3)]
    assert np.allclose(r["exact"][0, :3], expect, atol=1e-14)
    assert abs(r["exact"][0, 3] - (-math.expm1(-(a[0] + a[1])))) <= 1e-14


@pytest.mark.parametrize("n_ranks,slabs", [(4, 4), (3, 2), (5, 1)])
def test_segment_counts_on_interleaved_slabs(n_ranks, slabs):
    """Stress volume of the paper's weak-scaling test (Section 5, interleaved
    slabs): a ray along z crosses every slab once and consecutive slabs belong
    to different subdomains, so it has exactly n_ranks * slabs segments and
    meets every subdomain."""
    sc = synth.scene_slabs(n_ranks=n_ranks, slabs_per_rank=slabs, cells_per_slab=2, size=48)
    r = oracle.render(sc, pass2=False, segments=True)
    assert np.all(r["segments"][0] == n_ranks * slabs)
    assert np.all(r["segments"][1] == n_ranks)


def test_segment_counts_single_convex_subdomain():
    """One subdomain filling the unit cube (convex): one segment on every ray
    that meets it, none elsewhere."""
    sc = synth.scene_tiny()
    sc.mesh.tet_sub[:] = 0
    sc.mesh.n_sub = 1
    r = oracle.render(sc, pass2=False, segments=True)
    covered = r["moments"][0] > 0
    assert covered.all()
    assert np.all(r["segments"][0] == 1) and np.all(r["segments"][1] == 1)
