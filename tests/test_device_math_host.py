"""The library's moment-bound code (csrc/apc_mboit.h, the same source the HIP
kernels compile) built for the host and compared with the FP64 oracle on random
moment vectors: FP64 (used for m = 6, 8) to 1e-10, FP32 (used for m = 4) to the
transmittance level the image bar needs."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "libshim.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", str(out),
                           os.path.join(ROOT, "tests", "mboit_host_shim.cpp")])
    L = C.CDLL(str(out))
    L.shim_bound.restype = C.c_double
    L.shim_bound.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_double, C.c_double, C.c_int,
                             C.POINTER(C.c_int)]
    L.shim_roots.restype = C.c_int
    L.shim_roots.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    L.shim_zeros.restype = C.c_int
    L.shim_zeros.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p]
    L.shim_bound_cont.restype = C.c_int
    L.shim_bound_cont.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_double, C.c_void_p, C.c_int,
                                  C.c_void_p, C.c_void_p]
    L.shim_bound_table.restype = C.c_int
    L.shim_bound_table.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_double, C.c_void_p, C.c_int,
                                   C.c_void_p, C.c_void_p]
    return L


def _moments(rng, m, n_atoms):
    x = rng.uniform(-1, 1, n_atoms)
    w = rng.uniform(0.05, 1.0, n_atoms)
    w = w / w.sum() * rng.uniform(0.2, 4.0)
    return np.array([np.sum(w * x ** j) for j in range(m + 1)])


# m = 8: the biased 5x5 Hankel matrix has condition numbers up to ~1e9, so FP64 agrees to ~1e-8
@pytest.mark.parametrize("m,fp64,tol", [(4, 1, 1e-10), (6, 1, 1e-9), (8, 1, 1e-7), (4, 0, 2e-4)])
def test_bound_matches_oracle(shim, m, fp64, tol):
    rng = np.random.default_rng(40 + m + fp64)
    bias = np.ascontiguousarray(np.pad(synth.default_bias(m), (0, 8 - m)))
    fl = C.c_int(0)
    worst = 0.0
    for _ in range(2000):
        b = np.ascontiguousarray(_moments(rng, m, rng.integers(m // 2 + 1, 12)))
        zf, eta = rng.uniform(-1, 1), rng.uniform(0, 1)
        ref = oracle.bound(b, 5e-5, bias[:m], eta, zf)[0]
        got = shim.shim_bound(b.ctypes.data, m, 5e-5, bias.ctypes.data, eta, zf, fp64, C.byref(fl))
        worst = max(worst, abs(got - ref))
    assert worst <= tol, worst


@pytest.mark.parametrize("n", [2, 3, 4])
def test_closed_form_roots_match_numpy(shim, n):
    rng = np.random.default_rng(n)
    out = np.zeros(4)
    for _ in range(2000):
        r = np.sort(rng.uniform(-3, 3, n))
        q = np.poly(r)[::-1] * rng.uniform(0.1, 10)  # ascending coefficients with real simple roots
        q = np.ascontiguousarray(q)
        k = shim.shim_roots(q.ctypes.data, n, 1, out.ctypes.data)
        assert k == n
        assert np.allclose(np.sort(out[:k]), r, atol=1e-9 * max(1, np.abs(r).max()))


def test_vanishing_leading_coefficient_drops_a_root(shim):
    # x^4 coefficient far below the others: one node at infinity, three finite roots kept
    r = np.array([-0.7, 0.1, 0.5])
    q = np.concatenate([np.poly(r)[::-1], [1e-16]])
    out = np.zeros(4)
    k = shim.shim_roots(np.ascontiguousarray(q).ctypes.data, 4, 1, out.ctypes.data)
    assert k == 3 and np.allclose(np.sort(out[:3]), r, atol=1e-9)


def _rendered_moments(m, n_pix, seed):
    """Per-pixel moment vectors of a real frame (oracle, stage one only): the
    depth distributions the gap tables meet in practice."""
    sc = synth.scene_medium(size=128)
    sc.m = m
    sc.bias = synth.default_bias(m)
    pix = np.sort(np.random.default_rng(seed).choice(128 * 128, n_pix, replace=False))
    mom = oracle.render(sc, pixels=pix, pass2=False)["moments"]
    return mom[:, mom[0] > 0].T, sc


@pytest.mark.parametrize("m", [6, 8])
def test_gap_table_matches_closed_form_and_oracle(shim, m):
    """The table path (interpolated starts + Newton) gives the closed-form
    bound to 1e-9 at every depth across every gap, falls back rarely, and
    both agree with the oracle's own bound."""
    # 150 pixels: at m = 8 one of them has a nearly vanishing leading coefficient of K(., z) (a node near
    # 2.6e4), where a single Newton polish of the closed forms left F off by 8.7e-6
    moms, sc = _rendered_moments(m, 150, 7 + m)
    bias = np.ascontiguousarray(np.pad(synth.default_bias(m), (0, 8 - m)))
    n = 801
    z = np.ascontiguousarray(np.linspace(-1.0, 1.0, n))
    ft, fc = np.zeros(n), np.zeros(n)
    tabled = fallbacks = 0
    worst = worst_ref = 0.0
    for b in moms:
        b = np.ascontiguousarray(b)
        fb = shim.shim_bound_table(b.ctypes.data, m, sc.alpha, bias.ctypes.data, sc.eta, z.ctypes.data, n,
                                   ft.ctypes.data, fc.ctypes.data)
        if fb < 0:
            continue
        tabled += n
        fallbacks += fb
        worst = max(worst, float(np.abs(ft - fc).max()))
        for zf in z[::80]:
            ref = oracle.bound(b, sc.alpha, bias[:m], sc.eta, zf)[0]
            got = ft[np.searchsorted(z, zf)]
            worst_ref = max(worst_ref, abs(got - ref))
    assert tabled > 50 * n
    assert worst <= 1e-9, worst
    assert worst_ref <= (1e-9 if m == 6 else 1e-7), worst_ref
    assert fallbacks <= 2e-3 * tabled, (fallbacks, tabled)


def test_gap_table_on_random_atoms(shim):
    """Random discrete depth distributions (few, possibly clustered atoms):
    harder for the table than rendered pixels.  Against the oracle the table
    path must do at least as well as the closed forms' bar (1e-9 at m = 6,
    1e-7 at m = 8, where the quartic's resolvent loses digits)."""
    rng = np.random.default_rng(5)
    n = 401
    z = np.ascontiguousarray(np.linspace(-1.0, 1.0, n))
    ft, fc = np.zeros(n), np.zeros(n)
    for m, tol in ((6, 1e-9), (8, 1e-7)):
        bias = np.ascontiguousarray(np.pad(synth.default_bias(m), (0, 8 - m)))
        worst = worst_closed = 0.0
        for _ in range(200):
            b = np.ascontiguousarray(_moments(rng, m, rng.integers(m // 2 + 1, 12)))
            eta = rng.uniform(0, 1)
            if shim.shim_bound_table(b.ctypes.data, m, 5e-5, bias.ctypes.data, eta, z.ctypes.data, n,
                                     ft.ctypes.data, fc.ctypes.data) < 0:
                continue
            worst_closed = max(worst_closed, float(np.abs(ft - fc).max()))
            for i in range(0, n, 8):
                ref = oracle.bound(b, 5e-5, bias[:m], eta, z[i])[0]
                worst = max(worst, abs(ft[i] - ref))
        assert worst <= tol, (m, worst)
        assert worst_closed <= tol, (m, worst_closed)


@pytest.mark.parametrize("m", [6, 8])
def test_bound_on_and_near_the_zeros(shim, m):
    """Depths on and next to a zero of the degree-n orthonormal polynomial, where one node of the bound runs
    off to infinity and the kernel polynomial's leading coefficient vanishes: the closed forms (which divide
    the far root out instead of making the polynomial monic) match the oracle's companion-matrix roots."""
    rng = np.random.default_rng(70 + m)
    bias = np.ascontiguousarray(np.pad(synth.default_bias(m), (0, 8 - m)))
    fl = C.c_int(0)
    zs = np.zeros(4)
    worst, n = 0.0, 0
    for _ in range(300):
        b = np.ascontiguousarray(_moments(rng, m, rng.integers(m // 2 + 2, 12)))
        if shim.shim_zeros(b.ctypes.data, m, 5e-5, bias.ctypes.data, zs.ctypes.data) == 0:
            continue
        for t in zs[: m // 2]:
            for dz in (0.0, 1e-12, -1e-12, 1e-9, -1e-9, 1e-6, -1e-6, 1e-4, -1e-4):
                zf = float(t + dz)
                ref = oracle.bound(b, 5e-5, bias[:m], 0.3, zf)[0]
                got = shim.shim_bound(b.ctypes.data, m, 5e-5, bias.ctypes.data, 0.3, zf, 1, C.byref(fl))
                worst = max(worst, abs(got - ref))
                n += 1
    assert n > 1000
    assert worst <= 1e-7, worst


@pytest.mark.parametrize("m", [6, 8])
def test_continued_roots_match_oracle(shim, m):
    """The re-walk's root solve: each sample of a ray starts Newton from the previous sample's roots (in the
    gap's regularised coordinate), taking the closed forms in a new gap.  On rendered moment vectors, with
    the samples in runs of increasing depth in a random order (a ray meeting several subdomains), the bound
    matches the closed forms everywhere and the oracle wherever the two differ by more than rounding."""
    sc = synth.scene_medium(size=96)
    sc.m = m
    sc.bias = synth.default_bias(m)
    pix = np.random.default_rng(2).choice(96 * 96, 300, replace=False)
    ref = oracle.render(sc, pixels=pix, pass2=False)
    bias = np.ascontiguousarray(np.pad(synth.default_bias(m), (0, 8 - m)))
    rng = np.random.default_rng(4)
    total = closed = 0
    worst = 0.0
    for q in range(len(pix)):
        b = np.ascontiguousarray(ref["moments"][:, q])
        if b[0] <= 0:
            continue
        segs = np.sort(rng.uniform(-1, 1, (5, 2)), axis=1)
        z = np.ascontiguousarray(np.concatenate(
            [np.arange(a, e, rng.uniform(0.001, 0.01)) for a, e in segs[rng.permutation(5)]]))
        fc, fx = np.zeros(len(z)), np.zeros(len(z))
        n = shim.shim_bound_cont(b.ctypes.data, m, 5e-5, bias.ctypes.data, 0.3, z.ctypes.data, len(z),
                                 fc.ctypes.data, fx.ctypes.data)
        if n < 0:
            continue
        total += len(z)
        closed += n
        for i in np.where(np.abs(fc - fx) > 1e-10)[0]:
            worst = max(worst, abs(fc[i] - oracle.bound(b, 5e-5, bias[:m], 0.3, z[i])[0]))
        worst = max(worst, float(np.max(np.abs(fc - fx))) if np.all(np.abs(fc - fx) <= 1e-10) else 0.0)
    assert total > 20000
    assert closed <= 0.05 * total
    assert worst <= 1e-9, worst
