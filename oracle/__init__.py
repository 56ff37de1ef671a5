"""FP64 CPU oracle for the APC hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library (paper_2501_12581_amd) never imports, links
or calls it, and the two share no code; the only common dependency is the
seeded input generator in `synth`, which holds none of the method's arithmetic.

The renderer itself is plain C++ (oracle.cpp, FP64, OpenMP over screen tiles);
this module compiles it with g++ and calls it through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so next to it (g++, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class OView(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("projection", C.c_int32), ("pad", C.c_int32),
                ("eye", C.c_double * 3), ("dir", C.c_double * 3), ("right", C.c_double * 3),
                ("down", C.c_double * 3)]


class OScene(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_tets", C.c_int64), ("n_sub", C.c_int32), ("n_tf", C.c_int32),
                ("xyz", C.c_void_p), ("scalar", C.c_void_p), ("tets", C.c_void_p), ("tet_sub", C.c_void_p),
                ("tf", C.c_void_p), ("s_min", C.c_double), ("s_max", C.c_double), ("kappa", C.c_double),
                ("amax", C.c_double), ("step", C.c_double), ("view", OView), ("m", C.c_int32),
                ("renormalize", C.c_int32), ("alpha", C.c_double), ("eta", C.c_double),
                ("bias", C.c_double * 8)]


class OOut(C.Structure):
    _fields_ = [("pixels", C.c_void_p), ("n_pixels", C.c_int64), ("do_pass2", C.c_int32),
                ("do_exact", C.c_int32), ("n_threads", C.c_int32), ("pad", C.c_int32),
                ("moments_sub", C.c_void_p), ("moments", C.c_void_p), ("color_sub", C.c_void_p),
                ("color", C.c_void_p), ("rgba", C.c_void_p), ("exact", C.c_void_p),
                ("pieces_sub", C.c_void_p), ("n_pieces", C.c_int64), ("n_chords", C.c_int64),
                ("n_nonpd", C.c_int64), ("n_rank1", C.c_int64), ("t_near", C.c_double),
                ("t_far", C.c_double), ("segments", C.c_void_p)]


def lib():
    """The compiled oracle.  APC_ORACLE_LIB names another build of it instead: the planted-mistake test runs
    the oracle's pins against copies of oracle.cpp with one mistake each, which the pins must catch."""
    global _lib
    if _lib is None:
        path = os.environ.get("APC_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(path)
        d = C.c_double
        L.oracle_warp.restype = d
        L.oracle_warp.argtypes = [d, d, d]
        L.oracle_chord.restype = C.c_int
        L.oracle_chord.argtypes = [C.c_void_p] * 4
        L.oracle_roots.restype = C.c_int
        L.oracle_roots.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.oracle_bound.restype = d
        L.oracle_bound.argtypes = [C.c_void_p, C.c_int, d, C.c_void_p, d, d, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_int)]
        L.oracle_depth_range.restype = None
        L.oracle_depth_range.argtypes = [C.POINTER(OScene), C.c_void_p]
        L.oracle_render.restype = C.c_int
        L.oracle_render.argtypes = [C.POINTER(OScene), C.POINTER(OOut)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


# ----------------------------------------------------------------------------- building blocks

def warp(t, t_near, t_far) -> float:
    return lib().oracle_warp(float(t), float(t_near), float(t_far))


def chord(p4x3, o, d):
    """Chord [t0, t1] of the ray o + t d through the tet with vertices p4x3, or None."""
    p = np.ascontiguousarray(p4x3, dtype=np.float64).reshape(12)
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(2)
    ok = lib().oracle_chord(_ptr(p), _ptr(o), _ptr(d), _ptr(out))
    return (float(out[0]), float(out[1])) if ok else None


def roots(coef) -> np.ndarray:
    """Real parts of the roots of sum_j coef[j] x^j."""
    c = np.ascontiguousarray(coef, dtype=np.float64)
    r = np.zeros(max(len(c) - 1, 1))
    k = lib().oracle_roots(_ptr(c), len(c) - 1, _ptr(r))
    return r[:k]


def bound(b, alpha, bias, eta, zf):
    """Moment bound of Alg. 3 for the moment vector b[0..m] at warped depth zf.

    Returns (F, nodes[n+1], weights[n+1], flags) with flags bit0 = empty pixel,
    bit1 = single-depth (rank-one) branch, bit2 = non-positive pivot floored.
    """
    b = np.ascontiguousarray(b, dtype=np.float64)
    m = len(b) - 1
    bias = np.zeros(8) if bias is None else np.ascontiguousarray(np.pad(np.asarray(bias, np.float64), (0, 8 - m)))
    nodes = np.zeros(m // 2 + 1)
    weights = np.zeros(m // 2 + 1)
    flags = C.c_int(0)
    F = lib().oracle_bound(_ptr(b), m, float(alpha), _ptr(bias), float(eta), float(zf), _ptr(nodes),
                           _ptr(weights), C.byref(flags))
    return F, nodes, weights, flags.value


# ----------------------------------------------------------------------------- renderer

def _scene_struct(sc, keep):
    mesh = sc.mesh
    xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float32)
    scal = np.ascontiguousarray(mesh.scalar, dtype=np.float32)
    tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
    sub = np.ascontiguousarray(mesh.tet_sub, dtype=np.int32)
    tf = np.ascontiguousarray(sc.tf, dtype=np.float32)
    keep += [xyz, scal, tets, sub, tf]
    v = sc.view
    ov = OView(width=v["width"], height=v["height"], projection=v["projection"], pad=0,
               eye=(C.c_double * 3)(*v["eye"]), dir=(C.c_double * 3)(*v["dir"]),
               right=(C.c_double * 3)(*v["right"]), down=(C.c_double * 3)(*v["down"]))
    bias = np.zeros(8)
    bias[:sc.m] = sc.bias
    return OScene(n_vertices=mesh.n_vertices, n_tets=mesh.n_tets, n_sub=mesh.n_sub, n_tf=tf.shape[0],
                  xyz=_ptr(xyz), scalar=_ptr(scal), tets=_ptr(tets), tet_sub=_ptr(sub), tf=_ptr(tf),
                  s_min=sc.s_min, s_max=sc.s_max, kappa=sc.kappa, amax=sc.absorbance_max, step=sc.step,
                  view=ov, m=sc.m, renormalize=sc.renormalize, alpha=sc.alpha, eta=sc.eta,
                  bias=(C.c_double * 8)(*bias))


def depth_range(sc):
    keep = []
    s = _scene_struct(sc, keep)
    out = np.zeros(2)
    lib().oracle_depth_range(C.byref(s), _ptr(out))
    return float(out[0]), float(out[1])


def render(sc, pixels=None, pass2=True, exact=False, per_sub=False, threads=None, segments=False) -> dict:
    """Render a scene (see synth.Scene) in FP64.

    pixels: optional int64 array of pixel ids (row*W + col); default all pixels.
    Returns a dict with 'moments' [m+1, P], 'color' [P, 4] (additive sums),
    'rgba' [P, 4], optionally 'moments_sub' [S, m+1, P], 'color_sub' [S, P, 4],
    'exact' [P, 4], 'segments' [2, P] (segments per pixel ray, subdomains it
    meets), plus counters.  P is the number of rendered pixels.
    """
    keep = []
    s = _scene_struct(sc, keep)
    W, H = sc.view["width"], sc.view["height"]
    S, M1 = sc.mesh.n_sub, sc.m + 1
    if pixels is None:
        P = W * H
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        P = pix.size
    res = {"moments": np.zeros((M1, P)), "pieces_sub": np.zeros(S, dtype=np.int64)}
    if per_sub:
        res["moments_sub"] = np.zeros((S, M1, P))
    if segments:
        res["segments"] = np.zeros((2, P), dtype=np.int32)
    if pass2:
        res["color"] = np.zeros((P, 4))
        res["rgba"] = np.zeros((P, 4))
        if per_sub:
            res["color_sub"] = np.zeros((S, P, 4))
        if exact:
            res["exact"] = np.zeros((P, 4))
    threads = threads or (os.cpu_count() or 1)
    out = OOut(pixels=_ptr(pix), n_pixels=P, do_pass2=int(pass2), do_exact=int(exact), n_threads=threads,
               pad=0, moments_sub=_ptr(res.get("moments_sub")), moments=_ptr(res["moments"]),
               color_sub=_ptr(res.get("color_sub")), color=_ptr(res.get("color")), rgba=_ptr(res.get("rgba")),
               exact=_ptr(res.get("exact")), pieces_sub=_ptr(res["pieces_sub"]),
               segments=_ptr(res.get("segments")))
    rc = lib().oracle_render(C.byref(s), C.byref(out))
    if rc != 0:
        raise RuntimeError("oracle_render failed with code %d" % rc)
    res.update(n_pieces=out.n_pieces, n_chords=out.n_chords, n_nonpd=out.n_nonpd, n_rank1=out.n_rank1,
               t_near=out.t_near, t_far=out.t_far, threads=threads)
    return res
