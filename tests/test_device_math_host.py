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
