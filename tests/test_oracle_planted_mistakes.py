"""The oracle's pins catch plausible mistakes (CPU).  Each case copies oracle.cpp with one mistake planted
-- a dropped term, a wrong sign or index, a transposed operand -- compiles it, and runs the pin suite
(tests/test_oracle_pins.py) against that build: at least one pin must fail.  The mistakes live only in the
temporary copies; the oracle itself is untouched.  A case whose snippet no longer occurs in oracle.cpp fails,
so the list follows the source."""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

# (name, exact snippet of oracle.cpp, the same with the mistake)
MISTAKES = [
    ("warp runs from the far end",
     "2.0 * (std::log(t) - std::log(t_near))", "2.0 * (std::log(t_far) - std::log(t))"),
    ("face normal not turned outward", "if (dot(p[f] - a, n) > 0) n = -1.0 * n;", "if (dot(p[f] - a, n) < 0) n = -1.0 * n;"),
    ("barycentric weights of two vertices swapped",
     "sv[2] * l2 + sv[3] * l3", "sv[2] * l3 + sv[3] * l2"),
    ("transfer-function interpolation weights swapped",
     "(1.0 - f) * s.tf[4 * i0 + c] + f * s.tf[4 * (i0 + 1) + c]",
     "f * s.tf[4 * i0 + c] + (1.0 - f) * s.tf[4 * (i0 + 1) + c]"),
    ("lattice index off by one", "std::floor((t0 - t_near) / s.step) + 1.0", "std::floor((t0 - t_near) / s.step) + 2.0"),
    ("absorbance cap dropped", "std::min(s.kappa * rgba[3] * pc.len, s.amax)", "s.kappa * rgba[3] * pc.len"),
    ("piece depth at its start, not its middle", "pc.tm = 0.5 * (u + v);", "pc.tm = u;"),
    ("moment powers shifted by one", "double zp = 1.0;\n          for (int j = 0; j <= m; ++j) {\n            bl[j]",
     "double zp = z;\n          for (int j = 0; j <= m; ++j) {\n            bl[j]"),
    ("bias mixing without the (1 - alpha) factor", "(1.0 - alpha) * (b[j] / b[0]) + alpha * bias[j - 1]",
     "(b[j] / b[0]) + alpha * bias[j - 1]"),
    ("Hankel entry index shifted", "double sum = P.bp[j + k];", "double sum = P.bp[j + k + (j > 0)];"),
    ("Cholesky update sign", "sum -= P.L[j][l] * P.L[k][l];", "sum += P.L[j][l] * P.L[k][l];"),
    ("forward substitution with the transposed factor", "sum -= P.L[j][k] * y[k];", "sum -= P.L[k][j] * y[k];"),
    ("back substitution with the untransposed factor", "sum -= P.L[k][j] * q[k];", "sum -= P.L[j][k] * q[k];"),
    ("overestimation weight of the sample's own node dropped", "(i == 0) ? eta :", "(i == 0) ? 0.0 :"),
    ("nodes behind the sample counted instead of those in front", "(x[i] < zf ? 1.0 : 0.0)", "(x[i] > zf ? 1.0 : 0.0)"),
    ("single-depth branch reversed", "return z1 < zf ? 1.0 : 0.0;", "return z1 > zf ? 1.0 : 0.0;"),
    ("polynomial made monic by the wrong coefficient", "a[j] = c[j] / c[deg];", "a[j] = c[j] / c[0];"),
    ("transmittance without b0", "std::exp(-ps.b0 * F)", "std::exp(-F)"),
    ("colour not weighted by transmittance", "cl[c] += T * alpha_p * pc.rgb[c];", "cl[c] += alpha_p * pc.rgb[c];"),
    ("renormalisation dropped", "o4[c] = acc[c] * sc;", "o4[c] = acc[c];"),
    ("subdomain sum keeps only the last subdomain", "sum += bl[sub * M1 + j];", "sum = bl[sub * M1 + j];"),
    ("exact compositing attenuates a piece by itself", "double w = std::exp(-tau) * (-std::expm1(-e.a));",
     "double w = std::exp(-tau - e.a) * (-std::expm1(-e.a));"),
    ("every chord counted as a segment", "if (c[k].first > c[k - 1].second + 1e-9 * (1.0 + std::fabs(c[k - 1].second))) ++segs;",
     "++segs;"),
    ("depth range from half the bounding radius", "t_near = dist - r;", "t_near = dist - 0.5 * r;"),
]


def _run_case(tmp, k, name, old, new):
    src = open(SRC).read()
    if src.count(old) != 1:
        return name, "snippet found %d times" % src.count(old)
    path = os.path.join(tmp, "oracle_%d.cpp" % k)
    open(path, "w").write(src.replace(old, new))
    so = os.path.join(tmp, "liboracle_%d.so" % k)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", so, path])
    env = dict(os.environ, APC_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    return name, None if r.returncode == 1 else "pins passed (exit %d)" % r.returncode


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda a: _run_case(str(tmp_path), *a),
                              [(k,) + m for k, m in enumerate(MISTAKES)]))
    missed = [(n, why) for n, why in results if why]
    assert not missed, missed
