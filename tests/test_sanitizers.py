"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle (oracle/oracle.cpp) is built with both sanitizers and renders
  the tiny workload (both passes, per-subdomain images, exact compositing,
  segment counts) plus its building blocks in a child process.
* The library's host side (argument validation, mesh grouping, host face
  adjacency: csrc/apc_api.cpp) is built with both sanitizers by the host
  compiler and linked with the unsanitized gfx950 kernels; the C-ABI failure
  tests (tests/test_abi_errors.py) then run against it in a child process.

A sanitizer report aborts the child (halt_on_error), which fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _asan_runtime():
    return subprocess.check_output(["g++", "-print-file-name=libasan.so"]).decode().strip()


def _env():
    env = dict(os.environ)
    env["LD_PRELOAD"] = _asan_runtime()  # the runtime must come first in a non-instrumented python
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT
    return env


def _run(code, env, timeout=600):
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=timeout)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-std=c++17", "-fopenmp", "-fPIC", "-shared"] + SAN +
                          ["-o", lib, os.path.join(ROOT, "oracle", "oracle.cpp")])
    env = _env()
    env["APC_ORACLE_LIB"] = lib
    out = _run('''
import numpy as np, oracle, synth
sc = synth.scene_tiny()
r = oracle.render(sc, per_sub=True, exact=True, segments=True, threads=4)
assert r["n_pieces"] > 0 and np.isfinite(r["rgba"]).all()
sub = oracle.render(sc, pixels=np.arange(0, 128 * 128, 97), per_sub=True, threads=2)
for m in (4, 6, 8):
    b = np.array([1.0] + [0.3 ** j for j in range(1, m + 1)])
    for zf in (-0.9, 0.0, 0.31, 0.95):
        oracle.bound(b, 5e-5, synth.default_bias(m), 0.3, zf)
print(oracle.roots([1.0, -3.0, 2.0]), oracle.chord(np.eye(4, 3), (0.1, 0.1, -1.0), (0.0, 0.0, 1.0)))
import os
print("loaded", [l for l in open("/proc/self/maps").read().split() if l.endswith("liboracle_san.so")][:1])
''', env)
    assert "liboracle_san.so" in out


@pytest.mark.slow
def test_library_host_code_under_sanitizers(tmp_path):
    api_o, kern_o = str(tmp_path / "apc_api.o"), str(tmp_path / "apc_kernels.o")
    lib = str(tmp_path / "libapc_san.so")
    csrc = os.path.join(ROOT, "paper_2501_12581_amd", "csrc")
    # host side: the host compiler with both sanitizers (the HIP headers define two of the device-code
    # spellings only for the HIP compiler; the static device workspace becomes a plain host array here,
    # which no host-only call touches)
    subprocess.check_call(["g++", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-D__align__(x)=__attribute__((aligned(x)))", "-DHIP_SYMBOL(X)=X"] + SAN +
                          ["-c", os.path.join(csrc, "apc_api.cpp"), "-o", api_o])
    # kernels: gfx950 code as in the product build, no sanitizer
    hip = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    subprocess.check_call(hip + ["-c", os.path.join(csrc, "apc_kernels.hip"), "-o", kern_o],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call(["g++", "-shared", "-fsanitize=address,undefined", api_o, kern_o, "-L/opt/rocm/lib",
                           "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", lib])
    out = _run('''
import sys, pytest
import paper_2501_12581_amd as P
P.LIB_PATH = %r
rc = pytest.main(["-q", "-p", "no:cacheprovider", "tests/test_abi_errors.py"])
print("loaded", [l for l in open("/proc/self/maps").read().split() if l.endswith("libapc_san.so")][:1])
sys.exit(rc)
''' % lib, _env())
    assert "libapc_san.so" in out and " passed" in out
