"""The C ABI on the CPU: libapc.so loads, exports every entry point that
include/apc.h declares, and the binding's ctypes structures have the header's
layout (checked against a C program compiled from the header)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apc.h")


@pytest.fixture(scope="module")
def apc():
    import paper_2501_12581_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2501_12581_amd import build
        build.build()
    P.lib()
    return P


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function(apc):
    names = declared_functions()
    assert len(names) >= 14
    lib = C.CDLL(apc.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(apc.EXPORTS) == names


def test_version_string(apc):
    assert b"gfx950" in apc.lib().apc_version()


def test_struct_layouts_match_header(apc, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('''
#include <stdio.h>
#include <stddef.h>
#include "apc.h"
#define P(T, f) printf(#T "." #f " %zu\\n", offsetof(T, f));
int main(void) {
  printf("apc_mesh_desc %zu\\n", sizeof(apc_mesh_desc));
  printf("apc_view %zu\\n", sizeof(apc_view));
  printf("apc_tf %zu\\n", sizeof(apc_tf));
  printf("apc_mboit %zu\\n", sizeof(apc_mboit));
  printf("apc_mesh_info %zu\\n", sizeof(apc_mesh_info));
  printf("apc_counters %zu\\n", sizeof(apc_counters));
  printf("apc_timings %zu\\n", sizeof(apc_timings));
  P(apc_view, step) P(apc_view, t_near) P(apc_tf, rgba) P(apc_tf, absorbance_max)
  P(apc_mboit, eta) P(apc_mboit, bias) P(apc_mesh_desc, tet_subdomain) P(apc_mesh_info, device_bytes)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().splitlines())
    got = {"apc_mesh_desc": apc.MeshDesc, "apc_view": apc.View, "apc_tf": apc.TF, "apc_mboit": apc.Mboit,
           "apc_mesh_info": apc.MeshInfo, "apc_counters": apc.Counters, "apc_timings": apc.Timings}
    for name, cls in got.items():
        assert int(out[name]) == C.sizeof(cls), name
    for key, val in out.items():
        if "." in key:
            sname, field = key.split(".")
            assert getattr(got[sname], field).offset == int(val), key


def test_missing_library_fails_loudly(apc, monkeypatch):
    monkeypatch.setattr(apc, "_lib", None)
    monkeypatch.setattr(apc, "LIB_PATH", "/nonexistent/libapc.so")
    with pytest.raises(ImportError):
        apc.lib()


def test_flag_constants_match_the_header(apc):
    text = open(HEADER).read()
    defs = dict((k, int(v)) for k, v in re.findall(r"#define (APC_[A-Z0-9_]+) (\d+)u\b", text))
    names = ("APC_FINALIZE", "APC_MOMENTS_F16", "APC_MOMENTS_GLOBAL", "APC_KEEP_PIECES")
    for name in names:
        assert getattr(apc, name) == defs[name], name
    flags = [defs[n] for n in names]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == len(flags)  # distinct single bits
