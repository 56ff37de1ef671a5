"""Python binding of libapc.so, the MI355X (gfx950) library for the data-parallel
hot path of Approximate Puzzlepiece Compositing (see include/apc.h).

This module only marshals arguments: every step of the path (binning, tet
walk, moments, sums, moment-bound resolve) runs in the library's HIP kernels.
PyTorch supplies device memory and streams.  There is no CPU fallback: if
libapc.so is missing or cannot be loaded the import of any entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapc.so")

APC_ORTHOGRAPHIC = 0
APC_PERSPECTIVE = 1
APC_FINALIZE = 1
APC_MOMENTS_F16 = 2
APC_MOMENTS_GLOBAL = 8
APC_KEEP_PIECES = 16
APC_BY_PAIR = 32  # apc_resolve_pass: a workgroup per (tile, subdomain) pair, then the ordered colour sum
APC_DEVICE_NONE = -1   # apc_create: a host-only context (validates, launches nothing)
APC_MESH_DEVICE = 1    # apc_mesh_desc.flags: the mesh arrays are device memory
APC_DISPATCH_GRID = 0   # apc_set_dispatch: one workgroup per tile
APC_DISPATCH_QUEUE = 1  # apc_set_dispatch: persistent workgroups taking tiles from a work queue
STATUS = {0: "APC_OK", 1: "APC_E_ARG", 2: "APC_E_MESH", 3: "APC_E_NOMEM", 4: "APC_E_DEVICE",
          5: "APC_E_NUMERIC", 6: "APC_E_UNSUPPORTED"}
EXPORTS = ["apc_create", "apc_destroy", "apc_last_error", "apc_version", "apc_load_mesh", "apc_free_mesh",
           "apc_mesh_get_info", "apc_mesh_subdomain_info", "apc_moments_pass", "apc_sum_moments",
           "apc_resolve_pass", "apc_sum_images", "apc_pack_moments_f16", "apc_segment_counts", "apc_get_counters",
           "apc_get_timings", "apc_set_tile_shape", "apc_get_tile_shape", "apc_autotune_tile_shape",
           "apc_frame_graph_create", "apc_frame_graph_launch", "apc_frame_graph_counters", "apc_frame_graph_destroy",
           "apc_set_workspace_limit", "apc_resolve_pass_noalloc", "apc_get_workspace_bytes", "apc_set_dispatch",
           "apc_get_dispatch", "apc_moments_pass_tiles", "apc_sum_moment_tiles", "apc_autotune_launch",
           "apc_moments_pass_pairs"]


class ApcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_tets", C.c_int64), ("n_subdomains", C.c_int32),
                ("flags", C.c_int32), ("xyz", C.c_void_p), ("scalar", C.c_void_p),
                ("tet_vertices", C.c_void_p), ("tet_subdomain", C.c_void_p)]


class MeshInfo(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_tets", C.c_int64), ("n_boundary_faces", C.c_int64),
                ("n_subdomains", C.c_int32), ("pad", C.c_int32), ("bbox_lo", C.c_double * 3),
                ("bbox_hi", C.c_double * 3), ("device_bytes", C.c_int64)]


class View(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("projection", C.c_int32), ("pad", C.c_int32),
                ("eye", C.c_double * 3), ("dir", C.c_double * 3), ("right", C.c_double * 3),
                ("down", C.c_double * 3), ("t_near", C.c_double), ("t_far", C.c_double), ("step", C.c_double)]


class TF(C.Structure):
    _fields_ = [("n_entries", C.c_int32), ("pad", C.c_int32), ("rgba", C.c_void_p), ("s_min", C.c_float),
                ("s_max", C.c_float), ("kappa", C.c_float), ("absorbance_max", C.c_float)]


class Mboit(C.Structure):
    _fields_ = [("m", C.c_int32), ("renormalize", C.c_int32), ("alpha", C.c_double), ("bias", C.c_double * 8),
                ("eta", C.c_double)]


class Timings(C.Structure):
    _fields_ = [("bin_ms", C.c_double), ("moments_ms", C.c_double), ("sum_ms", C.c_double),
                ("resolve_ms", C.c_double), ("rewalk_ms", C.c_double), ("eval_ms", C.c_double)]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("pieces", "tet_steps", "entries", "bin_records", "walk_step_limit",
                                         "exit_fallback", "entry_overflow", "nonpd_pivots",
                                         "table_samples", "table_fallback", "segments")]


_lib = None


def lib():
    """Load libapc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libapc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        vp = C.c_void_p
        L.apc_version.restype = C.c_char_p
        L.apc_last_error.restype = C.c_char_p
        L.apc_last_error.argtypes = [vp]
        L.apc_create.restype = st
        L.apc_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.apc_destroy.restype = st
        L.apc_destroy.argtypes = [vp]
        L.apc_load_mesh.restype = st
        L.apc_load_mesh.argtypes = [vp, C.POINTER(MeshDesc), C.POINTER(vp), vp]
        L.apc_free_mesh.restype = st
        L.apc_free_mesh.argtypes = [vp, vp]
        L.apc_mesh_get_info.restype = st
        L.apc_mesh_get_info.argtypes = [vp, C.POINTER(MeshInfo)]
        L.apc_mesh_subdomain_info.restype = st
        L.apc_mesh_subdomain_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.apc_moments_pass.restype = st
        L.apc_moments_pass.argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.c_int32, vp, C.c_int32, vp,
                                       C.c_uint32, vp]
        L.apc_sum_moments.restype = st
        L.apc_sum_moments.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
        for name in ("apc_moments_pass_tiles", "apc_moments_pass_pairs"):
            getattr(L, name).restype = st
            getattr(L, name).argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.c_int32, vp, C.c_int32, vp, vp,
                                         C.c_int64, C.POINTER(C.c_int64), vp]
        L.apc_sum_moment_tiles.restype = st
        L.apc_sum_moment_tiles.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                           C.c_int32, vp, vp]
        L.apc_resolve_pass.restype = st
        L.apc_resolve_pass.argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.POINTER(Mboit), vp, vp,
                                       C.c_int32, vp, C.c_uint32, vp]
        L.apc_get_workspace_bytes.restype = st
        L.apc_get_workspace_bytes.argtypes = [vp, C.POINTER(C.c_int64)]
        L.apc_resolve_pass_noalloc.restype = st
        L.apc_resolve_pass_noalloc.argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.POINTER(Mboit), vp, vp,
                                               C.c_int32, vp, C.c_uint32, vp]
        L.apc_pack_moments_f16.restype = st
        L.apc_pack_moments_f16.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp]
        L.apc_set_workspace_limit.restype = st
        L.apc_set_workspace_limit.argtypes = [vp, C.c_int64]
        L.apc_frame_graph_create.restype = st
        L.apc_frame_graph_create.argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.POINTER(Mboit), vp, C.c_int32,
                                             vp, vp, vp, C.c_uint32, C.POINTER(vp)]
        L.apc_frame_graph_launch.restype = st
        L.apc_frame_graph_launch.argtypes = [vp, vp]
        L.apc_frame_graph_counters.restype = st
        L.apc_frame_graph_counters.argtypes = [vp, C.POINTER(Counters), C.c_int32]
        L.apc_frame_graph_destroy.restype = st
        L.apc_frame_graph_destroy.argtypes = [vp]
        L.apc_set_tile_shape.restype = st
        L.apc_set_tile_shape.argtypes = [vp, C.c_int32]
        L.apc_get_tile_shape.restype = st
        L.apc_get_tile_shape.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.apc_set_dispatch.restype = st
        L.apc_set_dispatch.argtypes = [vp, C.c_int32]
        L.apc_get_dispatch.restype = st
        L.apc_get_dispatch.argtypes = [vp, C.POINTER(C.c_int32)]
        L.apc_autotune_tile_shape.restype = st
        L.apc_autotune_tile_shape.argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.POINTER(Mboit), vp,
                                              C.c_int32, vp, vp, C.c_int32, C.POINTER(C.c_int32), vp, vp]
        L.apc_autotune_launch.restype = st
        L.apc_autotune_launch.argtypes = [vp, vp, C.POINTER(View), C.POINTER(TF), C.POINTER(Mboit), vp, C.c_int32,
                                          vp, vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp, vp]
        L.apc_segment_counts.restype = st
        L.apc_segment_counts.argtypes = [vp, vp, C.c_int32, C.c_int32, vp]
        L.apc_sum_images.restype = st
        L.apc_sum_images.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, C.POINTER(Mboit), vp, vp]
        L.apc_get_counters.restype = st
        L.apc_get_counters.argtypes = [vp, C.POINTER(Counters), C.c_int32]
        L.apc_get_timings.restype = st
        L.apc_get_timings.argtypes = [vp, C.POINTER(Timings)]
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != 0:
        raise ApcError(status, lib().apc_last_error(ctx).decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError("%s must be contiguous %s" % (name, dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return C.c_void_p(t.data_ptr())


def _ids(subdomains):
    a = np.ascontiguousarray(np.asarray(subdomains, dtype=np.int32).ravel())
    return a, C.c_void_p(a.ctypes.data)


def make_view(view: dict, step: float, t_near: float = 0.0, t_far: float = 0.0) -> View:
    """apc_view from a camera dict with width, height, projection, eye, dir, right, down."""
    return View(width=int(view["width"]), height=int(view["height"]), projection=int(view["projection"]), pad=0,
                eye=(C.c_double * 3)(*map(float, view["eye"])), dir=(C.c_double * 3)(*map(float, view["dir"])),
                right=(C.c_double * 3)(*map(float, view["right"])), down=(C.c_double * 3)(*map(float, view["down"])),
                t_near=float(t_near), t_far=float(t_far), step=float(step))


def make_tf(rgba_dev, s_min, s_max, kappa, absorbance_max) -> TF:
    import torch
    ptr = _dev_ptr(rgba_dev, torch.float32, name="tf table")
    return TF(n_entries=int(rgba_dev.shape[0]), pad=0, rgba=ptr, s_min=float(s_min), s_max=float(s_max),
              kappa=float(kappa), absorbance_max=float(absorbance_max))


def make_mboit(m, alpha, bias, eta, renormalize=1) -> Mboit:
    b = np.zeros(8)
    b[:m] = np.asarray(bias, dtype=np.float64)[:m]
    return Mboit(m=int(m), renormalize=int(renormalize), alpha=float(alpha), bias=(C.c_double * 8)(*b),
                 eta=float(eta))


class Mesh:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle

    def info(self) -> dict:
        mi = MeshInfo()
        _check(lib().apc_mesh_get_info(self.handle, C.byref(mi)))
        return dict(n_vertices=mi.n_vertices, n_tets=mi.n_tets, n_boundary_faces=mi.n_boundary_faces,
                    n_subdomains=mi.n_subdomains, bbox_lo=tuple(mi.bbox_lo), bbox_hi=tuple(mi.bbox_hi),
                    device_bytes=mi.device_bytes)

    def subdomain_info(self, sub) -> tuple:
        nt, nf = C.c_int64(0), C.c_int64(0)
        _check(lib().apc_mesh_subdomain_info(self.handle, int(sub), C.byref(nt), C.byref(nf)))
        return nt.value, nf.value

    def free(self):
        if self.handle:
            lib().apc_free_mesh(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """One library context on a HIP device (apc_create)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().apc_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().apc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, st):
        _check(st, self.handle)

    def load_mesh(self, xyz, scalar, tets, tet_sub, n_sub, stream=None) -> Mesh:
        """Host arrays (numpy), or device arrays (CUDA torch tensors, APC_MESH_DEVICE)."""
        dev = all(getattr(a, "is_cuda", False) for a in (xyz, scalar, tets, tet_sub))
        if dev:
            import torch
            xyz_p = _dev_ptr(xyz, torch.float32, name="xyz")
            sc_p = _dev_ptr(scalar, torch.float32, name="scalar")
            tv_p = _dev_ptr(tets, torch.int32, name="tets")
            ts_p = _dev_ptr(tet_sub, torch.int32, name="tet_sub")
            nv, nt = xyz.shape[0], tets.shape[0]
        else:
            xyz = np.ascontiguousarray(xyz, dtype=np.float32)
            scalar = np.ascontiguousarray(scalar, dtype=np.float32)
            tets = np.ascontiguousarray(tets, dtype=np.int32)
            tet_sub = np.ascontiguousarray(tet_sub, dtype=np.int32)
            xyz_p, sc_p, tv_p, ts_p = (a.ctypes.data for a in (xyz, scalar, tets, tet_sub))
            nv, nt = xyz.shape[0], tets.shape[0]
        d = MeshDesc(n_vertices=nv, n_tets=nt, n_subdomains=int(n_sub), flags=APC_MESH_DEVICE if dev else 0,
                     xyz=xyz_p, scalar=sc_p, tet_vertices=tv_p, tet_subdomain=ts_p)
        h = C.c_void_p()
        self._ck(lib().apc_load_mesh(self.handle, C.byref(d), C.byref(h), _stream(stream)))
        return Mesh(self, h)

    def moments_pass(self, mesh, view: View, tf: TF, m, subdomains, out, stream=None, keep=False,
                     global_sum=False):
        """Stage one; with keep its pieces are kept for the resolve pass of the same frame (APC_KEEP_PIECES).
        With global_sum (ascending subdomain ids), `out` is the global [m+1][H][W] image, summed by stage one
        itself (bitwise what sum_moments gives for the per-subdomain images), instead of [n][m+1][H][W]."""
        import torch
        ids, ptr = _ids(subdomains)
        shape = (m + 1, view.height, view.width) if global_sum else (len(ids), m + 1, view.height, view.width)
        flags = (APC_KEEP_PIECES if keep else 0) | (APC_MOMENTS_GLOBAL if global_sum else 0)
        self._ck(lib().apc_moments_pass(self.handle, mesh.handle, C.byref(view), C.byref(tf), int(m), ptr,
                                        len(ids), _dev_ptr(out, torch.float32, shape,
                                                           "moments" if global_sum else "moments_per_sub"),
                                        flags, _stream(stream)))

    def moments_pass_tiles(self, mesh, view: View, tf: TF, m, subdomains, tiles=None, pair_bin=None, stream=None,
                           by_pair=False):
        """Stage one in the tiles form (ascending subdomain ids): tiles [P][m+1][64] FP32 and pair_bin [P] int32
        for the P (tile, subdomain) pairs with binned faces.  Without buffers only counts the pairs.  Returns
        the pair count (raises ApcError, status APC_E_NOMEM, when the buffers are too small).  by_pair: a
        workgroup per pair (apc_moments_pass_pairs) instead of one per tile; the same tiles."""
        import torch
        ids, ptr = _ids(subdomains)
        n = C.c_int64(0)
        if tiles is None:
            tp, bp, cap = None, None, 0
        else:
            cap = int(tiles.shape[0])
            tp = _dev_ptr(tiles, torch.float32, (cap, m + 1, 64), "tiles")
            bp = _dev_ptr(pair_bin, torch.int32, (cap,), "pair_bin")
        fn = lib().apc_moments_pass_pairs if by_pair else lib().apc_moments_pass_tiles
        self._ck(fn(self.handle, mesh.handle, C.byref(view), C.byref(tf), int(m), ptr, len(ids), tp, bp, cap,
                    C.byref(n), _stream(stream)))
        return n.value

    def sum_moment_tiles(self, tiles, pair_bin, n_pairs, n_sub, m, height, width, out, stream=None):
        """Global [m+1][H][W] moments from the first n_pairs tiles (tile shape of this context)."""
        import torch
        tp = _dev_ptr(tiles, torch.float32, name="tiles") if n_pairs > 0 else None
        bp = _dev_ptr(pair_bin, torch.int32, name="pair_bin") if n_pairs > 0 else None
        if n_pairs > 0 and (tiles.numel() < n_pairs * (m + 1) * 64 or pair_bin.numel() < n_pairs):
            raise ValueError("tiles / pair_bin hold fewer than n_pairs pairs")
        self._ck(lib().apc_sum_moment_tiles(self.handle, tp, bp, int(n_pairs), int(n_sub), int(m), int(height),
                                            int(width), self.tile_shape()[0],
                                            _dev_ptr(out, torch.float32, (m + 1, height, width), "moments"),
                                            _stream(stream)))

    def sum_moments(self, per_sub, m, subdomains, out, stream=None):
        import torch
        n, m1, H, W = per_sub.shape
        ids, ptr = (None, None) if subdomains is None else _ids(subdomains)
        self._ck(lib().apc_sum_moments(self.handle, _dev_ptr(per_sub, torch.float32, name="moments_per_sub"), n,
                                       int(m), H, W, ptr, _dev_ptr(out, torch.float32, (m1, H, W), "moments"),
                                       _stream(stream)))

    def resolve_pass(self, mesh, view: View, tf: TF, mboit: Mboit, moments, subdomains, out, finalize=True,
                     stream=None, by_pair=False):
        """`moments`: the FP32 global image, or (torch.float16) the packed image of pack_moments_f16.
        by_pair: APC_BY_PAIR (plain form, FP32 moments)."""
        import torch
        ids, ptr = _ids(subdomains)
        f16 = moments.dtype == torch.float16
        flags = (APC_FINALIZE if finalize else 0) | (APC_MOMENTS_F16 if f16 else 0) | (APC_BY_PAIR if by_pair else 0)
        self._ck(lib().apc_resolve_pass(self.handle, mesh.handle, C.byref(view), C.byref(tf), C.byref(mboit),
                                        _dev_ptr(moments, torch.float16 if f16 else torch.float32,
                                                 (mboit.m + (3 if f16 else 1), view.height, view.width),
                                                 "moments"), ptr, len(ids),
                                        _dev_ptr(out, torch.float32, (view.height, view.width, 4), "rgba"),
                                        flags, _stream(stream)))

    def resolve_pass_noalloc(self, mesh, view: View, tf: TF, mboit: Mboit, moments, subdomains, out, finalize=True,
                             stream=None):
        """apc_resolve_pass_noalloc: the plain-form resolve with its binning state in the library's static
        device workspace (no device allocation)."""
        import torch
        ids, ptr = _ids(subdomains)
        f16 = moments.dtype == torch.float16
        flags = (APC_FINALIZE if finalize else 0) | (APC_MOMENTS_F16 if f16 else 0)
        self._ck(lib().apc_resolve_pass_noalloc(
            self.handle, mesh.handle, C.byref(view), C.byref(tf), C.byref(mboit),
            _dev_ptr(moments, torch.float16 if f16 else torch.float32,
                     (mboit.m + (3 if f16 else 1), view.height, view.width), "moments"), ptr, len(ids),
            _dev_ptr(out, torch.float32, (view.height, view.width, 4), "rgba"), flags, _stream(stream)))

    def workspace_bytes(self) -> int:
        """Device memory the context holds now (apc_get_workspace_bytes)."""
        b = C.c_int64(0)
        self._ck(lib().apc_get_workspace_bytes(self.handle, C.byref(b)))
        return b.value

    def set_workspace_limit(self, nbytes):
        """Cap the kept-piece pool (APC_KEEP_PIECES) at nbytes (0: default policy)."""
        self._ck(lib().apc_set_workspace_limit(self.handle, int(nbytes)))

    def set_dispatch(self, mode):
        """APC_DISPATCH_GRID (one workgroup per tile) or APC_DISPATCH_QUEUE (persistent work queue)."""
        self._ck(lib().apc_set_dispatch(self.handle, int(mode)))

    def dispatch(self):
        v = C.c_int32(0)
        self._ck(lib().apc_get_dispatch(self.handle, C.byref(v)))
        return v.value

    def set_tile_shape(self, tile_width):
        self._ck(lib().apc_set_tile_shape(self.handle, int(tile_width)))

    def tile_shape(self):
        w, h = C.c_int32(0), C.c_int32(0)
        self._ck(lib().apc_get_tile_shape(self.handle, C.byref(w), C.byref(h)))
        return w.value, h.value

    def autotune_tile_shape(self, mesh, view: View, tf: TF, mboit: Mboit, subdomains, moments, rgba, repeats=2,
                            stream=None):
        """Time whole frames (stage one summing the subdomains, then the finalising resolve) for tile widths
        2..32 and keep the fastest; moments [m+1][H][W] and rgba [H][W][4] are scratch.  Returns
        (width, {width: frame ms})."""
        import torch
        ids, ptr = _ids(subdomains)
        best = C.c_int32(0)
        ms = np.full(7, -1.0, dtype=np.float32)
        self._ck(lib().apc_autotune_tile_shape(self.handle, mesh.handle, C.byref(view), C.byref(tf),
                                               C.byref(mboit), ptr, len(ids),
                                               _dev_ptr(moments, torch.float32, name="moments"),
                                               _dev_ptr(rgba, torch.float32, name="rgba"), int(repeats),
                                               C.byref(best), C.c_void_p(ms.ctypes.data), _stream(stream)))
        return best.value, {1 << k: float(ms[k]) for k in range(7) if ms[k] >= 0}

    def autotune_launch(self, mesh, view: View, tf: TF, mboit: Mboit, subdomains, moments, rgba, repeats=1,
                        stream=None):
        """The tile-width search of autotune_tile_shape for both dispatch modes; sets the fastest width and mode.
        Returns (width, mode, {(mode, width): frame ms})."""
        import torch
        ids, ptr = _ids(subdomains)
        best, mode = C.c_int32(0), C.c_int32(0)
        ms = np.full(14, -1.0, dtype=np.float32)
        self._ck(lib().apc_autotune_launch(self.handle, mesh.handle, C.byref(view), C.byref(tf), C.byref(mboit), ptr,
                                           len(ids), _dev_ptr(moments, torch.float32, name="moments"),
                                           _dev_ptr(rgba, torch.float32, name="rgba"), int(repeats), C.byref(best),
                                           C.byref(mode), C.c_void_p(ms.ctypes.data), _stream(stream)))
        table = {(d, 1 << k): float(ms[d * 7 + k]) for d in range(2) for k in range(7) if ms[d * 7 + k] >= 0}
        return best.value, mode.value, table

    def segment_counts(self, height, width, stream=None):
        """[2][H][W] int32 of the last stage one: segments per pixel, subdomains met per pixel."""
        import torch
        out = torch.empty((2, height, width), dtype=torch.int32, device="cuda:%d" % self.device)
        self._ck(lib().apc_segment_counts(self.handle, _dev_ptr(out, torch.int32, name="segments"), height, width,
                                          _stream(stream)))
        return out

    def pack_moments_f16(self, moments, m, out, stream=None):
        """FP16 form of a global moment image ([m+3][H][W]): ln b0 and the mean depth, each as two halves, and
        the central moments of orders 2..m (include/apc.h)."""
        import torch
        m1, H, W = moments.shape
        self._ck(lib().apc_pack_moments_f16(self.handle, _dev_ptr(moments, torch.float32, (m1, H, W), "moments"),
                                            int(m), H, W, _dev_ptr(out, torch.float16, (m1 + 2, H, W), "packed"),
                                            _stream(stream)))

    def sum_images(self, partials, subdomains, moments, mboit: Mboit, out, stream=None):
        import torch
        n, H, W, _ = partials.shape
        ids, ptr = (None, None) if subdomains is None else _ids(subdomains)
        self._ck(lib().apc_sum_images(self.handle, _dev_ptr(partials, torch.float32, name="partials"), n, H, W,
                                      ptr, _dev_ptr(moments, torch.float32, name="moments"), C.byref(mboit),
                                      _dev_ptr(out, torch.float32, (H, W, 4), "rgba"), _stream(stream)))

    def timings(self) -> dict:
        t = Timings()
        self._ck(lib().apc_get_timings(self.handle, C.byref(t)))
        return {n: getattr(t, n) for n, _ in Timings._fields_}

    def counters(self, reset=False) -> dict:
        c = Counters()
        self._ck(lib().apc_get_counters(self.handle, C.byref(c), int(bool(reset))))
        return {n: getattr(c, n) for n, _ in Counters._fields_}


class FrameGraph:
    """A whole frame of a Renderer captured in a HIP graph (apc_frame_graph_create): one launch per frame,
    writing the Renderer's moment and image buffers."""

    def __init__(self, renderer, finalize=True, global_sum=False, keep=False):
        """global_sum: stage one sums the subdomains itself (per_sub is not written); keep: stage two evaluates
        the pieces stage one kept instead of walking again."""
        import torch
        r = renderer
        ids, ptr = _ids(r.subs)
        self._ids = ids
        h = C.c_void_p()
        _check(lib().apc_frame_graph_create(
            r.ctx.handle, r.mesh.handle, C.byref(r.view), C.byref(r.tf), C.byref(r.mboit), ptr, len(ids),
            None if global_sum else _dev_ptr(r.per_sub, torch.float32, name="moments_per_sub"),
            _dev_ptr(r.moments, torch.float32, name="moments"), _dev_ptr(r.rgba, torch.float32, name="rgba"),
            (APC_FINALIZE if finalize else 0) | (APC_MOMENTS_GLOBAL if global_sum else 0) |
            (APC_KEEP_PIECES if keep else 0), C.byref(h)), r.ctx.handle)
        self.handle = h
        self.renderer = r

    def launch(self, stream=None):
        _check(lib().apc_frame_graph_launch(self.handle, _stream(stream)))
        return self.renderer.rgba

    def counters(self, reset=False) -> dict:
        c = Counters()
        _check(lib().apc_frame_graph_counters(self.handle, C.byref(c), int(bool(reset))))
        return {name: getattr(c, name) for name, _ in Counters._fields_}

    def close(self):
        if self.handle:
            lib().apc_frame_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Renderer:
    """A resident mesh plus the per-scene device buffers of one workload.

    `frame()` runs the whole hot path once: stage one for all subdomains, the
    canonical moment sum, stage two with the final renormalised image.
    """

    def __init__(self, ctx: Context, scene, device="cuda"):
        import torch
        self.ctx = ctx
        self.scene = scene
        mesh = scene.mesh
        self.mesh = ctx.load_mesh(mesh.xyz, mesh.scalar, mesh.tets, mesh.tet_sub, mesh.n_sub)
        self.tf_dev = torch.as_tensor(np.ascontiguousarray(scene.tf, dtype=np.float32), device=device)
        self.view = make_view(scene.view, scene.step)
        self.tf = make_tf(self.tf_dev, scene.s_min, scene.s_max, scene.kappa, scene.absorbance_max)
        self.mboit = make_mboit(scene.m, scene.alpha, scene.bias, scene.eta, scene.renormalize)
        self.subs = np.arange(mesh.n_sub, dtype=np.int32)
        H, W, m = self.view.height, self.view.width, scene.m
        self._per_sub = None  # [S][m+1][H][W], allocated by the first frame that needs it (separate sum)
        self._device = device
        self.moments = torch.empty((m + 1, H, W), dtype=torch.float32, device=device)
        self.rgba = torch.empty((H, W, 4), dtype=torch.float32, device=device)
        self._tiles = self._pair_bin = None  # the tiles form's buffers (stage one by pairs), grown on demand

    @property
    def per_sub(self):
        """Per-subdomain moment images of the separate-sum form (17 GB at 2560^2, m = 8, 72 subdomains)."""
        if self._per_sub is None:
            import torch
            m1, H, W = self.moments.shape
            self._per_sub = torch.empty((len(self.subs), m1, H, W), dtype=torch.float32, device=self._device)
        return self._per_sub

    def moments_by_pair(self, subs, stream=None):
        """Stage one by (tile, subdomain) pairs into the tiles form, then their ordered FP64 sum into
        self.moments: bitwise the global moments of the other forms (ascending subdomain ids)."""
        import torch
        m = self.scene.m
        while True:
            if self._tiles is not None:
                try:
                    n = self.ctx.moments_pass_tiles(self.mesh, self.view, self.tf, m, subs, self._tiles,
                                                    self._pair_bin, stream, by_pair=True)
                    break
                except ApcError as e:
                    if e.status != 3:  # APC_E_NOMEM: grow the buffers below
                        raise
            n = self.ctx.moments_pass_tiles(self.mesh, self.view, self.tf, m, subs, stream=stream)
            cap = max(64, n + n // 4)
            dev = self.moments.device
            self._tiles = self._pair_bin = None
            self._tiles = torch.empty((cap, m + 1, 64), dtype=torch.float32, device=dev)
            self._pair_bin = torch.empty((cap,), dtype=torch.int32, device=dev)
        H, W = self.moments.shape[1:]
        self.ctx.sum_moment_tiles(self._tiles, self._pair_bin, n, len(subs), m, H, W, self.moments, stream)
        return n

    def frame(self, subdomains=None, finalize=True, stream=None, moments_f16=False, keep=False, global_sum=False,
              by_pair=False, resolve_by_pair=False):
        """One frame.  moments_f16: the resolve reads the FP16-packed moment image (self.moments_h); keep:
        stage one keeps its pieces and stage two evaluates them (else stage two walks the rays again, the
        plain form); global_sum (all subdomains, ascending): stage one writes the global moments itself and
        self.per_sub is not written; by_pair (ascending subdomains, no keep): stage one walks the (tile,
        subdomain) pairs in parallel into the tiles form and their ordered sum gives the global moments
        (the same bits); resolve_by_pair (plain form, FP32 moments): stage two walks the pairs in parallel
        too and sums their colours in order (the image to FP32 rounding)."""
        subs = self.subs if subdomains is None else np.asarray(subdomains, np.int32)
        if by_pair:
            if keep:
                raise ValueError("stage one by pairs keeps no pieces")
            self.moments_by_pair(subs, stream)
        elif global_sum:
            self.ctx.moments_pass(self.mesh, self.view, self.tf, self.scene.m, subs, self.moments, stream,
                                  keep=keep, global_sum=True)
        else:
            per_sub = self.per_sub if len(subs) == len(self.subs) else self.per_sub[:len(subs)]
            self.ctx.moments_pass(self.mesh, self.view, self.tf, self.scene.m, subs, per_sub, stream, keep=keep)
            self.ctx.sum_moments(per_sub, self.scene.m, subs, self.moments, stream)
        mom = self.moments
        if moments_f16:
            import torch
            if getattr(self, "moments_h", None) is None:
                m1, H, W = self.moments.shape
                self.moments_h = torch.empty((m1 + 2, H, W), dtype=torch.float16, device=self.moments.device)
            self.ctx.pack_moments_f16(self.moments, self.scene.m, self.moments_h, stream)
            mom = self.moments_h
        self.ctx.resolve_pass(self.mesh, self.view, self.tf, self.mboit, mom, subs, self.rgba,
                              finalize=finalize, stream=stream, by_pair=resolve_by_pair)
        return self.rgba
