// Host side of the C ABI declared in include/apc.h: argument validation,
// mesh residency (validation, grouping by subdomain, face adjacency on the
// device, per-subdomain boundary faces), per-call frame constants and the
// launch sequence of the two passes.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/apc.h"
#include "apc_internal.h"

using apc::FrameDev;
using apc::MeshDev;
using apc::SlotDev;

namespace {

thread_local std::string g_error = "no error";

apc_status fail(apc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

#define HIPCHK(x)                                                                                \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) return fail(APC_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_)); \
  } while (0)

template <class Fn>
void parallel_for(int64_t n, Fn fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 100000) nt = 1;
  std::vector<std::thread> th;
  for (unsigned k = 0; k < nt; ++k) {
    int64_t lo = n * k / nt, hi = n * (k + 1) / nt;
    th.emplace_back([=] { fn(lo, hi, int(k)); });
  }
  for (auto& t : th) t.join();
}

// Set while a frame is being captured into a HIP graph: workspace buffers
// are sized by an eager frame beforehand and must not be reallocated.
thread_local bool g_frozen = false;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need, bool slack = true) {
    if (need <= bytes) return hipSuccess;
    if (g_frozen) return hipErrorOutOfMemory;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      bytes = 0;
    }
    size_t nb = std::max<size_t>(slack ? need + need / 4 : need, 4096);
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) return e;
    bytes = nb;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

}  // namespace

// ---- the static workspace of apc_resolve_pass_noalloc
//
// Device memory in the library's own code object: every GPU the library runs
// on holds one copy of it (allocated when the code object is loaded, held
// until the process ends).  In host code `scratch` names a host-side stand-in,
// not a device address: its address on each device comes from
// hipGetSymbolAddress at context creation (apc_create), with that device
// current, and only that address is handed to kernels.
namespace {
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
hipError_t g_noalloc_err[NOALLOC_MAX_DEVICES] = {};
bool g_noalloc_done[NOALLOC_MAX_DEVICES] = {};

// once per device, with `device` current
void noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_done[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_noalloc_err[device] = e;
  g_noalloc_ptr[device] = e == hipSuccess ? ptr : nullptr;
  g_noalloc_done[device] = true;
}
}  // namespace

struct apc_ctx_s {
  int device = 0;
  bool host_only = false;  // APC_DEVICE_NONE: validates arguments, launches nothing
  DevBuf counts, offsets, cursors, records, scan_tmp, slots, order, counters;
  void* staging = nullptr;  // pinned host memory for small uploads
  size_t staging_bytes = 0;
  hipEvent_t staging_done = nullptr;
  int64_t bin_records = 0;  // (face, tile) records binned, counted on the host
  // event pairs around the launches: binning, moments, sum, resolve, re-walk, evaluation
  hipEvent_t ev[6][2] = {};
  bool ev_used[6] = {};
  // stage two: pieces per pixel (tile-major), 64-bit piece offsets, staged pieces
  // pieces per pixel of the last stage one (tile-major), for the evaluation of kept pieces
  DevBuf pcount;
  // tile shape of both passes: (1 << tw_log2) x (64 >> tw_log2) pixels per wavefront
  int tw_log2 = 3;
  // per-pixel segment statistics of the last stage one: [2][seg_h][seg_w]
  DevBuf segs;
  DevBuf gacc;  // FP64 [m+1][H][W] partial sums of APC_MOMENTS_GLOBAL
  int seg_h = 0, seg_w = 0;
  // the pieces per pixel in `pcount` belong to this (mesh, view, subdomain list)
  const void* pc_mesh = nullptr;
  apc_view pc_view;
  int pc_tw_log2 = -1;
  std::vector<int> pc_subs;
  bool pc_valid = false;
  // capture mode (see apc_frame_graph_create): no host round trips, no uploads, no event marks
  bool capturing = false;
  size_t store_slots = 0;     // pixels (tiles * 64) of the last stage one that kept pieces
  // pieces kept by stage one for stage two (see PieceStore)
  DevBuf pool, ptab, store_next;
  long long pool_chunks = 0;         // chunks the pool holds
  long long pool_target = 0;         // chunks wanted (grown after a frame did not fit)
  int maxc = 4096 / apc::PIECE_CHUNK;  // chunk slots per pixel (4096 pieces to start)
  bool store_ready = false;          // the last stage one kept its pieces (if none failed)
  apc_tf store_tf = {};              // the transfer function they were made with
  bool store_failed_last = false;    // the last resolve found that stage one could not keep every piece
  int64_t ws_limit = 0;              // bytes for the piece pool (0: up to 60 % of free memory)
  int dispatch = APC_DISPATCH_GRID;  // how both passes spread their tiles (apc_set_dispatch)
  DevBuf queue;                      // the work queue's per-XCD tile counters (APC_DISPATCH_QUEUE)
  DevBuf pidx;                       // tiles form: the pair number of each (tile, slot) bin
  DevBuf rpair, rpart;               // stage two by pairs: the pairs' bins, their colour sums [pairs][4][64]
  // the (tile, slot) bins in counts / offsets / records / slots were made for this mesh, view, tile shape
  // and subdomain list (stage two of a frame reuses stage one's)
  bool bins_valid = false;
  uint64_t bin_mesh = 0;
  apc_view bin_view = {};
  int bin_tw = -1;
  std::vector<int> bin_subs;
};

struct apc_graph_s {
  apc_ctx own = nullptr;         // private workspace, sized by the eager frame
  hipStream_t cs = nullptr;      // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
enum { EV_BIN = 0, EV_MOM, EV_SUM, EV_RES, EV_STG, EV_EVL, EV_COUNT };
hipError_t ev_mark(apc_ctx ctx, int k, int which, hipStream_t s) {
  if (ctx->capturing) return hipSuccess;
  if (which == 1) ctx->ev_used[k] = true;
  return hipEventRecord(ctx->ev[k][which], s);
}
}  // namespace

struct apc_mesh_s {
  apc_ctx ctx = nullptr;
  int64_t V = 0, T = 0, NB = 0;
  int32_t S = 0;
  float4* vert = nullptr;
  int4* tet = nullptr;
  int4* wrec = nullptr;  // [8T] walk records (128 bytes per tet)
  int* bface = nullptr;
  std::vector<int> sub_begin, face_begin;  // [S+1] each
  double lo[3], hi[3];
  int64_t device_bytes = 0;
  bool host_only = false;  // loaded by a host-only context: no device arrays
  uint64_t uid = 0;        // unique per load in the process (a freed mesh's address may be reused)
};

namespace {

// Copy `bytes` from host to device through the context's pinned staging
// buffer, ordered on `s`.  Waits for the previous staged copy first, so the
// staging buffer is never overwritten while a copy still reads it.
apc_status stage_upload(apc_ctx ctx, void* dst, const void* src, size_t bytes, hipStream_t s) {
  // capture mode: the data is resident from the sizing frame, which had the same arguments
  if (ctx->capturing) return APC_OK;
  if (ctx->staging_done) HIPCHK(hipEventSynchronize(ctx->staging_done));
  if (bytes > ctx->staging_bytes) {
    if (ctx->staging) HIPCHK(hipHostFree(ctx->staging));
    ctx->staging = nullptr;
    size_t nb = std::max<size_t>(bytes, 64 << 10);
    HIPCHK(hipHostMalloc(&ctx->staging, nb, hipHostMallocDefault));
    ctx->staging_bytes = nb;
  }
  std::memcpy(ctx->staging, src, bytes);
  HIPCHK(hipMemcpyAsync(dst, ctx->staging, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(ctx->staging_done, s));
  return APC_OK;
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// inverse of the 3x3 matrix with columns a, b, c; false when singular
bool inverse3(const double* a, const double* b, const double* c, double* inv) {
  double m[3][3] = {{a[0], b[0], c[0]}, {a[1], b[1], c[1]}, {a[2], b[2], c[2]}};
  double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
               m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
  double scale = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) *
                 std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) *
                 std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  if (!(std::fabs(det) > 1e-12 * scale)) return false;
  double id = 1.0 / det;
  inv[0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) * id;
  inv[1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
  inv[2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
  inv[3] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) * id;
  inv[4] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
  inv[5] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
  inv[6] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) * id;
  inv[7] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
  inv[8] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
  return true;
}

apc_status check_view_tf(const apc_view* v, const apc_tf* tf) {
  if (!v) return fail(APC_E_ARG, "view is NULL");
  if (v->width <= 0 || v->height <= 0 || int64_t(v->width) * v->height > (int64_t(1) << 30))
    return fail(APC_E_ARG, "image size %d x %d out of range", v->width, v->height);
  if (v->projection != APC_ORTHOGRAPHIC && v->projection != APC_PERSPECTIVE)
    return fail(APC_E_ARG, "unknown projection %d", v->projection);
  if (!finite3(v->eye) || !finite3(v->dir) || !finite3(v->right) || !finite3(v->down))
    return fail(APC_E_ARG, "camera vectors must be finite");
  if (!(v->step > 0.0) || !std::isfinite(v->step)) return fail(APC_E_ARG, "step must be positive");
  if (!tf) return fail(APC_E_ARG, "transfer function is NULL");
  if (tf->n_entries < 2 || tf->n_entries > apc::MAX_TF)
    return fail(APC_E_ARG, "transfer function needs 2..%d entries", apc::MAX_TF);
  if (!tf->rgba) return fail(APC_E_ARG, "transfer function table is NULL");
  if (!(tf->s_max > tf->s_min)) return fail(APC_E_ARG, "transfer function domain is empty");
  if (!(tf->kappa >= 0.0f) || !(tf->absorbance_max > 0.0f)) return fail(APC_E_ARG, "kappa/absorbance_max invalid");
  return APC_OK;
}

// Frame constants shared by both passes.
apc_status make_frame(const apc_mesh_s* m, const apc_view* v, const apc_tf* tf, int n_slots, int max_sub_tets,
                      int tw_log2, FrameDev& f) {
  std::memset(&f, 0, sizeof(f));
  f.W = v->width;
  f.H = v->height;
  f.proj = v->projection;
  f.tw_log2 = tw_log2;
  const int tw = 1 << tw_log2, th = 64 >> tw_log2;
  f.tiles_x = (v->width + tw - 1) / tw;
  f.tiles_y = (v->height + th - 1) / th;
  int64_t nt = int64_t(f.tiles_x) * f.tiles_y;
  if (nt * n_slots > (int64_t(1) << 31) - 1) return fail(APC_E_ARG, "too many tiles x subdomains");
  f.n_tiles = int(nt);
  f.n_slots = n_slots;
  f.n_tf = tf->n_entries;
  double dn = std::sqrt(v->dir[0] * v->dir[0] + v->dir[1] * v->dir[1] + v->dir[2] * v->dir[2]);
  if (!(dn > 0.0)) return fail(APC_E_ARG, "view direction is zero");
  double dir[3] = {v->dir[0], v->dir[1], v->dir[2]};
  if (v->projection == APC_ORTHOGRAPHIC)
    for (int k = 0; k < 3; ++k) dir[k] /= dn;
  f.ex = float(v->eye[0]);
  f.ey = float(v->eye[1]);
  f.ez = float(v->eye[2]);
  f.dx = float(dir[0]);
  f.dy = float(dir[1]);
  f.dz = float(dir[2]);
  f.rx = float(v->right[0]);
  f.ry = float(v->right[1]);
  f.rz = float(v->right[2]);
  f.wx = float(v->down[0]);
  f.wy = float(v->down[1]);
  f.wz = float(v->down[2]);
  f.half_w = 0.5f * float(v->width);
  f.half_h = 0.5f * float(v->height);
  for (int k = 0; k < 3; ++k) {
    f.ceye[k] = v->eye[k];
    f.cdir[k] = dir[k];
    f.cright[k] = v->right[k];
    f.cdown[k] = v->down[k];
  }
  double minv[9];
  if (!inverse3(dir, v->right, v->down, minv)) return fail(APC_E_ARG, "dir, right and down are not independent");
  for (int k = 0; k < 9; ++k) f.minv[k] = float(minv[k]);
  // the walk enters each subdomain through its boundary faces, so no ray may start inside the mesh: a
  // perspective eye lies outside the mesh's bounding box, an orthographic image plane has the box in front
  if (v->projection == APC_PERSPECTIVE) {
    bool inside = true;
    for (int k = 0; k < 3; ++k) inside = inside && v->eye[k] >= m->lo[k] && v->eye[k] <= m->hi[k];
    if (inside) return fail(APC_E_ARG, "camera inside the mesh's bounding box");
    // a ray is the half-line from the eye, but the walk's entry test (which side of each face edge the ray
    // passes) sees the whole line: the box must lie in front of the eye, every corner at a positive
    // coefficient of dir in (dir, right, down), so that no line crosses the mesh behind the eye (the
    // coefficient is linear in the point and the box convex)
    for (int c = 0; c < 8; ++c) {
      double l = 0.0;
      for (int k = 0; k < 3; ++k) l += minv[k] * (((c >> k) & 1 ? m->hi[k] : m->lo[k]) - v->eye[k]);
      if (!(l > 0.0)) return fail(APC_E_ARG, "the mesh's bounding box is not entirely in front of the camera");
    }
  } else {
    for (int c = 0; c < 8; ++c) {  // dir is normalised here
      double d = 0.0;
      for (int k = 0; k < 3; ++k) d += (((c >> k) & 1 ? m->hi[k] : m->lo[k]) - v->eye[k]) * dir[k];
      if (!(d > 0.0)) return fail(APC_E_ARG, "the mesh's bounding box is not in front of the image plane");
    }
  }
  // one depth range for every subdomain and both passes
  double tn = v->t_near, tfar = v->t_far;
  if (tn <= 0.0 && tfar <= 0.0) {
    double c[3], ext2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      c[k] = 0.5 * (m->lo[k] + m->hi[k]);
      ext2 += (m->hi[k] - m->lo[k]) * (m->hi[k] - m->lo[k]);
    }
    double R = 0.5 * std::sqrt(ext2), dist;
    if (v->projection == APC_PERSPECTIVE) {
      double e2 = 0.0;
      for (int k = 0; k < 3; ++k) e2 += (c[k] - v->eye[k]) * (c[k] - v->eye[k]);
      dist = std::sqrt(e2);
    } else {
      dist = 0.0;
      for (int k = 0; k < 3; ++k) dist += (c[k] - v->eye[k]) * dir[k];
    }
    tn = dist - R;
    tfar = dist + R;
  }
  if (!(tn > 0.0) || !(tfar > tn)) return fail(APC_E_ARG, "depth range [%g, %g] invalid (camera inside the mesh?)", tn, tfar);
  if ((tfar - tn) / v->step > double(1 << 22)) return fail(APC_E_ARG, "step too small for the depth range");
  const double tmid = 0.5 * (tn + tfar);
  f.t_mid = tmid;
  f.t_near = tn - tmid;
  f.step = v->step;
  f.inv_step = 1.0 / v->step;
  double lg0 = std::log2(tn), lg1 = std::log2(tfar);
  f.lg_near = float(lg0);
  f.warp_scale = float(2.0 / (lg1 - lg0));
  f.s_min = tf->s_min;
  f.tf_scale = float(double(tf->n_entries - 1) / (double(tf->s_max) - double(tf->s_min)));
  f.kappa = tf->kappa;
  f.amax = tf->absorbance_max;
  f.max_steps = std::min(max_sub_tets + 16, 1 << 22);
  return APC_OK;
}

apc_status check_subdomains(const apc_mesh_s* m, const int32_t* subs, int32_t n_sub) {
  if (!subs) return fail(APC_E_ARG, "subdomain list is NULL");
  if (n_sub < 1 || n_sub > m->S) return fail(APC_E_ARG, "n_sub %d out of range [1, %d]", n_sub, m->S);
  std::vector<char> seen(m->S, 0);
  for (int k = 0; k < n_sub; ++k) {
    if (subs[k] < 0 || subs[k] >= m->S) return fail(APC_E_ARG, "subdomain id %d out of range", subs[k]);
    if (seen[subs[k]]) return fail(APC_E_ARG, "subdomain id %d listed twice", subs[k]);
    seen[subs[k]] = 1;
  }
  return APC_OK;
}

// records the bin buffer holds
// the tile counters of a persistent launch, or null for one workgroup per tile
int* tile_queue(apc_ctx ctx) { return ctx->dispatch == APC_DISPATCH_QUEUE ? ctx->queue.as<int>() : nullptr; }
long long bin_cap(apc_ctx ctx) { return (long long)(ctx->records.bytes / sizeof(int)); }

// Where a frame's binning state lives: the context's growable buffers, or
// fixed slices of the static workspace (apc_resolve_pass_noalloc).
struct BinSpace {
  SlotDev* slots;
  int *counts, *offsets, *cursors, *tmp, *records;
  long long rec_cap;  // records the record buffer holds (sized after counting when `grow`)
  bool grow;          // records live in ctx->records and may be grown
};

// Bin the boundary faces of the listed subdomains into (tile, slot) bins:
// slot table upload, count pass, exclusive scan, the record total read back
// (to size or check the record buffer; not while capturing a graph, whose
// buffers were sized by an eager frame), fill pass.
apc_status bin_faces(apc_ctx ctx, const apc_mesh_s* m, const FrameDev& f, const int32_t* subs, int32_t n_sub,
                     BinSpace& B, hipStream_t s, MeshDev& md) {
  SlotDev sl_fixed[64];
  std::vector<SlotDev> sl_big;
  SlotDev* sl = sl_fixed;
  if (n_sub > 64) {
    sl_big.resize(n_sub);
    sl = sl_big.data();
  }
  int max_faces = 0;
  for (int k = 0; k < n_sub; ++k) {
    int id = subs[k];
    sl[k].tet_begin = m->sub_begin[id];
    sl[k].tet_end = m->sub_begin[id + 1];
    sl[k].face_begin = m->face_begin[id];
    sl[k].face_end = m->face_begin[id + 1];
    max_faces = std::max(max_faces, sl[k].face_end - sl[k].face_begin);
  }
  if (B.grow) {  // through the context's pinned staging buffer
    apc_status st = stage_upload(ctx, B.slots, sl, sizeof(SlotDev) * n_sub, s);
    if (st != APC_OK) return st;
  } else {  // a plain copy, complete once the record total has been read back below
    HIPCHK(hipMemcpyAsync(B.slots, sl, sizeof(SlotDev) * n_sub, hipMemcpyHostToDevice, s));
  }
  const int64_t nb = int64_t(f.n_tiles) * n_sub;
  md.vert = m->vert;
  md.tet = m->tet;
  md.wrec = m->wrec;
  md.n_vertices = m->V;
  md.n_tets = m->T;
  HIPCHK(ev_mark(ctx, EV_BIN, 0, s));
  HIPCHK(apc::launch_fill_i32(B.counts, 0, nb, s));
  HIPCHK(apc::launch_bin_count(md, f, B.slots, max_faces, m->bface, B.counts, s));
  HIPCHK(apc::launch_exclusive_scan(B.counts, B.offsets, nb, B.tmp, s));
  if (!ctx->capturing) {
    int tail[2];
    HIPCHK(hipMemcpyAsync(&tail[0], B.offsets + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tail[1], B.counts + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t total = int64_t(tail[0]) + tail[1];
    if (total < 0 || total > (int64_t(1) << 31) - 1)
      return fail(APC_E_NUMERIC, "bin records overflow (%lld)", (long long)total);
    if (B.grow) {
      HIPCHK(ctx->records.ensure(sizeof(int) * std::max<int64_t>(total, 1)));
      B.records = ctx->records.as<int>();
      B.rec_cap = bin_cap(ctx);
    } else if (total > B.rec_cap) {
      return fail(APC_E_NOMEM, "the frame bins %lld (face, tile) records; the static workspace holds %lld",
                  (long long)total, B.rec_cap);
    }
    ctx->bin_records += total;
  }
  HIPCHK(apc::launch_fill_i32(B.cursors, 0, nb, s));
  HIPCHK(apc::launch_bin_fill(md, f, B.slots, max_faces, m->bface, B.offsets, B.cursors, B.records, B.rec_cap, s));
  HIPCHK(ev_mark(ctx, EV_BIN, 1, s));
  return APC_OK;
}

// bin_faces into the context's growable buffers, unless they already hold the bins of this mesh, view, tile
// shape and subdomain list (stage two after stage one of the same frame); a captured frame always bins
apc_status build_bins(apc_ctx ctx, const apc_mesh_s* m, const apc_view* v, const FrameDev& f, const int32_t* subs,
                      int32_t n_sub, hipStream_t s, MeshDev& md) {
  if (!ctx->capturing && ctx->bins_valid && ctx->bin_mesh == m->uid && ctx->bin_tw == ctx->tw_log2 &&
      std::memcmp(&ctx->bin_view, v, sizeof(apc_view)) == 0 && ctx->bin_subs.size() == size_t(n_sub) &&
      std::equal(subs, subs + n_sub, ctx->bin_subs.begin())) {
    md.vert = m->vert;
    md.tet = m->tet;
    md.wrec = m->wrec;
    md.n_vertices = m->V;
    md.n_tets = m->T;
    return APC_OK;
  }
  ctx->bins_valid = false;
  const int64_t nb = int64_t(f.n_tiles) * n_sub;
  HIPCHK(ctx->slots.ensure(sizeof(SlotDev) * n_sub));
  HIPCHK(ctx->counts.ensure(sizeof(int) * nb));
  HIPCHK(ctx->offsets.ensure(sizeof(int) * (nb + 1)));
  HIPCHK(ctx->cursors.ensure(sizeof(int) * nb));
  HIPCHK(ctx->scan_tmp.ensure(sizeof(int) * apc::scan_tmp_elems(nb)));
  BinSpace B = {ctx->slots.as<SlotDev>(), ctx->counts.as<int>(), ctx->offsets.as<int>(), ctx->cursors.as<int>(),
                ctx->scan_tmp.as<int>(), ctx->records.as<int>(), bin_cap(ctx), true};
  const apc_status st = bin_faces(ctx, m, f, subs, n_sub, B, s, md);
  if (st == APC_OK && !ctx->capturing) {
    ctx->bins_valid = true;
    ctx->bin_mesh = m->uid;
    ctx->bin_view = *v;
    ctx->bin_tw = ctx->tw_log2;
    ctx->bin_subs.assign(subs, subs + n_sub);
  }
  return st;
}

void set_piece_key(apc_ctx ctx, const apc_mesh_s* m, const apc_view* v, const int32_t* subs, int32_t n_sub) {
  ctx->pc_mesh = m;
  ctx->pc_view = *v;
  ctx->pc_tw_log2 = ctx->tw_log2;
  ctx->pc_subs.assign(subs, subs + n_sub);
  ctx->pc_valid = true;
}

// Do the pieces per pixel in the context belong to this mesh, camera, lattice
// and subdomain list?  (They do not depend on the transfer function or m.)
bool piece_key_matches(apc_ctx ctx, const apc_mesh_s* m, const apc_view* v, const int32_t* subs, int32_t n_sub) {
  return ctx->pc_valid && ctx->pc_mesh == m && ctx->pc_tw_log2 == ctx->tw_log2 &&
         std::memcmp(&ctx->pc_view, v, sizeof(apc_view)) == 0 &&
         ctx->pc_subs.size() == size_t(n_sub) && std::equal(ctx->pc_subs.begin(), ctx->pc_subs.end(), subs);
}

int max_tets_of(const apc_mesh_s* m, const int32_t* subs, int32_t n_sub) {
  int mx = 0;
  for (int k = 0; k < n_sub; ++k) mx = std::max(mx, m->sub_begin[subs[k] + 1] - m->sub_begin[subs[k]]);
  return mx;
}

apc_status check_ctx(apc_ctx ctx) {
  if (!ctx) return fail(APC_E_ARG, "context is NULL");
  if (ctx->host_only) return APC_OK;
  HIPCHK(hipSetDevice(ctx->device));
  return APC_OK;
}

// A host-only context stops here, after every argument of the call was validated.
apc_status no_device(const char* call) {
  return fail(APC_E_DEVICE, "%s: host-only context (APC_DEVICE_NONE): the arguments are valid, nothing was launched",
              call);
}

// A mesh and a context must agree on having a device.
apc_status check_mesh(apc_ctx ctx, const apc_mesh_s* m) {
  if (!m) return fail(APC_E_ARG, "mesh is NULL");
  if (m->host_only != ctx->host_only)
    return fail(APC_E_ARG, "mesh and context differ in having a device (one is host-only)");
  return APC_OK;
}

// Face adjacency on the host (host-only contexts): through vertex -> tet
// incidence lists, every (tet, face) looks for the other tets holding the
// face's three vertices among those incident to its lowest vertex.  Returns
// false when a face is shared by more than two tets.
bool host_adjacency(const std::vector<int4>& tv, int64_t V, std::vector<int>& nbr) {
  const int64_t T = int64_t(tv.size());
  std::vector<int64_t> off(V + 1, 0);
  for (int64_t t = 0; t < T; ++t) {
    ++off[tv[t].x + 1];
    ++off[tv[t].y + 1];
    ++off[tv[t].z + 1];
    ++off[tv[t].w + 1];
  }
  for (int64_t v = 0; v < V; ++v) off[v + 1] += off[v];
  std::vector<int> inc(static_cast<size_t>(off[V]));
  {
    std::vector<int64_t> cur(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < T; ++t) {
      inc[cur[tv[t].x]++] = int(t);
      inc[cur[tv[t].y]++] = int(t);
      inc[cur[tv[t].z]++] = int(t);
      inc[cur[tv[t].w]++] = int(t);
    }
  }
  nbr.assign(size_t(4 * T), -1);
  std::vector<char> bad(16, 0);
  parallel_for(4 * T, [&](int64_t lo, int64_t hi, int k) {
    for (int64_t g = lo; g < hi; ++g) {
      const int t = int(g >> 2), fc = int(g & 3);
      const int v[4] = {tv[t].x, tv[t].y, tv[t].z, tv[t].w};
      int f3[3], q = 0;
      for (int i = 0; i < 4; ++i)
        if (i != fc) f3[q++] = v[i];
      const int a = std::min(f3[0], std::min(f3[1], f3[2]));
      int found = -1, n_found = 0;
      for (int64_t p = off[a]; p < off[a + 1]; ++p) {
        const int t2 = inc[size_t(p)];
        if (t2 == t) continue;
        const int w[4] = {tv[t2].x, tv[t2].y, tv[t2].z, tv[t2].w};
        int hit = 0, miss = -1;
        for (int i = 0; i < 4; ++i) {
          if (w[i] == f3[0] || w[i] == f3[1] || w[i] == f3[2])
            ++hit;
          else
            miss = i;
        }
        if (hit == 3) {
          found = (t2 << 2) | miss;
          ++n_found;
        }
      }
      if (n_found > 1) bad[k] = 1;
      nbr[size_t(g)] = n_found == 1 ? found : -1;
    }
  });
  for (char b : bad)
    if (b) return false;
  return true;
}

}  // namespace

extern "C" {

const char* apc_version(void) { return "apc-mi355x 0.1 (gfx950)"; }

const char* apc_last_error(apc_ctx) { return g_error.c_str(); }

apc_status apc_create(int device, apc_ctx* out) {
  if (!out) return fail(APC_E_ARG, "out is NULL");
  *out = nullptr;
  if (device == APC_DEVICE_NONE) {  // no HIP call at all
    apc_ctx c = new (std::nothrow) apc_ctx_s();
    if (!c) return fail(APC_E_NOMEM, "host allocation failed");
    c->device = APC_DEVICE_NONE;
    c->host_only = true;
    *out = c;
    return APC_OK;
  }
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(APC_E_ARG, "device %d not present (%d devices)", device, n);
  HIPCHK(hipSetDevice(device));
  apc_ctx c = new (std::nothrow) apc_ctx_s();
  if (!c) return fail(APC_E_NOMEM, "host allocation failed");
  c->device = device;
  noalloc_setup(device);
  hipError_t e = c->counters.ensure(sizeof(unsigned long long) * apc::C_COUNT);
  if (e == hipSuccess) e = hipMemset(c->counters.p, 0, c->counters.bytes);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming);
  for (int k = 0; k < EV_COUNT && e == hipSuccess; ++k)
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = hipEventCreate(&c->ev[k][w]);
  if (e != hipSuccess) {
    const char* msg = hipGetErrorString(e);
    apc_destroy(c);
    return fail(APC_E_DEVICE, "context set-up failed: %s", msg);
  }
  *out = c;
  return APC_OK;
}

apc_status apc_destroy(apc_ctx ctx) {
  if (!ctx) return APC_OK;
  if (ctx->host_only) {
    delete ctx;
    return APC_OK;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (DevBuf* b : {&ctx->counts, &ctx->offsets, &ctx->cursors, &ctx->records, &ctx->scan_tmp, &ctx->slots,
                    &ctx->order, &ctx->counters, &ctx->pcount, &ctx->segs, &ctx->gacc, &ctx->queue, &ctx->pidx,
                    &ctx->rpair, &ctx->rpart, &ctx->pool, &ctx->ptab, &ctx->store_next})
    b->release();
  if (ctx->staging) (void)hipHostFree(ctx->staging);
  if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
  for (int k = 0; k < EV_COUNT; ++k)
    for (int w = 0; w < 2; ++w)
      if (ctx->ev[k][w]) (void)hipEventDestroy(ctx->ev[k][w]);
  delete ctx;
  return APC_OK;
}

apc_status apc_load_mesh(apc_ctx ctx, const apc_mesh_desc* d, apc_mesh* out, void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!d || !out) return fail(APC_E_ARG, "desc/out is NULL");
  *out = nullptr;
  if (d->flags & ~int32_t(APC_MESH_DEVICE)) return fail(APC_E_ARG, "unknown mesh flags 0x%x", unsigned(d->flags));
  if (!d->xyz || !d->scalar || !d->tet_vertices || !d->tet_subdomain) return fail(APC_E_ARG, "mesh array is NULL");
  const int64_t V = d->n_vertices, T = d->n_tets;
  const int S = d->n_subdomains;
  if (V < 4 || V > (int64_t(1) << 31) - 1) return fail(APC_E_ARG, "n_vertices %lld out of range", (long long)V);
  if (T < 1 || T >= (int64_t(1) << 29)) return fail(APC_E_ARG, "n_tets %lld out of range", (long long)T);
  if (S < 1) return fail(APC_E_ARG, "n_subdomains must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t* tv = d->tet_vertices;
  const int32_t* ts = d->tet_subdomain;
  const float* xyz = d->xyz;
  const float* scal = d->scalar;
  // device arrays are validated from a host copy (the validation and the grouping run on the host)
  std::vector<float> h_xyz, h_scal;
  std::vector<int32_t> h_tv, h_ts;
  if (d->flags & APC_MESH_DEVICE) {
    if (ctx->host_only) return no_device("apc_load_mesh");
    try {
      h_xyz.resize(size_t(3 * V));
      h_scal.resize(size_t(V));
      h_tv.resize(size_t(4 * T));
      h_ts.resize(size_t(T));
    } catch (...) {
      return fail(APC_E_NOMEM, "host copy of the mesh arrays");
    }
    HIPCHK(hipMemcpyAsync(h_xyz.data(), xyz, sizeof(float) * 3 * V, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_scal.data(), scal, sizeof(float) * V, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_tv.data(), tv, sizeof(int32_t) * 4 * T, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_ts.data(), ts, sizeof(int32_t) * T, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    xyz = h_xyz.data();
    scal = h_scal.data();
    tv = h_tv.data();
    ts = h_ts.data();
  }
  // ---- validation (coordinates, then indices: nothing touches memory through an unchecked id)
  for (int64_t q = 0; q < 3 * V; ++q)
    if (!std::isfinite(xyz[q])) return fail(APC_E_MESH, "vertex %lld: coordinate is not finite", (long long)(q / 3));
  std::vector<int64_t> bad(16, -1);
  std::vector<int> why(16, 0);
  parallel_for(T, [&](int64_t lo, int64_t hi, int k) {
    for (int64_t t = lo; t < hi; ++t) {
      int reason = 0;
      const int32_t* v = tv + 4 * t;
      for (int q = 0; q < 4 && !reason; ++q)
        if (v[q] < 0 || v[q] >= V) reason = 1;
      if (!reason && (v[0] == v[1] || v[0] == v[2] || v[0] == v[3] || v[1] == v[2] || v[1] == v[3] || v[2] == v[3]))
        reason = 2;
      if (!reason && (ts[t] < 0 || ts[t] >= S)) reason = 3;
      if (!reason) {
        double p[4][3];
        for (int q = 0; q < 4; ++q)
          for (int c = 0; c < 3; ++c) p[q][c] = xyz[3 * int64_t(v[q]) + c];
        double a[3], b[3], c3[3];
        for (int c = 0; c < 3; ++c) {
          a[c] = p[1][c] - p[0][c];
          b[c] = p[2][c] - p[0][c];
          c3[c] = p[3][c] - p[0][c];
        }
        double vol = a[0] * (b[1] * c3[2] - b[2] * c3[1]) - a[1] * (b[0] * c3[2] - b[2] * c3[0]) +
                     a[2] * (b[0] * c3[1] - b[1] * c3[0]);
        if (!(vol > 0.0)) reason = 4;
      }
      if (reason) {
        bad[k] = t;
        why[k] = reason;
        return;
      }
    }
  });
  for (int k = 0; k < 16; ++k)
    if (bad[k] >= 0) {
      static const char* msg[] = {"", "vertex id out of range", "repeated vertex", "subdomain id out of range",
                                  "non-positive signed volume"};
      return fail(APC_E_MESH, "tet %lld: %s", (long long)bad[k], msg[why[k]]);
    }
  // ---- group tets by subdomain, keeping input order inside each (stable counting sort)
  static std::atomic<uint64_t> next_uid{1};
  apc_mesh_s* m = new (std::nothrow) apc_mesh_s();
  if (!m) return fail(APC_E_NOMEM, "host allocation failed");
  m->uid = next_uid.fetch_add(1);
  m->ctx = ctx;
  m->V = V;
  m->T = T;
  m->S = S;
  m->sub_begin.assign(S + 1, 0);
  for (int64_t t = 0; t < T; ++t) ++m->sub_begin[ts[t] + 1];
  for (int k = 0; k < S; ++k) m->sub_begin[k + 1] += m->sub_begin[k];
  std::vector<int4> tv_sorted(T);
  {
    std::vector<int> cur(m->sub_begin.begin(), m->sub_begin.end() - 1);
    for (int64_t t = 0; t < T; ++t) {
      const int32_t* v = tv + 4 * t;
      tv_sorted[cur[ts[t]]++] = make_int4(v[0], v[1], v[2], v[3]);
    }
  }
  for (int c = 0; c < 3; ++c) {
    m->lo[c] = 1e300;
    m->hi[c] = -1e300;
  }
  for (int64_t v = 0; v < V; ++v)
    for (int c = 0; c < 3; ++c) {
      m->lo[c] = std::min(m->lo[c], double(xyz[3 * v + c]));
      m->hi[c] = std::max(m->hi[c], double(xyz[3 * v + c]));
    }
  std::vector<float4> vert(V);
  for (int64_t v = 0; v < V; ++v) vert[v] = make_float4(xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2], scal[v]);
  // ---- face adjacency on the device through vertex -> tet incidence lists
  DevBuf d_tv, d_cnt, d_off, d_cur, d_inc, d_nbr, d_err, d_tmp;
  auto cleanup = [&]() {
    for (DevBuf* b : {&d_tv, &d_cnt, &d_off, &d_cur, &d_inc, &d_nbr, &d_err, &d_tmp}) b->release();
  };
  auto dev_fail = [&](hipError_t e, const char* what) {
    cleanup();
    if (m->vert) (void)hipFree(m->vert);
    if (m->tet) (void)hipFree(m->tet);
    if (m->wrec) (void)hipFree(m->wrec);
    if (m->bface) (void)hipFree(m->bface);
    delete m;
    return fail(e == hipErrorOutOfMemory ? APC_E_NOMEM : APC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  std::vector<int> nbr(4 * T);
  if (ctx->host_only) {
    if (!host_adjacency(tv_sorted, V, nbr)) {
      delete m;
      return fail(APC_E_MESH, "a face is shared by more than two tets (non-manifold mesh)");
    }
  } else {
    if ((e = d_tv.ensure(sizeof(int4) * T)) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_cnt.ensure(sizeof(int) * (V + 1))) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_off.ensure(sizeof(int) * (V + 1))) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_cur.ensure(sizeof(int) * V)) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_inc.ensure(sizeof(int) * 4 * T)) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_nbr.ensure(sizeof(int) * 4 * T)) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_err.ensure(sizeof(int))) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = d_tmp.ensure(sizeof(int) * apc::scan_tmp_elems(V + 1))) != hipSuccess) return dev_fail(e, "alloc");
    if ((e = hipMemcpyAsync(d_tv.p, tv_sorted.data(), sizeof(int4) * T, hipMemcpyHostToDevice, s)) != hipSuccess)
      return dev_fail(e, "upload");
    if ((e = apc::launch_fill_i32(d_cnt.as<int>(), 0, V + 1, s)) != hipSuccess) return dev_fail(e, "fill");
    if ((e = apc::launch_fill_i32(d_cur.as<int>(), 0, V, s)) != hipSuccess) return dev_fail(e, "fill");
    if ((e = apc::launch_fill_i32(d_err.as<int>(), 0, 1, s)) != hipSuccess) return dev_fail(e, "fill");
    if ((e = apc::launch_incidence_count(d_tv.as<int4>(), T, d_cnt.as<int>(), s)) != hipSuccess)
      return dev_fail(e, "incidence");
    if ((e = apc::launch_exclusive_scan(d_cnt.as<int>(), d_off.as<int>(), V + 1, d_tmp.as<int>(), s)) != hipSuccess)
      return dev_fail(e, "scan");
    if ((e = apc::launch_incidence_fill(d_tv.as<int4>(), T, d_off.as<int>(), d_cur.as<int>(), d_inc.as<int>(), s)) !=
        hipSuccess)
      return dev_fail(e, "incidence");
    if ((e = apc::launch_adjacency(d_tv.as<int4>(), T, d_off.as<int>(), d_inc.as<int>(), d_nbr.as<int>(),
                                   d_err.as<int>(), s)) != hipSuccess)
      return dev_fail(e, "adjacency");
    int err = 0;
    if ((e = hipMemcpyAsync(nbr.data(), d_nbr.p, sizeof(int) * 4 * T, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return dev_fail(e, "download");
    if ((e = hipMemcpyAsync(&err, d_err.p, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return dev_fail(e, "download");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return dev_fail(e, "adjacency");
    cleanup();
    if (err) {
      delete m;
      return fail(APC_E_MESH, "a face is shared by more than two tets (non-manifold mesh)");
    }
  }
  // ---- boundary faces of each subdomain: hull faces and faces shared with another subdomain
  std::vector<std::vector<int>> bf(S);
  {
    std::vector<std::thread> th;
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (unsigned w = 0; w < nt; ++w)
      th.emplace_back([&, w] {
        for (int k = int(w); k < S; k += int(nt)) {
          const int b0 = m->sub_begin[k], b1 = m->sub_begin[k + 1];
          for (int t = b0; t < b1; ++t)
            for (int fc = 0; fc < 4; ++fc) {
              const int nb = nbr[4 * int64_t(t) + fc];
              if (nb < 0 || (nb >> 2) < b0 || (nb >> 2) >= b1) bf[k].push_back((t << 2) | fc);
            }
        }
      });
    for (auto& t : th) t.join();
  }
  m->face_begin.assign(S + 1, 0);
  for (int k = 0; k < S; ++k) m->face_begin[k + 1] = m->face_begin[k] + int(bf[k].size());
  m->NB = m->face_begin[S];
  std::vector<int> bface(std::max<int64_t>(m->NB, 1));
  for (int k = 0; k < S; ++k) std::copy(bf[k].begin(), bf[k].end(), bface.begin() + m->face_begin[k]);
  if (ctx->host_only) {  // validated and grouped; nothing goes to a device
    m->host_only = true;
    *out = m;
    return APC_OK;
  }
  std::vector<int4> rec(2 * T);
  parallel_for(T, [&](int64_t lo, int64_t hi, int) {
    for (int64_t t = lo; t < hi; ++t) {
      rec[2 * t] = tv_sorted[t];
      rec[2 * t + 1] = make_int4(nbr[4 * t], nbr[4 * t + 1], nbr[4 * t + 2], nbr[4 * t + 3]);
    }
  });
  // ---- resident upload
  if ((e = hipMalloc(&m->vert, sizeof(float4) * V)) != hipSuccess) return dev_fail(e, "alloc");
  if ((e = hipMalloc(&m->tet, sizeof(int4) * 2 * T)) != hipSuccess) return dev_fail(e, "alloc");
  if ((e = hipMalloc(&m->bface, sizeof(int) * bface.size())) != hipSuccess) return dev_fail(e, "alloc");
  if ((e = hipMemcpyAsync(m->vert, vert.data(), sizeof(float4) * V, hipMemcpyHostToDevice, s)) != hipSuccess)
    return dev_fail(e, "upload");
  if ((e = hipMemcpyAsync(m->tet, rec.data(), sizeof(int4) * 2 * T, hipMemcpyHostToDevice, s)) != hipSuccess)
    return dev_fail(e, "upload");
  if ((e = hipMemcpyAsync(m->bface, bface.data(), sizeof(int) * bface.size(), hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return dev_fail(e, "upload");
  if ((e = hipMalloc(&m->wrec, sizeof(int4) * 8 * T)) != hipSuccess) return dev_fail(e, "alloc");
  if ((e = apc::launch_walk_records(m->tet, m->vert, T, m->wrec, s)) != hipSuccess) return dev_fail(e, "records");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return dev_fail(e, "upload");
  m->device_bytes = int64_t(sizeof(float4) * V + sizeof(int4) * 10 * T + sizeof(int) * bface.size());
  *out = m;
  return APC_OK;
}

apc_status apc_free_mesh(apc_ctx ctx, apc_mesh m) {
  if (!m) return APC_OK;
  if (m->host_only) {
    delete m;
    return APC_OK;
  }
  if (ctx) (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (m->vert) (void)hipFree(m->vert);
  if (m->tet) (void)hipFree(m->tet);
  if (m->wrec) (void)hipFree(m->wrec);
  if (m->bface) (void)hipFree(m->bface);
  delete m;
  return APC_OK;
}

apc_status apc_mesh_get_info(apc_mesh m, apc_mesh_info* out) {
  if (!m || !out) return fail(APC_E_ARG, "mesh/out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->n_vertices = m->V;
  out->n_tets = m->T;
  out->n_boundary_faces = m->NB;
  out->n_subdomains = m->S;
  for (int c = 0; c < 3; ++c) {
    out->bbox_lo[c] = m->lo[c];
    out->bbox_hi[c] = m->hi[c];
  }
  out->device_bytes = m->device_bytes;
  return APC_OK;
}

apc_status apc_mesh_subdomain_info(apc_mesh m, int32_t sub, int64_t* n_tets, int64_t* n_faces) {
  if (!m) return fail(APC_E_ARG, "mesh is NULL");
  if (sub < 0 || sub >= m->S) return fail(APC_E_ARG, "subdomain %d out of range", sub);
  if (n_tets) *n_tets = m->sub_begin[sub + 1] - m->sub_begin[sub];
  if (n_faces) *n_faces = m->face_begin[sub + 1] - m->face_begin[sub];
  return APC_OK;
}

// Grows the piece pool to pool_target chunks (capped by the workspace limit, else by 60 % of free memory)
// and the chunk table to `slots` pixels of maxc chunks.  Returns false when the memory cannot be had.
static bool grow_piece_store(apc_ctx ctx, size_t slots) {
  const size_t chunk_bytes = sizeof(float) * 3 * apc::PIECE_CHUNK;
  if (ctx->pool_chunks < ctx->pool_target && !ctx->capturing) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    const size_t limit =
        ctx->ws_limit > 0 ? size_t(ctx->ws_limit) : size_t(0.6 * double(free_b + ctx->pool.bytes));
    const size_t want = std::min(size_t(ctx->pool_target) * chunk_bytes, limit);
    if (want > ctx->pool.bytes) {
      ctx->pool.release();
      ctx->pool_chunks = 0;
      if (ctx->pool.ensure(want, ctx->ws_limit == 0) != hipSuccess) return false;
      ctx->pool_chunks = (long long)(ctx->pool.bytes / chunk_bytes);
    }
  }
  if (ctx->ptab.ensure(sizeof(int) * slots * ctx->maxc) != hipSuccess) return false;
  return ctx->store_next.ensure(4 * sizeof(unsigned long long)) == hipSuccess;
}

apc_status apc_moments_pass(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf, int32_t mm,
                            const int32_t* subs, int32_t n_sub, float* out, uint32_t flags, void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if ((st = check_mesh(ctx, m)) != APC_OK) return st;
  if ((st = check_view_tf(view, tf)) != APC_OK) return st;
  if (mm != 4 && mm != 6 && mm != 8) return fail(APC_E_ARG, "m = %d unsupported (4, 6 or 8)", mm);
  if ((st = check_subdomains(m, subs, n_sub)) != APC_OK) return st;
  if (!out) return fail(APC_E_ARG, "output is NULL");
  if (flags & ~(APC_KEEP_PIECES | APC_MOMENTS_GLOBAL)) return fail(APC_E_ARG, "unknown flags 0x%x", flags);
  const bool global = (flags & APC_MOMENTS_GLOBAL) != 0;
  if (global)
    for (int k = 1; k < n_sub; ++k)
      if (!(subs[k - 1] < subs[k])) return fail(APC_E_ARG, "APC_MOMENTS_GLOBAL needs ascending subdomain ids");
  FrameDev f;
  if ((st = make_frame(m, view, tf, n_sub, max_tets_of(m, subs, n_sub), ctx->tw_log2, f)) != APC_OK) return st;
  if (ctx->host_only) return no_device("apc_moments_pass");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MeshDev md;
  if ((st = build_bins(ctx, m, view, f, subs, n_sub, s, md)) != APC_OK) return st;
  HIPCHK(ctx->pcount.ensure(sizeof(int) * size_t(f.n_tiles) * 64));
  // keep the pieces for stage two unless asked not to (or the pool cannot be had)
  apc::PieceStore ps = {};
  ctx->store_ready = false;
  if (flags & APC_KEEP_PIECES) {
    const size_t slots = size_t(f.n_tiles) * 64;
    if (ctx->pool_target == 0)  // 128 pieces per pixel to start
      ctx->pool_target = (long long)(slots * 128 / apc::PIECE_CHUNK) + (long long)f.n_tiles * apc::STORE_BLOCK;
    const bool ok = grow_piece_store(ctx, slots);
    ctx->store_slots = slots;
    if (ok && ctx->pool_chunks > 0) {
      HIPCHK(apc::launch_fill_i32(ctx->store_next.as<int>(), 0, 8, s));
      ps.pool = ctx->pool.as<float>();
      ps.n_chunks = std::min<long long>(ctx->pool_chunks, (long long)INT32_MAX);
      ps.ptab = ctx->ptab.as<int>();
      ps.maxc = ctx->maxc;
      ps.next = ctx->store_next.as<unsigned long long>();
    }
  }
  HIPCHK(ctx->segs.ensure(sizeof(int) * 2 * size_t(view->width) * view->height));
  ctx->seg_h = view->height;
  ctx->seg_w = view->width;
  HIPCHK(ev_mark(ctx, EV_MOM, 0, s));
  if (global) {
    HIPCHK(ctx->gacc.ensure(sizeof(double) * size_t(mm + 1) * view->width * view->height));
    ctx->ev_used[EV_SUM] = false;  // no separate sum in this frame
  }
  HIPCHK(apc::launch_moments(mm, md, f, ctx->slots.as<SlotDev>(), ctx->offsets.as<int>(), ctx->counts.as<int>(),
                             ctx->records.as<int>(), bin_cap(ctx), tf->rgba, out,
                             global ? ctx->gacc.as<double>() : nullptr, ctx->pcount.as<int>(), ctx->segs.as<int>(), ps,
                             ctx->counters.as<unsigned long long>(), tile_queue(ctx), nullptr, nullptr, 0, s));
  HIPCHK(ev_mark(ctx, EV_MOM, 1, s));
  set_piece_key(ctx, m, view, subs, n_sub);
  ctx->store_ready = ps.pool != nullptr;
  ctx->store_tf = *tf;
  return APC_OK;
}

namespace {
// the tiles form; by_pair: a workgroup per (tile, subdomain) pair instead of one per tile
apc_status moments_tiles(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf, int32_t mm,
                         const int32_t* subs, int32_t n_sub, float* tiles, int32_t* pair_bin, int64_t max_pairs,
                         int64_t* n_pairs, void* stream, bool by_pair, const char* name) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if ((st = check_mesh(ctx, m)) != APC_OK) return st;
  if ((st = check_view_tf(view, tf)) != APC_OK) return st;
  if (mm != 4 && mm != 6 && mm != 8) return fail(APC_E_ARG, "m = %d unsupported (4, 6 or 8)", mm);
  if ((st = check_subdomains(m, subs, n_sub)) != APC_OK) return st;
  for (int k = 1; k < n_sub; ++k)
    if (!(subs[k - 1] < subs[k])) return fail(APC_E_ARG, "the tiles form needs ascending subdomain ids");
  if (!n_pairs) return fail(APC_E_ARG, "n_pairs is NULL");
  if (max_pairs < 0) return fail(APC_E_ARG, "max_pairs = %lld", (long long)max_pairs);
  if (max_pairs > 0 && (!tiles || !pair_bin)) return fail(APC_E_ARG, "tiles or pair_bin is NULL");
  FrameDev f;
  if ((st = make_frame(m, view, tf, n_sub, max_tets_of(m, subs, n_sub), ctx->tw_log2, f)) != APC_OK) return st;
  if (ctx->host_only) return no_device(name);
  hipStream_t s = static_cast<hipStream_t>(stream);
  MeshDev md;
  if ((st = build_bins(ctx, m, view, f, subs, n_sub, s, md)) != APC_OK) return st;
  // number the (tile, slot) bins that have faces: those are the pairs (the binning's cursors are free now)
  const int64_t nb = int64_t(f.n_tiles) * n_sub;
  HIPCHK(ctx->pidx.ensure(sizeof(int) * nb));
  HIPCHK(apc::launch_pair_scan(ctx->counts.as<int>(), nb, ctx->cursors.as<int>(), ctx->pidx.as<int>(),
                               ctx->scan_tmp.as<int>(), s));
  int tail[2];
  HIPCHK(hipMemcpyAsync(&tail[0], ctx->pidx.as<int>() + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&tail[1], ctx->cursors.as<int>() + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t pairs = int64_t(tail[0]) + tail[1];
  *n_pairs = pairs;
  if (max_pairs == 0 && !tiles) return APC_OK;  // a query: the caller sizes its buffers from *n_pairs
  if (pairs > max_pairs)
    return fail(APC_E_NOMEM, "the frame has %lld (tile, subdomain) pairs; the buffers hold %lld (nothing written)",
                (long long)pairs, (long long)max_pairs);
  ctx->store_ready = false;
  if (by_pair) {  // several workgroups per tile: no per-pixel piece or segment counts
    ctx->seg_h = ctx->seg_w = 0;
  } else {
    HIPCHK(ctx->pcount.ensure(sizeof(int) * size_t(f.n_tiles) * 64));
    HIPCHK(ctx->segs.ensure(sizeof(int) * 2 * size_t(view->width) * view->height));
    ctx->seg_h = view->height;
    ctx->seg_w = view->width;
  }
  HIPCHK(apc::launch_pair_list(ctx->counts.as<int>(), nb, ctx->pidx.as<int>(), pair_bin, s));
  HIPCHK(ev_mark(ctx, EV_MOM, 0, s));
  HIPCHK(apc::launch_moments(mm, md, f, ctx->slots.as<SlotDev>(), ctx->offsets.as<int>(), ctx->counts.as<int>(),
                             ctx->records.as<int>(), bin_cap(ctx), tf->rgba, tiles, nullptr,
                             by_pair ? nullptr : ctx->pcount.as<int>(), by_pair ? nullptr : ctx->segs.as<int>(),
                             apc::PieceStore{}, ctx->counters.as<unsigned long long>(),
                             by_pair ? nullptr : tile_queue(ctx), ctx->pidx.as<int>(), by_pair ? pair_bin : nullptr,
                             pairs, s));
  HIPCHK(ev_mark(ctx, EV_MOM, 1, s));
  set_piece_key(ctx, m, view, subs, n_sub);
  return APC_OK;
}
}  // namespace

apc_status apc_moments_pass_tiles(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf, int32_t mm,
                                  const int32_t* subs, int32_t n_sub, float* tiles, int32_t* pair_bin,
                                  int64_t max_pairs, int64_t* n_pairs, void* stream) {
  return moments_tiles(ctx, m, view, tf, mm, subs, n_sub, tiles, pair_bin, max_pairs, n_pairs, stream, false,
                       "apc_moments_pass_tiles");
}

apc_status apc_moments_pass_pairs(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf, int32_t mm,
                                  const int32_t* subs, int32_t n_sub, float* tiles, int32_t* pair_bin,
                                  int64_t max_pairs, int64_t* n_pairs, void* stream) {
  return moments_tiles(ctx, m, view, tf, mm, subs, n_sub, tiles, pair_bin, max_pairs, n_pairs, stream, true,
                       "apc_moments_pass_pairs");
}

apc_status apc_sum_moment_tiles(apc_ctx ctx, const float* tiles, const int32_t* pair_bin, int64_t n_pairs,
                                int32_t n_sub, int32_t mm, int32_t H, int32_t W, int32_t tile_width, float* outg,
                                void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!outg) return fail(APC_E_ARG, "moments_global is NULL");
  if (n_pairs > 0 && (!tiles || !pair_bin)) return fail(APC_E_ARG, "tiles or pair_bin is NULL");
  if (mm != 4 && mm != 6 && mm != 8) return fail(APC_E_ARG, "m = %d unsupported", mm);
  if (n_sub < 1 || H <= 0 || W <= 0 || n_pairs < 0) return fail(APC_E_ARG, "sizes out of range");
  int lg = -1;
  for (int k = 0; k <= 6; ++k)
    if (tile_width == (1 << k)) lg = k;
  if (lg < 0) return fail(APC_E_ARG, "tile width %d is not a power of two in 1..64", tile_width);
  const int64_t tiles_x = (int64_t(W) + (1 << lg) - 1) >> lg, tiles_y = (int64_t(H) + (64 >> lg) - 1) / (64 >> lg);
  if (n_pairs > tiles_x * tiles_y * n_sub)
    return fail(APC_E_ARG, "%lld pairs exceed the %lld (tile, subdomain) bins of a %d x %d image",
                (long long)n_pairs, (long long)(tiles_x * tiles_y * n_sub), W, H);
  if (ctx->host_only) return no_device("apc_sum_moment_tiles");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(ev_mark(ctx, EV_SUM, 0, s));
  HIPCHK(apc::launch_sum_tiles(tiles, pair_bin, n_pairs, n_sub, mm + 1, W, H, lg, outg, s));
  HIPCHK(ev_mark(ctx, EV_SUM, 1, s));
  return APC_OK;
}

apc_status apc_sum_moments(apc_ctx ctx, const float* in, int32_t n_sub, int32_t mm, int32_t H, int32_t W,
                           const int32_t* subs, float* outg, void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!in || !outg) return fail(APC_E_ARG, "buffer is NULL");
  if (mm != 4 && mm != 6 && mm != 8) return fail(APC_E_ARG, "m = %d unsupported", mm);
  if (n_sub < 1 || H <= 0 || W <= 0) return fail(APC_E_ARG, "sizes out of range");
  std::vector<int> order(n_sub);
  for (int k = 0; k < n_sub; ++k) order[k] = k;
  if (subs) {
    for (int k = 0; k < n_sub; ++k)
      for (int q = 0; q < k; ++q)
        if (subs[q] == subs[k]) return fail(APC_E_ARG, "subdomain id %d listed twice", subs[k]);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return subs[a] < subs[b]; });
  }
  if (ctx->host_only) return no_device("apc_sum_moments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(ctx->order.ensure(sizeof(int) * n_sub));
  if ((st = stage_upload(ctx, ctx->order.p, order.data(), sizeof(int) * n_sub, s)) != APC_OK) return st;
  HIPCHK(ev_mark(ctx, EV_SUM, 0, s));
  HIPCHK(apc::launch_sum_moments(in, n_sub, ctx->order.as<int>(), int64_t(mm + 1) * H * W, outg, s));
  HIPCHK(ev_mark(ctx, EV_SUM, 1, s));
  return APC_OK;
}

static apc_status bound_params(const apc_mboit* mb, apc::BoundParams& bp, int finalize) {
  if (!mb) return fail(APC_E_ARG, "mboit is NULL");
  if (mb->m != 4 && mb->m != 6 && mb->m != 8) return fail(APC_E_ARG, "m = %d unsupported", mb->m);
  if (!(mb->alpha >= 0.0 && mb->alpha < 1.0)) return fail(APC_E_ARG, "alpha must be in [0, 1)");
  if (!(mb->eta >= 0.0 && mb->eta <= 1.0)) return fail(APC_E_ARG, "eta must be in [0, 1]");
  std::memset(&bp, 0, sizeof(bp));
  bp.alpha = mb->alpha;
  bp.eta = mb->eta;
  for (int j = 0; j < 8; ++j) bp.bias[j] = j < mb->m ? mb->bias[j] : 0.0;
  bp.renormalize = mb->renormalize ? 1 : 0;
  bp.finalize = finalize;
  return APC_OK;
}

static apc_status resolve_frame(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                const apc_mboit* mb, const void* moments, const int32_t* subs, int32_t n_sub,
                                float* rgba, uint32_t flags, void* stream);

apc_status apc_resolve_pass(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf, const apc_mboit* mb,
                            const void* moments, const int32_t* subs, int32_t n_sub, float* rgba, uint32_t flags,
                            void* stream) {
  const apc_status st = resolve_frame(ctx, m, view, tf, mb, moments, subs, n_sub, rgba, flags, stream);
  // a frame whose pieces did not fit the store has sized it anew: grow it now, at the end of this frame,
  // so that the next frame's stage one does not allocate (an allocation waits for the whole device)
  if (st == APC_OK && !ctx->host_only && ctx->store_failed_last && !ctx->capturing && ctx->store_slots > 0)
    (void)grow_piece_store(ctx, ctx->store_slots);  // on failure the next stage one tries again
  return st;
}

// Validation shared by the resolve entry points; fills the bound parameters and the frame constants.  A
// host-only context stops here.
static apc_status check_resolve(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                const apc_mboit* mb, const void* moments, const int32_t* subs, int32_t n_sub,
                                const float* rgba, uint32_t flags, apc::BoundParams& bp, FrameDev& f,
                                const char* call, uint32_t allowed = APC_FINALIZE | APC_MOMENTS_F16) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if ((st = check_mesh(ctx, m)) != APC_OK) return st;
  if ((st = check_view_tf(view, tf)) != APC_OK) return st;
  if ((st = bound_params(mb, bp, (flags & APC_FINALIZE) ? 1 : 0)) != APC_OK) return st;
  if ((st = check_subdomains(m, subs, n_sub)) != APC_OK) return st;
  if (!moments || !rgba) return fail(APC_E_ARG, "buffer is NULL");
  if (reinterpret_cast<uintptr_t>(rgba) & 15) return fail(APC_E_ARG, "rgba_out must be 16-byte aligned");
  if (flags & ~allowed) return fail(APC_E_ARG, "unknown flags 0x%x for %s", flags, call);
  if ((flags & APC_BY_PAIR) && (flags & APC_MOMENTS_F16))
    return fail(APC_E_ARG, "stage two by pairs reads FP32 moments (APC_BY_PAIR with APC_MOMENTS_F16)");
  bp.moments_f16 = (flags & APC_MOMENTS_F16) ? 1 : 0;
  if (bp.moments_f16 && (reinterpret_cast<uintptr_t>(moments) & 1))
    return fail(APC_E_ARG, "packed FP16 moments must be 2-byte aligned");
  if ((st = make_frame(m, view, tf, n_sub, max_tets_of(m, subs, n_sub), ctx->tw_log2, f)) != APC_OK) return st;
  if (ctx->host_only) return no_device(call);
  return APC_OK;
}

static apc_status resolve_frame(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                const apc_mboit* mb, const void* moments, const int32_t* subs, int32_t n_sub,
                                float* rgba, uint32_t flags, void* stream) {
  apc::BoundParams bp;
  FrameDev f;
  apc_status st = check_resolve(ctx, m, view, tf, mb, moments, subs, n_sub, rgba, flags, bp, f, "apc_resolve_pass",
                                APC_FINALIZE | APC_MOMENTS_F16 | APC_BY_PAIR);
  if (st != APC_OK) return st;
  if ((flags & APC_BY_PAIR) && ctx->capturing)
    return fail(APC_E_ARG, "stage two by pairs reads its pair count back: not in a captured frame");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nt = f.n_tiles;
  unsigned long long* ctr = ctx->counters.as<unsigned long long>();
  ctx->ev_used[EV_STG] = false;
  ctx->ev_used[EV_EVL] = false;
  // stage one's kept pieces, when they belong to this geometry and transfer function and all fitted
  bool stored = ctx->store_ready && piece_key_matches(ctx, m, view, subs, n_sub) &&
                std::memcmp(&ctx->store_tf, tf, sizeof(apc_tf)) == 0;
  bool store_failed = false;
  if (stored && !ctx->capturing) {
    unsigned long long nx[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(nx, ctx->store_next.p, sizeof(nx), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    store_failed = nx[1] != 0;
    stored = !store_failed;
  }
  ctx->store_failed_last = store_failed;
  if (store_failed) {  // size the piece store for the next frame from this frame's counts
    std::vector<int> pc(size_t(nt) * 64);
    HIPCHK(hipMemcpyAsync(pc.data(), ctx->pcount.p, sizeof(int) * pc.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    long long chunks = 0;
    int most = 0;
    for (int c : pc) {
      chunks += (c + apc::PIECE_CHUNK - 1) / apc::PIECE_CHUNK;
      most = std::max(most, c);
    }
    ctx->pool_target = std::max(ctx->pool_target, chunks + chunks / 50 + (long long)nt * apc::STORE_BLOCK);
    ctx->maxc = std::max(ctx->maxc, (most + apc::PIECE_CHUNK - 1) / apc::PIECE_CHUNK + 8);
  }
  HIPCHK(ev_mark(ctx, EV_RES, 0, s));
  if (stored) {  // (in a replayed graph the kernel itself checks that no lane failed)
    apc::PieceStore ps = {ctx->pool.as<float>(), ctx->pool_chunks, ctx->ptab.as<int>(), ctx->maxc,
                          ctx->store_next.as<unsigned long long>()};
    HIPCHK(ev_mark(ctx, EV_EVL, 0, s));
    HIPCHK(apc::launch_eval(mb->m, f, 0, nt, ps, ctx->pcount.as<int>(), tf->rgba, moments, bp, rgba, ctr, s));
    HIPCHK(ev_mark(ctx, EV_EVL, 1, s));
    HIPCHK(ev_mark(ctx, EV_RES, 1, s));
    return APC_OK;
  }
  // the plain form: walk the rays again and evaluate every piece at once
  MeshDev md;
  if ((st = build_bins(ctx, m, view, f, subs, n_sub, s, md)) != APC_OK) return st;
  if (flags & APC_BY_PAIR) {
    // number the (tile, slot) bins with faces (the binning's cursors are free now), list them, walk each
    // pair in a workgroup of its own, then sum each pixel's pairs in slot order and finalise
    const int64_t nb = int64_t(f.n_tiles) * n_sub;
    HIPCHK(ctx->pidx.ensure(sizeof(int) * nb));
    HIPCHK(apc::launch_pair_scan(ctx->counts.as<int>(), nb, ctx->cursors.as<int>(), ctx->pidx.as<int>(),
                                 ctx->scan_tmp.as<int>(), s));
    int tail[2];
    HIPCHK(hipMemcpyAsync(&tail[0], ctx->pidx.as<int>() + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tail[1], ctx->cursors.as<int>() + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t pairs = int64_t(tail[0]) + tail[1];
    HIPCHK(ctx->rpair.ensure(sizeof(int) * size_t(std::max<int64_t>(pairs, 1))));
    HIPCHK(ctx->rpart.ensure(sizeof(float) * 4 * 64 * size_t(std::max<int64_t>(pairs, 1))));
    HIPCHK(apc::launch_pair_list(ctx->counts.as<int>(), nb, ctx->pidx.as<int>(), ctx->rpair.as<int>(), s));
    HIPCHK(ev_mark(ctx, EV_STG, 0, s));
    HIPCHK(apc::launch_resolve(mb->m, md, f, ctx->slots.as<SlotDev>(), ctx->offsets.as<int>(),
                               ctx->counts.as<int>(), ctx->records.as<int>(), bin_cap(ctx), tf->rgba, moments, bp,
                               rgba, ctr, nullptr, ctx->rpair.as<int>(), ctx->rpart.as<float>(), pairs, s));
    HIPCHK(apc::launch_sum_color_tiles(ctx->rpart.as<float>(), ctx->rpair.as<int>(), pairs, n_sub, f.W, f.H,
                                       ctx->tw_log2, static_cast<const float*>(moments), bp, rgba, s));
    HIPCHK(ev_mark(ctx, EV_STG, 1, s));
    HIPCHK(ev_mark(ctx, EV_RES, 1, s));
    return APC_OK;
  }
  HIPCHK(ev_mark(ctx, EV_STG, 0, s));
  HIPCHK(apc::launch_resolve(mb->m, md, f, ctx->slots.as<SlotDev>(), ctx->offsets.as<int>(), ctx->counts.as<int>(),
                             ctx->records.as<int>(), bin_cap(ctx), tf->rgba, moments, bp, rgba, ctr, tile_queue(ctx),
                             nullptr, nullptr, 0, s));
  HIPCHK(ev_mark(ctx, EV_STG, 1, s));
  HIPCHK(ev_mark(ctx, EV_RES, 1, s));
  return APC_OK;
}

apc_status apc_resolve_pass_noalloc(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                    const apc_mboit* mb, const void* moments, const int32_t* subs, int32_t n_sub,
                                    float* rgba, uint32_t flags, void* stream) {
  apc::BoundParams bp;
  FrameDev f;
  apc_status st =
      check_resolve(ctx, m, view, tf, mb, moments, subs, n_sub, rgba, flags, bp, f, "apc_resolve_pass_noalloc");
  if (st != APC_OK) return st;
  // the binning state's slices of the static workspace: slots, counts, offsets, cursors, scan scratch, then
  // the (face, tile) records in the rest
  const int64_t nb = int64_t(f.n_tiles) * n_sub;
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_counts = up(sizeof(SlotDev) * n_sub);
  const size_t o_offsets = o_counts + up(sizeof(int) * nb);
  const size_t o_cursors = o_offsets + up(sizeof(int) * (nb + 1));
  const size_t o_tmp = o_cursors + up(sizeof(int) * nb);
  const size_t o_rec = o_tmp + up(sizeof(int) * apc::scan_tmp_elems(nb));
  if (o_rec + sizeof(int) > NOALLOC_BYTES)
    return fail(APC_E_NOMEM,
                "a %d x %d frame of %d subdomains needs %zu bytes of binning state before its records; the static "
                "workspace holds %zu",
                view->width, view->height, n_sub, o_rec, NOALLOC_BYTES);
  const int dev = ctx->device;
  if (dev >= NOALLOC_MAX_DEVICES || !g_noalloc_ptr[dev])
    return fail(APC_E_DEVICE, "the static workspace has no address on device %d: %s", dev,
                dev < NOALLOC_MAX_DEVICES ? hipGetErrorString(g_noalloc_err[dev]) : "device id too large");
  unsigned char* base = static_cast<unsigned char*>(g_noalloc_ptr[dev]);
  BinSpace B = {reinterpret_cast<SlotDev*>(base), reinterpret_cast<int*>(base + o_counts),
                reinterpret_cast<int*>(base + o_offsets), reinterpret_cast<int*>(base + o_cursors),
                reinterpret_cast<int*>(base + o_tmp), reinterpret_cast<int*>(base + o_rec),
                (long long)((NOALLOC_BYTES - o_rec) / sizeof(int)), false};
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long* ctr = ctx->counters.as<unsigned long long>();
  ctx->ev_used[EV_STG] = false;
  ctx->ev_used[EV_EVL] = false;
  MeshDev md;
  HIPCHK(ev_mark(ctx, EV_RES, 0, s));
  if ((st = bin_faces(ctx, m, f, subs, n_sub, B, s, md)) != APC_OK) return st;
  HIPCHK(ev_mark(ctx, EV_STG, 0, s));
  HIPCHK(apc::launch_resolve(mb->m, md, f, B.slots, B.offsets, B.counts, B.records, B.rec_cap, tf->rgba, moments, bp,
                             rgba, ctr, tile_queue(ctx), nullptr, nullptr, 0, s));
  HIPCHK(ev_mark(ctx, EV_STG, 1, s));
  HIPCHK(ev_mark(ctx, EV_RES, 1, s));
  return APC_OK;
}

apc_status apc_frame_graph_destroy(apc_graph g) {
  if (!g) return APC_OK;
  if (g->own) (void)hipSetDevice(g->own->device);
  if (g->cs) (void)hipStreamSynchronize(g->cs);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cs) (void)hipStreamDestroy(g->cs);
  if (g->own) (void)apc_destroy(g->own);
  delete g;
  return APC_OK;
}

apc_status apc_frame_graph_create(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                  const apc_mboit* mb, const int32_t* subs, int32_t n_sub, float* moments_per_sub,
                                  float* moments_global, float* rgba_out, uint32_t flags, apc_graph* out) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!out) return fail(APC_E_ARG, "out is NULL");
  *out = nullptr;
  if (!mb) return fail(APC_E_ARG, "mboit is NULL");
  if (flags & ~(APC_FINALIZE | APC_MOMENTS_GLOBAL | APC_KEEP_PIECES))
    return fail(APC_E_ARG, "unknown flags 0x%x", flags);
  const bool global = (flags & APC_MOMENTS_GLOBAL) != 0;
  const uint32_t keep = flags & APC_KEEP_PIECES;
  if (!global && !moments_per_sub) return fail(APC_E_ARG, "moments_per_sub is NULL");
  if ((st = check_mesh(ctx, m)) != APC_OK) return st;
  if (ctx->host_only) return no_device("apc_frame_graph_create");
  apc_graph g = new (std::nothrow) apc_graph_s();
  if (!g) return fail(APC_E_NOMEM, "host allocation failed");
  if ((st = apc_create(ctx->device, &g->own)) != APC_OK) {
    delete g;
    return st;
  }
  g->own->tw_log2 = ctx->tw_log2;
  if ((st = apc_set_dispatch(g->own, ctx->dispatch)) != APC_OK) {
    apc_frame_graph_destroy(g);
    return st;
  }
  if (hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking) != hipSuccess) {
    apc_frame_graph_destroy(g);
    return fail(APC_E_DEVICE, "stream creation failed");
  }
  apc_ctx w = g->own;
  auto frame = [&]() -> apc_status {
    apc_status r;
    if (global) {
      r = apc_moments_pass(w, m, view, tf, mb->m, subs, n_sub, moments_global, APC_MOMENTS_GLOBAL | keep, g->cs);
    } else {
      r = apc_moments_pass(w, m, view, tf, mb->m, subs, n_sub, moments_per_sub, keep, g->cs);
      if (r == APC_OK)
        r = apc_sum_moments(w, moments_per_sub, n_sub, mb->m, view->height, view->width, subs, moments_global,
                            g->cs);
    }
    if (r == APC_OK)
      r = apc_resolve_pass(w, m, view, tf, mb, moments_global, subs, n_sub, rgba_out, flags & APC_FINALIZE, g->cs);
    return r;
  };
  // 1) eager frames size every workspace buffer (again while stage one's piece store overflowed: it grows
  //    after such a frame)
  for (int attempt = 0; attempt < 3; ++attempt) {
    st = frame();
    if (st == APC_OK && hipStreamSynchronize(g->cs) != hipSuccess) st = fail(APC_E_DEVICE, "sizing frame failed");
    if (st != APC_OK || !w->store_failed_last) break;
  }
  if (st == APC_OK && w->store_failed_last) st = fail(APC_E_NOMEM, "the frame's pieces do not fit the piece store");
  // 2) the same frame captured: kernels only (no uploads, host reads, event records or allocations)
  if (st == APC_OK) {
    if (hipStreamBeginCapture(g->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = fail(APC_E_DEVICE, "stream capture could not start");
    } else {
      w->capturing = true;
      g_frozen = true;
      st = frame();
      g_frozen = false;
      w->capturing = false;
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(g->cs, &gr);
      g->graph = gr;
      if (st == APC_OK && (e != hipSuccess || !gr)) st = fail(APC_E_DEVICE, "capture failed: %s", hipGetErrorString(e));
    }
  }
  if (st == APC_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    st = fail(APC_E_DEVICE, "graph instantiation failed");
  if (st != APC_OK) {
    apc_frame_graph_destroy(g);
    return st;
  }
  *out = g;
  return APC_OK;
}

apc_status apc_frame_graph_launch(apc_graph g, void* stream) {
  if (!g || !g->exec) return fail(APC_E_ARG, "graph is NULL");
  HIPCHK(hipSetDevice(g->own->device));
  HIPCHK(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return APC_OK;
}

apc_status apc_frame_graph_counters(apc_graph g, apc_counters* out, int32_t reset) {
  if (!g) return fail(APC_E_ARG, "graph is NULL");
  return apc_get_counters(g->own, out, reset);
}

apc_status apc_set_workspace_limit(apc_ctx ctx, int64_t bytes) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (bytes < 0) return fail(APC_E_ARG, "negative limit");
  ctx->ws_limit = bytes;
  if (ctx->host_only) return APC_OK;
  // a pool above the new limit is given back
  if (bytes > 0 && ctx->pool.bytes > size_t(bytes)) {
    HIPCHK(hipDeviceSynchronize());
    ctx->pool.release();
    ctx->pool_chunks = 0;
    ctx->store_ready = false;
  }
  return APC_OK;
}

apc_status apc_get_workspace_bytes(apc_ctx ctx, int64_t* bytes) {
  if (!ctx) return fail(APC_E_ARG, "context is NULL");
  if (!bytes) return fail(APC_E_ARG, "bytes is NULL");
  int64_t total = 0;
  for (const DevBuf* b : {&ctx->counts, &ctx->offsets, &ctx->cursors, &ctx->records, &ctx->scan_tmp, &ctx->slots,
                          &ctx->order, &ctx->counters, &ctx->pcount, &ctx->segs, &ctx->gacc, &ctx->queue, &ctx->pidx,
                          &ctx->rpair, &ctx->rpart, &ctx->pool, &ctx->ptab, &ctx->store_next})
    total += int64_t(b->bytes);
  *bytes = total;
  return APC_OK;
}

apc_status apc_set_dispatch(apc_ctx ctx, int32_t mode) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (mode != APC_DISPATCH_GRID && mode != APC_DISPATCH_QUEUE) return fail(APC_E_ARG, "unknown dispatch mode %d", mode);
  if (mode == APC_DISPATCH_QUEUE && !ctx->host_only) {  // the counters now, so that no pass allocates them
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(ctx->queue.ensure(sizeof(int) * apc::QUEUE_INTS));
  }
  ctx->dispatch = mode;
  return APC_OK;
}

apc_status apc_get_dispatch(apc_ctx ctx, int32_t* mode) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!mode) return fail(APC_E_ARG, "mode is NULL");
  *mode = ctx->dispatch;
  return APC_OK;
}

apc_status apc_set_tile_shape(apc_ctx ctx, int32_t tile_width) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  int lg = -1;
  for (int k = 0; k <= 6; ++k)
    if (tile_width == (1 << k)) lg = k;
  if (lg < 0) return fail(APC_E_ARG, "tile width %d is not a power of two in 1..64", tile_width);
  ctx->tw_log2 = lg;
  return APC_OK;
}

apc_status apc_get_tile_shape(apc_ctx ctx, int32_t* tile_width, int32_t* tile_height) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (tile_width) *tile_width = 1 << ctx->tw_log2;
  if (tile_height) *tile_height = 64 >> ctx->tw_log2;
  return APC_OK;
}

// Whole frames (stage one summing the subdomains itself, then the finalising resolve) timed with HIP events
// on `stream` for tile widths 2..32 and, with both_modes, both dispatch modes: the best of `repeats` after a
// warm-up frame per configuration.  Sets the fastest on the context (leaves it as it was on failure).
static apc_status autotune_frames(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                  const apc_mboit* mboit, const int32_t* subs, int32_t n_sub, float* moments,
                                  float* rgba_out, int32_t repeats, bool both_modes, int32_t* best_width,
                                  int32_t* best_dispatch, float* ms_table, void* stream, const char* who) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (repeats < 1 || repeats > 100) return fail(APC_E_ARG, "repeats must be in 1..100");
  if (!mboit) return fail(APC_E_ARG, "mboit is NULL");
  if ((st = check_mesh(ctx, m)) != APC_OK) return st;
  if (ctx->host_only) return no_device(who);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int old_lg = ctx->tw_log2, old_mode = ctx->dispatch;
  const int n_modes = both_modes ? 2 : 1;
  for (int k = 0; k < 7 * n_modes; ++k)
    if (ms_table) ms_table[k] = -1.0f;
  if (both_modes && (st = apc_set_dispatch(ctx, APC_DISPATCH_QUEUE)) != APC_OK) return st;  // its counters, once
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(APC_E_DEVICE, "event creation failed");
  }
  int best_lg = old_lg, best_mode = old_mode;
  float best_ms = -1.0f;
  apc_status res = APC_OK;
  for (int mi = 0; mi < n_modes && res == APC_OK; ++mi) {
    ctx->dispatch = both_modes ? (mi == 0 ? APC_DISPATCH_GRID : APC_DISPATCH_QUEUE) : old_mode;
    for (int lg = 1; lg <= 5 && res == APC_OK; ++lg) {  // 2x32 .. 32x2
      ctx->tw_log2 = lg;
      float t_min = 0.0f;
      for (int rep = 0; rep <= repeats && res == APC_OK; ++rep) {  // the first run is a warm-up
        if (hipEventRecord(e0, s) != hipSuccess) res = fail(APC_E_DEVICE, "event record failed");
        if (res == APC_OK)
          res = apc_moments_pass(ctx, m, view, tf, mboit->m, subs, n_sub, moments, APC_MOMENTS_GLOBAL, stream);
        if (res == APC_OK)
          res = apc_resolve_pass(ctx, m, view, tf, mboit, moments, subs, n_sub, rgba_out, APC_FINALIZE, stream);
        if (res == APC_OK && hipEventRecord(e1, s) != hipSuccess) res = fail(APC_E_DEVICE, "event record failed");
        float ms = 0.0f;
        if (res == APC_OK &&
            (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          res = fail(APC_E_DEVICE, "event timing failed");
        if (res == APC_OK && rep > 0) t_min = (rep == 1) ? ms : std::min(t_min, ms);
      }
      if (res != APC_OK) break;
      if (ms_table) ms_table[mi * 7 + lg] = t_min;
      if (best_ms < 0.0f || t_min < best_ms) {
        best_ms = t_min;
        best_lg = lg;
        best_mode = ctx->dispatch;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tw_log2 = res == APC_OK ? best_lg : old_lg;
  ctx->dispatch = res == APC_OK ? best_mode : old_mode;
  ctx->pc_valid = false;  // the piece counts of the last run belong to another tile shape
  if (res == APC_OK && best_width) *best_width = 1 << best_lg;
  if (res == APC_OK && best_dispatch) *best_dispatch = best_mode;
  return res;
}

apc_status apc_autotune_tile_shape(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                                   const apc_mboit* mboit, const int32_t* subs, int32_t n_sub, float* moments,
                                   float* rgba_out, int32_t repeats, int32_t* best_width, float* ms_per_width,
                                   void* stream) {
  return autotune_frames(ctx, m, view, tf, mboit, subs, n_sub, moments, rgba_out, repeats, false, best_width,
                         nullptr, ms_per_width, stream, "apc_autotune_tile_shape");
}

apc_status apc_autotune_launch(apc_ctx ctx, apc_mesh m, const apc_view* view, const apc_tf* tf,
                               const apc_mboit* mboit, const int32_t* subs, int32_t n_sub, float* moments,
                               float* rgba_out, int32_t repeats, int32_t* best_width, int32_t* best_dispatch,
                               float* ms_table, void* stream) {
  return autotune_frames(ctx, m, view, tf, mboit, subs, n_sub, moments, rgba_out, repeats, true, best_width,
                         best_dispatch, ms_table, stream, "apc_autotune_launch");
}

apc_status apc_segment_counts(apc_ctx ctx, int32_t* out, int32_t H, int32_t W, void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!out) return fail(APC_E_ARG, "out is NULL");
  if (ctx->seg_h == 0) return fail(APC_E_ARG, "no segment counts: no stage one has run on this context, or the last ran by pairs");
  if (H != ctx->seg_h || W != ctx->seg_w)
    return fail(APC_E_ARG, "image is %dx%d, the last stage one was %dx%d", W, H, ctx->seg_w, ctx->seg_h);
  if (ctx->host_only) return no_device("apc_segment_counts");
  HIPCHK(hipMemcpyAsync(out, ctx->segs.p, sizeof(int) * 2 * size_t(H) * W, hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return APC_OK;
}

apc_status apc_pack_moments_f16(apc_ctx ctx, const float* moments, int32_t mm, int32_t H, int32_t W, void* packed,
                                void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!moments || !packed) return fail(APC_E_ARG, "buffer is NULL");
  if (mm != 4 && mm != 6 && mm != 8) return fail(APC_E_ARG, "m = %d unsupported", mm);
  if (H <= 0 || W <= 0) return fail(APC_E_ARG, "sizes out of range");
  if (reinterpret_cast<uintptr_t>(packed) & 1) return fail(APC_E_ARG, "packed must be 2-byte aligned");
  if (ctx->host_only) return no_device("apc_pack_moments_f16");
  HIPCHK(apc::launch_pack_f16(moments, mm + 1, int64_t(H) * W, packed,
                              static_cast<hipStream_t>(stream)));
  return APC_OK;
}

apc_status apc_sum_images(apc_ctx ctx, const float* partials, int32_t n_sub, int32_t H, int32_t W,
                          const int32_t* subs, const float* moments, const apc_mboit* mb, float* rgba,
                          void* stream) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!partials || !moments || !rgba) return fail(APC_E_ARG, "buffer is NULL");
  if (n_sub < 1 || H <= 0 || W <= 0) return fail(APC_E_ARG, "sizes out of range");
  if ((reinterpret_cast<uintptr_t>(rgba) | reinterpret_cast<uintptr_t>(partials)) & 15)
    return fail(APC_E_ARG, "image buffers must be 16-byte aligned");
  apc::BoundParams bp;
  if ((st = bound_params(mb, bp, 1)) != APC_OK) return st;
  std::vector<int> order(n_sub);
  for (int k = 0; k < n_sub; ++k) order[k] = k;
  if (subs) {
    for (int k = 0; k < n_sub; ++k)
      for (int q = 0; q < k; ++q)
        if (subs[q] == subs[k]) return fail(APC_E_ARG, "subdomain id %d listed twice", subs[k]);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return subs[a] < subs[b]; });
  }
  if (ctx->host_only) return no_device("apc_sum_images");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(ctx->order.ensure(sizeof(int) * n_sub));
  if ((st = stage_upload(ctx, ctx->order.p, order.data(), sizeof(int) * n_sub, s)) != APC_OK) return st;
  HIPCHK(apc::launch_sum_images(partials, n_sub, ctx->order.as<int>(), int64_t(H) * W, moments, bp, rgba, s));
  return APC_OK;
}

apc_status apc_get_counters(apc_ctx ctx, apc_counters* out, int32_t reset) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!out) return fail(APC_E_ARG, "out is NULL");
  if (ctx->host_only) return no_device("apc_get_counters");
  HIPCHK(hipDeviceSynchronize());
  unsigned long long c[apc::C_COUNT];
  HIPCHK(hipMemcpy(c, ctx->counters.p, sizeof(c), hipMemcpyDeviceToHost));
  out->pieces = int64_t(c[apc::C_PIECES]);
  out->tet_steps = int64_t(c[apc::C_STEPS]);
  out->entries = int64_t(c[apc::C_ENTRIES]);
  out->bin_records = ctx->bin_records;
  out->walk_step_limit = int64_t(c[apc::C_STEPLIMIT]);
  out->exit_fallback = int64_t(c[apc::C_FALLBACK]);
  out->entry_overflow = int64_t(c[apc::C_OVERFLOW]);
  out->nonpd_pivots = int64_t(c[apc::C_NONPD]);
  out->table_samples = int64_t(c[apc::C_TABLED]);
  out->table_fallback = int64_t(c[apc::C_TABFB]);
  out->segments = int64_t(c[apc::C_SEGMENTS]);
  if (reset) {
    HIPCHK(hipMemset(ctx->counters.p, 0, sizeof(c)));
    ctx->bin_records = 0;
  }
  return APC_OK;
}

apc_status apc_get_timings(apc_ctx ctx, apc_timings* out) {
  apc_status st = check_ctx(ctx);
  if (st != APC_OK) return st;
  if (!out) return fail(APC_E_ARG, "out is NULL");
  if (ctx->host_only) return no_device("apc_get_timings");
  double ms[EV_COUNT] = {};
  for (int k = 0; k < EV_COUNT; ++k) {
    if (!ctx->ev_used[k]) continue;
    HIPCHK(hipEventSynchronize(ctx->ev[k][1]));
    float v = 0.0f;
    HIPCHK(hipEventElapsedTime(&v, ctx->ev[k][0], ctx->ev[k][1]));
    ms[k] = v;
  }
  out->bin_ms = ms[EV_BIN];
  out->moments_ms = ms[EV_MOM];
  out->sum_ms = ms[EV_SUM];
  out->resolve_ms = ms[EV_RES];
  out->rewalk_ms = ms[EV_STG];
  out->eval_ms = ms[EV_EVL];
  return APC_OK;
}

}  // extern "C"
