// HIP kernels (gfx950) for the APC hot path.
//
// One frame = for the listed subdomains:
//   k_bin        boundary faces of each subdomain -> (tile, subdomain) bins
//                (count pass, exclusive scan, fill pass)
//   k_moments    one 64-lane wavefront per 8x8 pixel tile: per subdomain,
//                collect the boundary faces where each pixel ray enters the
//                subdomain, walk the ray tet by tet from each entry to where
//                it leaves the subdomain, cut every chord at the global
//                sampling lattice and add a*z^j per piece (paper Alg. 2)
//                (with every subdomain on one GPU it also sums them: the
//                global image; else per-subdomain images, dense or as tiles
//                of the (tile, subdomain) pairs that have boundary faces)
//   k_sum_moments / k_sum_tiles  canonical-order FP64 sum of per-subdomain
//                images or tiles (the paper's moment Allreduce, Section 4.1)
//   k_resolve    stage two, plain form: per tile a walker wavefront walks the
//                rays again and hands each piece (depth, length, scalar)
//                through LDS to an evaluator wavefront, which forms the piece's
//                optical and warped depths as stage one did, evaluates the
//                moment bound of its pixel (Alg. 3) and weights the piece's
//                colour by T = exp(-b0 F) (Alg. 1 second loop, Section 4.2)
//   k_eval       the same evaluation over pieces stage one kept (variant)
//   k_sum_images canonical-order sum of partial images + renormalisation
//
// Geometry.  A ray crosses a face iff its Plücker side products with the
// face's three edges share one sign.  Every edge product is computed with one
// formula whose two orientations give exactly opposite values, and an exact
// zero counts as positive in the orientation from the lower vertex id to the
// higher; the entry test of one subdomain and the exit test of the walk in
// its neighbour therefore see identical signs for the face they share, so
// every ray crosses each subdomain interface exactly once (no gaps, no double
// counting).  The barycentric coordinates of the
// crossing point are the three edge products of the face, which give the
// depth t and the scalar at the crossing.  Functions whose results must agree
// bit for bit between the two passes or between the entry test and the walk
// are compiled without floating-point contraction.
#include <float.h>

#include "apc_internal.h"
#include "apc_mboit.h"

namespace apc {
namespace {

constexpr int WAVE = 64;
constexpr int E_MAX = 16;    // entries per ray held at once (more are handled in further rounds)
constexpr int CHUNK = 64;    // boundary faces staged in LDS at a time

// outward vertex order of the face opposite vertex f of a positively oriented tet
__device__ __constant__ int kFaceOut[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

__device__ __forceinline__ int sel4(const int4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
// The same as an OR of masked components: every component is read (the four
// come from one load), and no branch or indexed access is left.
__device__ __forceinline__ int sel4m(const int4& v, int i) {
  return (v.x & -int(i == 0)) | (v.y & -int(i == 1)) | (v.z & -int(i == 2)) | (v.w & -int(i == 3));
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  The tiles are handed out in runs of XCD_RUN consecutive tiles, so
// neighbouring tiles (which read the same tets) share one XCD's L2, and
// every XCD gets runs from all over the image: the work of a view is
// concentrated where the volume projects, and one contiguous band of the
// image per XCD gave the busiest XCD twice the mean work.  Round k of 8 runs
// (runs 8k .. 8k+7) goes to the XCDs rotated by k: with run c on XCD c % 8,
// an image row of 4 runs (2048 pixels of 8-wide tiles) put the same quarter
// of every row on one XCD.  The blocks beyond the last whole round take the
// remaining tiles in bands.
#ifndef APC_XCD_RUN
#define APC_XCD_RUN 64
#endif
constexpr int XCD_RUN = APC_XCD_RUN;
__device__ __forceinline__ int xcd_tile(int b, int nb, int run = XCD_RUN) {
  const int whole = nb / (8 * run) * (8 * run);
  if (b < whole) {
    const int x = b & 7, i = b >> 3;
    const int k = i / run;
    return (k * 8 + ((x + k) & 7)) * run + (i - k * run);
  }
  b -= whole;
  nb -= whole;
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, i = b >> 3;
  return whole + x * q + (x < r ? x : r) + i;
}

// Persistent launches (a work queue): as many workgroups as the device holds
// at once, each taking tile after tile until none is left.  The tiles are
// the ones the ordinary launch of nb workgroups would give, per XCD in the
// same order: XCD x owns the tiles of the workgroups b = 8k + x, handed out
// by its own counter q[x]; a workgroup whose XCD has none left takes the next
// one of the following XCDs.  Called by one lane; -1 when all are taken.
__device__ __forceinline__ int queue_take(int* q, int nb) {
  const int x = blockIdx.x & 7;
  for (int d = 0; d < 8; ++d) {
    const int y = (x + d) & 7;
    const int own = (nb - y + 7) >> 3;  // workgroups b < nb with b % 8 == y
    if (__hip_atomic_load(q + y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= own) continue;
    const int k = atomicAdd(q + y, 1);
    if (k < own) return xcd_tile(8 * k + y, nb);
  }
  return -1;
}

// A pixel ray in FP64: origin o (moved forward by t_mid), unit direction d,
// and unit vectors a, b = d x a perpendicular to d, so that (a, b, d) is a
// right-handed orthonormal frame.
struct Ray {
  double ox, oy, oz, dx, dy, dz;
  double ax, ay, az, bx, by, bz;
};

__device__ __forceinline__ Ray pixel_ray(const FrameDev& f, int i, int j) {
#pragma clang fp contract(off)
  const double a = double(j) + 0.5, b = double(i) + 0.5;
  Ray r;
  double dx, dy, dz;
  if (f.proj == 0) {
    r.ox = f.ceye[0] + a * f.cright[0] + b * f.cdown[0];
    r.oy = f.ceye[1] + a * f.cright[1] + b * f.cdown[1];
    r.oz = f.ceye[2] + a * f.cright[2] + b * f.cdown[2];
    dx = f.cdir[0];
    dy = f.cdir[1];
    dz = f.cdir[2];
  } else {
    r.ox = f.ceye[0];
    r.oy = f.ceye[1];
    r.oz = f.ceye[2];
    const double aa = a - 0.5 * double(f.W), bb = b - 0.5 * double(f.H);
    dx = f.cdir[0] + aa * f.cright[0] + bb * f.cdown[0];
    dy = f.cdir[1] + aa * f.cright[1] + bb * f.cdown[1];
    dz = f.cdir[2] + aa * f.cright[2] + bb * f.cdown[2];
  }
  const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  r.dx = dx * inv;
  r.dy = dy * inv;
  r.dz = dz * inv;
  {
    // a = d x h / |d x h| for a coordinate axis h far from parallel to d
    const bool xs = fabs(r.dx) < 0.9;
    const double hx = xs ? 1.0 : 0.0, hy = xs ? 0.0 : 1.0;
    const double ax = -r.dz * hy, ay = r.dz * hx, az = r.dx * hy - r.dy * hx;
    const double ia = 1.0 / sqrt(ax * ax + ay * ay + az * az);
    r.ax = ax * ia;
    r.ay = ay * ia;
    r.az = az * ia;
    r.bx = r.dy * r.az - r.dz * r.ay;
    r.by = r.dz * r.ax - r.dx * r.az;
    r.bz = r.dx * r.ay - r.dy * r.ax;
  }
  // depth 0 at the middle of the depth range
  r.ox = r.ox + f.t_mid * r.dx;
  r.oy = r.oy + f.t_mid * r.dy;
  r.oz = r.oz + f.t_mid * r.dz;
  return r;
}

// A vertex as seen from one ray: id, scalar, depth t = d.(P-o) (FP64) and its
// coordinates u = a.(P-o), v = b.(P-o) in the plane perpendicular to the ray,
// computed in FP64 and rounded to FP32 (near the ray |u|, |v| are about a
// cell's size, so the rounding is ~1e-7 of a cell, not of the distance to
// the eye).
struct VS {
  int id;
  float s, u, v;
  double t;
};

__device__ __forceinline__ VS vstate(const Ray& r, int id, float4 p) {
#pragma clang fp contract(off)
  VS v;
  v.id = id;
  v.s = p.w;
  const double px = double(p.x) - r.ox, py = double(p.y) - r.oy, pz = double(p.z) - r.oz;
  v.t = r.dx * px + r.dy * py + r.dz * pz;
  v.u = float(r.ax * px + r.ay * py + r.az * pz);
  v.v = float(r.bx * px + r.by * py + r.bz * pz);
  return v;
}

// Oriented Plücker side product d.((a-o) x (b-o)) of the ray with the edge
// a -> b: only the components perpendicular to d contribute, so it is the 2D
// cross product u_a v_b - v_a u_b.  Without contraction the two orientations
// of an edge give exactly opposite values (the products are the same two
// roundings in either order), so every test that meets the edge sees one
// value up to sign; an exact zero counts as positive in the orientation from
// the lower vertex id to the higher.
__device__ __forceinline__ float side(const VS& a, const VS& b) {
#pragma clang fp contract(off)
  const float p = a.u * b.v - a.v * b.u;
  return p == 0.0f ? (a.id < b.id ? FLT_MIN : -FLT_MIN) : p;
}

// Crossing point of the ray with the face (A, B, C) whose oriented products
// pAB, pBC, pCA are all positive: barycentric weights (pBC, pCA, pAB).  The
// sums start at the vertex with the smallest id, so a walk that leaves its
// subdomain (or the mesh) through a face and the entry test of the tet behind
// it (which list the face's vertices in different rotations) get the same
// depth bit for bit.
// The depth is that vertex's FP64 depth plus the weighted depth differences
// across the face (at most a cell's extent, so FP32 keeps them to ~1e-7 of a
// cell, the precision of the weights themselves).
__device__ __forceinline__ void face_point(const VS& A, const VS& B, const VS& C, float pAB, float pBC, float pCA,
                                           double& t, float& s) {
#pragma clang fp contract(off)
  float uA = fmaxf(pBC, 0.0f), uB = fmaxf(pCA, 0.0f), uC = fmaxf(pAB, 0.0f);
  const bool bmin = B.id < A.id && B.id < C.id, cmin = C.id < A.id && C.id < B.id;
  const float u0 = bmin ? uB : (cmin ? uC : uA), u1 = bmin ? uC : (cmin ? uA : uB), u2 = bmin ? uA : (cmin ? uB : uC);
  const double t0 = bmin ? B.t : (cmin ? C.t : A.t), t1 = bmin ? C.t : (cmin ? A.t : B.t),
               t2 = bmin ? A.t : (cmin ? B.t : C.t);
  const float s0 = bmin ? B.s : (cmin ? C.s : A.s), s1 = bmin ? C.s : (cmin ? A.s : B.s),
              s2 = bmin ? A.s : (cmin ? B.s : C.s);
  float sum = u0 + u1 + u2;
  if (!(sum > 0.0f)) {
    t = t0;
    s = s0;
    return;
  }
  float inv = __builtin_amdgcn_rcpf(sum);  // 1 ulp; both passes alike
  t = t0 + double((u1 * float(t1 - t0) + u2 * float(t2 - t0)) * inv);
  s = (u0 * s0 + u1 * s1 + u2 * s2) * inv;
}

// The same crossing with A as the base vertex: the depth and scalar a walk
// hands from one tet to the next inside a subdomain, where only this walk
// meets the face.  Where the walk leaves the subdomain (the neighbouring
// subdomain's entry test meets the face too) face_point's ordering is used.
__device__ __forceinline__ void face_point_a(const VS& A, const VS& B, const VS& C, float pAB, float pBC, float pCA,
                                             double& t, float& s) {
#pragma clang fp contract(off)
  const float uA = fmaxf(pBC, 0.0f), uB = fmaxf(pCA, 0.0f), uC = fmaxf(pAB, 0.0f);
  const float sum = uA + uB + uC;
  if (!(sum > 0.0f)) {
    t = A.t;
    s = A.s;
    return;
  }
  const float inv = __builtin_amdgcn_rcpf(sum);
  t = A.t + double((uB * float(B.t - A.t) + uC * float(C.t - A.t)) * inv);
  s = (uA * A.s + uB * B.s + uC * C.s) * inv;
}

// A boundary face staged in LDS, vertices in outward order of its tet.
struct FaceL {
  int code;  // (tet << 2) | face
  int id0, id1, id2;
  float4 p0, p1, p2;
};

// Does the ray enter the face's tet through it?  On success returns the
// entry state: the face in inward order (A, B, C) with its positive
// products, and the entry depth/scalar.
struct Entry {
  VS A, B, C;
  float pAB, pBC, pCA, s;
  double t;
};

__device__ __forceinline__ bool enter_face(const Ray& r, int id0, int id1, int id2, float4 p0, float4 p1,
                                           float4 p2, Entry& e) {
  VS a = vstate(r, id0, p0), b = vstate(r, id1, p1), c = vstate(r, id2, p2);
  float sab = side(a, b), sbc = side(b, c), sca = side(c, a);
  if (!(sab < 0.0f && sbc < 0.0f && sca < 0.0f)) return false;
  // inward order (a, c, b): pi(a->c) = -sca, pi(c->b) = -sbc, pi(b->a) = -sab
  e.A = a;
  e.B = c;
  e.C = b;
  e.pAB = -sca;
  e.pBC = -sbc;
  e.pCA = -sab;
  face_point(e.A, e.B, e.C, e.pAB, e.pBC, e.pCA, e.t, e.s);
  return true;
}

// Per-lane event counts, summed over the wavefront at the end of a kernel.  Events that are rare by design
// (a walk cut off by its step limit, an exit face chosen by the tie fallback, an entry list or buffer that
// overflowed) go straight to the device counters instead, so they hold no register in the walk.
struct LaneCount {
  unsigned pieces, steps, entries, nonpd, tabled, tab_fallback, segments;
  unsigned long long* ctr;
  __device__ void rare(int which, unsigned n = 1u) {
    if (n) atomicAdd(ctr + which, (unsigned long long)n);
  }
};

// Cut the chord [t0, t1] (scalar s0 -> s1) at the lattice t_near + k*step and
// hand each piece (mid depth, length, scalar at the mid point) to fn.  The cut
// points and mid depths are FP64 (depths are absolute positions along the
// ray); lengths and scalars are FP32.
template <class Fn>
__device__ __forceinline__ void cut_chord(const FrameDev& f, double t0, double t1, float s0, float s1, Fn&& fn) {
#pragma clang fp contract(off)
  const double len = t1 - t0;
  if (!(len > 0.0)) return;
  const float slope = (s1 - s0) * __builtin_amdgcn_rcpf(float(len));
  // the first lattice point after t0 (the rounded floor can fall one short)
  double kf = floor((t0 - f.t_near) * f.inv_step) + 1.0;
  if (!(f.t_near + kf * f.step > t0)) kf += 1.0;
  double u = t0;
  for (int guard = 0; u < t1 && guard < (1 << 22); ++guard) {
    const double nxt = f.t_near + kf * f.step;
    kf += 1.0;
    const double v = fmin(nxt, t1);
    const double tm = 0.5 * (u + v);
    const float s = s0 + slope * float(tm - t0);
    fn(tm, float(v - u), s);
    u = v;
  }
}

// Transfer-function table coordinate of scalar s: entry i0 and fraction fr.
__device__ __forceinline__ void tf_coord(const FrameDev& f, float s, int& i0, float& fr) {
#pragma clang fp contract(off)
  float u = (s - f.s_min) * f.tf_scale;
  u = __builtin_amdgcn_fmed3f(u, 0.0f, float(f.n_tf - 1));  // clamp to [0, n_tf - 1] in one instruction
  i0 = min(int(u), f.n_tf - 2);
  fr = u - float(i0);
}

// Optical depth of a piece (Alg. 2: absorbance capped) from the transfer
// function's alpha at its scalar and its length, and its warped depth (log
// depth rescaled to [-1, 1]) from its mid depth measured from the eye (wt =
// tm + t_mid, rounded to FP32).
__device__ __forceinline__ float piece_a(const FrameDev& f, float A, float len) {
#pragma clang fp contract(off)
  return __builtin_amdgcn_fmed3f(f.kappa * A * len, 0.0f, f.amax);  // min with the cap (the product is >= 0)
}
__device__ __forceinline__ float piece_z(const FrameDev& f, float wt) {
#pragma clang fp contract(off)
  const float z = (__log2f(wt) - f.lg_near) * f.warp_scale - 1.0f;
  return fminf(fmaxf(z, -1.0f), 1.0f);
}
__device__ __forceinline__ void piece_az(const FrameDev& f, double tm, float len, float A, float& a, float& z) {
  a = piece_a(f, A, len);
  z = piece_z(f, float(tm + f.t_mid));
}

// Opacity 1 - e^-a of a piece of optical depth a >= 0: below 0.35 the Taylor
// polynomial of degree 7 (the first omitted term is under 2e-8 of the value),
// above it the hardware exponential (no cancellation there: e^-a < 0.71).
__device__ __forceinline__ float opacity(float a) {
  float p = 1.0f / 5040.0f;
  p = fmaf(p, -a, 1.0f / 720.0f);
  p = fmaf(p, -a, 1.0f / 120.0f);
  p = fmaf(p, -a, 1.0f / 24.0f);
  p = fmaf(p, -a, 1.0f / 6.0f);
  p = fmaf(p, -a, 0.5f);
  p = fmaf(p, -a, 1.0f);
  return a < 0.35f ? a * p : 1.0f - __expf(-a);
}

__device__ __forceinline__ float lerp_nc(float a, float b, float fr) {
#pragma clang fp contract(off)
  return a * (1.0f - fr) + b * fr;
}

// Where a walk stands: the face (A, B, C) through which the ray entered the
// current tet, with its positive side products, and the tet with the local
// index of the vertex opposite that face.
// a or b, field by field (value selects: no store through a selected address)
__device__ __forceinline__ VS pick(bool c, const VS& a, const VS& b) {
  VS r;
  r.id = c ? a.id : b.id;
  r.s = c ? a.s : b.s;
  r.u = c ? a.u : b.u;
  r.v = c ? a.v : b.v;
  r.t = c ? a.t : b.t;
  return r;
}

struct WalkPos {
  VS A, B, C;
  float pAB, pBC, pCA;
  int tet, apex;
};

__device__ __forceinline__ WalkPos walk_start(const Entry& e, int tet, int apex) {
  return WalkPos{e.A, e.B, e.C, e.pAB, e.pBC, e.pCA, tet, apex};
}

// One step of the walk: the face through which the ray leaves the current
// tet and the depth and scalar where it does (tout >= tin); the position moves
// to the tet behind that face.  Returns false when that face lies on the mesh
// hull or leads out of the subdomain (tet range [t_lo, t_hi)).
__device__ __forceinline__ bool walk_step(const MeshDev& M, const Ray& r, WalkPos& w, double tin, int t_lo, int t_hi,
                                          double& tout, float& sout, LaneCount& cnt) {
  // ids, neighbours and the apex vertex come from one 128-byte record, so
  // the three loads go out together (no vertex load waiting on the ids)
  const int4* rec = M.wrec + 8 * size_t(w.tet);
  const int4 tv = rec[0];
  const int4 tn = rec[1];
  const float4 dp = reinterpret_cast<const float4*>(rec)[2 + w.apex];
  const int did = sel4m(tv, w.apex);
  const VS D = vstate(r, did, dp);
  const float qA = side(D, w.A), qB = side(D, w.B), qC = side(D, w.C);
  // exit through the face opposite X where q(next of X) > 0 > q(previous of X)
  int x;
  if (qB > 0.0f && qC < 0.0f)
    x = 0;
  else if (qC > 0.0f && qA < 0.0f)
    x = 1;
  else if (qA > 0.0f && qB < 0.0f)
    x = 2;
  else {  // sign pattern no line can have (rounding near a vertex): least-violated face
    float m0 = fminf(qB, -qC), m1 = fminf(qC, -qA), m2 = fminf(qA, -qB);
    x = (m0 >= m1 && m0 >= m2) ? 0 : (m1 >= m2 ? 1 : 2);
    cnt.rare(C_FALLBACK);
  }
  const int xid = x == 0 ? w.A.id : (x == 1 ? w.B.id : w.C.id);
  // The exit face replaces X by D in place: (D, B, C), (A, D, C) and
  // (A, B, D) are rotations of the exit faces (B, C, D), (C, A, D) and
  // (A, B, D), so the cyclic order with positive products is kept.
  const float nAB = x == 0 ? qB : (x == 1 ? -qA : w.pAB);
  const float nBC = x == 0 ? w.pBC : (x == 1 ? qC : -qB);
  const float nCA = x == 0 ? -qC : (x == 1 ? w.pCA : qA);
  w.A = pick(x == 0, D, w.A);
  w.B = pick(x == 1, D, w.B);
  w.C = pick(x == 2, D, w.C);
  w.pAB = nAB;
  w.pBC = nBC;
  w.pCA = nCA;
  ++cnt.steps;
  const int xl = tv.x == xid ? 0 : (tv.y == xid ? 1 : (tv.z == xid ? 2 : 3));
  const int nb = sel4m(tn, xl);
  const int t2 = nb >> 2;
  const bool stays = nb >= 0 && t2 >= t_lo && t2 < t_hi;
  if (stays)
    face_point_a(w.A, w.B, w.C, w.pAB, w.pBC, w.pCA, tout, sout);
  else
    face_point(w.A, w.B, w.C, w.pAB, w.pBC, w.pCA, tout, sout);
  if (!(tout >= tin)) tout = tin;
  if (!stays) return false;
  w.tet = t2;
  w.apex = nb & 3;
  return true;
}

// Walk the ray from an entry through the tets of one subdomain (tet range
// [t_lo, t_hi)) until it leaves the subdomain, handing every chord to sink.
// `apex` is the local index of the vertex opposite the entry face.  (The loop
// body repeats walk_step's, written out: the stage-one kernel keeps fewer
// registers that way.)
template <class Sink>
__device__ void walk(const MeshDev& M, const FrameDev& f, const Ray& r, int tet, int apex, Entry e, int t_lo,
                     int t_hi, Sink& sink, LaneCount& cnt) {
  VS A = e.A, B = e.B, C = e.C;
  float pAB = e.pAB, pBC = e.pBC, pCA = e.pCA, sin_ = e.s;
  double tin = e.t;
  for (int step = 0;; ++step) {
    if (step >= f.max_steps) {
      cnt.rare(C_STEPLIMIT);
      return;
    }
    const int4* rec = M.wrec + 8 * size_t(tet);
    const int4 tv = rec[0];
    const int4 tn = rec[1];
    const float4 dp = reinterpret_cast<const float4*>(rec)[2 + apex];
    int did = sel4(tv, apex);
    VS D = vstate(r, did, dp);
    float qA = side(D, A), qB = side(D, B), qC = side(D, C);
    int x;
    if (qB > 0.0f && qC < 0.0f)
      x = 0;
    else if (qC > 0.0f && qA < 0.0f)
      x = 1;
    else if (qA > 0.0f && qB < 0.0f)
      x = 2;
    else {
      float m0 = fminf(qB, -qC), m1 = fminf(qC, -qA), m2 = fminf(qA, -qB);
      x = (m0 >= m1 && m0 >= m2) ? 0 : (m1 >= m2 ? 1 : 2);
      cnt.rare(C_FALLBACK);
    }
    const int xid = x == 0 ? A.id : (x == 1 ? B.id : C.id);
    const float nAB = x == 0 ? qB : (x == 1 ? -qA : pAB);
    const float nBC = x == 0 ? pBC : (x == 1 ? qC : -qB);
    const float nCA = x == 0 ? -qC : (x == 1 ? pCA : qA);
    A = pick(x == 0, D, A);
    B = pick(x == 1, D, B);
    C = pick(x == 2, D, C);
    pAB = nAB;
    pBC = nBC;
    pCA = nCA;
    double tout;
    float sout;
    int xl = tv.x == xid ? 0 : (tv.y == xid ? 1 : (tv.z == xid ? 2 : 3));
    int nb = sel4m(tn, xl);
    int t2 = nb >> 2;
    const bool stays = nb >= 0 && t2 >= t_lo && t2 < t_hi;
    if (stays)
      face_point_a(A, B, C, pAB, pBC, pCA, tout, sout);
    else
      face_point(A, B, C, pAB, pBC, pCA, tout, sout);
    if (!(tout >= tin)) tout = tin;
    ++cnt.steps;
    sink.chord(tin, tout, sin_, sout);
    if (!stays) return;
    tet = t2;
    apex = nb & 3;
    tin = tout;
    sin_ = sout;
  }
}

// Per-lane list of entries (depth, face code) in LDS, kept sorted by
// (depth, code); lane-minor layout so the 64 lanes hit distinct banks.
struct EntryList {
  float* t;  // [E_MAX][WAVE]
  int* c;
  int lane;
  __device__ float& T(int e) { return t[e * WAVE + lane]; }
  __device__ int& Cd(int e) { return c[e * WAVE + lane]; }
};

__device__ __forceinline__ bool key_less(float ta, int ca, float tb, int cb) {
  return ta < tb || (ta == tb && ca < cb);
}

// Stage a chunk of boundary-face records of one bin into LDS.
__device__ __forceinline__ void stage_faces(const MeshDev& M, const int* rec, int n, FaceL* faces, int lane) {
  if (lane < n) {
    int code = rec[lane];
    int t = code >> 2, fc = code & 3;
    int4 tv = M.tet[2 * t];
    FaceL F;
    F.code = code;
    F.id0 = sel4(tv, kFaceOut[fc][0]);
    F.id1 = sel4(tv, kFaceOut[fc][1]);
    F.id2 = sel4(tv, kFaceOut[fc][2]);
    F.p0 = M.vert[F.id0];
    F.p1 = M.vert[F.id1];
    F.p2 = M.vert[F.id2];
    faces[lane] = F;
  }
}

// LDS writes of a wavefront visible to all its lanes (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The next (up to EMAX) entries of this lane's ray into one subdomain after
// the key (last_t, last_c), sorted by (depth, code) into L; returns how many,
// and sets `more` when there were others beyond them.  Must be called by the
// whole wavefront (it stages faces cooperatively into the wavefront's own LDS
// slice, so a workgroup may hold several wavefronts walking different tiles).
template <int EMAX>
__device__ int collect_entries(const MeshDev& M, const Ray& r, bool want, const int* rec, int n_rec, FaceL* faces,
                               EntryList& L, float last_t, int last_c, bool& more) {
  int n = 0;
  more = false;
  for (int c0 = 0; c0 < n_rec; c0 += CHUNK) {
    int nc = min(CHUNK, n_rec - c0);
    wave_sync();  // every lane is done with the previous chunk
    stage_faces(M, rec + c0, nc, faces, L.lane);
    wave_sync();
    if (!want) continue;
    for (int k = 0; k < nc; ++k) {
      const FaceL& F = faces[k];
      Entry e;
      if (!enter_face(r, F.id0, F.id1, F.id2, F.p0, F.p1, F.p2, e)) continue;
      const float et = float(e.t);  // sort key: the entry depth rounded to FP32
      if (!key_less(last_t, last_c, et, F.code)) continue;  // walked in an earlier round
      if (n == EMAX) {
        more = true;
        if (!key_less(et, F.code, L.T(n - 1), L.Cd(n - 1))) continue;
        --n;  // evict the largest
      }
      int pos = n;
      while (pos > 0 && key_less(et, F.code, L.T(pos - 1), L.Cd(pos - 1))) {
        L.T(pos) = L.T(pos - 1);
        L.Cd(pos) = L.Cd(pos - 1);
        --pos;
      }
      L.T(pos) = et;
      L.Cd(pos) = F.code;
      ++n;
    }
  }
  return n;
}

// Entry k of the list: the boundary face it crosses, as an entry state.
__device__ __forceinline__ bool list_entry(const MeshDev& M, const Ray& r, EntryList& L, int k, Entry& e, int& t,
                                           int& fc) {
  const int code = L.Cd(k);
  t = code >> 2;
  fc = code & 3;
  const int4 tv = M.tet[2 * t];
  const int i0 = sel4(tv, kFaceOut[fc][0]), i1 = sel4(tv, kFaceOut[fc][1]), i2 = sel4(tv, kFaceOut[fc][2]);
  return enter_face(r, i0, i1, i2, M.vert[i0], M.vert[i1], M.vert[i2], e);  // true: it was listed so
}

// All entries of this lane's ray into one subdomain, walked in (depth, code)
// order.  Handles more than E_MAX entries by repeated rounds that pick the
// next E_MAX entries after the last one walked.  Must be called by the whole
// wavefront.
template <class Sink>
__device__ void walk_subdomain(const MeshDev& M, const FrameDev& f, const Ray& r, bool valid, const int* rec,
                               int n_rec, const SlotDev& sl, FaceL* faces, EntryList& L, Sink& sink,
                               LaneCount& cnt) {
  float last_t = -FLT_MAX;
  int last_c = -1;
  bool more = true;
  while (true) {
    bool want = valid && more;
    if (!__any(want)) break;
    const int n = collect_entries<E_MAX>(M, r, want, rec, n_rec, faces, L, last_t, last_c, more);
    if (more) cnt.rare(C_OVERFLOW);
    for (int k = 0; k < n; ++k) {
      Entry e;
      int t, fc;
      if (!list_entry(M, r, L, k, e, t, fc)) continue;  // cannot happen
      ++cnt.entries;
      const unsigned before = sink.pieces;
      walk(M, f, r, t, fc, e, sl.tet_begin, sl.tet_end, sink, cnt);
      cnt.segments += sink.pieces > before ? 1u : 0u;  // a maximal ray interval inside the subdomain
    }
    if (n > 0) {
      last_t = L.T(n - 1);
      last_c = L.Cd(n - 1);
    }
  }
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ void flush_one(unsigned v, unsigned long long* slot) {
  unsigned s = wave_sum(v);
  if ((threadIdx.x & (WAVE - 1)) == 0 && s) atomicAdd(slot, (unsigned long long)s);
}

__device__ __forceinline__ void flush_counts(const LaneCount& c, unsigned long long* ctr) {
  flush_one(c.pieces, ctr + C_PIECES);
  flush_one(c.steps, ctr + C_STEPS);
  flush_one(c.entries, ctr + C_ENTRIES);
  flush_one(c.nonpd, ctr + C_NONPD);
  flush_one(c.tabled, ctr + C_TABLED);
  flush_one(c.tab_fallback, ctr + C_TABFB);
  flush_one(c.segments, ctr + C_SEGMENTS);
}

// ------------------------------------------------------------------ stage one

// The moments accumulate in FP64: a ray crosses hundreds of pieces per
// subdomain at the largest workloads, where FP32 sums would drift by ~1e-5 of
// b0; FP64 adds cost the same issue slot as FP32 ones here and need no
// compensation terms.
// A lane's share of the piece store: the chunk it is filling and the pieces
// it kept so far (over all subdomains, in walk order).  Chunks come from a
// block of STORE_BLOCK chunks that the wavefront takes with one atomic; the
// block's state lives in LDS (its lanes diverge, so no register copy of it
// stays current).  One atomic per chunk on a single counter was measured to
// serialise: stage one took 5x as long.
typedef __attribute__((address_space(3))) volatile unsigned long long lds_vu64;
typedef __attribute__((address_space(3))) volatile int lds_vi32;
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane(unsigned(v & 0xffffffffull), l);
  const unsigned hi = __builtin_amdgcn_readlane(unsigned(v >> 32), l);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}
struct LaneStore {
  PieceStore ps;
  size_t slot;     // tile * 64 + lane
  unsigned kept;
  float* cur;      // where the next piece goes in the current chunk
  bool keep;
  // LDS: first chunk of the wavefront's block and the chunks of it handed
  // out.  Written by one lane and read by others in later divergent regions,
  // so volatile; LDS-addressed, so a read waits for LDS only (a generic
  // access would also wait for every piece store still in flight).
  lds_vu64* blk_base;
  lds_vi32* blk_used;
  // append one piece; lanes that start a chunk at this point get consecutive
  // chunks of the wavefront's block (and a new block when it runs out)
  __device__ void put(float z, float a, float s, int lane) {
    if (!keep) return;
    if ((kept & (PIECE_CHUNK - 1)) == 0) {
      const unsigned long long need = __ballot(1);
      const int leader = __builtin_ffsll(static_cast<long long>(need)) - 1;
      const int n = __popcll(need);
      const int r = __popcll(need & ((1ull << lane) - 1));
      const unsigned long long base = *blk_base;  // every lane reads the same word
      const int used = *blk_used;
      const int rem = STORE_BLOCK - used;
      unsigned long long fresh = 0;
      if (n > rem) {
        unsigned long long got = 0;
        if (lane == leader) got = atomicAdd(ps.next, (unsigned long long)STORE_BLOCK);
        fresh = readlane_u64(got, leader);
      }
      const unsigned long long id = r < rem ? base + used + r : fresh + (r - rem);
      if (lane == leader) {
        if (n > rem) {
          *blk_base = fresh;
          *blk_used = n - rem;
        } else {
          *blk_used = used + n;
        }
      }
      const unsigned k = kept / PIECE_CHUNK;
      if (id < static_cast<unsigned long long>(ps.n_chunks) && k < unsigned(ps.maxc)) {
        ps.ptab[slot * ps.maxc + k] = int(id);
        cur = ps.pool + size_t(id) * (PIECE_CHUNK * 3);
      } else {
        keep = false;
        atomicAdd(ps.next + 1, 1ull);
        return;
      }
    }
    cur[0] = z;
    cur[1] = a;
    cur[2] = s;
    cur += 3;
    ++kept;
  }
};

// KEEP: stage one also keeps every piece for stage two (the pieces then need
// not be walked again); fixed per launch, so the store costs no registers
// when it is off.
template <int M1, bool KEEP>
struct MomentSink {
  const FrameDev* f;
  const float* tfa;  // LDS alpha column of the table
  double b[M1];
  unsigned pieces;
  LaneStore st;      // st.keep false: pieces are not kept
  int lane;
  __device__ void chord(double t0, double t1, float s0, float s1) {
    cut_chord(*f, t0, t1, s0, s1, [&](double tm, float len, float s) {
      int i0;
      float fr, a, z;
      tf_coord(*f, s, i0, fr);
      float A = lerp_nc(tfa[i0], tfa[i0 + 1], fr);
      piece_az(*f, tm, len, A, a, z);
      double term = a;  // the powers in FP64 too: one conversion per piece, not one per moment
      const double zd = z;
#pragma unroll
      for (int j = 0; j < M1; ++j) {  // Alg. 2: moment j gains absorbance * depth^j
        b[j] += term;
        term *= zd;
      }
      if constexpr (KEEP) st.put(z, a, s, lane);
      ++pieces;
    });
  }
};

// Waves per SIMD the walk kernels are compiled for (register budget 512 / n).
#ifndef APC_WALK_WAVES
#define APC_WALK_WAVES 3
#endif

template <int M1, bool KEEP, bool QUEUE>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(APC_WALK_WAVES, 8))) void k_moments(MeshDev M, FrameDev f, const SlotDev* __restrict__ slots,
                                                  const int* __restrict__ offsets, const int* __restrict__ counts,
                                                  const int* __restrict__ records, const float* __restrict__ tf_rgba,
                                                  float* __restrict__ out, double* __restrict__ gacc,
                                                  int* __restrict__ pcount, int* __restrict__ segs, long long bin_cap,
                                                  PieceStore ps, unsigned long long* ctr, int* queue,
                                                  const int* __restrict__ pair_idx, const int* __restrict__ pair_list) {
  extern __shared__ float4 dyn_lds[];
  float* tfa = reinterpret_cast<float*>(dyn_lds);  // [n_tf] alpha column
  __shared__ FaceL faces[CHUNK];
  __shared__ float ent_t[E_MAX * WAVE];
  __shared__ int ent_c[E_MAX * WAVE];
  const int lane = threadIdx.x;
  for (int i = lane; i < f.n_tf; i += WAVE) tfa[i] = tf_rgba[4 * i + 3];
  __shared__ unsigned long long blk_base;
  __shared__ int blk_used;
  if (lane == 0) {
    blk_base = 0;
    blk_used = STORE_BLOCK;  // no block yet
  }
  __syncthreads();
  // a pair list (tiles form): this workgroup walks the one (tile, subdomain) pair blockIdx.x names;
  // else every subdomain of its tile
  int k_first = 0, k_end = f.n_slots;
  int tile = QUEUE ? __builtin_amdgcn_readfirstlane(lane == 0 ? queue_take(queue, f.n_tiles) : 0)
                   : xcd_tile(blockIdx.x, gridDim.x);
  if (!QUEUE && pair_list) {
    const int bin = pair_list[blockIdx.x];
    tile = bin / f.n_slots;
    k_first = bin - tile * f.n_slots;
    k_end = k_first + 1;
  }
  for (; tile >= 0;
       tile = QUEUE ? __builtin_amdgcn_readfirstlane(lane == 0 ? queue_take(queue, f.n_tiles) : 0) : -1) {
  const int tx = tile % f.tiles_x, ty = tile / f.tiles_x;
  const int px = (tx << f.tw_log2) + (lane & ((1 << f.tw_log2) - 1)),
            py = ty * (WAVE >> f.tw_log2) + (lane >> f.tw_log2);
  const bool valid = px < f.W && py < f.H;
  const Ray r = pixel_ray(f, valid ? py : 0, valid ? px : 0);
  const size_t HW = size_t(f.W) * f.H, pix = size_t(py) * f.W + px;
  EntryList L{ent_t, ent_c, lane};
  LaneCount cnt = {};
  cnt.ctr = ctr;
  int covering = 0;  // subdomains with at least one piece on this ray
  // the global sum's FP64 partials: in registers for m <= 6 (room within the register budget of 3
  // wavefronts per SIMD), else in the per-pixel scratch gacc; the same additions either way
  constexpr bool REG_ACC = M1 <= 7;
  double acc[REG_ACC ? M1 : 1];
  MomentSink<M1, KEEP> sink;  // one sink for all subdomains: its piece store runs across them
  sink.f = &f;
  sink.tfa = tfa;
  sink.st = LaneStore{ps, size_t(tile) * WAVE + lane, 0u, nullptr, ps.pool != nullptr && valid, (lds_vu64*)&blk_base,
                      (lds_vi32*)&blk_used};
  sink.lane = lane;
  for (int k = k_first; k < k_end; ++k) {
    const int bin = tile * f.n_slots + k;
    const int n_rec = counts[bin];
    sink.pieces = 0;
#pragma unroll
    for (int j = 0; j < M1; ++j) sink.b[j] = 0.0;
    if (n_rec > 0 && offsets[bin] + n_rec <= bin_cap) {
      const SlotDev sl = slots[k];
      walk_subdomain(M, f, r, valid, records + offsets[bin], n_rec, sl, faces, L, sink, cnt);
    } else if (n_rec > 0) {
      cnt.rare(C_OVERFLOW);  // binned beyond the record capacity (never on an eagerly sized workspace)
    }
    cnt.pieces += sink.pieces;
    if (gacc) {
      // the global sum in slot order, one FP64 partial per pixel: a subdomain without pieces adds an exact
      // zero, so only the others are read and written, and the first one needs no read
      if (valid && sink.pieces > 0) {
        double* g = gacc + pix;
#pragma unroll
        for (int j = 0; j < M1; ++j) {
          const double v = double(float(sink.b[j]));
          if constexpr (REG_ACC)
            acc[j] = covering > 0 ? acc[j] + v : v;
          else
            g[size_t(j) * HW] = covering > 0 ? g[size_t(j) * HW] + v : v;
        }
      }
    } else if (pair_idx) {  // tiles form: only pairs with binned faces, every lane (zeros outside the image)
      if (n_rec > 0) {
        const int p = pair_idx[bin];
        float* o = out + size_t(p) * M1 * WAVE + lane;
#pragma unroll
        for (int j = 0; j < M1; ++j) o[j * WAVE] = float(sink.b[j]);
      }
    } else if (valid) {
      float* o = out + size_t(k) * M1 * HW + pix;
#pragma unroll
      for (int j = 0; j < M1; ++j) o[size_t(j) * HW] = float(sink.b[j]);
    }
    covering += sink.pieces > 0 ? 1 : 0;
  }
  if (gacc && valid) {
    float* o = out + pix;
#pragma unroll
    for (int j = 0; j < M1; ++j) {
      double t = 0.0;
      if (covering > 0) {
        if constexpr (REG_ACC)
          t = acc[j];
        else
          t = gacc[size_t(j) * HW + pix];
      }
      o[size_t(j) * HW] = float(t);
    }
  }
  if (pcount) pcount[size_t(tile) * WAVE + lane] = int(cnt.pieces);
  if (segs && valid) {  // [2][H][W]: segments, covering subdomains
    segs[pix] = int(cnt.segments);
    segs[HW + pix] = covering;
  }
  flush_counts(cnt, ctr);
  }  // tiles
}

// ------------------------------------------------------------------ stage two, kept pieces
//
// When stage one kept its pieces, stage two evaluates them without a walk:
// one wavefront per tile takes the tile's pixels one at a time, and its 64
// lanes evaluate 64 consecutive pieces of that pixel with the pixel's factor
// from LDS; every pixel then adds its own contributions in a fixed order, so
// the sum is deterministic.

__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

template <int N, class R>
using LdsBound = apcm::Bound<N, R, apcm::StridedStore<(N + 1) * (N + 2) / 2, R, WAVE>>;

__device__ __forceinline__ float4 finalize_px(float4 acc, float b0, int finalize, int renormalize) {
  if (!finalize) return acc;
  if (!renormalize) return acc;
  float A = -expm1f(-b0);
  float sc = acc.w > 1e-30f ? A / acc.w : 0.0f;
  return make_float4(acc.x * sc, acc.y * sc, acc.z * sc, A);
}

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// The global moments b_0..b_2N of one pixel (zero for an invalid lane), from
// the FP32 image [2N+1][H][W] or its packed FP16 form [2N+3][H][W] (ln b0 and
// the mean, each as two halves, and the central moments); returns b0 in FP32.
template <int N, class R>
__device__ __forceinline__ float pixel_moments(const void* moments, int f16, bool valid, size_t pix, size_t HW,
                                               R* b) {
  constexpr int M1 = 2 * N + 1;
  float b0f;
  if (f16) {
    const _Float16* hm = static_cast<const _Float16*>(moments);
    const double lb0 = valid ? double(hm[pix]) + double(hm[HW + pix]) : -HUGE_VAL;
    b0f = float(exp(lb0));  // exp(-inf) = 0: background
    double c[M1];
    c[0] = 1.0;
    c[1] = 0.0;
#pragma unroll
    for (int k = 2; k < M1; ++k) c[k] = valid ? double(hm[size_t(k + 2) * HW + pix]) : 0.0;
    const double mu = valid ? double(hm[2 * HW + pix]) + double(hm[3 * HW + pix]) : 0.0;
    b[0] = R(b0f);
#pragma unroll
    for (int j = 1; j < M1; ++j) {  // beta_j = E[z^j] = sum_k C(j, k) mu^(j-k) E[(z - mu)^k]
      double sum = 0.0, binom = 1.0, pw = 1.0;
#pragma unroll
      for (int k = j; k >= 0; --k) {  // term k: C(j, k) c_k mu^(j-k)
        sum += binom * c[k] * pw;
        pw *= mu;
        binom = binom * double(k) / double(j - k + 1);
      }
      b[j] = R(sum * double(b0f));
    }
  } else {
    const float* fm = static_cast<const float*>(moments);
#pragma unroll
    for (int j = 0; j < M1; ++j) b[j] = valid ? R(fm[size_t(j) * HW + pix]) : R(0);
    b0f = valid ? fm[pix] : 0.0f;
  }
  return b0f;
}

// Moment bound for every staged piece of a tile and the per-pixel colour
// sums (Alg. 1 second loop, Alg. 3).  The tile's pixels are taken one at a
// time: the 64 lanes evaluate that pixel's consecutive pieces (so they share
// the pixel's factor and, with nearby depths, mostly the same branches), each
// lane keeps a partial sum, and a fixed butterfly adds the partials, so the
// result does not depend on scheduling.  For n >= 3 a pixel with at least
// TABLE_MIN_PIECES pieces first fills its gap table (one node per lane) and
// its pieces take their roots from it.
// Waves per SIMD the FP64 evaluation is compiled for (register budget 512 / n):
// the closed-form root solver is out of line, which keeps n = 4 within 168.
#ifndef APC_EVAL_WAVES
#define APC_EVAL_WAVES 3
#endif
#ifndef APC_EVAL_WAVES_N4
#define APC_EVAL_WAVES_N4 3
#endif
#ifndef APC_TABLE_MIN_PIECES
#define APC_TABLE_MIN_PIECES 128
#endif

// Wavefronts per workgroup of the evaluation: they share one copy of the
// transfer-function table in LDS (the per-pixel state is per wavefront).
constexpr int EVAL_WPB = 4;

template <int N, class R>
__global__ __launch_bounds__(WAVE * EVAL_WPB) __attribute__((amdgpu_waves_per_eu(N >= 4 ? APC_EVAL_WAVES_N4 : APC_EVAL_WAVES, 8))) void k_eval(
    FrameDev f, int tile_lo, int tile_hi, PieceStore ps, const int* __restrict__ pcount,
                                               const float* __restrict__ tf_rgba, const void* __restrict__ moments,
                                               BoundParams bp, float* __restrict__ rgba,
                                               unsigned long long* ctr) {
  extern __shared__ float4 dyn_lds[];
  float4* tf = dyn_lds;  // [n_tf] RGBA
  constexpr int M1 = 2 * N + 1;
  constexpr int NL = (N + 1) * (N + 2) / 2;
  constexpr bool TABLES = N >= 3;
  constexpr int TAB_ENTRIES = TABLES ? apcm::Gaps<N>::NODES * apcm::Gaps<N>::NC : 1;
  __shared__ R li_all[EVAL_WPB][NL * WAVE];  // per-pixel inverse Cholesky factors, lane-minor
  __shared__ R zs_all[EVAL_WPB][N * WAVE];   // per-pixel sorted zeros of the degree-N orthonormal polynomial
  __shared__ R b0_all[EVAL_WPB][WAVE], z1_all[EVAL_WPB][WAVE];
  __shared__ R tab_all[EVAL_WPB][TAB_ENTRIES];  // gap table of the pixel being evaluated
  __shared__ int mode_all[EVAL_WPB][WAVE];
  __shared__ int off_all[EVAL_WPB][WAVE + 1];  // piece offsets of the tile's pixels, relative to the tile
  for (int i = threadIdx.x; i < f.n_tf; i += WAVE * EVAL_WPB)
    tf[i] = make_float4(tf_rgba[4 * i], tf_rgba[4 * i + 1], tf_rgba[4 * i + 2], tf_rgba[4 * i + 3]);
  __syncthreads();  // the only workgroup barrier: every later wait is within a wavefront
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int tile = tile_lo + xcd_tile(blockIdx.x, gridDim.x, (XCD_RUN + EVAL_WPB - 1) / EVAL_WPB) * EVAL_WPB + wv;
  if (tile >= tile_hi) return;
  R* li_lds = li_all[wv];
  R* zs_lds = zs_all[wv];
  R* b0_lds = b0_all[wv];
  R* z1_lds = z1_all[wv];
  R* tab_lds = tab_all[wv];
  int* mode_lds = mode_all[wv];
  int* off_lds = off_all[wv];
  const int tx = tile % f.tiles_x, ty = tile / f.tiles_x;
  const int px = (tx << f.tw_log2) + (lane & ((1 << f.tw_log2) - 1)),
            py = ty * (WAVE >> f.tw_log2) + (lane >> f.tw_log2);
  const bool valid = px < f.W && py < f.H;
  const size_t HW = size_t(f.W) * f.H, pix = size_t(py) * f.W + px;
  const size_t slot0 = size_t(tile) * WAVE;
  // per-pixel offsets within the tile: scan of the piece counts.  A lane of stage one that could not keep
  // its pieces leaves its chunk table unset: then nothing is read (counted)
  const bool staged = ps.next[1] == 0;
  {
    int c = staged ? pcount[slot0 + lane] : 0;
    const int own = c;
    for (int o = 1; o < WAVE; o <<= 1) {
      const int up = __shfl_up(c, o, WAVE);
      if (lane >= o) c += up;
    }
    off_lds[lane] = c - own;
    if (lane == WAVE - 1) off_lds[WAVE] = c;
  }
  LaneCount cnt = {};
  cnt.ctr = ctr;
  if (!staged && lane == 0) cnt.rare(C_OVERFLOW);
  // per-pixel part of Alg. 3, once per pixel instead of once per sample
  float b0f = 0.0f;
  {
    LdsBound<N, R> bound;
    bound.Li.base = li_lds + lane;
    R b[M1], bias[2 * N], zs[N];
    b0f = pixel_moments<N, R>(moments, bp.moments_f16, valid, pix, HW, b);
#pragma unroll
    for (int j = 0; j < 2 * N; ++j) bias[j] = R(bp.bias[j]);
    cnt.nonpd += bound.setup(b, R(bp.alpha), bias, zs);
    b0_lds[lane] = bound.b0;
    z1_lds[lane] = bound.z1;
#pragma unroll
    for (int i = 0; i < N; ++i) zs_lds[i * WAVE + lane] = zs[i];
    mode_lds[lane] = valid ? bound.mode : 0;
  }
  wave_sync();
  const R eta = R(bp.eta);
  float4 mine = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int p = 0; p < WAVE; ++p) {  // uniform loop over the tile's pixels
    const int lo = off_lds[p], hi = off_lds[p + 1];
    const int md = mode_lds[p];
    if (lo == hi || md == 0) continue;
    // the pixel's factor, uniform over the wavefront: held in scalar registers
    apcm::Bound<N, R> bound;
#pragma unroll
    for (int k = 0; k < NL; ++k) bound.Li[k] = wave_uniform(li_lds[k * WAVE + p]);
    bound.b0 = b0_lds[p];
    bound.z1 = z1_lds[p];
    bound.mode = md;
    const apcm::StridedStore<N, R, WAVE> zs{zs_lds + p};
    bound.xlo = md == 2 ? zs[0] : R(1);
    bound.xhi = md == 2 ? zs[N - 1] : R(-1);
    // no zeros found (never expected for a positive definite factor): no shortcut, no table
    if (md == 2 && !(zs[0] < zs[N - 1])) {
      bound.xlo = R(1);
      bound.xhi = R(-1);
    }
    bool use_table = false;
    if constexpr (TABLES) {
      use_table = md == 2 && bound.xlo < bound.xhi && hi - lo >= APC_TABLE_MIN_PIECES;
      if (use_table) {
        apcm::TablePtr<N, R> tab{tab_lds};
        if (lane < apcm::Gaps<N>::NODES) bound.gap_node(zs, lane, tab);
        wave_sync();
      }
    }
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    const int* chunks = ps.ptab + (slot0 + p) * size_t(ps.maxc);
    // the pixel's first 64 chunk ids, one per lane, fetched before the loop
    const int n_ch = (hi - lo + PIECE_CHUNK - 1) / PIECE_CHUNK;
    const int my_ch = (lane < n_ch && lane < ps.maxc) ? chunks[lane] : 0;
    // the piece of step ib for this lane (z, a, s), or ok = false past the pixel's end.  Steps start at
    // lo + 64 k and a chunk holds 64 pieces, so a step's pieces are exactly chunk k of the pixel: its id is
    // the same for the whole wavefront (a scalar), and lane l reads the chunk's l-th record
    static_assert(PIECE_CHUNK == WAVE, "one evaluation step reads one chunk");
    auto fetch = [&](int ib, float& z, float& a, float& s, bool& ok) {
      ok = ib + lane < hi;
      const int k = (ib - lo) / PIECE_CHUNK;  // uniform
      const int ch = k < WAVE ? __builtin_amdgcn_readlane(my_ch, k) : __builtin_amdgcn_readfirstlane(chunks[k]);
      if (unsigned(ch) >= unsigned(ps.n_chunks)) {  // cannot happen when every lane kept its pieces; never read
        if (ok) cnt.rare(C_OVERFLOW);
        ok = false;
        return;
      }
      const float* pr = ps.pool + (size_t(ch) * PIECE_CHUNK + lane) * 3;
      if (!ok) return;
      z = pr[0];
      a = pr[1];
      s = pr[2];
    };
    float nz = 0.0f, na = 0.0f, ns = 0.0f;
    bool nok = false;
    if (lo < hi) fetch(lo, nz, na, ns, nok);
    for (int ib = lo; ib < hi; ib += WAVE) {  // uniform loop; the next step's piece is loaded first
      const float z = nz, a = na, s = ns;
      const bool ok = nok;
      if (ib + WAVE < hi) fetch(ib + WAVE, nz, na, ns, nok);
      if (!ok) continue;
      R F = R(0);
      bool closed = true;
      if constexpr (TABLES) {
        if (use_table) {
          closed = !bound.frac_before_tab(R(z), eta, zs, apcm::TablePtr<N, R>{tab_lds}, F);
          ++cnt.tabled;
          cnt.tab_fallback += closed ? 1u : 0u;
        }
      }
      if (closed) F = bound.frac_before(R(z), eta);  // the one inlined copy of the closed forms
      float T = __expf(-float(bound.b0 * F));
      T = fminf(fmaxf(T, 0.0f), 1.0f);
      int i0;
      float fr;
      tf_coord(f, s, i0, fr);
      const float4 t0 = tf[i0], t1 = tf[i0 + 1];
      const float w = T * opacity(a);
      a0 += w * lerp_nc(t0.x, t1.x, fr);
      a1 += w * lerp_nc(t0.y, t1.y, fr);
      a2 += w * lerp_nc(t0.z, t1.z, fr);
      a3 += w;
    }
    if (use_table) wave_sync();  // the next pixel's table overwrites this one
    a0 = wave_sum_f(a0);
    a1 = wave_sum_f(a1);
    a2 = wave_sum_f(a2);
    a3 = wave_sum_f(a3);
    if (lane == p) mine = make_float4(a0, a1, a2, a3);
  }
  if (valid) reinterpret_cast<float4*>(rgba)[pix] = finalize_px(mine, b0f, bp.finalize, bp.renormalize);
  flush_counts(cnt, ctr);
}

// ------------------------------------------------------------------ stage two, fused re-walk
//
// The plain form of stage two (Alg. 1 second loop, Section 4.2): every ray is
// walked again exactly like stage one (the same pieces with bit for bit the
// same warped depths and optical depths), and each piece is weighted at once
// by the transmittance the moment bound gives at its depth.  Per pixel nothing
// but (m + 1) moments in and 4 colour sums out, whatever the depth
// complexity; no piece is written to memory.
//
// Each tile is one workgroup of two wavefronts, a walker and an evaluator.
// The walk is bound by its dependent record loads and the evaluation by FP64
// arithmetic, and the evaluation's per-pixel state (inverse Cholesky factor,
// zeros of the degree-n orthonormal polynomial, continuation of the roots) is
// what limits how many wavefronts a SIMD holds.  Split this way neither
// wavefront holds the other's registers (three workgroups of two per SIMD,
// where one wavefront doing both fits two), and the evaluator's arithmetic
// fills the issue slots the walker spends waiting on memory.  The pieces pass
// through a ring of PQ slots per lane in LDS.  The two wavefronts meet at
// phase boundaries (workgroup barriers): at each the walker publishes how many
// pieces each lane has produced and the evaluator how many it has evaluated;
// between two boundaries the evaluator takes only pieces published at the
// earlier one and the walker writes only ring slots evaluated before it, so
// they never touch the same slot.  Per lane the pieces are evaluated in walk
// order, each with the roots the previous one left
// (apcm::Bound::frac_before_cont, n >= 3).
#ifndef APC_RES_EMAX
#define APC_RES_EMAX 8
#endif
constexpr int RES_EMAX = APC_RES_EMAX;  // entries per ray held at once in the re-walk
// walk steps a lane takes per iteration while its ring has room for another chord's pieces
#ifndef APC_RES_BURST
#define APC_RES_BURST 4
#endif
constexpr int RES_ROOM = 3;  // ring slots a walk step needs free (a chord of one tet rarely has more pieces)
#ifndef APC_PAIR_QUEUE
#define APC_PAIR_QUEUE 16
#endif
// evaluation rounds per phase at most (one piece per lane per round).  Measured on the large frame (m = 8):
// 4 rounds 148 ms, 6 130, 7 126, 8 132, 12 156, 16 192: fewer rounds keep the walker waiting for room, more
// keep it waiting at the boundary
#ifndef APC_PAIR_ROUNDS
#define APC_PAIR_ROUNDS 7
#endif
// the walker ends its phase once this many 64ths of its lanes that still walk cannot take a step
#ifndef APC_PAIR_BLOCKED
#define APC_PAIR_BLOCKED 16
#endif
// wavefronts per SIMD the kernel is compiled for (register budget 512 / n)
#ifndef APC_PAIR_WAVES
#define APC_PAIR_WAVES 3
#endif
constexpr int PQ = APC_PAIR_QUEUE;
static_assert((PQ & (PQ - 1)) == 0, "the ring size is a power of two");

struct PairLDS {
  float q[3][PQ * WAVE];  // wt, len, s of ring slot j of lane l at j * WAVE + l (the 64 lanes hit distinct banks)
  int tail[2][WAVE];      // pieces lane l has produced, published at the boundaries of each parity
  int head[2][WAVE];      // pieces of lane l evaluated
  int done[2];            // the walker has no more pieces
};

// The walker's side: the chord being cut (bit for bit cut_chord's arithmetic,
// resumable when the ring is full) and the ring position.  A piece goes into
// the ring raw -- depth from the eye, length, scalar -- and the evaluator
// forms its optical depth and warped depth (piece_a, piece_z, the arithmetic
// of stage one): the walker's divergent cutting loop stays short.
struct Producer {
  PairLDS* sh;
  int lane, parity;
  int tail;   // pieces produced
  int limit;  // ring slots free up to here (evaluated count at the last boundary + PQ)
  unsigned pieces;
  bool cutting;
  double cu, ckf, ct0, ct1;
  float cs0, cslope;
  int cguard;

  __device__ __forceinline__ void start_cut(const FrameDev& f, double t0, double t1, float s0, float s1) {
#pragma clang fp contract(off)
    const double len_c = t1 - t0;
    cutting = len_c > 0.0;
    if (!cutting) return;
    cslope = (s1 - s0) * __builtin_amdgcn_rcpf(float(len_c));  // as cut_chord
    ckf = floor((t0 - f.t_near) * f.inv_step) + 1.0;
    if (!(f.t_near + ckf * f.step > t0)) ckf += 1.0;
    cu = t0;
    ct0 = t0;
    ct1 = t1;
    cs0 = s0;
    cguard = 0;
  }
  // ring the pieces of the chord being cut until it ends or the ring is full
  __device__ __forceinline__ void cut_more(const FrameDev& f) {
#pragma clang fp contract(off)
    while (cutting && tail < limit) {
      if (!(cu < ct1) || cguard >= (1 << 22)) {
        cutting = false;
        break;
      }
      ++cguard;
      const double nxt = f.t_near + ckf * f.step;
      ckf += 1.0;
      const double v = fmin(nxt, ct1);
      const double tm = 0.5 * (cu + v);
      const float s = cs0 + cslope * float(tm - ct0);
      const int slot = (tail & (PQ - 1)) * WAVE + lane;
      sh->q[0][slot] = float(tm + f.t_mid);
      sh->q[1][slot] = float(v - cu);
      sh->q[2][slot] = s;
      ++tail;
      ++pieces;
      cu = v;
    }
  }
  __device__ __forceinline__ bool can_step() const { return tail <= limit - RES_ROOM; }
  // phase boundary (the whole walker wavefront): publish, meet the evaluator, learn what it evaluated
  __device__ __forceinline__ void boundary(bool finished) {
    sh->tail[parity][lane] = tail;
    if (lane == 0) sh->done[parity] = finished ? 1 : 0;
    __syncthreads();
    limit = sh->head[parity][lane] + PQ;
    parity ^= 1;
  }
};

// All entries of this lane's ray into one subdomain, walked in (depth, code)
// order as in walk_subdomain (same pieces, same order), one entry start, the
// rest of a chord or a few walk steps per lane per iteration of a loop the
// whole walker wavefront runs; a lane whose ring has no room waits, and the
// wavefront ends its phase when enough of its lanes wait.
__device__ void walk_subdomain_paired(const MeshDev& M, const FrameDev& f, const Ray& r, bool valid, const int* rec,
                                      int n_rec, const SlotDev& sl, FaceL* faces, EntryList& L, Producer& q,
                                      LaneCount& cnt) {
  float last_t = -FLT_MAX;
  int last_c = -1;
  bool more = true;
  while (true) {
    const bool want = valid && more;
    if (!__any(want)) break;
    const int n = collect_entries<RES_EMAX>(M, r, want, rec, n_rec, faces, L, last_t, last_c, more);
    if (more) cnt.rare(C_OVERFLOW);
    int k = 0, steps = 0;
    bool walking = false, open = false;  // a walk in progress; an entry whose segment is still counted
    unsigned seg_start = 0;
    WalkPos w;
    double tin = 0.0;
    float sin_ = 0.0f;
    while (true) {
      const bool busy = q.cutting || walking || k < n;
      const unsigned long long act = __ballot(busy);
      if (!act) break;
      if (!q.cutting && !walking && k < n) {  // the next entry
        Entry e;
        int t, fc;
        if (list_entry(M, r, L, k, e, t, fc)) {
          ++cnt.entries;
          w = walk_start(e, t, fc);
          tin = e.t;
          sin_ = e.s;
          walking = true;
          steps = 0;
          open = true;
          seg_start = q.pieces;
        }
        ++k;
      }
      if (q.cutting) q.cut_more(f);  // the rest of a chord that did not fit the ring
      for (int burst = 0; burst < APC_RES_BURST; ++burst) {  // a uniform loop: lanes that stop just idle
        const bool act = !q.cutting && walking && q.can_step();
        if (!__any(act)) break;
        if (act) {
          if (steps >= f.max_steps) {
            cnt.rare(C_STEPLIMIT);
            walking = false;
          } else {
            double tout;
            float sout;
            walking = walk_step(M, r, w, tin, sl.tet_begin, sl.tet_end, tout, sout, cnt);
            ++steps;
            q.start_cut(f, tin, tout, sin_, sout);
            q.cut_more(f);
            tin = tout;
            sin_ = sout;
          }
        }
      }
      if (open && !walking && !q.cutting) {  // a maximal ray interval inside the subdomain ended
        cnt.segments += q.pieces > seg_start ? 1u : 0u;
        open = false;
      }
      // lanes that still have work here but no room to go on
      const bool stuck = (q.cutting || walking || k < n) && !(q.cutting ? q.tail < q.limit : q.can_step());
      const unsigned long long blocked = __ballot(stuck);
      const unsigned long long still = __ballot(q.cutting || walking || k < n);
      if (blocked && (blocked == still || __popcll(blocked) * 64 >= APC_PAIR_BLOCKED * __popcll(still)))
        q.boundary(false);
    }
    if (n > 0) {
      last_t = L.T(n - 1);
      last_c = L.Cd(n - 1);
    }
  }
}

template <int N, class R, bool QUEUE, bool PAIRS>
__global__ __launch_bounds__(2 * WAVE) __attribute__((amdgpu_waves_per_eu(APC_PAIR_WAVES, 8))) void k_resolve(
    MeshDev M, FrameDev f, const SlotDev* __restrict__ slots, const int* __restrict__ offsets,
    const int* __restrict__ counts, const int* __restrict__ records, long long bin_cap,
    const float* __restrict__ tf_rgba, const void* __restrict__ moments, BoundParams bp, float* __restrict__ rgba,
    unsigned long long* ctr, int* queue, const int* __restrict__ pair_list, float* __restrict__ part) {
  extern __shared__ float4 dyn_lds[];
  float4* tf = dyn_lds;  // [n_tf] RGBA
  __shared__ FaceL faces[CHUNK];
  __shared__ float ent_t[RES_EMAX * WAVE];
  __shared__ int ent_c[RES_EMAX * WAVE];
  __shared__ PairLDS sh;
  __shared__ int next_tile;
  for (int i = threadIdx.x; i < f.n_tf; i += 2 * WAVE)
    tf[i] = make_float4(tf_rgba[4 * i], tf_rgba[4 * i + 1], tf_rgba[4 * i + 2], tf_rgba[4 * i + 3]);
  // PAIRS (a launch over pair_list): this workgroup walks the one (tile, subdomain) pair `pair` and writes
  // its colour sums, unfinalised, to part[pair]; else every subdomain of its tile, into the image
  int pair = 0, k_first = 0, k_end = f.n_slots;
  if constexpr (PAIRS) {
    pair = xcd_tile(blockIdx.x, gridDim.x);
    k_first = pair_list[pair] % f.n_slots;
    k_end = k_first + 1;
  }
  if (threadIdx.x == 0)
    next_tile = QUEUE ? queue_take(queue, f.n_tiles)
                      : PAIRS ? pair_list[pair] / f.n_slots : xcd_tile(blockIdx.x, gridDim.x);
  __syncthreads();
  for (int tile = next_tile; tile >= 0;) {  // the same tiles for both wavefronts of the workgroup
  const bool walker = threadIdx.x < WAVE;
  const int lane = threadIdx.x % WAVE;
  const int tx = tile % f.tiles_x, ty = tile / f.tiles_x;
  const int px = (tx << f.tw_log2) + (lane & ((1 << f.tw_log2) - 1)),
            py = ty * (WAVE >> f.tw_log2) + (lane >> f.tw_log2);
  const bool valid = px < f.W && py < f.H;
  LaneCount cnt = {};
  cnt.ctr = ctr;
  if (walker) {
    const Ray r = pixel_ray(f, valid ? py : 0, valid ? px : 0);
    Producer q;
    q.sh = &sh;
    q.lane = lane;
    q.parity = 0;
    q.tail = 0;
    q.limit = PQ;
    q.pieces = 0u;
    q.cutting = false;
    EntryList L{ent_t, ent_c, lane};
    for (int k = k_first; k < k_end; ++k) {
      const int bin = tile * f.n_slots + k;
      const int n_rec = counts[bin];
      if (n_rec > 0 && offsets[bin] + n_rec <= bin_cap)
        walk_subdomain_paired(M, f, r, valid, records + offsets[bin], n_rec, slots[k], faces, L, q, cnt);
      else if (n_rec > 0)
        cnt.rare(C_OVERFLOW);  // binned beyond the record capacity (never on an eagerly sized workspace)
    }
    q.boundary(true);
    cnt.pieces += q.pieces;
  } else {
    const size_t HW = size_t(f.W) * f.H, pix = size_t(py) * f.W + px;
    // per-pixel part of Alg. 3, once per pixel instead of once per sample; the bound, its zeros and the
    // continuation are separate locals (a structure holding a run-time indexed array would live in scratch)
    apcm::Bound<N, R> bound;
    apcm::RegArray<N, R> zs;
    typename apcm::Bound<N, R>::Cont cont;
    cont.k = -1;
#pragma unroll
    for (int c = 0; c < int(sizeof(cont.v) / sizeof(R)); ++c) cont.v[c] = R(0);
    float b0f;
    {
      R b[2 * N + 1], bias[2 * N], zsr[N];
      b0f = pixel_moments<N, R>(moments, bp.moments_f16, valid, pix, HW, b);
#pragma unroll
      for (int j = 0; j < 2 * N; ++j) bias[j] = R(bp.bias[j]);
      cnt.nonpd += bound.setup(b, R(bp.alpha), bias, zsr);
#pragma unroll
      for (int i = 0; i < N; ++i) zs.v[i] = zsr[i];
      // no zeros found (never expected for a positive definite factor): no shortcut, every sample solves
      if (bound.mode == 2 && !(zsr[0] < zsr[N - 1])) {
        bound.xlo = -R(HUGE_VAL);
        bound.xhi = R(HUGE_VAL);
      }
    }
    const R eta = R(bp.eta);
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    unsigned solved = 0u, closed_used = 0u;  // samples needing roots; of those, by the closed forms
    int head = 0, avail = 0, parity = 0;
    auto eval_one = [&]() {  // Alg. 1 second loop with Alg. 3's bound, for the piece at `head`
      const int slot = (head & (PQ - 1)) * WAVE + lane;
      const float wt = sh.q[0][slot], len = sh.q[1][slot], s = sh.q[2][slot];
      ++head;
      if (bound.mode == 0) return;  // no absorbance on the ray: every piece has a = 0
      int i0;
      float fr;
      tf_coord(f, s, i0, fr);
      const float4 c0 = tf[i0], c1 = tf[i0 + 1];
      const float a = piece_a(f, lerp_nc(c0.w, c1.w, fr), len), z = piece_z(f, wt);  // as stage one
      R F;
      if constexpr (N >= 3) {
        int how;
        F = bound.frac_before_cont(R(z), eta, zs, cont, how);
        solved += how != 0 ? 1u : 0u;
        closed_used += how == 2 ? 1u : 0u;
      } else {
        F = bound.frac_before(R(z), eta);
      }
      float T = __expf(-float(bound.b0 * F));
      T = fminf(fmaxf(T, 0.0f), 1.0f);
      const float w = T * opacity(a);
      a0 += w * lerp_nc(c0.x, c1.x, fr);
      a1 += w * lerp_nc(c0.y, c1.y, fr);
      a2 += w * lerp_nc(c0.z, c1.z, fr);
      a3 += w;
    };
    while (true) {  // one phase per iteration, as many as the walker has
      for (int round = 0; round < APC_PAIR_ROUNDS && __any(head < avail); ++round)
        if (head < avail) eval_one();
      sh.head[parity][lane] = head;
      __syncthreads();
      avail = sh.tail[parity][lane];
      const bool fin = sh.done[parity] != 0;
      parity ^= 1;
      if (fin) break;
    }
    while (__any(head < avail))
      if (head < avail) eval_one();
    cnt.tabled += solved;
    cnt.tab_fallback += closed_used;
    if constexpr (PAIRS) {  // [pairs][4][64], every lane
      float* o = part + size_t(pair) * 4 * WAVE + lane;
      o[0] = a0;
      o[WAVE] = a1;
      o[2 * WAVE] = a2;
      o[3 * WAVE] = a3;
    } else if (valid) {
      reinterpret_cast<float4*>(rgba)[pix] =
          finalize_px(make_float4(a0, a1, a2, a3), b0f, bp.finalize, bp.renormalize);
    }
  }
  flush_counts(cnt, ctr);
  if (!QUEUE) break;
  // both wavefronts are done with the tile (and with next_tile): take the next one
  __syncthreads();
  if (threadIdx.x == 0) next_tile = queue_take(queue, f.n_tiles);
  __syncthreads();
  tile = next_tile;
  }  // tiles
}

// walk records: [ids][neighbours][v0][v1][v2][v3], 8 x 16 bytes per tet
__global__ void k_walk_records(const int4* __restrict__ tet, const float4* __restrict__ vert, int64_t n,
                               int4* __restrict__ wrec) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int4 tv = tet[2 * t];
  int4* o = wrec + 8 * t;
  o[0] = tv;
  o[1] = tet[2 * t + 1];
  float4* ov = reinterpret_cast<float4*>(o + 2);
  ov[0] = vert[tv.x];
  ov[1] = vert[tv.y];
  ov[2] = vert[tv.z];
  ov[3] = vert[tv.w];
}

// ------------------------------------------------------------------ binning

__device__ __forceinline__ void project_px(const FrameDev& f, float4 p, float& col, float& row, bool& ok) {
  const float* Minv = f.minv;
  // solve [dir right down] (l, la, lb)^T = p - eye
  float yx = p.x - f.ex, yy = p.y - f.ey, yz = p.z - f.ez;
  float l = Minv[0] * yx + Minv[1] * yy + Minv[2] * yz;
  float la = Minv[3] * yx + Minv[4] * yy + Minv[5] * yz;
  float lb = Minv[6] * yx + Minv[7] * yy + Minv[8] * yz;
  if (f.proj == 0) {
    col = la - 0.5f;
    row = lb - 0.5f;
    ok = true;
  } else {
    ok = l > 1e-6f;
    float il = 1.0f / l;
    col = la * il + f.half_w - 0.5f;
    row = lb * il + f.half_h - 0.5f;
  }
}

__global__ void k_bin(MeshDev M, FrameDev f, const SlotDev* __restrict__ slots,
                      const int* __restrict__ bface, int* __restrict__ counts, const int* __restrict__ offsets,
                      int* __restrict__ cursors, int* __restrict__ records, int fill, long long rec_cap) {
  const int k = blockIdx.y;
  const SlotDev sl = slots[k];
  const int i = sl.face_begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sl.face_end) return;
  const int code = bface[i];
  const int t = code >> 2, fc = code & 3;
  const int4 tv = M.tet[2 * t];
  const float4 a = M.vert[sel4(tv, kFaceOut[fc][0])];
  const float4 b = M.vert[sel4(tv, kFaceOut[fc][1])];
  const float4 c = M.vert[sel4(tv, kFaceOut[fc][2])];
  // conservative back-face cull: drop faces every ray crosses outwards
  {
    float ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z, vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
    float nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
    float nn = sqrtf(nx * nx + ny * ny + nz * nz);
    float gx, gy, gz;
    if (f.proj == 0) {
      gx = f.dx;
      gy = f.dy;
      gz = f.dz;
    } else {
      gx = a.x - f.ex;
      gy = a.y - f.ey;
      gz = a.z - f.ez;
    }
    float gn = sqrtf(gx * gx + gy * gy + gz * gz);
    if (gx * nx + gy * ny + gz * nz > 1e-4f * gn * nn) return;
  }
  float cmin = FLT_MAX, cmax = -FLT_MAX, rmin = FLT_MAX, rmax = -FLT_MAX;
  bool all_ok = true;
  const float4 pts[3] = {a, b, c};
  for (int q = 0; q < 3; ++q) {
    float col, row;
    bool ok;
    project_px(f, pts[q], col, row, ok);
    all_ok = all_ok && ok;
    cmin = fminf(cmin, col);
    cmax = fmaxf(cmax, col);
    rmin = fminf(rmin, row);
    rmax = fmaxf(rmax, row);
  }
  int c0, c1, r0, r1;
  if (!all_ok || !(cmax - cmin < 1e7f) || !(rmax - rmin < 1e7f)) {
    c0 = 0;
    r0 = 0;
    c1 = f.W - 1;
    r1 = f.H - 1;
  } else {
    if (cmax < -2.0f || rmax < -2.0f || cmin > float(f.W) + 1.0f || rmin > float(f.H) + 1.0f) return;
    c0 = max(0, int(floorf(cmin)) - 1);
    r0 = max(0, int(floorf(rmin)) - 1);
    c1 = min(f.W - 1, int(ceilf(cmax)) + 1);
    r1 = min(f.H - 1, int(ceilf(rmax)) + 1);
    if (c0 > c1 || r0 > r1) return;
  }
  const int th = WAVE >> f.tw_log2;
  for (int ty = r0 / th; ty <= r1 / th; ++ty)
    for (int tx = c0 >> f.tw_log2; tx <= (c1 >> f.tw_log2); ++tx) {
      const int bin = (ty * f.tiles_x + tx) * f.n_slots + k;
      if (!fill) {
        atomicAdd(counts + bin, 1);
      } else {
        const int pos = offsets[bin] + atomicAdd(cursors + bin, 1);
        if (pos < rec_cap) records[pos] = code;  // the walks skip bins beyond the capacity
      }
    }
}

// ------------------------------------------------------------------ sums

__global__ void k_sum_moments(const float* __restrict__ in, int n_slots, const int* __restrict__ order,
                              int64_t elems, float* __restrict__ out) {
  int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
  if (i >= elems) return;
  if (i + 4 <= elems && (elems & 3) == 0) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int k = 0; k < n_slots; ++k) {
      const float4 v = *reinterpret_cast<const float4*>(in + int64_t(order[k]) * elems + i);
      s0 += v.x;
      s1 += v.y;
      s2 += v.z;
      s3 += v.w;
    }
    *reinterpret_cast<float4*>(out + i) = make_float4(float(s0), float(s1), float(s2), float(s3));
  } else {
    for (int64_t e = i; e < elems && e < i + 4; ++e) {
      double s = 0;
      for (int k = 0; k < n_slots; ++k) s += in[int64_t(order[k]) * elems + e];
      out[e] = float(s);
    }
  }
}

// The tiles form's pairs: bin b = tile * n_slots + slot with binned faces is pair pidx[b] (exclusive scan of
// the flags, so in bin order); pair_bin lists the bins of the pairs in that order.
__global__ void k_pair_flags(const int* __restrict__ counts, int64_t nb, int* __restrict__ flags) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b < nb) flags[b] = counts[b] > 0 ? 1 : 0;
}
__global__ void k_pair_list(const int* __restrict__ counts, int64_t nb, const int* __restrict__ pidx,
                            int* __restrict__ pair_bin) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b < nb && counts[b] > 0) pair_bin[pidx[b]] = int(b);
}

// Global moments from the tiles form: pixel (tile t, lane l) adds, for the pairs of tile t in slot order
// (ascending subdomain ids), tile p's value at lane l in FP64 -- the additions of k_sum_moments without the
// pairs' zeros (adding an exact 0 changes nothing), so the result is bitwise the dense form's.  A tile's
// pairs are contiguous in pair_bin (ascending): found by binary search.
__global__ void k_sum_tiles(const float* __restrict__ tiles, const int* __restrict__ pair_bin, int64_t n_pairs,
                            int n_slots, int m1, int W, int H, int tw_log2, float* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t HW = int64_t(W) * H;
  if (i >= HW) return;
  const int y = int(i / W), x = int(i - int64_t(y) * W);
  const int tw = 1 << tw_log2, th = WAVE >> tw_log2;
  const int tiles_x = (W + tw - 1) / tw;
  const int tile = (y / th) * tiles_x + (x >> tw_log2);
  const int lane = (y % th) * tw + (x & (tw - 1));
  const int64_t first_bin = int64_t(tile) * n_slots;
  int64_t lo = 0, hi = n_pairs;  // first pair with pair_bin >= first_bin
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (pair_bin[mid] < first_bin)
      lo = mid + 1;
    else
      hi = mid;
  }
  double acc[9];
  for (int j = 0; j < m1; ++j) acc[j] = 0.0;
  for (int64_t p = lo; p < n_pairs && pair_bin[p] < first_bin + n_slots; ++p) {
    const float* t = tiles + p * m1 * WAVE + lane;
    for (int j = 0; j < m1; ++j) acc[j] += double(t[j * WAVE]);
  }
  for (int j = 0; j < m1; ++j) out[int64_t(j) * HW + i] = float(acc[j]);
}

// FP16 moment image, planes [m+3][pixels]: ln b0 (-inf on background) and the mean depth mu = beta_1, each as
// two FP16 halves (hi, and the rest lo); the central moments E[(z - mu)^k] (mu = hi + lo), k = 2..m.  Central
// moments keep the spread of a concentrated depth distribution at FP16's relative precision, which raw moments
// (all near mu^j) lose; the split ln b0 keeps the opacity 1 - exp(-b0) near FP32 precision.
__global__ void k_pack_f16(const float* __restrict__ in, int m1, int64_t pixels, _Float16* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= pixels) return;
  const float b0 = in[i];
  const bool bg = !(b0 > 0.0f);
  const double lb0 = bg ? 0.0 : log(double(b0));
  const _Float16 lhi = _Float16(lb0);
  out[i] = bg ? _Float16(-HUGE_VALF) : lhi;
  out[pixels + i] = bg ? _Float16(0.0f) : _Float16(lb0 - double(lhi));
  const double inv = bg ? 0.0 : 1.0 / double(b0);
  double beta[9];
  beta[0] = 1.0;
  for (int j = 1; j < m1; ++j) beta[j] = double(in[int64_t(j) * pixels + i]) * inv;
  const _Float16 hi = _Float16(beta[1]);
  const _Float16 lo = _Float16(beta[1] - double(hi));
  const double mu = double(hi) + double(lo);
  out[2 * pixels + i] = bg ? _Float16(0.0f) : hi;
  out[3 * pixels + i] = bg ? _Float16(0.0f) : lo;
  for (int k = 2; k < m1; ++k) {
    // E[(z - mu)^k] = sum_i C(k, i) (-mu)^(k-i) beta_i, Horner in (-mu) with running binomials
    double c = 0.0, binom = 1.0, pw = 1.0;
    for (int t = k; t >= 0; --t) {  // term t: C(k, t) beta_t (-mu)^(k-t)
      c += binom * beta[t] * pw;
      pw *= -mu;
      binom = binom * double(t) / double(k - t + 1);
    }
    out[int64_t(k + 2) * pixels + i] = bg ? _Float16(0.0f) : _Float16(c);
  }
}

// Stage two by pairs: pixel (tile t, lane l) adds the colour sums of tile t's pairs at lane l in slot order
// (ascending subdomain ids) in FP64, then finalises with its b0 (FP32 moment image plane 0) -- the
// per-subdomain partial images' canonical sum, taken over the pairs only (a subdomain without a pair on
// the tile has no piece there).
__global__ void k_sum_color_tiles(const float* __restrict__ part, const int* __restrict__ pair_bin, int64_t n_pairs,
                                  int n_slots, int W, int H, int tw_log2, const float* __restrict__ b0,
                                  BoundParams bp, float4* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t HW = int64_t(W) * H;
  if (i >= HW) return;
  const int y = int(i / W), x = int(i - int64_t(y) * W);
  const int tw = 1 << tw_log2, th = WAVE >> tw_log2;
  const int tiles_x = (W + tw - 1) / tw;
  const int tile = (y / th) * tiles_x + (x >> tw_log2);
  const int lane = (y % th) * tw + (x & (tw - 1));
  const int64_t first_bin = int64_t(tile) * n_slots;
  int64_t lo = 0, hi = n_pairs;  // first pair with pair_bin >= first_bin
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (pair_bin[mid] < first_bin)
      lo = mid + 1;
    else
      hi = mid;
  }
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int64_t p = lo; p < n_pairs && pair_bin[p] < first_bin + n_slots; ++p) {
    const float* t = part + p * 4 * WAVE + lane;
    s0 += t[0];
    s1 += t[WAVE];
    s2 += t[2 * WAVE];
    s3 += t[3 * WAVE];
  }
  out[i] = finalize_px(make_float4(float(s0), float(s1), float(s2), float(s3)), b0[i], bp.finalize, bp.renormalize);
}

__global__ void k_sum_images(const float4* __restrict__ in, int n_slots, const int* __restrict__ order,
                             int64_t pixels, const float* __restrict__ b0, BoundParams bp,
                             float4* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= pixels) return;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int k = 0; k < n_slots; ++k) {
    const float4 v = in[int64_t(order[k]) * pixels + i];
    s0 += v.x;
    s1 += v.y;
    s2 += v.z;
    s3 += v.w;
  }
  out[i] = finalize_px(make_float4(float(s0), float(s1), float(s2), float(s3)), b0[i], 1, bp.renormalize);
}

// ------------------------------------------------------------------ scan / fill

constexpr int SCAN_THREADS = 256, SCAN_ITEMS = 8, SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_local(const int* __restrict__ in, int* __restrict__ out,
                                                             int64_t n, int* __restrict__ sums) {
  __shared__ int part[SCAN_THREADS];
  const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int tot = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    tot += v[k];
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < SCAN_THREADS; o <<= 1) {  // Hillis-Steele inclusive scan
    int add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int run = part[threadIdx.x] - tot;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1) sums[blockIdx.x] = part[threadIdx.x];
}

__global__ void k_scan_add(int* __restrict__ out, int64_t n, const int* __restrict__ sums) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / SCAN_TILE];
}

__global__ void k_fill(int* p, int v, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ mesh residency

__global__ void k_inc_count(const int4* __restrict__ tv, int64_t n_tets, int* __restrict__ counts) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tets) return;
  const int4 v = tv[t];
  atomicAdd(counts + v.x, 1);
  atomicAdd(counts + v.y, 1);
  atomicAdd(counts + v.z, 1);
  atomicAdd(counts + v.w, 1);
}

__global__ void k_inc_fill(const int4* __restrict__ tv, int64_t n_tets, const int* __restrict__ offsets,
                           int* __restrict__ cursors, int* __restrict__ inc) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tets) return;
  const int4 v = tv[t];
  inc[offsets[v.x] + atomicAdd(cursors + v.x, 1)] = int(t);
  inc[offsets[v.y] + atomicAdd(cursors + v.y, 1)] = int(t);
  inc[offsets[v.z] + atomicAdd(cursors + v.z, 1)] = int(t);
  inc[offsets[v.w] + atomicAdd(cursors + v.w, 1)] = int(t);
}

// neighbour of every (tet, face): the other tet holding the face's 3 vertices
__global__ void k_adjacency(const int4* __restrict__ tv, int64_t n_tets, const int* __restrict__ offsets,
                            const int* __restrict__ inc, int* __restrict__ nbr, int* __restrict__ err) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= 4 * n_tets) return;
  const int t = int(g >> 2), fc = int(g & 3);
  const int4 v = tv[t];
  int f3[3], q = 0;
  for (int k = 0; k < 4; ++k)
    if (k != fc) f3[q++] = sel4(v, k);
  int a = min(f3[0], min(f3[1], f3[2]));
  int found = -1, n_found = 0;
  for (int p = offsets[a]; p < offsets[a + 1]; ++p) {
    const int t2 = inc[p];
    if (t2 == t) continue;
    const int4 w = tv[t2];
    int hit = 0, miss = -1;
    for (int k = 0; k < 4; ++k) {
      const int x = sel4(w, k);
      if (x == f3[0] || x == f3[1] || x == f3[2])
        ++hit;
      else
        miss = k;
    }
    if (hit == 3) {
      found = (t2 << 2) | miss;
      ++n_found;
    }
  }
  if (n_found > 1) atomicOr(err, 1);
  nbr[g] = n_found == 1 ? found : -1;
}

inline unsigned grid1(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_bin_count(const MeshDev& m, const FrameDev& f, const SlotDev* slots, int max_faces,
                            const int* bface, int* counts, hipStream_t s) {
  if (max_faces <= 0 || f.n_slots <= 0) return hipSuccess;
  dim3 grid(grid1(max_faces, 256), f.n_slots);
  hipLaunchKernelGGL(k_bin, grid, dim3(256), 0, s, m, f, slots, bface, counts, (const int*)nullptr, (int*)nullptr,
                     (int*)nullptr, 0, 0ll);
  return hipGetLastError();
}

hipError_t launch_bin_fill(const MeshDev& m, const FrameDev& f, const SlotDev* slots, int max_faces,
                           const int* bface, const int* offsets, int* cursors, int* records, long long rec_cap,
                           hipStream_t s) {
  if (max_faces <= 0 || f.n_slots <= 0) return hipSuccess;
  dim3 grid(grid1(max_faces, 256), f.n_slots);
  hipLaunchKernelGGL(k_bin, grid, dim3(256), 0, s, m, f, slots, bface, (int*)nullptr, offsets, cursors, records,
                     1, rec_cap);
  return hipGetLastError();
}

// Workgroups of `kernel` the device holds at once (the grid of a persistent launch), at least one.
template <class K>
static int resident_blocks(K kernel, int block, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess)
    return 1;
  return cus * per_cu > 0 ? cus * per_cu : 1;
}

// the 8 per-XCD tile counters of a persistent launch start at zero (a fill kernel, not a memset: the
// launch may be captured in a graph)
static hipError_t reset_queue(int* queue, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, queue, 0, int64_t(QUEUE_INTS));
  return hipGetLastError();
}

hipError_t launch_moments(int mm, const MeshDev& m, const FrameDev& f, const SlotDev* slots, const int* offsets,
                          const int* counts, const int* records, long long bin_cap, const float* tf_rgba, float* out,
                          double* gacc, int* pcount, int* segs, const PieceStore& store,
                          unsigned long long* counters, int* queue, const int* pair_idx, const int* pair_list,
                          int64_t n_pairs, hipStream_t s) {
  const size_t lds = size_t(f.n_tf) * sizeof(float);
  const dim3 block(WAVE);
  if (pair_list) {
    queue = nullptr;  // a workgroup per pair
    if (n_pairs <= 0) return hipSuccess;
  }
  const dim3 grid(pair_list ? unsigned(n_pairs) : unsigned(f.n_tiles));
  if (queue) {
    const hipError_t e = reset_queue(queue, s);
    if (e != hipSuccess) return e;
  }
#define APC_LAUNCH_MOMENTS_K(M1, KP)                                                                    \
  do {                                                                                                  \
    if (queue)                                                                                          \
      hipLaunchKernelGGL((k_moments<M1, KP, true>), dim3(resident_blocks(k_moments<M1, KP, true>, WAVE, lds)), \
                         block, lds, s, m, f, slots, offsets, counts, records, tf_rgba, out, gacc, pcount, \
                         segs, bin_cap, store, counters, queue, pair_idx, nullptr);                     \
    else                                                                                                \
      hipLaunchKernelGGL((k_moments<M1, KP, false>), grid, block, lds, s, m, f, slots, offsets, counts,   \
                         records, tf_rgba, out, gacc, pcount, segs, bin_cap, store, counters, queue, pair_idx, \
                         pair_list);                                                                    \
  } while (0)
#define APC_LAUNCH_MOMENTS(M1)                                                                          \
  do {                                                                                                  \
    if (store.pool)                                                                                     \
      APC_LAUNCH_MOMENTS_K(M1, true);                                                                   \
    else                                                                                                \
      APC_LAUNCH_MOMENTS_K(M1, false);                                                                  \
  } while (0)
  if (mm == 4)
    APC_LAUNCH_MOMENTS(5);
  else if (mm == 6)
    APC_LAUNCH_MOMENTS(7);
  else
    APC_LAUNCH_MOMENTS(9);
#undef APC_LAUNCH_MOMENTS
#undef APC_LAUNCH_MOMENTS_K
  return hipGetLastError();
}

hipError_t launch_eval(int mm, const FrameDev& f, int tile_lo, int tile_hi, const PieceStore& store,
                       const int* pcount, const float* tf_rgba, const void* moments, const BoundParams& bp,
                       float* rgba, unsigned long long* counters, hipStream_t s) {
  if (tile_hi <= tile_lo) return hipSuccess;
  const size_t lds = size_t(f.n_tf) * sizeof(float4);
  const dim3 grid((tile_hi - tile_lo + EVAL_WPB - 1) / EVAL_WPB), block(WAVE * EVAL_WPB);
  if (mm == 4)
    hipLaunchKernelGGL((k_eval<2, float>), grid, block, lds, s, f, tile_lo, tile_hi, store, pcount, tf_rgba, moments,
                       bp, rgba, counters);
  else if (mm == 6)
    hipLaunchKernelGGL((k_eval<3, double>), grid, block, lds, s, f, tile_lo, tile_hi, store, pcount, tf_rgba,
                       moments, bp, rgba, counters);
  else
    hipLaunchKernelGGL((k_eval<4, double>), grid, block, lds, s, f, tile_lo, tile_hi, store, pcount, tf_rgba,
                       moments, bp, rgba, counters);
  return hipGetLastError();
}

hipError_t launch_resolve(int mm, const MeshDev& m, const FrameDev& f, const SlotDev* slots, const int* offsets,
                          const int* counts, const int* records, long long bin_cap, const float* tf_rgba,
                          const void* moments, const BoundParams& bp, float* rgba, unsigned long long* counters,
                          int* queue, const int* pair_list, float* part, int64_t n_pairs, hipStream_t s) {
  const size_t lds = size_t(f.n_tf) * sizeof(float4);
  const dim3 block(2 * WAVE);  // a tile (or a pair) per workgroup at a time: its walker and its evaluator
  if (pair_list) {
    queue = nullptr;
    if (n_pairs <= 0) return hipSuccess;
  }
  const dim3 grid(pair_list ? unsigned(n_pairs) : unsigned(f.n_tiles));
  if (queue) {
    const hipError_t e = reset_queue(queue, s);
    if (e != hipSuccess) return e;
  }
#define APC_LAUNCH_RESOLVE(N, R)                                                                               \
  do {                                                                                                         \
    if (pair_list)                                                                                             \
      hipLaunchKernelGGL((k_resolve<N, R, false, true>), grid, block, lds, s, m, f, slots, offsets, counts,   \
                         records, bin_cap, tf_rgba, moments, bp, rgba, counters, nullptr, pair_list, part);   \
    else if (queue)                                                                                            \
      hipLaunchKernelGGL((k_resolve<N, R, true, false>),                                                      \
                         dim3(resident_blocks(k_resolve<N, R, true, false>, 2 * WAVE, lds)), block, lds, s, m, \
                         f, slots, offsets, counts, records, bin_cap, tf_rgba, moments, bp, rgba, counters,    \
                         queue, nullptr, nullptr);                                                             \
    else                                                                                                       \
      hipLaunchKernelGGL((k_resolve<N, R, false, false>), grid, block, lds, s, m, f, slots, offsets, counts,  \
                         records, bin_cap, tf_rgba, moments, bp, rgba, counters, nullptr, nullptr, nullptr);  \
  } while (0)
  if (mm == 4)
    APC_LAUNCH_RESOLVE(2, float);
  else if (mm == 6)
    APC_LAUNCH_RESOLVE(3, double);
  else
    APC_LAUNCH_RESOLVE(4, double);
#undef APC_LAUNCH_RESOLVE
  return hipGetLastError();
}

hipError_t launch_pack_f16(const float* in, int m1, int64_t pixels, void* out_f16, hipStream_t s) {
  if (pixels <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_f16, dim3(grid1(pixels, 256)), dim3(256), 0, s, in, m1, pixels,
                     static_cast<_Float16*>(out_f16));
  return hipGetLastError();
}

hipError_t launch_walk_records(const int4* tet, const float4* vert, int64_t n_tets, int4* wrec, hipStream_t s) {
  if (n_tets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_walk_records, dim3(grid1(n_tets, 256)), dim3(256), 0, s, tet, vert, n_tets, wrec);
  return hipGetLastError();
}

hipError_t launch_sum_moments(const float* in, int n_slots, const int* order, int64_t elems, float* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_sum_moments, dim3(grid1((elems + 3) / 4, 256)), dim3(256), 0, s, in, n_slots, order, elems,
                     out);
  return hipGetLastError();
}

hipError_t launch_pair_scan(const int* counts, int64_t nb, int* flags, int* pidx, int* tmp, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_flags, dim3(grid1(nb, 256)), dim3(256), 0, s, counts, nb, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_exclusive_scan(flags, pidx, nb, tmp, s);
}

hipError_t launch_pair_list(const int* counts, int64_t nb, const int* pidx, int* pair_bin, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_list, dim3(grid1(nb, 256)), dim3(256), 0, s, counts, nb, pidx, pair_bin);
  return hipGetLastError();
}

hipError_t launch_sum_tiles(const float* tiles, const int* pair_bin, int64_t n_pairs, int n_slots, int m1, int W,
                            int H, int tw_log2, float* out, hipStream_t s) {
  const int64_t HW = int64_t(W) * H;
  if (HW <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_tiles, dim3(grid1(HW, 256)), dim3(256), 0, s, tiles, pair_bin, n_pairs, n_slots, m1, W, H,
                     tw_log2, out);
  return hipGetLastError();
}

hipError_t launch_sum_color_tiles(const float* part, const int* pair_bin, int64_t n_pairs, int n_slots, int W, int H,
                                 int tw_log2, const float* b0, const BoundParams& bp, float* out, hipStream_t s) {
  const int64_t HW = int64_t(W) * H;
  if (HW <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_color_tiles, dim3(grid1(HW, 256)), dim3(256), 0, s, part, pair_bin, n_pairs, n_slots, W,
                     H, tw_log2, b0, bp, reinterpret_cast<float4*>(out));
  return hipGetLastError();
}

hipError_t launch_sum_images(const float* in, int n_slots, const int* order, int64_t pixels, const float* b0,
                             const BoundParams& bp, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_images, dim3(grid1(pixels, 256)), dim3(256), 0, s, reinterpret_cast<const float4*>(in),
                     n_slots, order, pixels, b0, bp, reinterpret_cast<float4*>(out));
  return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t total = 0;
  while (n > 1) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    total += 2 * n + 1;
  }
  return total + 1;
}

hipError_t launch_exclusive_scan(const int* in, int* out, int64_t n, int* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  int* sums = tmp;
  int* sums_scan = tmp + nb;
  hipLaunchKernelGGL(k_scan_local, dim3(unsigned(nb)), dim3(SCAN_THREADS), 0, s, in, out, n, sums);
  if (nb > 1) {
    hipError_t e = launch_exclusive_scan(sums, sums_scan, nb, tmp + 2 * nb + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3(grid1(n, 256)), dim3(256), 0, s, out, n, (const int*)sums_scan);
  }
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid1(n, 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_incidence_count(const int4* tv, int64_t n_tets, int* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_inc_count, dim3(grid1(n_tets, 256)), dim3(256), 0, s, tv, n_tets, counts);
  return hipGetLastError();
}

hipError_t launch_incidence_fill(const int4* tv, int64_t n_tets, const int* offsets, int* cursors, int* inc,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_inc_fill, dim3(grid1(n_tets, 256)), dim3(256), 0, s, tv, n_tets, offsets, cursors, inc);
  return hipGetLastError();
}

hipError_t launch_adjacency(const int4* tv, int64_t n_tets, const int* offsets, const int* inc, int* nbr,
                            int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_adjacency, dim3(grid1(4 * n_tets, 256)), dim3(256), 0, s, tv, n_tets, offsets, inc, nbr,
                     err);
  return hipGetLastError();
}

}  // namespace apc
