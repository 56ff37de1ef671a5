// Declarations shared by the host side of the C ABI (apc_api.cpp) and the
// HIP kernels (apc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apc {

// Device-resident mesh.  Tets are grouped by subdomain; tet record t is two
// int4 at tet[2t] (vertex ids, positively oriented) and tet[2t+1] (neighbour
// code per face: face f is opposite vertex f; code = (nbr_tet << 2) | face
// index of the shared face in nbr_tet, or -1 on the mesh hull).
struct MeshDev {
  const float4* vert;  // [V]: x, y, z, scalar
  const int4* tet;     // [2T]
  // [8T]: the walk's record of tet t, one 128-byte line: vertex ids, neighbour
  // codes, then the four vertices (x, y, z, scalar) in vertex-id order
  const int4* wrec;
  int64_t n_vertices;
  int64_t n_tets;
};

// One subdomain taking part in a call.
struct SlotDev {
  int tet_begin, tet_end;    // tet range of the subdomain
  int face_begin, face_end;  // range in the boundary-face array
};

// Per-call constants: the camera (FP32 for binning, FP64 for the rays), the
// lattice, the warp and the transfer-function parameters.
struct FrameDev {
  int W, H, proj, tiles_x, tiles_y, n_tiles, n_slots, n_tf;
  int tw_log2;          // a tile (one wavefront) is (1 << tw_log2) x (64 >> tw_log2) pixels
  float ex, ey, ez;     // eye (perspective origin / orthographic image-plane origin)
  float dx, dy, dz;     // forward direction (unit for orthographic)
  float rx, ry, rz;     // right
  float wx, wy, wz;     // down
  float half_w, half_h; // W/2, H/2
  // The walk's ray geometry is FP64: the camera below, the ray's orthonormal
  // frame, every vertex depth and the lattice cuts.  A grazing ray's chord
  // through a face changes by the lateral ray error over the tangent of the
  // incidence angle, so FP32 rays (~3e-7 lateral error at distance 2) moved
  // silhouette moments by up to 6e-4 of b0; in FP64 only the FP32 side
  // products remain (~1e-7 of a face's size).
  double ceye[3], cdir[3], cright[3], cdown[3];
  // Depths inside the kernels are measured from a ray origin moved forward by
  // t_mid = (t_near + t_far) / 2.  t_near below is the lattice origin in
  // those shifted units (t_near - t_mid).
  double t_mid, t_near, step, inv_step;
  float lg_near, warp_scale;  // log2(t_near), 2 / (log2 t_far - log2 t_near), absolute units
  float s_min, tf_scale;      // table coordinate = (s - s_min) * tf_scale
  float kappa, amax;
  int max_steps;
  float minv[9];  // inverse of the 3x3 matrix with columns dir, right, down (screen projection)
};

// Pieces kept by stage one for stage two: a pool of PIECE_CHUNK-piece chunks
// handed out by a device counter, and per pixel (tile-major slot) the ids of
// its chunks in walk order.  A lane that cannot get a chunk stops keeping
// pieces and counts a failure; stage two then walks the frame again.
constexpr int PIECE_CHUNK = 64;
// chunks a wavefront takes from the pool at a time; the unused rest of its
// last block is lost for the frame, so a pool needs n_tiles * STORE_BLOCK
// chunks beyond the pieces themselves
constexpr int STORE_BLOCK = 64;
struct PieceStore {
  float* pool;               // [n_chunks][PIECE_CHUNK][3]: z, a, s
  long long n_chunks;
  int* ptab;                 // [n_tiles * 64][maxc]
  int maxc;
  unsigned long long* next;  // [0]: chunks handed out, [1]: lanes that failed
};

// Moment-bound parameters in the precision of the resolve pass.
struct BoundParams {
  double alpha, eta;
  double bias[8];
  int renormalize, finalize;
  int moments_f16;  // the moment image is the packed FP16 form (ln b0, b_j / b0)
};

// Diagnostic counters (device memory, int64 each), in apc_counters order.
enum { C_PIECES = 0, C_STEPS, C_ENTRIES, C_BINREC, C_STEPLIMIT, C_FALLBACK, C_OVERFLOW, C_NONPD, C_TABLED,
       C_TABFB, C_SEGMENTS, C_COUNT };

constexpr int MAX_TF = 1024;

// ---- frame kernels (apc_kernels.hip)
hipError_t launch_bin_count(const MeshDev& m, const FrameDev& f, const SlotDev* slots, int max_faces,
                            const int* bface, int* counts, hipStream_t s);
hipError_t launch_bin_fill(const MeshDev& m, const FrameDev& f, const SlotDev* slots, int max_faces,
                           const int* bface, const int* offsets, int* cursors, int* records, long long rec_cap,
                           hipStream_t s);
// stage one; pcount (tile-major [n_tiles * 64], may be null) receives the pieces per pixel, segs
// ([2][H][W], may be null) the segments per pixel and the subdomains with pieces on each ray.  With gacc
// ([m+1][H][W] FP64 scratch) set, out is the global [m+1][H][W] image: the slots' FP32 moments summed in
// FP64 in slot order; else out is [n_slots][m+1][H][W]
hipError_t launch_moments(int mm, const MeshDev& m, const FrameDev& f, const SlotDev* slots, const int* offsets,
                          const int* counts, const int* records, long long bin_cap, const float* tf_rgba, float* out,
                          double* gacc, int* pcount, int* segs, const PieceStore& store,
                          unsigned long long* counters, int* queue, const int* pair_idx, const int* pair_list,
                          int64_t n_pairs, hipStream_t s);
// pair_idx (tiles form, gacc null): per bin with faces its pair number; out is then [pairs][m+1][64]
// (lane-minor), every lane of every pair written.  pair_list (tiles form, may be null): the bin of each of
// the n_pairs pairs; a workgroup per pair then walks that pair alone (pcount and segs must be null)
// queue (both passes): null for one workgroup per tile; else QUEUE_INTS device ints that the launch
// resets and a persistent launch (as many workgroups as the device holds) takes the tiles from
constexpr int QUEUE_INTS = 8;
// stage two, plain form: the rays are walked again and every piece is evaluated at once (no piece
// is kept); rgba [H][W][4] receives the listed subdomains' colour sums, finalised with bp.finalize.
// pair_list (may be null): the bins of n_pairs (tile, subdomain) pairs, ascending; a workgroup per pair then
// writes that pair's unfinalised colour sums to part [n_pairs][4][64] instead of rgba (queue ignored)
hipError_t launch_resolve(int mm, const MeshDev& m, const FrameDev& f, const SlotDev* slots, const int* offsets,
                          const int* counts, const int* records, long long bin_cap, const float* tf_rgba,
                          const void* moments, const BoundParams& bp, float* rgba, unsigned long long* counters,
                          int* queue, const int* pair_list, float* part, int64_t n_pairs, hipStream_t s);
// the image from stage two's pair colour sums: per pixel its tile's pairs summed in FP64 in slot order, then
// finalised with bp.finalize and b0 [H][W] (plane 0 of the FP32 moment image)
hipError_t launch_sum_color_tiles(const float* part, const int* pair_bin, int64_t n_pairs, int n_slots, int W, int H,
                                 int tw_log2, const float* b0, const BoundParams& bp, float* out, hipStream_t s);
// stage two from the pieces stage one kept (store, pcount per pixel) for tiles [tile_lo, tile_hi)
hipError_t launch_eval(int mm, const FrameDev& f, int tile_lo, int tile_hi, const PieceStore& store,
                       const int* pcount, const float* tf_rgba, const void* moments, const BoundParams& bp,
                       float* rgba, unsigned long long* counters, hipStream_t s);
// FP16 packing of a global moment image
hipError_t launch_pack_f16(const float* in, int m1, int64_t pixels, void* out_f16, hipStream_t s);
hipError_t launch_sum_moments(const float* in, int n_slots, const int* order, int64_t elems, float* out,
                              hipStream_t s);
hipError_t launch_sum_images(const float* in, int n_slots, const int* order, int64_t pixels, const float* b0,
                             const BoundParams& bp, float* out, hipStream_t s);
// 128-byte walk records from the tet records and the vertices
hipError_t launch_walk_records(const int4* tet, const float4* vert, int64_t n_tets, int4* wrec, hipStream_t s);
// exclusive scan of n int32 values; tmp must hold scan_tmp_elems(n) ints
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_exclusive_scan(const int* in, int* out, int64_t n, int* tmp, hipStream_t s);
// tiles form: pidx[b] = pair number of bin b when counts[b] > 0 (bins with faces, numbered in bin order; the
// pair count is pidx[nb-1] + flags[nb-1]); flags: nb ints; tmp as for the scan.  Then pair_bin[p] = its bin.
hipError_t launch_pair_scan(const int* counts, int64_t nb, int* flags, int* pidx, int* tmp, hipStream_t s);
hipError_t launch_pair_list(const int* counts, int64_t nb, const int* pidx, int* pair_bin, hipStream_t s);
// global [m1][H][W] moments from n_pairs tiles (pair_bin ascending, n_slots slots per tile, ascending ids)
hipError_t launch_sum_tiles(const float* tiles, const int* pair_bin, int64_t n_pairs, int n_slots, int m1, int W,
                            int H, int tw_log2, float* out, hipStream_t s);
hipError_t launch_fill_i32(int* p, int value, int64_t n, hipStream_t s);

// ---- mesh residency kernels
hipError_t launch_incidence_count(const int4* tv, int64_t n_tets, int* counts, hipStream_t s);
hipError_t launch_incidence_fill(const int4* tv, int64_t n_tets, const int* offsets, int* cursors, int* inc,
                                 hipStream_t s);
hipError_t launch_adjacency(const int4* tv, int64_t n_tets, const int* offsets, const int* inc, int* nbr,
                            int* err, hipStream_t s);

}  // namespace apc
