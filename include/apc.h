/*
 * apc.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of Approximate Puzzlepiece Compositing (APC).
 *
 * The method (paper Sections 3 and 4): every subdomain of a distributed tet
 * mesh is rendered twice.  Stage one (Section 4.1) traces rays through the
 * subdomain's own cells and sums, per pixel, power moments of optical depth
 * over log-warped depth (Alg. 2); the per-subdomain moment images are added
 * into one global moment image, which is order independent because addition
 * commutes.  Stage two (Section 4.2) traces the same rays again and weights
 * each sample by the transmittance that the global moments imply at the
 * sample's depth (Alg. 3: normalise and bias the moments, Cholesky-factor the
 * Hankel matrix, find the roots of the kernel polynomial, weight the nodes
 * and read off the absorbance in front); the per-subdomain colour images are
 * then simply added (Alg. 1) and renormalised by the total opacity
 * (Section 4.3).
 *
 * Here every subdomain that the paper places on its own MPI rank lives on one
 * GPU; the two MPI reductions of the paper become device sums in canonical
 * subdomain order.
 *
 * Conventions
 *  - Every call returns apc_status; nothing aborts or throws across the ABI.
 *    On failure the reason is available from apc_last_error() on the calling
 *    thread.  All argument validation happens before any device work, so a
 *    call that fails validation writes nothing.
 *  - "device" pointers are HIP device memory owned by the caller (for example
 *    torch tensors on cuda:0); "host" pointers are ordinary host memory read
 *    during the call only.  `stream` is a hipStream_t (NULL = default
 *    stream); work is stream ordered like the HIP APIs, and outputs are ready
 *    when that stream reaches the end of the call's work.  The library never
 *    keeps a caller pointer after a call returns.
 *  - A device-side failure (launch error, fault) reported by HIP is returned
 *    as APC_E_DEVICE by the call that observes it.
 *  - Image layout: pixel (row i, column j) of a W x H image has index
 *    i*W + j.  Moment images are planar: element (j, pixel) of an [m+1][H][W]
 *    image is at j*H*W + pixel.
 */
#ifndef APC_H
#define APC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum apc_status {
  APC_OK = 0,
  APC_E_ARG = 1,         /* invalid argument (null pointer, size, id, unsupported m) */
  APC_E_MESH = 2,        /* invalid mesh: index out of range, non-positive volume, non-manifold face */
  APC_E_NOMEM = 3,       /* device or host allocation failed */
  APC_E_DEVICE = 4,      /* HIP runtime error */
  APC_E_NUMERIC = 5,     /* numeric failure in strict mode (walk step limit hit) */
  APC_E_UNSUPPORTED = 6  /* valid request the library does not implement */
} apc_status;

typedef struct apc_ctx_s* apc_ctx;   /* one per device: workspace and diagnostic counters */
typedef struct apc_mesh_s* apc_mesh; /* device-resident mesh of all subdomains, owned by the library */

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  The context owns growable device
 * workspace; calls on one context must not overlap in time (one host thread
 * at a time, one stream at a time).
 * device = APC_DEVICE_NONE creates a host-only context, which makes no HIP
 * call at all: every call validates its arguments exactly as on a device and
 * then returns APC_E_DEVICE ("nothing was launched") instead of doing device
 * work, so requests can be checked where no GPU is present.  apc_load_mesh
 * on such a context validates and groups the mesh on the host (face
 * adjacency included) and returns a mesh that holds no device memory; it can
 * only be passed to host-only calls. */
#define APC_DEVICE_NONE (-1)
apc_status apc_create(int device, apc_ctx* out);
apc_status apc_destroy(apc_ctx ctx);

/* Message describing the last failed call on this thread (never NULL). */
const char* apc_last_error(apc_ctx ctx);

/* Library version string. */
const char* apc_version(void);

/* ------------------------------------------------------------------ mesh */

/* A tetrahedral mesh split into disjoint subdomains (Section 4: each rank
 * holds one subdomain; subdomains may be non-convex and their bounding boxes
 * may overlap, but no cell belongs to two subdomains -- Section 6 notes that
 * overlapping volumes are not supported). */
typedef struct apc_mesh_desc {
  int64_t n_vertices;           /* V >= 4 */
  int64_t n_tets;               /* 1 <= T < 2^29 */
  int32_t n_subdomains;         /* S >= 1 */
  int32_t flags;                /* 0: the four arrays are host memory; APC_MESH_DEVICE: device memory */
  const float* xyz;             /* [V][3] vertex positions */
  const float* scalar;          /* [V] vertex scalars, linearly interpolated inside each tet */
  const int32_t* tet_vertices;  /* [T][4] vertex ids; every tet must have positive signed volume
                                   det(v1-v0, v2-v0, v3-v0) > 0 */
  const int32_t* tet_subdomain; /* [T] subdomain id in [0, S) */
} apc_mesh_desc;
#define APC_MESH_DEVICE 1 /* apc_mesh_desc.flags: the arrays are device memory (copied to the host to validate) */

/* Copy a mesh to the device and build its residency structures: face
 * adjacency (each face is shared by at most two tets), tets grouped by
 * subdomain (the input order is kept inside each subdomain, so pass tets in a
 * spatially coherent order such as Morton order), and per subdomain the list
 * of boundary faces -- faces on the mesh hull or shared with another
 * subdomain -- through which rays enter it.
 * Errors: APC_E_ARG (null pointers, sizes, unknown flags), APC_E_MESH
 * (vertex id out of range, repeated vertex in a tet, non-positive volume,
 * subdomain id out of range, non-finite coordinate, a face shared by more
 * than two tets), APC_E_NOMEM, APC_E_DEVICE.  A failed call creates no mesh.
 * Synchronous (the validation reads the arrays on the host; device arrays are
 * first copied there on `stream`): the caller may free its arrays when the
 * call returns. */
apc_status apc_load_mesh(apc_ctx ctx, const apc_mesh_desc* desc, apc_mesh* out, void* stream);
apc_status apc_free_mesh(apc_ctx ctx, apc_mesh mesh);

typedef struct apc_mesh_info {
  int64_t n_vertices, n_tets, n_boundary_faces;
  int32_t n_subdomains, pad;
  double bbox_lo[3], bbox_hi[3];     /* global bounding box of all vertices */
  int64_t device_bytes;              /* resident device memory held by the mesh */
} apc_mesh_info;
apc_status apc_mesh_get_info(apc_mesh mesh, apc_mesh_info* out);
/* Number of tets and boundary faces of one subdomain. */
apc_status apc_mesh_subdomain_info(apc_mesh mesh, int32_t subdomain, int64_t* n_tets, int64_t* n_boundary_faces);

/* ------------------------------------------------------------------ frame parameters */

#define APC_ORTHOGRAPHIC 0
#define APC_PERSPECTIVE 1

/* Camera.  Pixel (row i, column j), a = j + 1/2, b = i + 1/2:
 *   orthographic: origin = eye + a*right + b*down, direction = dir/|dir|
 *   perspective:  origin = eye, direction = normalise(dir + (a - W/2)*right + (b - H/2)*down)
 * Ray depth t is the distance along the unit direction.  The log-depth warp
 * of Alg. 2/3 maps [t_near, t_far] to [-1, 1]; the sampling lattice is
 * t_near + k*step.  If t_near <= 0 and t_far <= 0 both are derived from the
 * bounding sphere of the whole mesh (centre c, radius R of its bounding box):
 * t_near = dist - R, t_far = dist + R with dist = |c - eye| (perspective) or
 * (c - eye).dir/|dir| (orthographic).  The same range must be used by every
 * subdomain and by both passes.  t_near must come out positive.  Every ray
 * must start outside the mesh (the walk enters each subdomain through its
 * boundary faces): a perspective eye outside the mesh's bounding box, an
 * orthographic image plane with the whole box in front of it; APC_E_ARG
 * otherwise.  A perspective view must also have the whole box in front of
 * the eye (every corner at a positive coefficient of dir when written in
 * (dir, right, down)): a ray is the half-line from the eye, and no line may
 * cross the mesh behind it; APC_E_ARG otherwise.  Depths outside
 * [t_near, t_far] warp outside [-1, 1]. */
typedef struct apc_view {
  int32_t width, height;
  int32_t projection;   /* APC_ORTHOGRAPHIC or APC_PERSPECTIVE */
  int32_t pad;
  double eye[3], dir[3], right[3], down[3];
  double t_near, t_far; /* <= 0: derive from the mesh */
  double step;          /* world-space lattice spacing, > 0 */
} apc_view;

/* Transfer function: a table of n_entries RGBA values over [s_min, s_max],
 * linearly interpolated and clamped.  Extinction per unit length is
 * kappa * A; a sample of length l has optical depth
 * min(kappa * A * l, absorbance_max) (Alg. 2 caps the absorbance). */
typedef struct apc_tf {
  int32_t n_entries;    /* 2..1024 */
  int32_t pad;
  const float* rgba;    /* device [n_entries][4] */
  float s_min, s_max, kappa, absorbance_max;
} apc_tf;

/* Moment-bound parameters (Alg. 3 and Section 4.3).  The moments are
 * normalised by b0 and mixed with a bias vector: beta' = (1-alpha)*b/b0 +
 * alpha*bias; the node at the sample's own depth is weighted by eta
 * ("overestimation"). */
typedef struct apc_mboit {
  int32_t m;            /* number of power moments: 4, 6 or 8 */
  int32_t renormalize;  /* finalised output: 1 = rgb * (1 - exp(-b0)) / sum(T*a), 0 = literal Alg. 1 sums */
  double alpha;         /* bias mixing strength, 0 <= alpha < 1 */
  double bias[8];       /* b*_1..b*_m */
  double eta;           /* overestimation weight, 0..1 */
} apc_mboit;

/* ------------------------------------------------------------------ the hot path */

/* Stage one for a list of subdomains (Section 4.1, Alg. 2).  For each listed
 * subdomain s (slot k = position in `subdomains`), every pixel ray is walked
 * through the tets of s from each boundary face where it enters s; the chord
 * in each tet is cut at the lattice t_near + k*step into pieces, and each
 * piece of optical depth a at warped depth z adds a*z^j to moment j.
 *   subdomains      host [n_sub] distinct subdomain ids
 *   moments_per_sub device [n_sub][m+1][H][W] FP32, fully written (zero where
 *                   subdomain k is not hit)
 * m is 4, 6 or 8.
 * flags: 0, or any of
 *   APC_MOMENTS_GLOBAL: the listed subdomains are all that the frame has and
 *     stage one sums them itself: `moments_per_sub` is then the global image
 *     device [m+1][H][W] FP32, bitwise what apc_sum_moments returns for the
 *     per-subdomain images of the same call (each subdomain's FP32 value added
 *     in FP64 in ascending subdomain-id order).  The ids must be listed in
 *     ascending order (APC_E_ARG otherwise).  Needs an FP64 accumulator of
 *     8*(m+1)*H*W bytes in context-owned device memory; the per-subdomain
 *     images are never formed.
 *   APC_KEEP_PIECES: also keep every piece (12 bytes each, in chunks of 64, in
 *     context-owned device memory grown after a frame that did not fit) so that
 *     apc_resolve_pass of the same geometry, camera, transfer function and
 *     subdomain list evaluates them instead of walking the rays again.  A
 *     variant that trades memory (about 67 GB at 2560^2 on a 100M-tet mesh)
 *     for the second walk; results equal the plain form's to rounding.
 * Without APC_KEEP_PIECES nothing per piece is stored (the paper's method: the
 * per-pixel state is the m + 1 moments). */
apc_status apc_moments_pass(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf, int32_t m,
                            const int32_t* subdomains, int32_t n_sub, float* moments_per_sub, uint32_t flags,
                            void* stream);

/* Global moments = sum of the per-subdomain moment images (Section 4.1; the
 * paper's MPI_Allreduce).  The sum runs in FP64 over the slots in ascending
 * subdomain-id order, whatever their order in the buffer, so the result is
 * bitwise independent of the order in which subdomains were rendered.
 *   moments_per_sub device [n_sub][m+1][H][W] FP32
 *   subdomains      host [n_sub] ids of the slots (NULL: slot order is canonical)
 *   moments_global  device [m+1][H][W] FP32 */
apc_status apc_sum_moments(apc_ctx ctx, const float* moments_per_sub, int32_t n_sub, int32_t m, int32_t height,
                           int32_t width, const int32_t* subdomains, float* moments_global, void* stream);

#define APC_FINALIZE 1u
#define APC_MOMENTS_F16 2u
#define APC_MOMENTS_GLOBAL 8u
#define APC_KEEP_PIECES 16u
#define APC_BY_PAIR 32u

/* Pack a global moment image for FP16 storage, m + 3 planes each rounded to
 * the nearest FP16 value: planes 0 and 1 hold ln(b0) as two halves (hi, then
 * the rest lo; plane 0 is -inf and the others 0 where b0 <= 0); planes 2 and
 * 3 the mean warped depth mu = b1 / b0 as two halves (mu = hi + lo); planes
 * 4..m+2 the central moments E[(z - mu)^k] for k = 2..m of the pixel's
 * normalised depth distribution.  Central moments keep a concentrated
 * distribution's spread at FP16's relative precision, which raw moments
 * b_j / b0 (all near mu^j) lose; the split ln b0 keeps the opacity near FP32
 * precision.  2(m + 3) bytes per pixel instead of 4(m + 1); apc_resolve_pass
 * reads it with APC_MOMENTS_F16.  The rounding perturbs the moments by up to
 * about 2^-11 relative, far beyond the FP32 bar: the resulting image error is
 * a property of the variant, not a parity result.
 *   moments_global  device [m+1][H][W] FP32 (from apc_sum_moments)
 *   packed          device [m+3][H][W] FP16 (2-byte aligned), written */
apc_status apc_pack_moments_f16(apc_ctx ctx, const float* moments_global, int32_t m, int32_t height, int32_t width,
                                void* packed, void* stream);

/* Stage two for a list of subdomains (Section 4.2, Alg. 1 second loop and
 * Alg. 3).  The rays are walked again exactly like stage one (the same pieces,
 * bit for bit the same depths and optical depths), and each piece of opacity
 * alpha_p = 1 - exp(-a) and colour c (transfer-function RGB) adds
 * T * alpha_p * (c, 1) to its pixel at once, where T = clamp(exp(-b0 * F))
 * and F is the moment bound at the piece's warped depth computed from
 * `moments_global`; nothing per piece is stored.  When the preceding
 * apc_moments_pass on this context kept its pieces (APC_KEEP_PIECES) for the
 * same mesh, camera, transfer function and subdomain list, those pieces are
 * evaluated instead of walking again.
 *   moments_global  device [m+1][H][W] FP32 (from apc_sum_moments), or with
 *                   APC_MOMENTS_F16 the FP16 image of apc_pack_moments_f16
 *                   ([m+3][H][W])
 *   rgba_out        device [H][W][4] FP32, 16-byte aligned.  Without
 *                   APC_FINALIZE: the additive partial image (sum T*a*rgb,
 *                   sum T*a) of the listed subdomains.  With APC_FINALIZE:
 *                   the final image of those subdomains (renormalised when
 *                   mboit->renormalize, see apc_mboit).
 * The per-pixel Hankel/Cholesky set-up and the per-piece solve run in FP64
 * when m = 6 or 8 and in FP32 when m = 4; everything else runs in FP32, the
 * walk's ray geometry in FP64.
 * APC_BY_PAIR (plain form; ignored when kept pieces are evaluated): one
 * workgroup walks one (tile, subdomain) pair with binned faces and writes
 * its unfinalised colour sums to a context buffer, then each pixel's pairs
 * are summed in FP64 in slot order and finalised.  For frames of few tiles
 * (one chain of dependent steps per tile through every subdomain otherwise);
 * the same pieces, the image equal to the per-tile form's to FP32 rounding
 * (another grouping of the colour sums, and each pair's root solver starts
 * afresh).  Reads the pair count back (one stream synchronisation); not with
 * APC_MOMENTS_F16 or in a captured frame (APC_E_ARG).
 * flags: APC_FINALIZE, APC_MOMENTS_F16, APC_BY_PAIR. */
apc_status apc_resolve_pass(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf,
                            const apc_mboit* mboit, const void* moments_global, const int32_t* subdomains,
                            int32_t n_sub, float* rgba_out, uint32_t flags, void* stream);

/* apc_resolve_pass for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the plain form only (stage two walks the rays again; kept
 * pieces are never used), with the same arguments, flags, validation and
 * results bit for bit.  Its binning state lives in a static device workspace
 * of 64 MiB in the library's code object (every GPU the library runs on holds
 * one, until the process ends) instead of the context's growable buffers, so
 * the call allocates nothing.  The call reads back the number of binned
 * (face, tile) records (one stream synchronisation) before it walks.
 * Limits: the slot table, 3 x 4 bytes per (tile, subdomain) pair and the
 * binned records must fit the 64 MiB (about 16 subdomains at 2048^2 or all
 * 72 of a 100M-tet mesh at 1024^2); a frame beyond them returns APC_E_NOMEM
 * with the sizes in the message and writes nothing to rgba_out.  Every call on
 * one GPU shares that GPU's workspace: calls that overlap in time on one GPU
 * (any contexts, any streams) race.  Everything it needs is cleared by its own
 * kernels on every call. */
apc_status apc_resolve_pass_noalloc(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf,
                                    const apc_mboit* mboit, const void* moments_global,
                                    const int32_t* subdomains, int32_t n_sub, float* rgba_out, uint32_t flags,
                                    void* stream);

/* Stage one in the tiles form: the per-subdomain moments as the message a
 * rank would send (Section 4.3: only non-empty tiles are exchanged) -- one
 * tile of 64 pixels x (m+1) moments per (tile, subdomain) pair that has
 * boundary faces of the subdomain binned to it, instead of dense
 * [n_sub][m+1][H][W] images that are mostly zero (92 % at 2560^2 over 72
 * subdomains).  Same pieces and per-pixel sums as apc_moments_pass: a pair's
 * tile holds exactly the dense image's values of its 64 pixels (0 on pixels
 * with no piece or outside the image), and every pixel of a tile without a
 * pair is 0 there.
 *   subdomains  host [n_sub], ascending ids (else APC_E_ARG)
 *   tiles       device [max_pairs][m+1][64] FP32: pair p's moment j of
 *               lane l (the tile's pixel (l mod w, l / w) for the context's
 *               tile shape w x 64/w) at tiles[(p*(m+1) + j)*64 + l]
 *   pair_bin    device [max_pairs] int32: pair p's bin, tile*n_sub + slot
 *               (slot = index into `subdomains`), ascending
 *   max_pairs   capacity of tiles and pair_bin; with tiles == NULL and
 *               max_pairs == 0 the call only counts the pairs (a query)
 *   n_pairs     host out: the frame's pair count (also on APC_E_NOMEM)
 * More pairs than max_pairs: APC_E_NOMEM, nothing written.  Reads the pair
 * count back (one stream synchronisation) before it walks. */
apc_status apc_moments_pass_tiles(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf, int32_t m,
                                  const int32_t* subdomains, int32_t n_sub, float* tiles, int32_t* pair_bin,
                                  int64_t max_pairs, int64_t* n_pairs, void* stream);

/* The tiles form walked pair by pair: the same arguments, results and
 * errors as apc_moments_pass_tiles (bitwise the same tiles), but one
 * workgroup walks one (tile, subdomain) pair instead of all the pairs of
 * its tile in turn.  A small image has few tiles, each a long chain of
 * dependent walk steps through every subdomain on its rays; by pair the
 * chains are short and many.  (Section 4.1's per-rank stage one, every
 * subdomain a rank.)  Keeps no per-pixel segment counts
 * (apc_segment_counts then fails with APC_E_ARG); ignores the work-queue
 * dispatch setting. */
apc_status apc_moments_pass_pairs(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf, int32_t m,
                                  const int32_t* subdomains, int32_t n_sub, float* tiles, int32_t* pair_bin,
                                  int64_t max_pairs, int64_t* n_pairs, void* stream);

/* The global [m+1][H][W] moments from the tiles form: per pixel the pairs of
 * its tile summed in FP64 in slot (ascending id) order -- bitwise what
 * apc_sum_moments gives for the dense images of the same stage one.
 * tile_width is the tile shape the tiles were made with. */
apc_status apc_sum_moment_tiles(apc_ctx ctx, const float* tiles, const int32_t* pair_bin, int64_t n_pairs,
                                int32_t n_sub, int32_t m, int32_t height, int32_t width, int32_t tile_width,
                                float* moments_global, void* stream);

/* Final image = sum of partial images (Section 4.2; the paper's
 * MPI_Reduce), in ascending subdomain-id order, then finalised like
 * apc_resolve_pass with APC_FINALIZE.
 *   partials        device [n_sub][H][W][4] additive partial images
 *   subdomains      host [n_sub] ids of the partial images (NULL: canonical)
 *   moments_global  device [m+1][H][W] (b0 plane used for the opacity)
 *   rgba_out        device [H][W][4] */
apc_status apc_sum_images(apc_ctx ctx, const float* partials, int32_t n_sub, int32_t height, int32_t width,
                          const int32_t* subdomains, const float* moments_global, const apc_mboit* mboit,
                          float* rgba_out, void* stream);

/* Bound the context's kept-piece pool (APC_KEEP_PIECES) to `bytes` (0: it
 * may take up to 60 % of the free device memory, the default).  A frame whose
 * pieces exceed the pool walks again in stage two (same results).  Lets
 * several contexts (e.g. a server's slots) share one GPU with a known
 * footprint. */
apc_status apc_set_workspace_limit(apc_ctx ctx, int64_t bytes);

/* Device memory the context holds now (binning state, FP64 moment partials,
 * segment statistics, the kept-piece pool): it grows to what the largest
 * frame so far needed and is kept for the next frames.  A server adds it to
 * a request's own buffers to admit requests by their HBM footprint. */
apc_status apc_get_workspace_bytes(apc_ctx ctx, int64_t* bytes);

/* ------------------------------------------------------------------ frame graphs */

/* A whole frame (apc_moments_pass, apc_sum_moments, apc_resolve_pass for one
 * mesh, camera, transfer-function buffer, moment parameters and subdomain
 * list, into the given buffers) captured once in a HIP graph and replayed
 * with one launch.  The graph owns a private workspace, sized by one eager
 * frame that create runs first (so create is synchronous and its buffers
 * hold that frame's results), and all its kernels take their sizes from the
 * device: no host round trip, upload or allocation happens in a replay.  The
 * camera, parameters and buffer addresses are fixed at capture; the contents
 * of the transfer-function table and of the mesh may change between replays
 * as long as the binned boundary faces do not (the mesh's geometry and the
 * camera fix them; with APC_KEEP_PIECES also the piece counts per pixel: a
 * piece beyond the pool of the sizing frame is not kept, and that pixel's
 * pieces are then left out and counted in entry_overflow).  Calls that
 * overlap on one graph race.
 *   flags  APC_FINALIZE or 0, as for apc_resolve_pass, and/or APC_MOMENTS_GLOBAL:
 *          stage one sums the subdomains itself (as apc_moments_pass with that
 *          flag: ascending ids; moments_per_sub is not used and may be NULL),
 *          and/or APC_KEEP_PIECES: stage two evaluates the pieces stage one kept
 *          (else it walks again, the plain form)
 * Errors: APC_E_NOMEM when APC_KEEP_PIECES is set and the frame's pieces do
 * not fit the pool. */
typedef struct apc_graph_s* apc_graph;
apc_status apc_frame_graph_create(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf,
                                  const apc_mboit* mboit, const int32_t* subdomains, int32_t n_sub,
                                  float* moments_per_sub, float* moments_global, float* rgba_out, uint32_t flags,
                                  apc_graph* out);
apc_status apc_frame_graph_launch(apc_graph graph, void* stream);
apc_status apc_frame_graph_destroy(apc_graph graph);

/* ------------------------------------------------------------------ tile shape */

/* Every pass maps one wavefront (64 lanes) to a tile of tile_width x
 * (64 / tile_width) pixels; the shape changes which rays walk together, not
 * any result (default 8 x 8).  The shape is a property of the context and
 * applies to later passes; the resolve pass must run with the shape of the
 * stage one whose piece counts it reuses (it counts again otherwise). */
apc_status apc_set_tile_shape(apc_ctx ctx, int32_t tile_width);  /* 1, 2, 4, ..., 64; else APC_E_ARG */
apc_status apc_get_tile_shape(apc_ctx ctx, int32_t* tile_width, int32_t* tile_height);

/* ------------------------------------------------------------------ dispatch */

/* How both passes hand their tiles (tile x subdomain-list work units, the
 * batching of Section 5.3's uneven partitions) to the GPU; a property of the
 * context for later passes, frame graphs included.  Results are identical
 * either way (each tile is computed by the same code in the same order).
 *   APC_DISPATCH_GRID   one workgroup per tile, handed out by the hardware
 *                       (default).
 *   APC_DISPATCH_QUEUE  persistent: as many workgroups as the device holds
 *                       at once, each taking tile after tile from a work
 *                       queue of per-XCD counters (the order of
 *                       APC_DISPATCH_GRID per XCD; an XCD whose tiles are
 *                       gone takes the next XCD's).  The counters (32 bytes)
 *                       are allocated by this call, so that no pass
 *                       allocates them; they are reset on the caller's
 *                       stream by a kernel before each pass, so two passes
 *                       of one context must not overlap in time.
 * Other modes: APC_E_ARG. */
#define APC_DISPATCH_GRID 0
#define APC_DISPATCH_QUEUE 1
apc_status apc_set_dispatch(apc_ctx ctx, int32_t mode);
apc_status apc_get_dispatch(apc_ctx ctx, int32_t* mode);

/* Autotuner: times whole frames -- stage one summing the subdomains itself
 * (APC_MOMENTS_GLOBAL: `subdomains` ascending, else APC_E_ARG) followed by
 * the finalising resolve, as a frame on one GPU runs them -- for tile widths
 * 2, 4, 8, 16, 32 (one warm-up frame per width, then the best of `repeats`,
 * HIP events on `stream`), sets the fastest on the context and returns it.
 * Synchronous.  The tile shape changes both passes' cost (which rays walk
 * together in stage one; which pieces stage two reads together), so a frame,
 * not stage one alone, is timed.
 *   moments       device [m+1][H][W] FP32 scratch (overwritten), m = mboit->m
 *   rgba_out      device [H][W][4] FP32 scratch (overwritten)
 *   ms_per_width  host [7] or NULL: entry k = frame milliseconds for width
 *                 2^k, -1 where not timed */
apc_status apc_autotune_tile_shape(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf,
                                   const apc_mboit* mboit, const int32_t* subdomains, int32_t n_sub, float* moments,
                                   float* rgba_out, int32_t repeats, int32_t* best_width, float* ms_per_width,
                                   void* stream);

/* The same search over tile widths 2..32 for both dispatch modes
 * (APC_DISPATCH_GRID, APC_DISPATCH_QUEUE), setting the fastest width and
 * mode on the context.  ms_table: host [2][7] or NULL, entry [d][k] = frame
 * milliseconds for mode d and width 2^k, -1 where not timed.  Allocates the
 * work queue's counters (as apc_set_dispatch does).  Synchronous. */
apc_status apc_autotune_launch(apc_ctx ctx, apc_mesh mesh, const apc_view* view, const apc_tf* tf,
                               const apc_mboit* mboit, const int32_t* subdomains, int32_t n_sub, float* moments,
                               float* rgba_out, int32_t repeats, int32_t* best_width, int32_t* best_dispatch,
                               float* ms_table, void* stream);

/* ------------------------------------------------------------------ diagnostics */

/* Per-pixel segment statistics of the last apc_moments_pass on this context
 * (its subdomains only).  A segment is a maximal interval of a pixel ray
 * inside one subdomain that holds at least one piece: the number of colour
 * fragments a sort-last compositor would have to exchange and order for that
 * pixel (Section 6, segment counts), while APC exchanges one moment vector
 * and one colour per subdomain that the ray meets.
 *   out  device [2][H][W] int32: plane 0 segments, plane 1 subdomains with at
 *        least one piece on the ray
 * Errors: APC_E_ARG when no stage one has run or H, W differ from its view. */
apc_status apc_segment_counts(apc_ctx ctx, int32_t* out, int32_t height, int32_t width, void* stream);

typedef struct apc_counters {
  int64_t pieces;           /* samples (pieces) generated, by every walk (stage one, and stage two when it walks) */
  int64_t tet_steps;        /* tets walked, every walk */
  int64_t entries;          /* (ray, boundary face) entries walked, every walk */
  int64_t bin_records;      /* (face, tile) records binned */
  int64_t walk_step_limit;  /* walks cut off by the step limit (should be 0) */
  int64_t exit_fallback;    /* exit faces chosen by the tie fallback (should be ~0) */
  int64_t entry_overflow;   /* per-ray entry lists refilled in extra rounds (results stay correct), plus
                               stage-two re-walks whose piece count differed from the count (never expected) */
  int64_t nonpd_pivots;     /* Cholesky pivots floored in the resolve pass */
  int64_t table_samples;    /* samples (m >= 6) whose moment bound needed roots, found by Newton from a
                               start: their pixel's gap table (kept pieces) or the ray's previous sample
                               (re-walk) */
  int64_t table_fallback;   /* of those, samples that took the closed-form roots: a start that did not
                               converge (~1e-4 with tables), and in the re-walk every first sample of a ray
                               in a new gap of the bound (a few percent) */
  int64_t segments;         /* maximal ray intervals inside one subdomain with at least one piece, every walk */
} apc_counters;

/* Read (and with reset != 0, clear) the counters accumulated by this context.
 * Synchronises the device. */
apc_status apc_get_counters(apc_ctx ctx, apc_counters* out, int32_t reset);
/* Counters of a frame graph's private workspace (see apc_frame_graph_create). */
apc_status apc_frame_graph_counters(apc_graph graph, apc_counters* out, int32_t reset);

/* Durations in milliseconds of the kernels of the most recent calls on this
 * context, measured with HIP events recorded on the caller's stream around
 * each launch.  Waits for those events.  A kernel that has not run yet
 * reports 0. */
typedef struct apc_timings {
  double bin_ms;       /* binning of the most recent pass (count + scan + fill) */
  double moments_ms;   /* stage-one walk kernel of the last apc_moments_pass */
  double sum_ms;       /* last apc_sum_moments (0 after an APC_MOMENTS_GLOBAL stage one) */
  double resolve_ms;   /* everything after binning in the last apc_resolve_pass */
  double rewalk_ms;    /* its walk-and-evaluate kernel (0 when it evaluated kept pieces) */
  double eval_ms;      /* its evaluation of kept pieces (0 when it walked again) */
} apc_timings;
apc_status apc_get_timings(apc_ctx ctx, apc_timings* out);

#ifdef __cplusplus
}
#endif

#endif /* APC_H */
