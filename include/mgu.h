/*
 * mgu.h - C ABI of libmgu: the per-frame dynamic mesh-Gaussian update on one
 * AMD MI355X (gfx950).
 *
 * Paper: "Real-Time Physics Simulation with Dynamic Mesh-Gaussian
 * Reconstructions" (arXiv 2606.00444).  A fixed-topology physics mesh drives
 * a Gaussian render representation (Sec. 3.2); acceleration structures are
 * built once from the template faces and reused (Sec. 3.4, Initialization);
 * each frame only rewrites the vertex buffer, normals being recomputed on
 * demand inside collision queries (Sec. 3.4, per-frame steps 1-3); varying
 * topology instead destroys and rebuilds the collision structures every frame
 * (Sec. 4.1).
 *
 * Conventions for every entry point:
 *  - All array pointers are DEVICE pointers unless marked "host".  The caller
 *    allocates everything (inputs, outputs, BVH buffers, workspaces); the
 *    library never allocates, frees or synchronises, so every call may be
 *    captured into a HIP graph.
 *  - Layout is structure-of-arrays: "[k][n]" means k planes of n contiguous
 *    values (vertices [3][n_verts] float32 x/y/z planes; faces [3][n_faces]
 *    int32 vertex ids).  Counts are int32 and must be >= 0 and < 2^30.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued asynchronously on it; outputs are valid once the stream
 *    reaches that point.
 *  - Arguments are checked on the host before any HIP call; a bad argument
 *    returns a status and enqueues nothing.  Index ranges inside arrays are
 *    NOT checked by the compute calls (mg_validate_indices does that on
 *    request); out-of-range ids are undefined behaviour.  A failed kernel
 *    launch returns MG_ERR_HIP.  No C++ exception crosses this boundary.
 *  - n == 0 is a valid no-op for every call.
 */
#ifndef MGU_H
#define MGU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mg_status;

#define MG_OK                       0
#define MG_ERR_INVALID_ARGUMENT     1  /* null pointer, negative or too large count, bad flag */
#define MG_ERR_WORKSPACE_TOO_SMALL  2  /* a caller buffer is smaller than the size query says */
#define MG_ERR_INDEX_OUT_OF_RANGE   3  /* reported by mg_validate_indices */
#define MG_ERR_NONFINITE_INPUT      4  /* reported by mg_validate_finite */
#define MG_ERR_TOPOLOGY_MISMATCH    5  /* BVH used with a different primitive count or kind */
#define MG_ERR_HIP                  6  /* a HIP runtime call failed (launch, copy) */
#define MG_ERR_UNSUPPORTED_DEVICE   7  /* current device is not gfx950 */

#define MG_PRIM_TRIANGLES 0  /* primitives are faces [3][n] into a vertex array */
#define MG_PRIM_POINTS    1  /* primitives are the points [3][n] themselves */

/* Human-readable name of a status code (static storage). */
const char *mg_status_string(mg_status s);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t mg_version(void);

/* Returns MG_OK if the current HIP device is a gfx950 (MI355X class) GPU. */
mg_status mg_check_device(void);

/* ------------------------------------------------------------------------
 * Frame selection and vertex-buffer update (Sec. 3.3 MaGS paragraph:
 * k = floor(t * f_recon); Sec. 3.4 per-frame steps 1-2).
 * ---------------------------------------------------------------------- */

/* Host-only integer arithmetic: t = step / f_sim seconds, f_recon =
 * f_recon_num / f_recon_den frames per second, *k_out (host) =
 * min(floor(step * f_recon_num / (f_sim * f_recon_den)), n_frames - 1).
 * Invalid: step < 0, f_recon_num < 0, f_recon_den <= 0, f_sim <= 0,
 * n_frames <= 0, k_out == NULL. */
mg_status mg_frame_index(int64_t step, int64_t f_recon_num, int64_t f_recon_den, int64_t f_sim,
                         int32_t n_frames, int32_t *k_out);

/* live[3][n_verts] <- frames[k][3][n_verts] (a bitwise O(N_v) copy on the
 * device).  frames is a [n_frames][3][n_verts] store; 0 <= k < n_frames.
 * live must not overlap frame k. */
mg_status mg_vertex_buffer_update(const float *frames, int32_t n_frames, int32_t n_verts, int32_t k,
                                  float *live, void *stream);

/* x[n] <- value on the device (a kernel, not a memset, so it may sit in a
 * captured HIP graph); used to clear gradient accumulators. */
mg_status mg_fill(float *x, int64_t n, float value, void *stream);

/* out[n] = wa a[n] + wb b[n] on the device (out may alias a or b).  The
 * re-anchoring of temporal correspondence tracking (Sec. 3.3, Strategy 1:
 * every 50 frames, 80% tracked motion blended with 20% template projection). */
mg_status mg_blend(const float *a, const float *b, float wa, float wb, float *out, int64_t n, void *stream);

/* ------------------------------------------------------------------------
 * Face-bound Gaussian re-pose (render side of the dual representation,
 * Sec. 3.2).  The paper states no binding formula; the library computes, per
 * Gaussian g bound to face f = gface[g] with vertices (v0, v1, v2) in stored
 * order:
 *   triangle frame  e1 = v1 - v0, e2 = v2 - v0, n = e1 x e2, t = e1/|e1|,
 *                   nh = n/|n|, b = nh x t, R_f = [t b nh] (columns);
 *                   |e1| == 0 or |n| == 0 gives R_f = I, nh = 0;
 *   mean            mu = (1 - b1 - b2) v0 + b1 v1 + b2 v2 + offset * nh;
 *   rotation        R_g = R_f R(q_l), q_l = (w,x,y,z) normalised; quat =
 *                   Shepperd's extraction of R_g, sign fixed so w > 0 (w == 0:
 *                   first non-zero of x, y, z positive);
 *   covariance      Sigma = R_g diag(exp(2 log_scale)) R_g^T packed as
 *                   (xx, xy, xz, yy, yz, zz).
 * ---------------------------------------------------------------------- */

/* Inputs: verts [3][n_verts], faces [3][n_faces], gface [n_gauss] (face of
 * each Gaussian, any order; sorted by face is fastest), bary [2][n_gauss]
 * (b1, b2), q_local [4][n_gauss], log_scale [3][n_gauss], offset [n_gauss]
 * or NULL (zero).  Outputs: mean [3][n_gauss] (required), quat [4][n_gauss],
 * cov [6][n_gauss], rot [9][n_gauss] (row-major R_g), each NULL to skip.
 * flags must be 0. */
mg_status mg_mesh_gaussian_update(const float *verts, int32_t n_verts, const int32_t *faces,
                                  int32_t n_faces, const int32_t *gface, const float *bary,
                                  const float *q_local, const float *log_scale, const float *offset,
                                  int32_t n_gauss, uint32_t flags, float *mean, float *quat,
                                  float *cov, float *rot, void *stream);

/* Backward of mg_mesh_gaussian_update w.r.t. the vertices: g_verts [3][n_verts]
 * is ACCUMULATED into (+=) from g_mean [3][G], g_rot [9][G] (row-major
 * dL/dR_g) and g_cov [6][G] (dL/d packed Sigma), each NULL for zero (all
 * three NULL: no-op).  The quaternion output is not differentiated.  Uses float atomics:
 * results are reproducible to rounding, not bitwise. */
mg_status mg_mesh_gaussian_update_backward(const float *verts, int32_t n_verts, const int32_t *faces,
                                           int32_t n_faces, const int32_t *gface, const float *bary,
                                           const float *q_local, const float *log_scale,
                                           const float *offset, int32_t n_gauss, const float *g_mean,
                                           const float *g_rot, const float *g_cov, float *g_verts,
                                           void *stream);

/* ------------------------------------------------------------------------
 * Linear BVH (Karras 2012) over triangles or points.  Built once from the
 * template faces and then only refit per frame (Sec. 3.4); rebuilt every frame
 * on the varying-topology comparison path (Sec. 4.1).
 *
 * Construction, all on the device: per-axis bounds of s = (v0 + v1) + v2
 * (points: s = p); 30-bit Morton codes defined in IEEE binary32 (scale =
 * 1024/(hi - lo) or 0, q = min(1023, trunc((s - lo) * scale)), x bits most
 * significant); stable LSD radix sort of (code, primitive id); Karras binary
 * radix tree with the leaf index as tie-break; leaf permutation; refit.
 *
 * A BVH lives in ONE caller-allocated device buffer of
 * mg_lbvh_layout_query()->total_bytes, 256-byte aligned; section offsets (in
 * bytes from its start) are returned so callers may read it:
 *   header      mg_lbvh_header (below)
 *   codes       uint32 [n]       sorted Morton codes
 *   prim        int32  [n]       leaf -> original primitive id
 *   leaf_faces  int32  [3][n]    vertex ids of each leaf's face (triangles only)
 *   leaf_parent int32  [n]       (parent << 1) | slot, -1 when n == 1
 *   node_parent int32  [n-1]     (parent << 1) | slot, -1 for the root (node 0)
 *   nodes       float4 [n-1][6]  per internal node, slot 0 = left child (float4
 *                                0..2), slot 1 = right child (float4 3..5):
 *                                internal child (triangles): (lo.xyz, ref) (hi.xyz, a) (d.xyz, b)
 *                                internal child (points):    (lo.xyz, ref) (hi.xyz, 0) (unused)
 *                                leaf triangle:  (v0.xyz, ref) (v1.xyz, id) (v2.xyz, 0)
 *                                leaf point:     (p.xyz, ref)  (p.xyz, id)  (unused)
 *                                ref (int bits): >= 0 internal node, < 0 leaf ~ref;
 *                                id: original primitive id.  A leaf's box is the
 *                                min/max of its vertices.  Normal slab of an
 *                                internal child: d is the unit sum of the area-
 *                                weighted normals of the faces below it (for the
 *                                vertices of the last build/refit; zero with
 *                                a = -inf, b = +inf when that sum vanishes), and
 *                                a <= d.x <= b for every point x of those faces
 *                                (a conservative bound, formed bottom-up from the
 *                                children's slabs and the node's box).  The
 *                                refit rewrites all of it.
 *   node_aux    int32  [n-1]     refit schedule: index among the "top" nodes (those
 *                                with more than 2^chunk_log2 leaves), or -1
 *   child       int32  [2][n-1]  child references of each internal node, as in the
 *                                records (>= 0 internal node, < 0 leaf ~i)
 *   top_nodes   int32  [n]       node id of each top node (header.n_top of them)
 *   top_child   int32  [4][n]    plane s < 2, per top node: its child in slot s,
 *                                as that child's top index, or ~k for the root of
 *                                subtree k; plane 2 + s: that child's node id when
 *                                it is a top node (0 otherwise)
 *   subtrees    int32  [3][n]    per subtree (header.n_sub): root reference, first
 *                                and last leaf; the subtrees (at most 2^chunk_log2
 *                                leaves, children of top nodes) cut the tree
 *   deposits    float4 [n][3]    refit scratch: each subtree root's summary (box,
 *                                normal direction and sum length, slab)
 *   top_scratch float4 [n][3] + uint32 [n]  refit scratch for the top nodes when
 *                                they are too many for the workgroup's LDS
 *   inv_prim    int32  [n]       original primitive id -> leaf (inverse of prim)
 * ---------------------------------------------------------------------- */

typedef struct mg_lbvh_header {
    int32_t n_prims;
    int32_t prim_kind;
    int32_t status;        /* device-side error word, 0 = fine; bits: 4 inconsistent
                              tree, 8 bad refit schedule, 16 a query found an id
                              without a leaf or a bounded wait ran out, 32 a refit
                              or query was given a vertex count other than the
                              build's, 64 a traversal stack overflowed (with 16,
                              32 or 64 set, results may be wrong) */
    int32_t n_verts;       /* vertex count of the build (the points for MG_PRIM_POINTS) */
    float root_lo[3];      /* root box (the only box not stored in a node record) */
    float pad0;
    float root_hi[3];
    float pad1;
    float quant_lo[3];     /* Morton quantisation of the last build: lo, scale */
    float quant_scale[3];
    uint32_t bounds_enc[6];/* build scratch: order-preserving encodings of lo/hi */
    uint32_t tile_counter[4];
    int32_t chunk_log2;    /* refit: subtrees of at most 2^chunk_log2 leaves */
    int32_t n_top;         /* number of top nodes */
    int32_t n_sub;         /* number of subtrees (n_top + 1 when n > 2^chunk_log2) */
    uint32_t refit_arrivals; /* refit scratch: subtrees finished in the running refit (0 between refits) */
    int32_t reserved[8];
} mg_lbvh_header;

typedef struct mg_lbvh_layout {
    int64_t total_bytes;
    int64_t off_header;
    int64_t off_codes;
    int64_t off_prim;
    int64_t off_leaf_faces;
    int64_t off_leaf_parent;
    int64_t off_node_parent;
    int64_t off_nodes;
    int64_t off_node_aux;
    int64_t off_child;
    int64_t off_top_nodes;
    int64_t off_top_child;
    int64_t off_subtrees;
    int64_t off_deposits;
    int64_t off_top_scratch;
    int64_t off_inv_prim;
} mg_lbvh_layout;

/* Host-only: section offsets and total size of a BVH over n_prims primitives
 * of the given kind.  out is a host pointer. */
mg_status mg_lbvh_layout_query(int32_t n_prims, int32_t prim_kind, mg_lbvh_layout *out);

/* Host-only: bytes of device workspace mg_lbvh_build needs (ws_bytes host). */
mg_status mg_lbvh_workspace_size(int32_t n_prims, int32_t prim_kind, size_t *ws_bytes);

/* Build a BVH.  verts [3][n_verts] (points: the primitives themselves, then
 * n_prims == n_verts and faces == NULL); faces [3][n_prims] for triangles.
 * bvh: device buffer of at least layout.total_bytes; ws: device workspace of
 * at least mg_lbvh_workspace_size bytes (contents need not be initialised,
 * may be reused after the call completes on the stream). */
mg_status mg_lbvh_build(const float *verts, int32_t n_verts, const int32_t *faces, int32_t n_prims,
                        int32_t prim_kind, void *bvh, size_t bvh_bytes, void *ws, size_t ws_bytes,
                        void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): mg_lbvh_build with the sort
 * workspace taken from a static device array that the library holds on each
 * device until the process ends (about 17 MiB), instead of a caller buffer.
 * n_prims at most MG_LBVH_STATIC_MAX_PRIMS (2^20), else MG_ERR_INVALID_ARGUMENT;
 * the other arguments and the result are as for mg_lbvh_build.  The call
 * allocates nothing; the first call on a device looks up that device's copy of
 * the array.  All calls on one device share the array: calls that may overlap in
 * time on one device (different streams without ordering) race and build wrong
 * trees, so order them on one stream. */
#define MG_LBVH_STATIC_MAX_PRIMS (1 << 20)
mg_status mg_lbvh_build_static(const float *verts, int32_t n_verts, const int32_t *faces,
                               int32_t n_prims, int32_t prim_kind, void *bvh, size_t bvh_bytes,
                               void *stream);

/* Refit in place: recompute every box of a built BVH for new vertex positions
 * (same n_prims and prim_kind as the build; topology unchanged).  One kernel: a
 * workgroup per subtree, the last of them also refits the top nodes.  verts must
 * hold exactly the n_verts of the build: the faces stored at build time index
 * them.  The refit and every query compare n_verts with the build's
 * (header.n_verts) and set status bit 32 when they differ; vertex ids are then
 * clamped into [0, n_verts), so a wrong count gives wrong boxes and results but
 * never a read outside the caller's array.
 * Refits (and builds) of one BVH must not run concurrently: they share its
 * scratch sections. */
mg_status mg_lbvh_refit(const float *verts, int32_t n_verts, void *bvh, size_t bvh_bytes,
                        int32_t n_prims, int32_t prim_kind, void *stream);

/* The per-frame update of a fixed-topology mesh in one launch (Sec. 3.4: the
 * vertex buffer written from the current reconstruction frame, the render
 * Gaussians re-posed from their faces, the collision BVH refit, O(N_v)):
 * copies frame k of frames [n_frames][3][n_verts] into live [3][n_verts],
 * re-poses the n_gauss Gaussians bound to faces [3][n_faces] (arguments and
 * outputs as for mg_mesh_gaussian_update, flags 0; n_gauss may be 0) and refits
 * bvh, a MG_PRIM_TRIANGLES BVH built over those faces and n_verts vertices.
 * All three read the vertices from frame k itself, so they run side by side in
 * one kernel; the results are bitwise those of mg_vertex_buffer_update,
 * mg_mesh_gaussian_update and mg_lbvh_refit called in turn.  live must not
 * overlap frame k.  The refit's rules hold (no concurrent refit of one BVH;
 * a vertex count other than the build's sets status bit 32). */
mg_status mg_frame_update(const float *frames, int32_t n_frames, int32_t n_verts, int32_t k, float *live,
                          const int32_t *faces, int32_t n_faces, const int32_t *gface, const float *bary,
                          const float *q_local, const float *log_scale, const float *offset,
                          int32_t n_gauss, float *mean, float *quat, float *cov, float *rot, void *bvh,
                          size_t bvh_bytes, void *stream);

/* Traversal choice for the query calls (NULL options = MG_QUERY_AUTO).
 *   MG_QUERY_LANE   one query per lane, depth-first, nearer child first
 *   MG_QUERY_BATCH  one wave per `batch` queries (1, 2, 4, 8, 16 or 32) sharing
 *                   an LDS work stack, up to 64 node expansions per step; suits
 *                   few queries or queries with many near-equidistant faces
 *   MG_QUERY_AUTO   BATCH with the default batch and seed on
 * batch == 0 means the default: the largest of 16, 8, 4, 2, 1 with
 * n_queries >= 2048 batch (at least 512 workgroups of four waves).  NULL
 * options also turn the seed on; with options given, seed is as set.  seed != 0 (BATCH only): each query first descends
 * greedily (nearer child first) to one leaf to start from a tight bound before
 * the wide expansion.  order (device int32 [n_queries] permutation, or NULL):
 * queries are processed in the order order[0], order[1], ... - e.g. the prim
 * section of a MG_PRIM_POINTS BVH built over the queries, i.e. Morton order -
 * and every result is still written at the query's own index.  counters
 * (device uint64 [4], or NULL): += node expansions, leaf bound tests, exact
 * leaf tests, queries.  queue (device uint32 [1], or NULL; BATCH only): the
 * waves stay resident and take query batches one at a time from this counter,
 * which the call zeroes on its stream before the traversal (no initial value
 * needed); calls that may overlap in time must use different words.  Without a
 * queue, batches are dealt to the waves statically.  hint (device int32
 * [n_queries], or NULL): an original primitive id per query (-1 or out of range:
 * none), e.g. the previous frame's result; each query starts from that
 * primitive's distance instead of the seed descent, which makes frame-to-frame
 * queries on a slowly moving mesh cheap.  hint may be the output id array of
 * the same call (a query reads its hint before writing its result).  warm
 * (mg_chamfer only, which ignores hint): non-zero means nn_ab and nn_ba hold
 * earlier answers on entry (e.g. the previous call's) that start the queries
 * of their directions.  waves (BATCH on triangles): the batch kernel's register
 * allocation; 0 picks five resident waves per SIMD when the batches outnumber
 * four waves on every SIMD (more than 4,096 batches) and four otherwise, 4 or
 * 5 forces one; any other value is MG_ERR_INVALID_ARGUMENT.  Results do not
 * depend on any of these choices except among exact ties, which all pick the
 * lowest original id. */
#define MG_QUERY_AUTO  0
#define MG_QUERY_LANE  1
#define MG_QUERY_BATCH 2

typedef struct mg_query_options {
    int32_t kernel;
    int32_t batch;
    int32_t seed;
    int32_t warm;
    const int32_t *order;
    uint64_t *counters;
    uint32_t *queue;
    const int32_t *hint;
    int32_t waves;
} mg_query_options;

/* ------------------------------------------------------------------------
 * Closest point on a triangle mesh (NearestSurface with barycentric
 * interpolation, Sec. 3.3 Eq. 1-2, read as the single nearest face) with the
 * face normal computed on demand (Sec. 3.4 step 3).  A face is the closed
 * triangle, the hull of its vertices: a face with two equal vertices is the
 * segment between the distinct ones (and has no normal).  Exact ties of the
 * float32 squared distance go to the lowest original face id.  Per query q:
 *   face[q]   original face id, -1 if no face has d^2 <= max_dist2
 *   point     [3][nq] closest point (the query itself when face == -1)
 *   bary      [2][nq] (w1, w2): point = (1-w1-w2) v0 + w1 v1 + w2 v2 (0 when none)
 *   dist2     [nq] squared distance (+inf when none)
 *   normal    [3][nq] unit normal of the face, zero if degenerate or none
 * point, bary, dist2, normal may each be NULL to skip.  max_dist2 >= 0
 * (+inf allowed).  bvh must be a MG_PRIM_TRIANGLES BVH built/refit on verts
 * (leaf triangles are read from the BVH, the winner's from verts).  opts: host
 * pointer or NULL.
 * ---------------------------------------------------------------------- */
mg_status mg_closest_point_query(const void *bvh, size_t bvh_bytes, int32_t n_prims,
                                 const float *verts, int32_t n_verts, const float *queries,
                                 int32_t n_queries, float max_dist2, int32_t *face, float *point,
                                 float *bary, float *dist2, float *normal,
                                 const mg_query_options *opts, void *stream);

/* Same contract as mg_closest_point_query but tests every face for every query
 * (no BVH; for self-checks on small meshes).  faces [3][n_faces]. */
mg_status mg_closest_point_bruteforce(const float *verts, int32_t n_verts, const int32_t *faces,
                                      int32_t n_faces, const float *queries, int32_t n_queries,
                                      float max_dist2, int32_t *face, float *point, float *bary,
                                      float *dist2, float *normal, void *stream);

/* k-NN weighted surface projection (the weighted nearest-neighbour variant of
 * NearestSurface in Sec. 3.3; the paper states neither k nor the weights).
 * For every query, the k faces of a MG_PRIM_TRIANGLES BVH nearest
 * to it (1 <= k <= 8; ties of the squared distance to the lowest original face
 * id; faces farther than max_dist2 are ignored), and their closest points c_i
 * at distances d_i combined as point = sum w_i c_i / sum w_i with
 * w_i = 1 / (d_i + eps) (eps >= 0; a face at distance exactly 0 gives its point).
 * Outputs (device): face_k [k][n_queries] (-1 where fewer than k faces exist or
 * lie within max_dist2), dist2_k [k][n_queries] or NULL (+inf for -1 entries),
 * point [3][n_queries] or NULL (the query itself when no face qualifies).
 * counters: NULL or a device uint64 [4] accumulating node expansions, leaf
 * bound tests, exact leaf tests and queries (as mg_query_options.counters).
 * One query per lane; k = 1 gives the single closest point (unweighted). */
mg_status mg_knn_surface_query(const void *bvh, size_t bvh_bytes, int32_t n_prims, const float *verts,
                               int32_t n_verts, const float *queries, int32_t n_queries, int32_t k,
                               float eps, float max_dist2, int32_t *face_k, float *dist2_k, float *point,
                               uint64_t *counters, void *stream);

/* Nearest point of a MG_PRIM_POINTS BVH built over points [3][n_prims]:
 * index[q] (lowest index on exact ties, -1 if none within max_dist2) and
 * dist2[q] (+inf if none); dist2 may be NULL.  opts as for mg_closest_point_query. */
mg_status mg_nearest_point_query(const void *bvh, size_t bvh_bytes, int32_t n_prims,
                                 const float *points, const float *queries, int32_t n_queries,
                                 float max_dist2, int32_t *index, float *dist2,
                                 const mg_query_options *opts, void *stream);

/* ------------------------------------------------------------------------
 * Index signed-distance grid: the SDF the paper builds from the template
 * faces beside the BVH (Sec. 3.4, Initialization: structures that store only
 * indices and serve every frame).  An nx x ny x nz grid (each >= 2, at most
 * 2^31 - 1 nodes) with node (i, j, k) at lo + h (i, j, k), node index
 * i + nx (j + ny k).  At initialisation every node stores the ids of its k
 * nearest template faces (mg_knn_surface_query on the node positions); per
 * frame mg_sdf_update recomputes each node's signed distance from those faces'
 * current vertices: the minimum point-to-triangle distance over them (ties to
 * the lowest slot), positive where the winning face's normal points (and on
 * its plane), negative behind it.  Exact while a node's nearest face stays
 * among its k; an upper bound of the unsigned distance otherwise.
 * ---------------------------------------------------------------------- */

/* points [3][nx ny nz] (device) <- the node positions. */
mg_status mg_grid_points(float lo_x, float lo_y, float lo_z, float h, int32_t nx, int32_t ny, int32_t nz,
                         float *points, void *stream);

/* sdf [nx ny nz] (device) <- signed distances of the nodes to their faces
 * face_k [k][nx ny nz] (1 <= k <= 64; ids outside [0, n_faces) are ignored;
 * a node with no valid face gets +inf); face [nx ny nz] (device, or NULL) <-
 * the winning face id (-1 if none).  verts [3][n_verts], faces [3][n_faces]. */
mg_status mg_sdf_update(const float *verts, int32_t n_verts, const int32_t *faces, int32_t n_faces,
                        const int32_t *face_k, int32_t k, float lo_x, float lo_y, float lo_z, float h,
                        int32_t nx, int32_t ny, int32_t nz, float *sdf, int32_t *face, void *stream);

/* out [n_queries] (device) <- trilinear interpolation of the node values sdf at
 * queries [3][n_queries]; +inf for a query outside the grid's box. */
mg_status mg_sdf_sample(const float *sdf, float lo_x, float lo_y, float lo_z, float h, int32_t nx, int32_t ny,
                        int32_t nz, const float *queries, int32_t n_queries, float *out, void *stream);

/* ------------------------------------------------------------------------
 * Sphere-mesh contact step from on-demand face normals: collision response
 * for spheres dropped on the mesh (the falling-sphere simulation of Sec. 4.1;
 * face normals computed on demand, Sec. 3.4 step 3).  A step of spheres of
 * radius r: mg_particles_integrate, then mg_closest_point_query at the new
 * positions (point, face and normal outputs), then mg_contact_response.
 * Positions x and velocities v are [3][n] float32 device arrays.
 * ---------------------------------------------------------------------- */

/* v <- v + g dt, then x <- x + v dt (semi-implicit Euler); dt >= 0. */
mg_status mg_particles_integrate(float *x, float *v, int32_t n, float gx, float gy, float gz, float dt,
                                 void *stream);

/* With c = point, n = normal (unit, zero for a degenerate face), face (-1 for
 * none) from mg_closest_point_query at x: side = (x - c) . n; a sphere is in
 * contact when face >= 0, n != 0 and (side < 0 or |x - c| < radius).  Then
 * nh = (x - c)/|x - c| if side >= 0 and |x - c| > 0, else n; x <- c + radius nh;
 * if v . nh < 0, v <- v - (1 + restitution)(v . nh) nh.  restitution in
 * [0, 1], radius >= 0; contact [n] (device int32, or NULL) <- 1 / 0. */
mg_status mg_contact_response(float *x, float *v, int32_t n, const float *point, const float *normal,
                              const int32_t *face, float radius, float restitution, int32_t *contact,
                              void *stream);

/* ------------------------------------------------------------------------
 * Losses for differentiable template projection.  Chamfer distance is used
 * by the paper as a metric (Sec. 4.2) without a formula; the library's is
 * CD(A,B) = mean_a min_b |a-b|^2 + mean_b min_a |a-b|^2.
 * ---------------------------------------------------------------------- */

/* Workspace bytes (host out) for mg_mean / mg_chamfer over up to n values. */
mg_status mg_reduce_workspace_size(int64_t n, size_t *ws_bytes);

/* out[0] (device, float64) = mean of x[n] (0 when n == 0), deterministic:
 * fixed-order per-block float64 partial sums, then one block sums them. */
mg_status mg_mean(const float *x, int64_t n, double *out, void *ws, size_t ws_bytes, void *stream);

/* The two-sided Chamfer distance (Sec. 4.2's geometric metric, read as the
 * sum of the two mean squared nearest distances):
 * nn_ab[i] / d_ab[i]: nearest b of a_i and its squared distance (via bvh_b,
 * a MG_PRIM_POINTS BVH over b); nn_ba / d_ba likewise via bvh_a over a;
 * out (device float64 [3]): out[0] = mean d_ab, out[1] = mean d_ba,
 * out[2] = (out[0] + out[1]) + add[0], where add (device float64, or NULL for
 * 0) is another loss term to fold in, e.g. the point-to-mesh term of the
 * template projection.  opts as for mg_nearest_point_query (applies to both
 * directions) except hint, which is ignored: with opts->warm set, the entries
 * of nn_ab and nn_ba on entry are the hints of their directions (ids out of
 * range count as none). */
mg_status mg_chamfer(const float *a, int32_t na, const void *bvh_a, size_t bvh_a_bytes,
                     const float *b, int32_t nb, const void *bvh_b, size_t bvh_b_bytes,
                     int32_t *nn_ab, float *d_ab, int32_t *nn_ba, float *d_ba, double *out,
                     const double *add, void *ws, size_t ws_bytes, const mg_query_options *opts,
                     void *stream);

/* g_verts [3][n_verts] += scale * g * sum_q -2 w_k (y_q - c_q) on the three
 * vertices of each query's face (queries with face == -1 contribute nothing).
 * face/point/bary as returned by mg_closest_point_query on the same mesh.
 * g_loss: optional device float64 scalar (the upstream gradient of the loss,
 * read on the device so autograd needs no host sync); NULL means g = 1.
 * Accumulates with float32 atomics, so the summation order (last bits) may
 * vary between runs. */
mg_status mg_point_mesh_backward(const float *verts, int32_t n_verts, const int32_t *faces,
                                 int32_t n_faces, const float *queries, int32_t n_queries,
                                 const int32_t *face, const float *point, const float *bary,
                                 float scale, const double *g_loss, float *g_verts, void *stream);

/* g_a [3][na] += g * (2 scale_ab (a_i - b_nn_ab(i)) + 2 scale_ba sum_{j: nn_ba(j)=i} (a_i - b_j)),
 * g = *g_loss (device float64) or 1 when g_loss is NULL.  Swapping the roles
 * of a and b (and of the two maps and scales) gives the gradient w.r.t. b. */
mg_status mg_chamfer_backward(const float *a, int32_t na, const float *b, int32_t nb,
                              const int32_t *nn_ab, const int32_t *nn_ba, float scale_ab,
                              float scale_ba, const double *g_loss, float *g_a, void *stream);

/* Adam (Kingma & Ba 2015) in torch.optim.Adam's order, in place on param/m/v
 * [n] float32; step counts from 1. */
mg_status mg_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int32_t step,
                       float lr, float beta1, float beta2, float eps, void *stream);

/* ------------------------------------------------------------------------
 * Batched form: many scenes x frames of uneven size in one persistent launch.
 * Per scene-frame it does what the plain per-frame path does - Gaussian
 * re-pose, refit of the scene's template BVH, closest-point queries - reading
 * frame t's vertices in place from the frame store (the vertex buffer of
 * Sec. 3.4 step 2 aliases the frame) and writing every frame's results to its
 * own output block.  Work items are taken in index order from one atomic queue
 * in four phases (refit chunks, Gaussian tiles, refit top nodes, query tiles);
 * a top item waits for its scene-frame's chunks and a query item for its
 * refit, so every wait is on earlier items held by running workgroups.
 * Results are bitwise those of the plain calls with the same query options.
 * ---------------------------------------------------------------------- */

typedef struct mg_batch_scene {
    const float *frames;        /* [n_frames][3][n_verts] */
    int32_t n_frames;
    int32_t n_verts;
    const int32_t *faces;       /* [3][n_faces] */
    int32_t n_faces;
    int32_t n_gauss;
    const int32_t *gface;       /* [n_gauss] */
    const float *bary;          /* [2][n_gauss] */
    const float *q_local;       /* [4][n_gauss] */
    const float *log_scale;     /* [3][n_gauss] */
    const float *queries;       /* [3][n_queries] */
    int32_t n_queries;
    int32_t batch;              /* this scene's queries per wave (1, 2, 4, 8, 16); 0: the plan's */
    int32_t seed;               /* this scene's seed descent: 0 off, 1 on, -1: the plan's */
    int32_t query_tile;         /* this scene's queries per work item, a multiple of 4 * its
                                   batch; 0: the plan's */
    const void *bvh;            /* MG_PRIM_TRIANGLES BVH built over this scene's faces: only
                                   its topology is used, its boxes are untouched */
    size_t bvh_bytes;
    float *nodes;               /* out [n_frames][n_faces-1][24]: per-frame node records */
    float *roots;               /* out [n_frames][8]: per-frame root box (lo xyz, 0, hi xyz, 0) */
    float *mean;                /* out [n_frames][3][n_gauss] */
    float *quat;                /* out [n_frames][4][n_gauss] or NULL */
    float *cov;                 /* out [n_frames][6][n_gauss] or NULL */
    int32_t *face;              /* out [n_frames][n_queries] */
    float *point;               /* out [n_frames][3][n_queries] or NULL */
    float *qbary;               /* out [n_frames][2][n_queries] or NULL */
    float *dist2;               /* out [n_frames][n_queries] or NULL */
    float *normal;              /* out [n_frames][3][n_queries] or NULL */
} mg_batch_scene;

/* Plan-wide defaults; a scene's own batch / seed / query_tile fields override
 * them (the autotuner picks the traversal per scene). */
typedef struct mg_batch_options {
    int32_t batch;              /* queries per wave of the batch traversal: 1, 2, 4, 8, 16 (0: 4) */
    int32_t seed;               /* greedy seed descent: 0 off, otherwise on */
    int32_t gauss_tile;         /* Gaussians per work item, multiple of 256 (0: 2048) */
    int32_t query_tile;         /* queries per work item, multiple of 4 * batch (0: 256) */
    int32_t reserved[4];        /* must be 0 */
} mg_batch_options;

/* Bytes of the device plan for these scenes (scenes: host array).  Reads each
 * scene BVH's top-node count from its device header (a synchronous copy):
 * scenes with more than 384 top nodes get second-phase refit scratch in the
 * plan.  A scene may have at most 262,144 faces (the batched refit keeps
 * subtrees of up to 512 leaves in LDS); larger ones give
 * MG_ERR_INVALID_ARGUMENT. */
mg_status mg_batch_plan_size(const mg_batch_scene *scenes, int32_t n_scenes, size_t *plan_bytes);

/* Validate the scenes and write the device plan (scene table, work-item
 * counts, dependency counters).  scenes/opts are host pointers (opts may be
 * NULL); plan is a device buffer of mg_batch_plan_size bytes.  Copies the
 * table with the stream and synchronises it (initialisation only).  Every
 * scene needs n_faces >= 1, n_frames >= 1 and a built BVH over exactly its
 * faces and n_verts vertices (else MG_ERR_TOPOLOGY_MISMATCH); the BVH must not
 * be rebuilt between plan_init and the runs. */
mg_status mg_batch_plan_init(const mg_batch_scene *scenes, int32_t n_scenes, const mg_batch_options *opts,
                             void *plan, size_t plan_bytes, void *stream);

/* One run over all scenes x frames: a small reset kernel, then the
 * persistent kernel.  Asynchronous; capturable in a HIP graph.  Runs on the
 * same plan must not overlap.  A scene's queries in frame t > 0 start from
 * their faces of frame t - 1 when those are already computed (the results are
 * the same either way); the face outputs are written with device-coherent
 * stores for that. */
mg_status mg_batch_run(void *plan, size_t plan_bytes, void *stream);

/* Host-only: device address of the plan's int32 error word (0 = fine; a
 * non-zero value means a dependency wait timed out or a scene's BVH does not
 * match the plan). */
mg_status mg_batch_status_word(void *plan, int32_t **status);

/* ------------------------------------------------------------------------
 * Validation helpers (asynchronous; the result lands in a device int32).
 * ---------------------------------------------------------------------- */

/* *status_out (device int32) is set to MG_ERR_INDEX_OUT_OF_RANGE if any of
 * idx[n] lies outside [0, bound), else left unchanged (caller zeroes it). */
mg_status mg_validate_indices(const int32_t *idx, int64_t n, int32_t bound, int32_t *status_out,
                              void *stream);

/* *status_out (device int32) is set to MG_ERR_NONFINITE_INPUT if any of x[n]
 * is NaN or infinite, else left unchanged. */
mg_status mg_validate_finite(const float *x, int64_t n, int32_t *status_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MGU_H */
