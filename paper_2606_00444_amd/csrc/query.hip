// Closest point on a triangle mesh / nearest point of a point set through the
// LBVH, and an all-faces brute force for self-checks (gfx950).
//
// NearestSurface of the paper (Sec. 3.3, Eq. 1-2) projects a point onto a mesh
// with barycentric interpolation; it is read as the single nearest face.  The
// face normal is computed on demand from the three vertices of the winning
// face (Sec. 3.4 step 3), never stored.
//
// Traversal: one query per lane, depth-first, nearer child first.  A child is
// visited when its box distance is <= best * (1 + 2^-20): the slack keeps a
// float32 rounding of the box distance from pruning a face whose float32 distance
// ties the best (ties go to the lowest original id, which the node record
// carries next to each leaf child's box).  Leaf children are tested as soon as
// their box passes, so the bound tightens before descending.  The stack lives
// in LDS ([depth][lane], conflict-free) for the first 32 entries and in a
// private array beyond; Karras trees over 30-bit codes with index tie-break are
// at most 62 levels deep, so 64 entries always suffice.
#include "mgu_internal.hpp"

#include <climits>

namespace mgu {
namespace {

constexpr int kQueryBlock = 64;
constexpr int kLdsStack = 32;
constexpr int kMaxStack = 64;
constexpr float kPruneSlack = 1.0f + 1.0f / 1048576.0f;

struct QueryArgs {
    const float4 *nodes;
    const mg_lbvh_header *hdr;
    const int32_t *leaf_faces;   // [3][n] (triangles) or nullptr (points)
    const int32_t *prim;         // [n]
    const float *verts;          // mesh vertices or the points
    int64_t nv, n;
    const float *queries;
    int64_t nq;
    float maxd2;
    int32_t *face;
    float *point, *bary, *dist2, *normal;
};

template <bool kTri>
__global__ __launch_bounds__(kQueryBlock) void traverse_kernel(QueryArgs a) {
    __shared__ int32_t s_stack[kLdsStack][kQueryBlock];
    int32_t deep[kMaxStack - kLdsStack];
    const int lane = threadIdx.x;
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kQueryBlock + lane;
    if (q >= a.nq) return;
    const f3 p = load3(a.queries, a.nq, q);
    float best = a.maxd2;
    int32_t best_id = INT_MAX, best_leaf = -1;

    auto test_leaf = [&](int32_t leaf, int32_t id) {
        float d2;
        if (kTri) {
            const f3 A = load3(a.verts, a.nv, a.leaf_faces[leaf]);
            const f3 B = load3(a.verts, a.nv, a.leaf_faces[a.n + leaf]);
            const f3 C = load3(a.verts, a.nv, a.leaf_faces[2 * a.n + leaf]);
            float w1, w2;
            d2 = tri_closest(p, A, B, C, w1, w2);
        } else {
            const f3 d = p - load3(a.verts, a.nv, id);
            d2 = dot(d, d);
        }
        if (d2 < best || (d2 == best && id < best_id)) {
            best = d2;
            best_id = id;
            best_leaf = leaf;
        }
    };

    if (a.n == 1) {
        test_leaf(0, a.prim[0]);
    } else if (a.n > 1) {
        const f3 rlo = f3{a.hdr->root_lo[0], a.hdr->root_lo[1], a.hdr->root_lo[2]};
        const f3 rhi = f3{a.hdr->root_hi[0], a.hdr->root_hi[1], a.hdr->root_hi[2]};
        int sp = 0;
        int32_t node = box_dist2(p, rlo, rhi) <= best * kPruneSlack ? 0 : -1;
        // Each internal node is visited at most once in a valid tree; the step cap
        // and the reference range checks keep a corrupted buffer from looping or
        // reading out of bounds.
        const int64_t max_steps = a.n + 64;
        for (int64_t step = 0; node >= 0 && node < a.n - 1 && step < max_steps; ++step) {
            const float4 *rec = a.nodes + 4 * static_cast<int64_t>(node);
            const float4 l0 = rec[0], l1 = rec[1], r0 = rec[2], r1 = rec[3];
            const float dl = box_dist2(p, f3{l0.x, l0.y, l0.z}, f3{l1.x, l1.y, l1.z});
            const float dr = box_dist2(p, f3{r0.x, r0.y, r0.z}, f3{r1.x, r1.y, r1.z});
            const int32_t lref = __float_as_int(l0.w), rref = __float_as_int(r0.w);
            if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) break;
            float bound = best * kPruneSlack;
            bool gl = dl <= bound, gr = dr <= bound;
            if (gl && lref < 0) { test_leaf(~lref, __float_as_int(l1.w)); gl = false; }
            if (gr && rref < 0) { test_leaf(~rref, __float_as_int(r1.w)); gr = false; }
            bound = best * kPruneSlack;
            gl = gl && dl <= bound;
            gr = gr && dr <= bound;
            if (gl && gr) {
                const bool left_first = dl <= dr;
                const int32_t far = left_first ? rref : lref;
                node = left_first ? lref : rref;
                if (sp < kLdsStack) s_stack[sp][lane] = far;
                else if (sp < kMaxStack) deep[sp - kLdsStack] = far;
                sp = sp < kMaxStack ? sp + 1 : sp;   // unreachable bound (depth <= 62)
            } else if (gl) {
                node = lref;
            } else if (gr) {
                node = rref;
            } else if (sp > 0) {
                --sp;
                node = sp < kLdsStack ? s_stack[sp][lane] : deep[sp - kLdsStack];
            } else {
                node = -1;
            }
        }
    }

    if (kTri) {
        if (best_leaf >= 0) {
            const f3 A = load3(a.verts, a.nv, a.leaf_faces[best_leaf]);
            const f3 B = load3(a.verts, a.nv, a.leaf_faces[a.n + best_leaf]);
            const f3 C = load3(a.verts, a.nv, a.leaf_faces[2 * a.n + best_leaf]);
            float w1, w2;
            const float d2 = tri_closest(p, A, B, C, w1, w2);
            const float w0 = 1.0f - w1 - w2;
            a.face[q] = best_id;
            if (a.point)
                store3(a.point, a.nq, q, f3{w0 * A.x + w1 * B.x + w2 * C.x, w0 * A.y + w1 * B.y + w2 * C.y,
                                            w0 * A.z + w1 * B.z + w2 * C.z});
            if (a.bary) { a.bary[q] = w1; a.bary[a.nq + q] = w2; }
            if (a.dist2) a.dist2[q] = d2;
            if (a.normal) store3(a.normal, a.nq, q, tri_normal(A, B, C));
        } else {
            a.face[q] = -1;
            if (a.point) store3(a.point, a.nq, q, p);
            if (a.bary) { a.bary[q] = 0.0f; a.bary[a.nq + q] = 0.0f; }
            if (a.dist2) a.dist2[q] = INFINITY;
            if (a.normal) store3(a.normal, a.nq, q, f3{0.0f, 0.0f, 0.0f});
        }
    } else {
        a.face[q] = best_leaf >= 0 ? best_id : -1;
        if (a.dist2) a.dist2[q] = best_leaf >= 0 ? best : INFINITY;
    }
}

// Every face for every query, in original face order (strict < keeps the
// lowest id on exact ties).
__global__ __launch_bounds__(256) void bruteforce_kernel(const float *__restrict__ verts, int64_t nv,
                                                         const int32_t *__restrict__ faces, int64_t nf,
                                                         const float *__restrict__ queries, int64_t nq,
                                                         float maxd2, int32_t *face, float *point,
                                                         float *bary, float *dist2, float *normal) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const f3 p = load3(queries, nq, q);
    float best = INFINITY;
    int64_t bf = -1;
    for (int64_t f = 0; f < nf; ++f) {
        const f3 A = load3(verts, nv, faces[f]);
        const f3 B = load3(verts, nv, faces[nf + f]);
        const f3 C = load3(verts, nv, faces[2 * nf + f]);
        float w1, w2;
        const float d2 = tri_closest(p, A, B, C, w1, w2);
        if (d2 < best) { best = d2; bf = f; }
    }
    if (bf >= 0 && best <= maxd2) {
        const f3 A = load3(verts, nv, faces[bf]);
        const f3 B = load3(verts, nv, faces[nf + bf]);
        const f3 C = load3(verts, nv, faces[2 * nf + bf]);
        float w1, w2;
        const float d2 = tri_closest(p, A, B, C, w1, w2);
        const float w0 = 1.0f - w1 - w2;
        face[q] = static_cast<int32_t>(bf);
        if (point)
            store3(point, nq, q, f3{w0 * A.x + w1 * B.x + w2 * C.x, w0 * A.y + w1 * B.y + w2 * C.y,
                                    w0 * A.z + w1 * B.z + w2 * C.z});
        if (bary) { bary[q] = w1; bary[nq + q] = w2; }
        if (dist2) dist2[q] = d2;
        if (normal) store3(normal, nq, q, tri_normal(A, B, C));
    } else {
        face[q] = -1;
        if (point) store3(point, nq, q, p);
        if (bary) { bary[q] = 0.0f; bary[nq + q] = 0.0f; }
        if (dist2) dist2[q] = INFINITY;
        if (normal) store3(normal, nq, q, f3{0.0f, 0.0f, 0.0f});
    }
}

template <typename T>
inline const T *cat(const void *base, int64_t off) {
    return reinterpret_cast<const T *>(static_cast<const char *>(base) + off);
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_closest_point_query(const void *bvh, size_t bvh_bytes, int32_t n_prims,
                                            const float *verts, int32_t n_verts, const float *queries,
                                            int32_t n_queries, float max_dist2, int32_t *face,
                                            float *point, float *bary, float *dist2, float *normal,
                                            void *stream) {
    if (bad_count(n_prims) || bad_count(n_verts) || bad_count(n_queries) || !bvh || !(max_dist2 >= 0.0f))
        return MG_ERR_INVALID_ARGUMENT;
    mg_lbvh_layout L;
    mg_lbvh_layout_query(n_prims, MG_PRIM_TRIANGLES, &L);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (n_queries == 0) return MG_OK;
    if (!queries || !face || (n_prims > 0 && (!verts || n_verts == 0))) return MG_ERR_INVALID_ARGUMENT;
    QueryArgs a;
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.hdr = cat<mg_lbvh_header>(bvh, L.off_header);
    a.leaf_faces = cat<int32_t>(bvh, L.off_leaf_faces);
    a.prim = cat<int32_t>(bvh, L.off_prim);
    a.verts = verts; a.nv = n_verts; a.n = n_prims;
    a.queries = queries; a.nq = n_queries; a.maxd2 = max_dist2;
    a.face = face; a.point = point; a.bary = bary; a.dist2 = dist2; a.normal = normal;
    hipLaunchKernelGGL(traverse_kernel<true>, dim3(blocks_for(n_queries, kQueryBlock)), dim3(kQueryBlock), 0,
                       as_stream(stream), a);
    return launch_status();
}

extern "C" mg_status mg_nearest_point_query(const void *bvh, size_t bvh_bytes, int32_t n_prims,
                                            const float *points, const float *queries, int32_t n_queries,
                                            float max_dist2, int32_t *index, float *dist2, void *stream) {
    if (bad_count(n_prims) || bad_count(n_queries) || !bvh || !(max_dist2 >= 0.0f))
        return MG_ERR_INVALID_ARGUMENT;
    mg_lbvh_layout L;
    mg_lbvh_layout_query(n_prims, MG_PRIM_POINTS, &L);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (n_queries == 0) return MG_OK;
    if (!queries || !index || (n_prims > 0 && !points)) return MG_ERR_INVALID_ARGUMENT;
    QueryArgs a;
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.hdr = cat<mg_lbvh_header>(bvh, L.off_header);
    a.leaf_faces = nullptr;
    a.prim = cat<int32_t>(bvh, L.off_prim);
    a.verts = points; a.nv = n_prims; a.n = n_prims;
    a.queries = queries; a.nq = n_queries; a.maxd2 = max_dist2;
    a.face = index; a.point = nullptr; a.bary = nullptr; a.dist2 = dist2; a.normal = nullptr;
    hipLaunchKernelGGL(traverse_kernel<false>, dim3(blocks_for(n_queries, kQueryBlock)), dim3(kQueryBlock), 0,
                       as_stream(stream), a);
    return launch_status();
}

extern "C" mg_status mg_closest_point_bruteforce(const float *verts, int32_t n_verts, const int32_t *faces,
                                                 int32_t n_faces, const float *queries, int32_t n_queries,
                                                 float max_dist2, int32_t *face, float *point, float *bary,
                                                 float *dist2, float *normal, void *stream) {
    if (bad_count(n_verts) || bad_count(n_faces) || bad_count(n_queries) || !(max_dist2 >= 0.0f))
        return MG_ERR_INVALID_ARGUMENT;
    if (n_queries == 0) return MG_OK;
    if (!queries || !face || (n_faces > 0 && (!verts || !faces || n_verts == 0)))
        return MG_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(bruteforce_kernel, dim3(blocks_for(n_queries, 256)), dim3(256), 0, as_stream(stream),
                       verts, (int64_t)n_verts, faces, (int64_t)n_faces, queries, (int64_t)n_queries, max_dist2,
                       face, point, bary, dist2, normal);
    return launch_status();
}
