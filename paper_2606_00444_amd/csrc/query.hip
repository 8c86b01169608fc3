// Closest point on a triangle mesh / nearest point of a point set through the
// LBVH, and an all-faces brute force for self-checks (gfx950).
//
// NearestSurface of the paper (Sec. 3.3, Eq. 1-2) projects a point onto a mesh
// with barycentric interpolation; it is read as the single nearest face.  The
// face normal is computed on demand from the three vertices of the winning
// face (Sec. 3.4 step 3), never stored.
//
// Pruning: a child is expanded when its lower bound is <= prune_bound(best)
// (traverse.hpp), a slack that keeps faces whose float32 distance ties the
// best, so ties go to the lowest original id (carried in the node record beside
// each leaf child) in every traversal.  Leaf children hold their triangle, so a
// leaf is tested with the data of the record that referenced it.
//
// Two traversals (chosen per call, see mg_query_options):
//  * lane:  one query per lane, depth-first, nearer child first; stack in LDS
//           for the first 32 entries and in a private array beyond (Karras trees
//           over 30-bit codes with index tie-break are at most 62 levels deep).
//  * batch: one wave owns M queries and a shared LDS stack of (query, node, box
//           distance) entries; each round the wave pops up to 64 entries, one per
//           lane, expands them and pushes the surviving children with ballots.
//           A query's best is a 64-bit LDS atomic min over (float bits of d^2,
//           original id): non-negative floats order like their bit patterns, so
//           this is the lexicographic (d^2, id) minimum.  A query near the middle
//           of a closed surface has thousands of near-equidistant faces; here they
//           are expanded 64 at a time instead of one lane walking them serially.
#include "traverse.hpp"

#include <atomic>

namespace mgu {
namespace {

// ---------------------------------------------------------------- lane kernel
template <bool kTri>
__global__ __launch_bounds__(kLaneBlock) void traverse_lane_kernel(QueryArgs a) {
    __shared__ int32_t s_stack[kLdsStack][kLaneBlock];
    int32_t deep[kMaxStack - kLdsStack];
    const int lane = threadIdx.x;
    check_vertex_count(a);
    const int64_t pos = static_cast<int64_t>(blockIdx.x) * kLaneBlock + lane;
    if (pos >= a.nq) return;
    const int64_t q = query_at(a, pos);
    if (q < 0) return;
    const f3 p = load3(a.queries, a.nq, q);
    const float dq = slab_query_margin(p);
    float best = a.maxd2;
    int32_t best_id = INT_MAX, best_leaf = -1;
    unsigned long long n_exp = 0, n_lbox = 0, n_lex = 0;
    {
        const unsigned long long h = hint_best<kTri>(a, q, p, pack_best(a.maxd2, INT_MAX));
        if (h != pack_best(a.maxd2, INT_MAX)) {
            best = __uint_as_float(static_cast<uint32_t>(h >> 32));
            best_id = static_cast<int32_t>(h & 0xffffffffull);
            best_leaf = a.inv_prim[best_id];
        }
    }

    auto consider = [&](float d2, int32_t id, int32_t leaf) {
        ++n_lex;
        if (d2 < best || (d2 == best && id < best_id)) {
            best = d2;
            best_id = id;
            best_leaf = leaf;
        }
    };

    if (a.n == 1) {
        consider(single_leaf_dist2<kTri>(a, p), a.prim[0], 0);
    } else if (a.n > 1) {
        const f3 rlo = f3{a.root[0], a.root[1], a.root[2]};
        const f3 rhi = f3{a.root[4], a.root[5], a.root[6]};
        int sp = 0;
        const float qm = qnorm1(p);
        int32_t node = box_dist2(p, rlo, rhi) <= prune_bound(best, qm) ? 0 : -1;
        // each internal node is visited at most once in a valid tree: the step cap
        // and the reference checks keep a corrupted buffer from looping or faulting
        for (int64_t step = 0; node >= 0 && node < a.n - 1 && step < a.n + 64; ++step) {
            const float4 *rec = a.nodes + 6 * static_cast<int64_t>(node);
            const float4 l0 = rec[0], l1 = rec[1], l2 = rec[2], r0 = rec[3], r1 = rec[4], r2 = rec[5];
            const int32_t lref = __float_as_int(l0.w), rref = __float_as_int(r0.w);
            if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) break;
            ++n_exp;
            n_lbox += (lref < 0) + (rref < 0);
            if (lref < 0 && leaf_box_dist2<kTri>(p, l0, l1, l2) <= prune_bound(best, qm))
                consider(leaf_dist2<kTri>(p, l0, l1, l2), __float_as_int(l1.w), ~lref);
            if (rref < 0 && leaf_box_dist2<kTri>(p, r0, r1, r2) <= prune_bound(best, qm))
                consider(leaf_dist2<kTri>(p, r0, r1, r2), __float_as_int(r1.w), ~rref);
            const float bound = prune_bound(best, qm);
            const float dl = lref >= 0 ? child_bound<kTri>(p, dq, l0, l1, l2) : INFINITY;
            const float dr = rref >= 0 ? child_bound<kTri>(p, dq, r0, r1, r2) : INFINITY;
            const bool gl = lref >= 0 && dl <= bound, gr = rref >= 0 && dr <= bound;
            if (gl && gr) {
                const bool left_first = dl <= dr;
                const int32_t far = left_first ? rref : lref;
                node = left_first ? lref : rref;
                if (sp < kLdsStack) s_stack[sp][lane] = far;
                else if (sp < kMaxStack) deep[sp - kLdsStack] = far;
                else atomicOr(a.status, 64);   // past the depth bound of a valid tree
                sp = sp < kMaxStack ? sp + 1 : sp;
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
    write_result<kTri>(a, q, p, best_leaf, best_id, best);
    if (a.counters) add_counters(a, n_exp, n_lbox, n_lex, 1);
}

// kMinWaves: the fewest waves per SIMD the register allocation must allow (4:
// at most 128 VGPRs, what the triangle kernel needs without spills; 5 trades a
// few spills outside the round loop for a fifth resident wave, which pays only
// when the launch has more waves than four per SIMD hold).
template <bool kTri, int M, int kMinWaves>
__global__ __launch_bounds__(64 * kBatchWaves) __attribute__((amdgpu_waves_per_eu(kMinWaves))) void traverse_batch_kernel(QueryArgs a) {
    __shared__ BatchLds<M> lds;
    check_vertex_count(a);
    const int64_t per_block = static_cast<int64_t>(kBatchWaves) * M;
    batch_loop<kTri, M>(a, static_cast<int64_t>(blockIdx.x) * per_block, static_cast<int64_t>(gridDim.x) * per_block,
                        a.nq, lds);
}

// ----------------------------------------------------------------- k nearest
// One query per lane, depth-first like the lane kernel, keeping the K best
// (d^2, original id, leaf) in registers sorted by (d^2, id); a child is pruned
// against the k-th best (k <= K at run time).  At the end the k closest points
// are combined with inverse-distance weights 1 / (d + eps) (the weighted
// nearest-neighbour NearestSurface of Sec. 3.3); a face at distance 0 gives its
// own point.
template <int K>
__global__ __launch_bounds__(kLaneBlock) void knn_lane_kernel(QueryArgs a, int k, float eps, int32_t *face_k,
                                                              float *dist2_k) {
    unsigned long long n_exp = 0, n_lbox = 0, n_lex = 0;
    __shared__ int32_t s_stack[kLdsStack][kLaneBlock];
    int32_t deep[kMaxStack - kLdsStack];
    const int lane = threadIdx.x;
    check_vertex_count(a);
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kLaneBlock + lane;
    if (q >= a.nq) return;
    const f3 p = load3(a.queries, a.nq, q);
    const float dq = slab_query_margin(p);
    float bd[K];
    int32_t bid[K], bleaf[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        bd[j] = a.maxd2;
        bid[j] = INT_MAX;
        bleaf[j] = -1;
    }
    // the k-th best (registers are not indexed at run time)
    auto kth = [&]() {
        float b = bd[0];
#pragma unroll
        for (int j = 1; j < K; ++j)
            if (j == k - 1) b = bd[j];
        return b;
    };
    auto consider = [&](float d2, int32_t id, int32_t leaf) {
        ++n_lex;
        const bool in = d2 < bd[K - 1] || (d2 == bd[K - 1] && id < bid[K - 1]);
        if (!in) return;
        bd[K - 1] = d2;
        bid[K - 1] = id;
        bleaf[K - 1] = leaf;
#pragma unroll
        for (int j = K - 1; j > 0; --j) {
            const bool up = bd[j] < bd[j - 1] || (bd[j] == bd[j - 1] && bid[j] < bid[j - 1]);
            if (up) {
                const float td = bd[j]; bd[j] = bd[j - 1]; bd[j - 1] = td;
                const int32_t ti = bid[j]; bid[j] = bid[j - 1]; bid[j - 1] = ti;
                const int32_t tl = bleaf[j]; bleaf[j] = bleaf[j - 1]; bleaf[j - 1] = tl;
            }
        }
    };

    if (a.n == 1) {
        consider(single_leaf_dist2<true>(a, p), a.prim[0], 0);
    } else if (a.n > 1) {
        const f3 rlo = f3{a.root[0], a.root[1], a.root[2]};
        const f3 rhi = f3{a.root[4], a.root[5], a.root[6]};
        int sp = 0;
        const float qm = qnorm1(p);
        int32_t node = box_dist2(p, rlo, rhi) <= prune_bound(kth(), qm) ? 0 : -1;
        for (int64_t step = 0; node >= 0 && node < a.n - 1 && step < a.n + 64; ++step) {
            const float4 *rec = a.nodes + 6 * static_cast<int64_t>(node);
            const float4 l0 = rec[0], l1 = rec[1], l2 = rec[2], r0 = rec[3], r1 = rec[4], r2 = rec[5];
            const int32_t lref = __float_as_int(l0.w), rref = __float_as_int(r0.w);
            if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) break;
            ++n_exp;
            n_lbox += (lref < 0) + (rref < 0);
            if (lref < 0 && leaf_box_dist2<true>(p, l0, l1, l2) <= prune_bound(kth(), qm))
                consider(leaf_dist2<true>(p, l0, l1, l2), __float_as_int(l1.w), ~lref);
            if (rref < 0 && leaf_box_dist2<true>(p, r0, r1, r2) <= prune_bound(kth(), qm))
                consider(leaf_dist2<true>(p, r0, r1, r2), __float_as_int(r1.w), ~rref);
            const float bound = prune_bound(kth(), qm);
            const float dl = lref >= 0 ? child_bound<true>(p, dq, l0, l1, l2) : INFINITY;
            const float dr = rref >= 0 ? child_bound<true>(p, dq, r0, r1, r2) : INFINITY;
            const bool gl = lref >= 0 && dl <= bound, gr = rref >= 0 && dr <= bound;
            if (gl && gr) {
                const bool left_first = dl <= dr;
                const int32_t far = left_first ? rref : lref;
                node = left_first ? lref : rref;
                if (sp < kLdsStack) s_stack[sp][lane] = far;
                else if (sp < kMaxStack) deep[sp - kLdsStack] = far;
                else atomicOr(a.status, 64);   // past the depth bound of a valid tree
                sp = sp < kMaxStack ? sp + 1 : sp;
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
    f3 num = f3{0.0f, 0.0f, 0.0f};
    float den = 0.0f;
    bool hit = false;                       // a face at distance 0: its point, unweighted
    f3 on = p;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= k) break;
        const int32_t leaf = bleaf[j];
        const bool ok = leaf >= 0 && leaf < a.n;
        face_k[j * a.nq + q] = ok ? bid[j] : -1;
        if (dist2_k) dist2_k[j * a.nq + q] = ok ? bd[j] : INFINITY;
        if (!ok) continue;
        const f3 A = vload(a.verts, a.nv, a.leaf_faces[leaf]);
        const f3 B = vload(a.verts, a.nv, a.leaf_faces[a.n + leaf]);
        const f3 C = vload(a.verts, a.nv, a.leaf_faces[2 * a.n + leaf]);
        float w1, w2;
        const float d2 = tri_closest(p, A, B, C, w1, w2);
        const f3 c = tri_point(A, B, C, w1, w2);
        if ((d2 == 0.0f || k == 1) && !hit) {   // k = 1: the closest point itself, unweighted
            hit = true;
            on = c;
        }
        const float w = 1.0f / (sqrtf(d2) + eps);
        num = num + w * c;
        den += w;
    }
    if (a.point) store3(a.point, a.nq, q, hit ? on : (den > 0.0f ? (1.0f / den) * num : p));
    if (a.counters) add_counters(a, n_exp, n_lbox, n_lex, 1);
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
        face[q] = static_cast<int32_t>(bf);
        if (point) store3(point, nq, q, tri_point(A, B, C, w1, w2));
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

// Default traversal when the caller gives no options: the batch kernel with a
// greedy seed descent and the largest batch (16, 8, 4, 2 or 1 queries per wave)
// that leaves at least 512 workgroups of four waves (the autotuner's choice on
// the workloads measured; it refines per workload).
inline void resolve(const mg_query_options *o, int64_t nq, int &kernel, int &batch, int &seed) {
    kernel = o ? o->kernel : MG_QUERY_AUTO;
    batch = o ? o->batch : 0;
    seed = o ? (o->seed != 0) : 1;
    if (kernel == MG_QUERY_AUTO) kernel = MG_QUERY_BATCH;
    if (batch <= 0) {
        // the largest batch that still gives at least 512 workgroups (two per CU)
        batch = 16;
        while (batch > 1 && nq < static_cast<int64_t>(2048) * batch) batch >>= 1;
    }
}

__global__ void zero_word_kernel(uint32_t *w) { *w = 0u; }

// Without a queue: one workgroup per kBatchWaves batches (at most 4096
// workgroups, striding beyond).  With a queue: as many workgroups as can be
// resident at once, each wave taking batches until none is left.
template <bool kTri, int M, int kMinWaves>
mg_status launch_batch_variant(const QueryArgs &a, hipStream_t s) {
    const int64_t per_block = static_cast<int64_t>(M) * kBatchWaves;
    int64_t grid = std::min<int64_t>((a.nq + per_block - 1) / per_block, 256 * 16);
    if (a.queue) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, traverse_batch_kernel<kTri, M, kMinWaves>,
                                                         64 * kBatchWaves, 0) != hipSuccess)
            return MG_ERR_HIP;
        grid = std::max<int64_t>(1, std::min<int64_t>(grid, static_cast<int64_t>(cus) * std::max(per_cu, 1)));
        hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(1), 0, s, a.queue);
    }
    hipLaunchKernelGGL((traverse_batch_kernel<kTri, M, kMinWaves>), dim3(static_cast<unsigned>(grid)),
                       dim3(64 * kBatchWaves), 0, s, a);
    return launch_status();
}

// Compute units of the current device, read once per device (a partitioned
// device has fewer than the full chip's 256).
int device_cus() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev].store(v, std::memory_order_relaxed);
    return v;
}

// The triangle kernel takes the five-wave allocation when its batches outnumber
// four waves on every SIMD (CUs x 4 SIMDs x 4 waves; 4,096 on a whole MI355X):
// 1M queries in batches of 16 ran 7% faster, while launches that fit in four
// waves per SIMD ran up to 2% slower with it.
// waves: 0 by that rule, 4 or 5 forced (the batched launch's tuner times the
// plain traversal with the four-wave allocation its own kernel has).
template <bool kTri, int M>
mg_status launch_batch(const QueryArgs &a, int waves, hipStream_t s) {
    if constexpr (kTri) {
        const int64_t four_wave_slots = static_cast<int64_t>(device_cus()) * 4 * 4;
        if (waves == 5 || (waves == 0 && (a.nq + M - 1) / M > four_wave_slots))
            return launch_batch_variant<kTri, M, 5>(a, s);
    }
    return launch_batch_variant<kTri, M, 4>(a, s);
}

template <bool kTri>
mg_status launch_traverse(QueryArgs a, const mg_query_options *opts, hipStream_t s) {
    int kernel, batch;
    resolve(opts, a.nq, kernel, batch, a.seed);
    const int waves = opts ? opts->waves : 0;
    a.order = opts ? opts->order : nullptr;
    a.counters = opts ? reinterpret_cast<unsigned long long *>(opts->counters) : nullptr;
    a.queue = opts ? opts->queue : nullptr;
    a.hint = opts ? opts->hint : nullptr;
    if (kernel == MG_QUERY_LANE) {
        hipLaunchKernelGGL(traverse_lane_kernel<kTri>, dim3(blocks_for(a.nq, kLaneBlock)), dim3(kLaneBlock), 0, s, a);
        return launch_status();
    }
    switch (batch) {
        case 1: return launch_batch<kTri, 1>(a, waves, s);
        case 2: return launch_batch<kTri, 2>(a, waves, s);
        case 4: return launch_batch<kTri, 4>(a, waves, s);
        case 8: return launch_batch<kTri, 8>(a, waves, s);
        case 16: return launch_batch<kTri, 16>(a, waves, s);
        case 32: return launch_batch<kTri, 32>(a, waves, s);
        default: return MG_ERR_INVALID_ARGUMENT;
    }
}

inline bool bad_options(const mg_query_options *o) {
    if (!o) return false;
    if (o->kernel < MG_QUERY_AUTO || o->kernel > MG_QUERY_BATCH) return true;
    if (o->waves != 0 && o->waves != 4 && o->waves != 5) return true;
    return !(o->batch == 0 || o->batch == 1 || o->batch == 2 || o->batch == 4 || o->batch == 8 || o->batch == 16 ||
             o->batch == 32);
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_closest_point_query(const void *bvh, size_t bvh_bytes, int32_t n_prims,
                                            const float *verts, int32_t n_verts, const float *queries,
                                            int32_t n_queries, float max_dist2, int32_t *face,
                                            float *point, float *bary, float *dist2, float *normal,
                                            const mg_query_options *opts, void *stream) {
    if (bad_count(n_prims) || bad_count(n_verts) || bad_count(n_queries) || !bvh || !(max_dist2 >= 0.0f) ||
        bad_options(opts))
        return MG_ERR_INVALID_ARGUMENT;
    mg_lbvh_layout L;
    mg_lbvh_layout_query(n_prims, MG_PRIM_TRIANGLES, &L);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (n_queries == 0) return MG_OK;
    if (!queries || !face || (n_prims > 0 && (!verts || n_verts == 0))) return MG_ERR_INVALID_ARGUMENT;
    QueryArgs a{};
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.root = cat<mg_lbvh_header>(bvh, L.off_header)->root_lo;
    a.leaf_faces = cat<int32_t>(bvh, L.off_leaf_faces);
    a.prim = cat<int32_t>(bvh, L.off_prim);
    a.inv_prim = cat<int32_t>(bvh, L.off_inv_prim);
    a.status = &const_cast<mg_lbvh_header *>(cat<mg_lbvh_header>(bvh, L.off_header))->status;
    a.hdr_nv = &cat<mg_lbvh_header>(bvh, L.off_header)->n_verts;
    a.verts = verts; a.nv = n_verts; a.n = n_prims;
    a.queries = queries; a.nq = n_queries; a.maxd2 = max_dist2;
    a.face = face; a.point = point; a.bary = bary; a.dist2 = dist2; a.normal = normal;
    return launch_traverse<true>(a, opts, as_stream(stream));
}

extern "C" mg_status mg_nearest_point_query(const void *bvh, size_t bvh_bytes, int32_t n_prims,
                                            const float *points, const float *queries, int32_t n_queries,
                                            float max_dist2, int32_t *index, float *dist2,
                                            const mg_query_options *opts, void *stream) {
    if (bad_count(n_prims) || bad_count(n_queries) || !bvh || !(max_dist2 >= 0.0f) || bad_options(opts))
        return MG_ERR_INVALID_ARGUMENT;
    mg_lbvh_layout L;
    mg_lbvh_layout_query(n_prims, MG_PRIM_POINTS, &L);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (n_queries == 0) return MG_OK;
    if (!queries || !index || (n_prims > 0 && !points)) return MG_ERR_INVALID_ARGUMENT;
    QueryArgs a{};
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.root = cat<mg_lbvh_header>(bvh, L.off_header)->root_lo;
    a.leaf_faces = nullptr;
    a.prim = cat<int32_t>(bvh, L.off_prim);
    a.inv_prim = cat<int32_t>(bvh, L.off_inv_prim);
    a.status = &const_cast<mg_lbvh_header *>(cat<mg_lbvh_header>(bvh, L.off_header))->status;
    a.hdr_nv = &cat<mg_lbvh_header>(bvh, L.off_header)->n_verts;
    a.verts = points; a.nv = n_prims; a.n = n_prims;
    a.queries = queries; a.nq = n_queries; a.maxd2 = max_dist2;
    a.face = index; a.point = nullptr; a.bary = nullptr; a.dist2 = dist2; a.normal = nullptr;
    return launch_traverse<false>(a, opts, as_stream(stream));
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

extern "C" mg_status mg_knn_surface_query(const void *bvh, size_t bvh_bytes, int32_t n_prims, const float *verts,
                                          int32_t n_verts, const float *queries, int32_t n_queries, int32_t k,
                                          float eps, float max_dist2, int32_t *face_k, float *dist2_k,
                                          float *point, uint64_t *counters, void *stream) {
    if (bad_count(n_prims) || bad_count(n_verts) || bad_count(n_queries) || !bvh || k < 1 || k > 8 ||
        !(eps >= 0.0f) || !(max_dist2 >= 0.0f))
        return MG_ERR_INVALID_ARGUMENT;
    mg_lbvh_layout L;
    mg_lbvh_layout_query(n_prims, MG_PRIM_TRIANGLES, &L);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (n_queries == 0) return MG_OK;
    if (!queries || !face_k || (n_prims > 0 && (!verts || n_verts == 0))) return MG_ERR_INVALID_ARGUMENT;
    QueryArgs a{};
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.root = cat<mg_lbvh_header>(bvh, L.off_header)->root_lo;
    a.leaf_faces = cat<int32_t>(bvh, L.off_leaf_faces);
    a.prim = cat<int32_t>(bvh, L.off_prim);
    a.inv_prim = cat<int32_t>(bvh, L.off_inv_prim);
    a.status = &const_cast<mg_lbvh_header *>(cat<mg_lbvh_header>(bvh, L.off_header))->status;
    a.hdr_nv = &cat<mg_lbvh_header>(bvh, L.off_header)->n_verts;
    a.verts = verts; a.nv = n_verts; a.n = n_prims;
    a.queries = queries; a.nq = n_queries; a.maxd2 = max_dist2;
    a.point = point;
    a.counters = reinterpret_cast<unsigned long long *>(counters);
    const dim3 g(static_cast<unsigned>(blocks_for(n_queries, kLaneBlock))), b(kLaneBlock);
    hipStream_t s = as_stream(stream);
    if (k <= 1) hipLaunchKernelGGL(knn_lane_kernel<1>, g, b, 0, s, a, k, eps, face_k, dist2_k);
    else if (k <= 2) hipLaunchKernelGGL(knn_lane_kernel<2>, g, b, 0, s, a, k, eps, face_k, dist2_k);
    else if (k <= 4) hipLaunchKernelGGL(knn_lane_kernel<4>, g, b, 0, s, a, k, eps, face_k, dist2_k);
    else hipLaunchKernelGGL(knn_lane_kernel<8>, g, b, 0, s, a, k, eps, face_k, dist2_k);
    return launch_status();
}
