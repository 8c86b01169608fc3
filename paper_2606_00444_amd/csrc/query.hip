// Closest point on a triangle mesh / nearest point of a point set through the
// LBVH, and an all-faces brute force for self-checks (gfx950).
//
// NearestSurface of the paper (Sec. 3.3, Eq. 1-2) projects a point onto a mesh
// with barycentric interpolation; it is read as the single nearest face.  The
// face normal is computed on demand from the three vertices of the winning
// face (Sec. 3.4 step 3), never stored.
//
// Pruning: a child is expanded when its box distance is <= best * (1 + 2^-20);
// the slack keeps a float32 rounding of a box distance from pruning a face whose
// float32 distance ties the best (ties go to the lowest original id, carried in
// the node record beside each leaf child).  Leaf children hold their triangle,
// so a leaf is tested with the data of the record that referenced it.
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
#include "mgu_internal.hpp"

#include <climits>

namespace mgu {
namespace {

constexpr int kLaneBlock = 64;
constexpr int kLdsStack = 32;
constexpr int kMaxStack = 64;
constexpr float kPruneSlack = 1.0f + 1.0f / 1048576.0f;

constexpr int kBatchWaves = 2;          // waves per workgroup of the batch kernel
constexpr int kBatchCap = 512;          // stack entries before the pop width shrinks
constexpr int kBatchAlloc = kBatchCap + 64;

struct QueryArgs {
    const float4 *nodes;                // [n-1][6]
    const mg_lbvh_header *hdr;
    const int32_t *leaf_faces;          // [3][n] (triangles) or nullptr (points)
    const int32_t *prim;                // [n]
    const float *verts;                 // mesh vertices or the points
    int64_t nv, n;
    const float *queries;
    int64_t nq;
    float maxd2;
    int32_t *face;
    float *point, *bary, *dist2, *normal;
    int seed;                           // batch kernel: greedy descent first
    const int32_t *order;               // processing order (permutation) or nullptr
    unsigned long long *counters;       // [4] statistics or nullptr
};

// Query processed in position i (order[i], or i); -1 if the order entry is out of range.
__device__ __forceinline__ int64_t query_at(const QueryArgs &a, int64_t i) {
    if (!a.order) return i;
    const int32_t q = a.order[i];
    return (q >= 0 && q < a.nq) ? q : -1;
}

__device__ __forceinline__ void add_counters(const QueryArgs &a, unsigned long long e, unsigned long long lb,
                                             unsigned long long lx, unsigned long long nq) {
    atomicAdd(a.counters + 0, e);
    atomicAdd(a.counters + 1, lb);
    atomicAdd(a.counters + 2, lx);
    atomicAdd(a.counters + 3, nq);
}

__device__ __forceinline__ f3 xyz(float4 v) { return f3{v.x, v.y, v.z}; }

// Exact squared distance to the leaf child stored in a record slot.
template <bool kTri>
__device__ __forceinline__ float leaf_dist2(f3 p, float4 f0, float4 f1, float4 f2) {
    if (kTri) {
        float w1, w2;
        return tri_closest(p, xyz(f0), xyz(f1), xyz(f2), w1, w2);
    }
    const f3 d = p - xyz(f0);
    return dot(d, d);
}

// Box distance of a leaf child (its triangle's bounds, or the point itself).
template <bool kTri>
__device__ __forceinline__ float leaf_box_dist2(f3 p, float4 f0, float4 f1, float4 f2) {
    if (kTri) {
        const f3 lo = fmin3(fmin3(xyz(f0), xyz(f1)), xyz(f2));
        const f3 hi = fmax3(fmax3(xyz(f0), xyz(f1)), xyz(f2));
        return box_dist2(p, lo, hi);
    }
    const f3 d = p - xyz(f0);
    return dot(d, d);
}

__device__ __forceinline__ unsigned long long pack_best(float d2, int32_t id) {
    return (static_cast<unsigned long long>(__float_as_uint(d2)) << 32) | static_cast<uint32_t>(id);
}

// Final record of query q: recomputed from the winning leaf's face (triangles)
// or point, which the BVH stores bit-identically.
template <bool kTri>
__device__ void write_result(const QueryArgs &a, int64_t q, f3 p, int32_t leaf, int32_t id, float d2) {
    if (kTri) {
        if (leaf >= 0) {
            const f3 A = load3(a.verts, a.nv, a.leaf_faces[leaf]);
            const f3 B = load3(a.verts, a.nv, a.leaf_faces[a.n + leaf]);
            const f3 C = load3(a.verts, a.nv, a.leaf_faces[2 * a.n + leaf]);
            float w1, w2;
            const float dd = tri_closest(p, A, B, C, w1, w2);
            const float w0 = 1.0f - w1 - w2;
            a.face[q] = id;
            if (a.point)
                store3(a.point, a.nq, q, f3{w0 * A.x + w1 * B.x + w2 * C.x, w0 * A.y + w1 * B.y + w2 * C.y,
                                            w0 * A.z + w1 * B.z + w2 * C.z});
            if (a.bary) { a.bary[q] = w1; a.bary[a.nq + q] = w2; }
            if (a.dist2) a.dist2[q] = dd;
            if (a.normal) store3(a.normal, a.nq, q, tri_normal(A, B, C));
        } else {
            a.face[q] = -1;
            if (a.point) store3(a.point, a.nq, q, p);
            if (a.bary) { a.bary[q] = 0.0f; a.bary[a.nq + q] = 0.0f; }
            if (a.dist2) a.dist2[q] = INFINITY;
            if (a.normal) store3(a.normal, a.nq, q, f3{0.0f, 0.0f, 0.0f});
        }
    } else {
        a.face[q] = leaf >= 0 ? id : -1;
        if (a.dist2) a.dist2[q] = leaf >= 0 ? d2 : INFINITY;
    }
}

// Test of the single leaf of a one-primitive BVH (no records exist).
template <bool kTri>
__device__ __forceinline__ float single_leaf_dist2(const QueryArgs &a, f3 p) {
    if (kTri) {
        float w1, w2;
        return tri_closest(p, load3(a.verts, a.nv, a.leaf_faces[0]), load3(a.verts, a.nv, a.leaf_faces[a.n]),
                           load3(a.verts, a.nv, a.leaf_faces[2 * a.n]), w1, w2);
    }
    const f3 d = p - load3(a.verts, a.nv, a.prim[0]);
    return dot(d, d);
}

// ---------------------------------------------------------------- lane kernel
template <bool kTri>
__global__ __launch_bounds__(kLaneBlock) void traverse_lane_kernel(QueryArgs a) {
    __shared__ int32_t s_stack[kLdsStack][kLaneBlock];
    int32_t deep[kMaxStack - kLdsStack];
    const int lane = threadIdx.x;
    const int64_t pos = static_cast<int64_t>(blockIdx.x) * kLaneBlock + lane;
    if (pos >= a.nq) return;
    const int64_t q = query_at(a, pos);
    if (q < 0) return;
    const f3 p = load3(a.queries, a.nq, q);
    float best = a.maxd2;
    int32_t best_id = INT_MAX, best_leaf = -1;
    unsigned long long n_exp = 0, n_lbox = 0, n_lex = 0;

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
        const f3 rlo = f3{a.hdr->root_lo[0], a.hdr->root_lo[1], a.hdr->root_lo[2]};
        const f3 rhi = f3{a.hdr->root_hi[0], a.hdr->root_hi[1], a.hdr->root_hi[2]};
        int sp = 0;
        int32_t node = box_dist2(p, rlo, rhi) <= best * kPruneSlack ? 0 : -1;
        // each internal node is visited at most once in a valid tree: the step cap
        // and the reference checks keep a corrupted buffer from looping or faulting
        for (int64_t step = 0; node >= 0 && node < a.n - 1 && step < a.n + 64; ++step) {
            const float4 *rec = a.nodes + 6 * static_cast<int64_t>(node);
            const float4 l0 = rec[0], l1 = rec[1], l2 = rec[2], r0 = rec[3], r1 = rec[4], r2 = rec[5];
            const int32_t lref = __float_as_int(l0.w), rref = __float_as_int(r0.w);
            if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) break;
            ++n_exp;
            n_lbox += (lref < 0) + (rref < 0);
            if (lref < 0 && leaf_box_dist2<kTri>(p, l0, l1, l2) <= best * kPruneSlack)
                consider(leaf_dist2<kTri>(p, l0, l1, l2), __float_as_int(l1.w), ~lref);
            if (rref < 0 && leaf_box_dist2<kTri>(p, r0, r1, r2) <= best * kPruneSlack)
                consider(leaf_dist2<kTri>(p, r0, r1, r2), __float_as_int(r1.w), ~rref);
            const float bound = best * kPruneSlack;
            const float dl = lref >= 0 ? box_dist2(p, xyz(l0), xyz(l1)) : INFINITY;
            const float dr = rref >= 0 ? box_dist2(p, xyz(r0), xyz(r1)) : INFINITY;
            const bool gl = lref >= 0 && dl <= bound, gr = rref >= 0 && dr <= bound;
            if (gl && gr) {
                const bool left_first = dl <= dr;
                const int32_t far = left_first ? rref : lref;
                node = left_first ? lref : rref;
                if (sp < kLdsStack) s_stack[sp][lane] = far;
                else if (sp < kMaxStack) deep[sp - kLdsStack] = far;
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

// --------------------------------------------------------------- batch kernel
template <bool kTri, int M>
__global__ __launch_bounds__(64 * kBatchWaves) void traverse_batch_kernel(QueryArgs a) {
    __shared__ int32_t s_node[kBatchWaves][kBatchAlloc];
    __shared__ float s_dist[kBatchWaves][kBatchAlloc];
    __shared__ uint8_t s_slot[kBatchWaves][kBatchAlloc];
    __shared__ unsigned long long s_best[kBatchWaves][M];
    __shared__ int32_t s_leaf[kBatchWaves][M];
    __shared__ float s_q[kBatchWaves][3][M];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const uint64_t lt = lanemask_lt();
    const int64_t waves_total = static_cast<int64_t>(gridDim.x) * kBatchWaves;
    const unsigned long long none = pack_best(a.maxd2, INT_MAX);
    unsigned long long n_exp = 0, n_lbox = 0, n_lex = 0, n_q = 0;   // statistics (wave-uniform)

    for (int64_t qb = (static_cast<int64_t>(blockIdx.x) * kBatchWaves + w) * M; qb < a.nq; qb += waves_total * M) {
        const int nb = static_cast<int>(a.nq - qb < M ? a.nq - qb : M);
        const int64_t qid = lane < nb ? query_at(a, qb + lane) : -1;
        const bool own = qid >= 0;
        f3 p = f3{0.0f, 0.0f, 0.0f};
        if (own) {
            p = load3(a.queries, a.nq, qid);
            s_q[w][0][lane] = p.x; s_q[w][1][lane] = p.y; s_q[w][2][lane] = p.z;
            s_best[w][lane] = none;
            s_leaf[w][lane] = -1;
        }
        int sp = 0;
        if (a.n == 1) {
            if (own) {
                const unsigned long long c = pack_best(single_leaf_dist2<kTri>(a, p), a.prim[0]);
                if (c < none) { s_best[w][lane] = c; s_leaf[w][lane] = 0; }
            }
        } else if (a.n > 1) {
            unsigned long long seeded = none;
            if (a.seed && own) {
                // one greedy root-to-leaf walk (nearer internal child first) gives an
                // upper bound before the wide expansion starts
                int32_t cleaf = -1, node = 0;
                for (int lvl = 0; lvl < 64 && node >= 0 && node < a.n - 1; ++lvl) {
                    const float4 *rec = a.nodes + 6 * static_cast<int64_t>(node);
                    const float4 l0 = rec[0], l1 = rec[1], l2 = rec[2], r0 = rec[3], r1 = rec[4], r2 = rec[5];
                    const int32_t lref = __float_as_int(l0.w), rref = __float_as_int(r0.w);
                    if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) break;
                    if (a.counters) {   // per-lane path: count directly
                        const unsigned long long nl = (lref < 0) + (rref < 0);
                        add_counters(a, 1, nl, nl, 0);
                    }
                    if (lref < 0) {
                        const unsigned long long c = pack_best(leaf_dist2<kTri>(p, l0, l1, l2), __float_as_int(l1.w));
                        if (c < seeded) { seeded = c; cleaf = ~lref; }
                    }
                    if (rref < 0) {
                        const unsigned long long c = pack_best(leaf_dist2<kTri>(p, r0, r1, r2), __float_as_int(r1.w));
                        if (c < seeded) { seeded = c; cleaf = ~rref; }
                    }
                    const float dl = lref >= 0 ? box_dist2(p, xyz(l0), xyz(l1)) : INFINITY;
                    const float dr = rref >= 0 ? box_dist2(p, xyz(r0), xyz(r1)) : INFINITY;
                    node = (lref >= 0 && dl <= dr) ? lref : (rref >= 0 ? rref : -1);
                }
                if (seeded < none) { s_best[w][lane] = seeded; s_leaf[w][lane] = cleaf; }
            }
            const f3 rlo = f3{a.hdr->root_lo[0], a.hdr->root_lo[1], a.hdr->root_lo[2]};
            const f3 rhi = f3{a.hdr->root_hi[0], a.hdr->root_hi[1], a.hdr->root_hi[2]};
            const float rd = own ? box_dist2(p, rlo, rhi) : INFINITY;
            const float rb = (seeded < none ? __uint_as_float(static_cast<uint32_t>(seeded >> 32)) : a.maxd2);
            const bool push = own && rd <= rb * kPruneSlack;
            const uint64_t bm = __ballot(push);
            if (push) {
                const int pos = __popcll(bm & lt);
                s_node[w][pos] = 0;
                s_dist[w][pos] = rd;
                s_slot[w][pos] = static_cast<uint8_t>(lane);
            }
            sp = __popcll(bm);
        }
        // the stack never exceeds kBatchCap + 62: a round of width k pushes at most
        // 2k entries, widths are cut to (kBatchCap - sp) / 2, and width-1 rounds are
        // a plain depth-first walk whose growth is bounded by the tree depth
        // each query expands each internal node at most once: the round cap only
        // stops a corrupted buffer from looping
        for (int64_t round = 0; sp > 0 && round < static_cast<int64_t>(M + 1) * a.n + 64; ++round) {
            int take = sp < 64 ? sp : 64;
            const int room = (kBatchCap - sp) / 2;
            if (take > room) take = room > 1 ? room : 1;
            const bool pop = lane < take;
            const int idx = sp - 1 - lane;
            int32_t node = 0, slot = 0;
            float nd = INFINITY;
            if (pop) {
                node = s_node[w][idx];
                nd = s_dist[w][idx];
                slot = s_slot[w][idx];
            }
            sp -= take;
            bool act = pop && node >= 0 && node < a.n - 1;
            unsigned long long best = act ? s_best[w][slot] : 0ull;
            act = act && nd <= __uint_as_float(static_cast<uint32_t>(best >> 32)) * kPruneSlack;
            float4 l0, l1, l2, r0, r1, r2;
            int32_t lref = 0, rref = 0;
            f3 qp = f3{0.0f, 0.0f, 0.0f};
            unsigned long long cand = ~0ull;
            int32_t cand_leaf = -1;
            if (act) {
                qp = f3{s_q[w][0][slot], s_q[w][1][slot], s_q[w][2][slot]};
                const float4 *rec = a.nodes + 6 * static_cast<int64_t>(node);
                l0 = rec[0]; l1 = rec[1]; l2 = rec[2]; r0 = rec[3]; r1 = rec[4]; r2 = rec[5];
                lref = __float_as_int(l0.w);
                rref = __float_as_int(r0.w);
                if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) act = false;
            }
            const float pbound = __uint_as_float(static_cast<uint32_t>(best >> 32)) * kPruneSlack;
            const bool tl = act && lref < 0 && leaf_box_dist2<kTri>(qp, l0, l1, l2) <= pbound;
            const bool tr = act && rref < 0 && leaf_box_dist2<kTri>(qp, r0, r1, r2) <= pbound;
            if (a.counters) {
                n_exp += __popcll(__ballot(act));
                n_lbox += __popcll(__ballot(act && lref < 0)) + __popcll(__ballot(act && rref < 0));
                n_lex += __popcll(__ballot(tl)) + __popcll(__ballot(tr));
            }
            if (tl) {
                cand = pack_best(leaf_dist2<kTri>(qp, l0, l1, l2), __float_as_int(l1.w));
                cand_leaf = ~lref;
            }
            if (tr) {
                const unsigned long long c = pack_best(leaf_dist2<kTri>(qp, r0, r1, r2), __float_as_int(r1.w));
                if (c < cand) { cand = c; cand_leaf = ~rref; }
            }
            if (cand != ~0ull) atomicMin(&s_best[w][slot], cand);
            // the lane holding the minimum records its leaf (ids are unique, so at
            // most one lane per query matches); a later round may overwrite it
            if (cand != ~0ull && s_best[w][slot] == cand) s_leaf[w][slot] = cand_leaf;
            best = act ? s_best[w][slot] : 0ull;
            const float bound = __uint_as_float(static_cast<uint32_t>(best >> 32)) * kPruneSlack;
            const float dl = (act && lref >= 0) ? box_dist2(qp, xyz(l0), xyz(l1)) : INFINITY;
            const float dr = (act && rref >= 0) ? box_dist2(qp, xyz(r0), xyz(r1)) : INFINITY;
            const bool pl = act && lref >= 0 && dl <= bound;
            const bool pr = act && rref >= 0 && dr <= bound;
            const uint64_t bl = __ballot(pl), br = __ballot(pr);
            const int off = sp + __popcll(bl & lt) + __popcll(br & lt);
            if (pl && pr) {
                const bool left_near = dl <= dr;   // nearer child on top of the stack
                s_node[w][off] = left_near ? rref : lref;
                s_dist[w][off] = left_near ? dr : dl;
                s_slot[w][off] = static_cast<uint8_t>(slot);
                s_node[w][off + 1] = left_near ? lref : rref;
                s_dist[w][off + 1] = left_near ? dl : dr;
                s_slot[w][off + 1] = static_cast<uint8_t>(slot);
            } else if (pl || pr) {
                s_node[w][off] = pl ? lref : rref;
                s_dist[w][off] = pl ? dl : dr;
                s_slot[w][off] = static_cast<uint8_t>(slot);
            }
            sp += __popcll(bl) + __popcll(br);
        }
        if (own) {
            const unsigned long long b = s_best[w][lane];
            const int32_t id = static_cast<int32_t>(b & 0xffffffffull);
            const int32_t leaf = id == INT_MAX ? -1 : s_leaf[w][lane];
            write_result<kTri>(a, qid, p, leaf, id, __uint_as_float(static_cast<uint32_t>(b >> 32)));
        }
        if (a.counters) n_q += __popcll(__ballot(own));
    }
    if (a.counters && lane == 0) add_counters(a, n_exp, n_lbox, n_lex, n_q);
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

// Default traversal when the caller gives no options: batches of 4 queries per
// wave with a greedy seed descent (the best or close to it on every workload
// measured; the autotuner refines per workload).
inline void resolve(const mg_query_options *o, int64_t nq, int &kernel, int &batch, int &seed) {
    kernel = o ? o->kernel : MG_QUERY_AUTO;
    batch = o ? o->batch : 0;
    seed = o ? (o->seed != 0) : 1;
    if (kernel == MG_QUERY_AUTO) kernel = MG_QUERY_BATCH;
    if (batch <= 0) batch = 4;
}

template <bool kTri>
mg_status launch_traverse(QueryArgs a, const mg_query_options *opts, hipStream_t s) {
    int kernel, batch;
    resolve(opts, a.nq, kernel, batch, a.seed);
    a.order = opts ? opts->order : nullptr;
    a.counters = opts ? reinterpret_cast<unsigned long long *>(opts->counters) : nullptr;
    if (kernel == MG_QUERY_LANE) {
        hipLaunchKernelGGL(traverse_lane_kernel<kTri>, dim3(blocks_for(a.nq, kLaneBlock)), dim3(kLaneBlock), 0, s, a);
        return launch_status();
    }
    const int64_t per_block = static_cast<int64_t>(batch) * kBatchWaves;
    const int grid = static_cast<int>(std::min<int64_t>((a.nq + per_block - 1) / per_block, 256 * 16));
    const dim3 g(grid), b(64 * kBatchWaves);
    switch (batch) {
        case 1: hipLaunchKernelGGL((traverse_batch_kernel<kTri, 1>), g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL((traverse_batch_kernel<kTri, 2>), g, b, 0, s, a); break;
        case 4: hipLaunchKernelGGL((traverse_batch_kernel<kTri, 4>), g, b, 0, s, a); break;
        case 8: hipLaunchKernelGGL((traverse_batch_kernel<kTri, 8>), g, b, 0, s, a); break;
        case 16: hipLaunchKernelGGL((traverse_batch_kernel<kTri, 16>), g, b, 0, s, a); break;
        case 32: hipLaunchKernelGGL((traverse_batch_kernel<kTri, 32>), g, b, 0, s, a); break;
        default: return MG_ERR_INVALID_ARGUMENT;
    }
    return launch_status();
}

inline bool bad_options(const mg_query_options *o) {
    if (!o) return false;
    if (o->kernel < MG_QUERY_AUTO || o->kernel > MG_QUERY_BATCH) return true;
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
    QueryArgs a;
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.hdr = cat<mg_lbvh_header>(bvh, L.off_header);
    a.leaf_faces = cat<int32_t>(bvh, L.off_leaf_faces);
    a.prim = cat<int32_t>(bvh, L.off_prim);
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
    QueryArgs a;
    a.nodes = cat<float4>(bvh, L.off_nodes);
    a.hdr = cat<mg_lbvh_header>(bvh, L.off_header);
    a.leaf_faces = nullptr;
    a.prim = cat<int32_t>(bvh, L.off_prim);
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
