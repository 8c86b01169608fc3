// Closest-point / nearest-point traversal pieces shared by the plain query
// kernels and the batched persistent kernel.
//
// Pruning: a child is expanded when its box distance is <= best * (1 + 2^-20);
// the slack keeps a float32 rounding of a box distance from pruning a face whose
// float32 distance ties the best (ties go to the lowest original id, carried in
// the node record beside each leaf child).  Leaf children hold their triangle,
// so a leaf is tested with the data of the record that referenced it.
#pragma once

#include "mgu_internal.hpp"

#include <climits>

namespace mgu {

constexpr int kLaneBlock = 64;
constexpr int kLdsStack = 32;
constexpr int kMaxStack = 64;
constexpr float kPruneSlack = 1.0f + 1.0f / 1048576.0f;

constexpr int kBatchWaves = 2;          // waves per workgroup of the batch kernel
constexpr int kBatchCap = 512;          // stack entries before the pop width shrinks
constexpr int kBatchAlloc = kBatchCap + 64;

struct QueryArgs {
    const float4 *nodes;                // [n-1][6]
    const float *root;                  // root box: lo at [0..2], hi at [4..6]
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
        if (leaf >= 0 && leaf < a.n) {
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

// --------------------------------------------------------------- batch kernel
// Per-wave LDS of the batch traversal.
template <int M>
struct WaveStack {
    int32_t node[kBatchAlloc];
    float dist[kBatchAlloc];
    uint8_t slot[kBatchAlloc];
    unsigned long long best[M];
    int32_t leaf[M];
    float q[3][M];
};

// One wave processes the query batches [qb, qb + M) for qb = start, start +
// stride, ... below q_end (positions in the processing order).
template <bool kTri, int M>
__device__ void batch_loop(const QueryArgs &a, int64_t start, int64_t stride, int64_t q_end, WaveStack<M> &S) {
    const int lane = threadIdx.x % 64;
    const uint64_t lt = lanemask_lt();
    const unsigned long long none = pack_best(a.maxd2, INT_MAX);
    unsigned long long n_exp = 0, n_lbox = 0, n_lex = 0, n_q = 0;   // statistics (wave-uniform)

    for (int64_t qb = start; qb < q_end; qb += stride) {
        const int nb = static_cast<int>(q_end - qb < M ? q_end - qb : M);
        const int64_t qid = lane < nb ? query_at(a, qb + lane) : -1;
        const bool own = qid >= 0;
        f3 p = f3{0.0f, 0.0f, 0.0f};
        if (own) {
            p = load3(a.queries, a.nq, qid);
            S.q[0][lane] = p.x; S.q[1][lane] = p.y; S.q[2][lane] = p.z;
            S.best[lane] = none;
            S.leaf[lane] = -1;
        }
        int sp = 0;
        if (a.n == 1) {
            if (own) {
                const unsigned long long c = pack_best(single_leaf_dist2<kTri>(a, p), a.prim[0]);
                if (c < none) { S.best[lane] = c; S.leaf[lane] = 0; }
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
                if (seeded < none) { S.best[lane] = seeded; S.leaf[lane] = cleaf; }
            }
            const f3 rlo = f3{a.root[0], a.root[1], a.root[2]};
            const f3 rhi = f3{a.root[4], a.root[5], a.root[6]};
            const float rd = own ? box_dist2(p, rlo, rhi) : INFINITY;
            const float rb = (seeded < none ? __uint_as_float(static_cast<uint32_t>(seeded >> 32)) : a.maxd2);
            const bool push = own && rd <= rb * kPruneSlack;
            const uint64_t bm = __ballot(push);
            if (push) {
                const int pos = __popcll(bm & lt);
                S.node[pos] = 0;
                S.dist[pos] = rd;
                S.slot[pos] = static_cast<uint8_t>(lane);
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
                node = S.node[idx];
                nd = S.dist[idx];
                slot = S.slot[idx];
                if (slot >= M) { node = -1; slot = 0; }
            }
            sp -= take;
            bool act = pop && node >= 0 && node < a.n - 1;
            unsigned long long best = act ? S.best[slot] : 0ull;
            act = act && nd <= __uint_as_float(static_cast<uint32_t>(best >> 32)) * kPruneSlack;
            float4 l0, l1, l2, r0, r1, r2;
            int32_t lref = 0, rref = 0;
            f3 qp = f3{0.0f, 0.0f, 0.0f};
            unsigned long long cand = ~0ull;
            int32_t cand_leaf = -1;
            if (act) {
                qp = f3{S.q[0][slot], S.q[1][slot], S.q[2][slot]};
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
            if (cand != ~0ull) atomicMin(&S.best[slot], cand);
            // the lane holding the minimum records its leaf (ids are unique, so at
            // most one lane per query matches); a later round may overwrite it
            if (cand != ~0ull && S.best[slot] == cand) S.leaf[slot] = cand_leaf;
            best = act ? S.best[slot] : 0ull;
            const float bound = __uint_as_float(static_cast<uint32_t>(best >> 32)) * kPruneSlack;
            const float dl = (act && lref >= 0) ? box_dist2(qp, xyz(l0), xyz(l1)) : INFINITY;
            const float dr = (act && rref >= 0) ? box_dist2(qp, xyz(r0), xyz(r1)) : INFINITY;
            const bool pl = act && lref >= 0 && dl <= bound;
            const bool pr = act && rref >= 0 && dr <= bound;
            const uint64_t bl = __ballot(pl), br = __ballot(pr);
            const int off = sp + __popcll(bl & lt) + __popcll(br & lt);
            // The bound above only holds for a valid tree; the clamp keeps a
            // corrupted buffer from writing past this wave's stack.
            if (pl && pr) {
                const bool left_near = dl <= dr;   // nearer child on top of the stack
                if (off < kBatchAlloc) {
                    S.node[off] = left_near ? rref : lref;
                    S.dist[off] = left_near ? dr : dl;
                    S.slot[off] = static_cast<uint8_t>(slot);
                }
                if (off + 1 < kBatchAlloc) {
                    S.node[off + 1] = left_near ? lref : rref;
                    S.dist[off + 1] = left_near ? dl : dr;
                    S.slot[off + 1] = static_cast<uint8_t>(slot);
                }
            } else if ((pl || pr) && off < kBatchAlloc) {
                S.node[off] = pl ? lref : rref;
                S.dist[off] = pl ? dl : dr;
                S.slot[off] = static_cast<uint8_t>(slot);
            }
            sp += __popcll(bl) + __popcll(br);
            sp = sp < kBatchAlloc ? sp : kBatchAlloc;
        }
        if (own) {
            const unsigned long long b = S.best[lane];
            const int32_t id = static_cast<int32_t>(b & 0xffffffffull);
            const int32_t leaf = id == INT_MAX ? -1 : S.leaf[lane];
            write_result<kTri>(a, qid, p, leaf, id, __uint_as_float(static_cast<uint32_t>(b >> 32)));
        }
        if (a.counters) n_q += __popcll(__ballot(own));
    }
    if (a.counters && lane == 0) add_counters(a, n_exp, n_lbox, n_lex, n_q);
}

}  // namespace mgu
