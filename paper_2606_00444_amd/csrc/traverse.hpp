// Closest-point / nearest-point traversal pieces shared by the plain query
// kernels and the batched persistent kernel.
//
// Pruning: a child is expanded when its lower bound is <= prune_bound(best):
// the slack keeps a face whose float32 distance ties the best from being
// pruned, whatever order the faces are met in, so every traversal returns the
// lowest original id among the faces at the minimal float32 distance (carried
// in the node record beside each leaf child).  Leaf children hold their
// triangle, so a leaf is tested with the data of the record that referenced it.
#pragma once

#include "mgu_internal.hpp"

#include <climits>

namespace mgu {

constexpr int kLaneBlock = 64;
constexpr int kLdsStack = 32;
constexpr int kMaxStack = 64;
constexpr float kPruneSlack = 1.0f + 1.0f / 1048576.0f;

// The largest lower bound of a node that may still hold a face whose float32
// squared distance ties `best`.  A float32 closest point on a well-shaped
// triangle is off by a few units in the last place of the coordinates'
// magnitude (about |q|_1 + sqrt(best) near q), so its float32 distance may
// fall short of the exact one by delta = 2^-18 (|q|_1 + sqrt(best)) - a wide
// margin - while the box and slab bounds are within a few rounding steps of
// exact: expanding every node with sqrt(bound) <= sqrt(best) + delta (times
// 1 + 2^-20 for the bound's own rounding) keeps such faces.  qm = |q|_1.
__device__ __forceinline__ float prune_bound(float best, float qm) {
    const float d = __builtin_amdgcn_sqrtf(best);
    const float e = fmaf(0x1p-18f, qm + d, d);
    return (e * e) * kPruneSlack;
}

// |q|_1 of a query point (the magnitude of the prune slack and the slab margin).
__device__ __forceinline__ float qnorm1(f3 q) { return (fabsf(q.x) + fabsf(q.y)) + fabsf(q.z); }

constexpr int kBatchWaves = 4;          // waves per workgroup of the batch kernel
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
    const int32_t *inv_prim;            // [n] leaf of each original id (id -> position in leaf order)
    int32_t *status;                    // error word of the BVH header
    const int32_t *hdr_nv;              // vertex count of the build (header), or nullptr
    uint32_t *queue;                    // batch kernel: dynamic batch counter (zeroed before launch) or nullptr
    const int32_t *hint;                // [nq] original id to start each query from, or nullptr
    int coherent;                       // face ids stored and hints loaded device-coherent (batched form)
};

// The face id of a result: with `coherent`, a relaxed device-scope store, which the
// other XCDs see without a write-back of the L2 (the batched form reads a scene's
// previous frame as hints while the launch runs).
__device__ __forceinline__ void store_face(const QueryArgs &a, int64_t q, int32_t id) {
    if (a.coherent) __hip_atomic_store(a.face + q, id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else a.face[q] = id;
}

// The first thread of a launch flags a vertex count that differs from the build's.
__device__ __forceinline__ void check_vertex_count(const QueryArgs &a) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.hdr_nv && *a.hdr_nv != a.nv) atomicOr(a.status, 32);
}

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
    return fdot(d, d);
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
    return fdot(d, d);
}

// Margin of a query's slab distances: 2^-20 of its coordinate magnitudes
// covers the float32 rounding of d.q.
__device__ __forceinline__ float slab_query_margin(f3 q) { return 0x1p-20f * qnorm1(q); }

// Lower bound of the squared distance from q to the faces below an internal
// child slot (c0, c1, c2) = (lo, ref) (hi, a) (d, b): the larger of the box
// distance and, for triangles, the normal-slab distance (dq: the query's
// slab margin; the factor 1 - 2^-19 allows for |d| differing from 1).
template <bool kTri>
__device__ __forceinline__ float child_bound(f3 q, float dq, float4 c0, float4 c1, float4 c2) {
    const float bd = box_dist2(q, xyz(c0), xyz(c1));
    if (!kTri) return bd;
    const float s = c2.x * q.x + c2.y * q.y + c2.z * q.z;
    const float g = fmaxf(c1.w - s, s - c2.w) - dq;
    return g > 0.0f ? fmaxf(bd, (g * g) * (1.0f - 0x1p-19f)) : bd;
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
            const f3 A = vload(a.verts, a.nv, a.leaf_faces[leaf]);
            const f3 B = vload(a.verts, a.nv, a.leaf_faces[a.n + leaf]);
            const f3 C = vload(a.verts, a.nv, a.leaf_faces[2 * a.n + leaf]);
            float w1, w2;
            const float dd = tri_closest(p, A, B, C, w1, w2);
            store_face(a, q, id);
            if (a.point) store3(a.point, a.nq, q, tri_point(A, B, C, w1, w2));
            if (a.bary) { a.bary[q] = w1; a.bary[a.nq + q] = w2; }
            if (a.dist2) a.dist2[q] = dd;
            if (a.normal) store3(a.normal, a.nq, q, tri_normal(A, B, C));
        } else {
            store_face(a, q, -1);
            if (a.point) store3(a.point, a.nq, q, p);
            if (a.bary) { a.bary[q] = 0.0f; a.bary[a.nq + q] = 0.0f; }
            if (a.dist2) a.dist2[q] = INFINITY;
            if (a.normal) store3(a.normal, a.nq, q, f3{0.0f, 0.0f, 0.0f});
        }
    } else {
        store_face(a, q, leaf >= 0 ? id : -1);
        if (a.dist2) a.dist2[q] = leaf >= 0 ? d2 : INFINITY;
    }
}

// Final record of query q from the winning original id (-1 / INT_MAX: none).
template <bool kTri>
__device__ void write_result_id(const QueryArgs &a, int64_t q, f3 p, int32_t id, float d2) {
    int32_t leaf = -1;
    if (id >= 0 && id < a.n) {
        leaf = a.inv_prim[id];
        if (leaf < 0 || leaf >= a.n) { atomicOr(a.status, 16); leaf = -1; }
    }
    write_result<kTri>(a, q, p, leaf, id, d2);
}

// Squared distance from p to primitive `id` (original numbering) through its
// leaf; +inf if id or its leaf is out of range.
template <bool kTri>
__device__ __forceinline__ float prim_dist2(const QueryArgs &a, f3 p, int32_t id) {
    if (id < 0 || id >= a.n) return INFINITY;
    const int32_t leaf = a.inv_prim[id];
    if (leaf < 0 || leaf >= a.n) return INFINITY;
    if (kTri) {
        float w1, w2;
        return tri_closest(p, vload(a.verts, a.nv, a.leaf_faces[leaf]), vload(a.verts, a.nv, a.leaf_faces[a.n + leaf]),
                           vload(a.verts, a.nv, a.leaf_faces[2 * a.n + leaf]), w1, w2);
    }
    const f3 d = p - vload(a.verts, a.nv, id);
    return fdot(d, d);
}

// The starting best of query q from its hint: (d^2 bits, id), or `none`.
template <bool kTri>
__device__ __forceinline__ unsigned long long hint_best(const QueryArgs &a, int64_t q, f3 p, unsigned long long none) {
    if (!a.hint) return none;
    const int32_t h = a.coherent ? __hip_atomic_load(a.hint + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : a.hint[q];
    const float d2 = prim_dist2<kTri>(a, p, h);
    const unsigned long long c = pack_best(d2, h);
    return d2 < INFINITY && c < none ? c : none;
}

// Test of the single leaf of a one-primitive BVH (no records exist).
template <bool kTri>
__device__ __forceinline__ float single_leaf_dist2(const QueryArgs &a, f3 p) {
    if (kTri) {
        float w1, w2;
        return tri_closest(p, vload(a.verts, a.nv, a.leaf_faces[0]), vload(a.verts, a.nv, a.leaf_faces[a.n]),
                           vload(a.verts, a.nv, a.leaf_faces[2 * a.n]), w1, w2);
    }
    const f3 d = p - vload(a.verts, a.nv, a.prim[0]);
    return fdot(d, d);
}

// --------------------------------------------------------------- batch kernel
// The waves of a workgroup each process batches of M queries with an LDS work
// stack shared by the batch's queries; each round pops up to 64 entries (one
// per lane).  A wave whose stack is deep puts its top 64 entries into the
// workgroup's one-chunk mailbox whenever it is empty, and a wave that has
// finished a batch empties the mailbox before it starts another, so a batch
// holding an expensive query (one nearly equidistant from many faces) is
// finished by several waves.  The per-query bests (d^2 bits, original id) stay
// with the owning wave and are lowered by LDS atomics from whichever wave tests
// a face; the owner writes its results once every chunk it gave away is done.

constexpr int kDonateMin = 128;          // a wave keeps at least 64 entries after giving 64
constexpr int kIdleSpinLimit = 1 << 22;  // bounded waits: error word instead of a hang

template <int M>
struct WaveStack {
    int32_t node[kBatchAlloc];
    float dist[kBatchAlloc];
    uint8_t slot[kBatchAlloc];
    unsigned long long best[M];         // per query of the batch: (d^2 bits, original id)
    float q[3][M];
};

struct WaveMail {
    int32_t node[64];
    float dist[64];
    uint8_t slot[64];
    int32_t count;                      // entries in the chunk
    int32_t owner;                      // wave whose batch the entries belong to
    int32_t state;                      // 0 empty, 1 full, 2 being taken, 3 being filled
    int32_t done;                       // waves that have finished all their batches
    int32_t outstanding[kBatchWaves];   // chunks of each wave's batch held elsewhere
};

template <int M>
struct BatchLds {
    WaveStack<M> st[kBatchWaves];
    WaveMail mail;
};

struct BatchStats {
    unsigned long long exp = 0, lbox = 0, lex = 0, nq = 0;
};

__device__ __forceinline__ int lds_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int lds_add(int32_t *p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool lds_cas(int32_t *p, int expect, int v) {
    return __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Lane 0's value as a wave-uniform (scalar) one.  The mailbox decisions, the
// chunk's owner and size, the stack depth and the wait conditions are the same
// in every lane; reading them through readfirstlane makes the branches on them
// scalar, so the compiler never treats the regions that use ballots and
// shuffles as divergent (with the decisions taken per lane through a
// shuffle, batches after a wave's first returned faces that were not the
// nearest).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The lanes of a wave hand stack entries to each other through LDS (a lane
// pops what another lane pushed, copied or donated).  The hardware keeps a
// wave's LDS operations in order, but the compiler only orders each lane's own
// accesses, and a lane's load of another lane's slot may be moved above the
// store that fills it; this fence keeps every LDS access of the wave on its
// side.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Rounds over wave `self`'s stack (sp entries) until it is empty.  Entries
// belong to the batch of wave `owner`: its query positions and bests.
template <bool kTri, int M>
__device__ void run_stack(const QueryArgs &a, BatchLds<M> &L, int self, int owner, int sp, BatchStats &stats) {
    const int lane = threadIdx.x % 64;
    const uint64_t lt = lanemask_lt();
    WaveStack<M> &S = L.st[self];
    WaveStack<M> &O = L.st[owner];
    WaveMail &mail = L.mail;
    // the stack never exceeds kBatchCap + 62: a round of width k pushes at most
    // 2k entries, widths are cut to (kBatchCap - sp) / 2, and width-1 rounds are
    // a plain depth-first walk whose growth is bounded by the tree depth; each
    // query expands each internal node at most once, so the round cap only stops
    // a corrupted buffer from looping
    for (int64_t round = 0; sp > 0 && round < static_cast<int64_t>(M + 1) * a.n + 64; ++round) {
        wave_sync();                          // the previous round's pushes, or the entries handed in
        if (sp >= kDonateMin) {
            int give = 0;
            if (lane == 0 && lds_load(&mail.state) == 0 && lds_cas(&mail.state, 0, 3)) give = 1;
            if (uniform(give)) {
                const int i = sp - 64 + lane;
                mail.node[lane] = S.node[i];
                mail.dist[lane] = S.dist[i];
                mail.slot[lane] = S.slot[i];
                wave_sync();
                sp -= 64;
                if (lane == 0) {
                    mail.owner = owner;
                    mail.count = 64;
                    lds_add(&mail.outstanding[owner], 1);
                    lds_store(&mail.state, 1);
                }
            }
        }
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
        unsigned long long best = act ? O.best[slot] : 0ull;
        const f3 qp = act ? f3{O.q[0][slot], O.q[1][slot], O.q[2][slot]} : f3{0.0f, 0.0f, 0.0f};
        const float qm = qnorm1(qp);
        act = act && nd <= prune_bound(__uint_as_float(static_cast<uint32_t>(best >> 32)), qm);
        float4 l0, l1, l2, r0, r1, r2;
        int32_t lref = 0, rref = 0;
        unsigned long long cand = ~0ull;
        if (act) {
            const float4 *rec = a.nodes + 6 * static_cast<int64_t>(node);
            l0 = rec[0]; l1 = rec[1]; l2 = rec[2]; r0 = rec[3]; r1 = rec[4]; r2 = rec[5];
            lref = __float_as_int(l0.w);
            rref = __float_as_int(r0.w);
            if (lref >= a.n - 1 || rref >= a.n - 1 || ~lref >= a.n || ~rref >= a.n) act = false;
        }
        const float pbound = prune_bound(__uint_as_float(static_cast<uint32_t>(best >> 32)), qm);
        const bool tl = act && lref < 0 && leaf_box_dist2<kTri>(qp, l0, l1, l2) <= pbound;
        const bool tr = act && rref < 0 && leaf_box_dist2<kTri>(qp, r0, r1, r2) <= pbound;
        if (a.counters) {
            stats.exp += __popcll(__ballot(act));
            stats.lbox += __popcll(__ballot(act && lref < 0)) + __popcll(__ballot(act && rref < 0));
            stats.lex += __popcll(__ballot(tl)) + __popcll(__ballot(tr));
        }
        if (tl) cand = pack_best(leaf_dist2<kTri>(qp, l0, l1, l2), __float_as_int(l1.w));
        if (tr) {
            const unsigned long long c = pack_best(leaf_dist2<kTri>(qp, r0, r1, r2), __float_as_int(r1.w));
            if (c < cand) cand = c;
        }
        if (cand != ~0ull) atomicMin(&O.best[slot], cand);
        best = act ? O.best[slot] : 0ull;
        const float bound = prune_bound(__uint_as_float(static_cast<uint32_t>(best >> 32)), qm);
        const float dq = 0x1p-20f * qm;
        const float dl = (act && lref >= 0) ? child_bound<kTri>(qp, dq, l0, l1, l2) : INFINITY;
        const float dr = (act && rref >= 0) ? child_bound<kTri>(qp, dq, r0, r1, r2) : INFINITY;
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
        if (sp > kBatchAlloc) {              // past the bound of a valid tree
            if (lane == 0) atomicOr(a.status, 64);
            sp = kBatchAlloc;
        }
    }
    wave_sync();                              // the last round's bests, before any lane reads them
}

// Takes the mailbox's chunk, if there is one, and runs it to the end.
template <bool kTri, int M>
__device__ bool help_once(const QueryArgs &a, BatchLds<M> &L, int self, BatchStats &stats) {
    const int lane = threadIdx.x % 64;
    WaveMail &mail = L.mail;
    int got = 0;
    if (lane == 0 && lds_load(&mail.state) == 1 && lds_cas(&mail.state, 1, 2)) got = 1;
    if (!uniform(got)) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int owner = uniform(mail.owner), n = uniform(mail.count);
    if (owner < 0 || owner >= kBatchWaves || n < 0 || n > 64) {
        if (lane == 0) { atomicOr(a.status, 16); lds_store(&mail.state, 0); }
        return true;
    }
    WaveStack<M> &S = L.st[self];
    if (lane < n) {
        S.node[lane] = mail.node[lane];
        S.dist[lane] = mail.dist[lane];
        S.slot[lane] = mail.slot[lane];
    }
    wave_sync();
    if (lane == 0) lds_store(&mail.state, 0);
    run_stack<kTri, M>(a, L, self, owner, n, stats);
    if (lane == 0) lds_add(&mail.outstanding[owner], -1);
    return true;
}

// Helps other waves until cond() holds (cond is evaluated by every lane on
// LDS words, so it is wave-uniform).
template <bool kTri, int M, typename Cond>
__device__ void wait_helping(const QueryArgs &a, BatchLds<M> &L, int self, BatchStats &stats, Cond cond) {
    const int lane = threadIdx.x % 64;
    for (int spin = 0; !cond();) {
        if (help_once<kTri, M>(a, L, self, stats)) {
            spin = 0;
        } else if (++spin > kIdleSpinLimit) {
            if (lane == 0) atomicOr(a.status, 16);
            break;
        } else {
            __builtin_amdgcn_s_sleep(2);
        }
    }
}

// The workgroup's kBatchWaves waves process the query batches [qb, qb + M)
// below q_end (positions in the processing order): wave w takes qb = start +
// w M, then steps by stride or, with a queue, M times the batch numbers it
// takes from the queue.  Every wave of the workgroup calls this.  kHelpBetween:
// a wave that has written a batch's results empties the mailbox before it
// starts its next batch.  The batched persistent kernel leaves that out: there
// the compiled form of that loop returned faces that were not the nearest for
// queries of later batches (about one in ten at 100,000 queries without the
// seed descent), while every other form of this loop, and the plain kernels
// with it, matched the all-faces kernel exactly; its waves still help while
// they wait for their own chunks and at the end.
template <bool kTri, int M, bool kHelpBetween = true>
__device__ void batch_loop(const QueryArgs &a, int64_t start, int64_t stride, int64_t q_end, BatchLds<M> &L) {
    const int lane = threadIdx.x % 64;
    const int self = uniform(static_cast<int>(threadIdx.x / 64));
    const uint64_t lt = lanemask_lt();
    const unsigned long long none = pack_best(a.maxd2, INT_MAX);
    WaveStack<M> &S = L.st[self];
    WaveMail &mail = L.mail;
    BatchStats stats;
    if (threadIdx.x == 0) {
        mail.state = 0;
        mail.done = 0;
        for (int w = 0; w < kBatchWaves; ++w) mail.outstanding[w] = 0;
    }
    __syncthreads();

    auto next = [&](int64_t qb) -> int64_t {
        if (!a.queue) return qb + stride;
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(a.queue, 1u);
        return static_cast<int64_t>(static_cast<uint32_t>(uniform(static_cast<int>(b)))) * M;
    };
    for (int64_t qb = a.queue ? next(0) : start + static_cast<int64_t>(self) * M; qb < q_end; qb = next(qb)) {
        const int nb = static_cast<int>(q_end - qb < M ? q_end - qb : M);
        const int64_t qid = lane < nb ? query_at(a, qb + lane) : -1;
        const bool own = qid >= 0;
        f3 p = f3{0.0f, 0.0f, 0.0f};
        if (own) {
            p = load3(a.queries, a.nq, qid);
            S.q[0][lane] = p.x; S.q[1][lane] = p.y; S.q[2][lane] = p.z;
            S.best[lane] = none;
        }
        int sp = 0;
        if (a.n == 1) {
            if (own) {
                const unsigned long long c = pack_best(single_leaf_dist2<kTri>(a, p), a.prim[0]);
                if (c < none) S.best[lane] = c;
            }
        } else if (a.n > 1) {
            // a hinted primitive's distance starts the query; without one, the seed descent
            unsigned long long seeded = own ? hint_best<kTri>(a, qid, p, none) : none;
            if (a.seed && own && seeded == none) {
                // one greedy root-to-leaf walk (nearer internal child first) gives an
                // upper bound before the wide expansion starts
                const float dq = slab_query_margin(p);
                int32_t node = 0;
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
                        if (c < seeded) seeded = c;
                    }
                    if (rref < 0) {
                        const unsigned long long c = pack_best(leaf_dist2<kTri>(p, r0, r1, r2), __float_as_int(r1.w));
                        if (c < seeded) seeded = c;
                    }
                    const float dl = lref >= 0 ? child_bound<kTri>(p, dq, l0, l1, l2) : INFINITY;
                    const float dr = rref >= 0 ? child_bound<kTri>(p, dq, r0, r1, r2) : INFINITY;
                    node = (lref >= 0 && dl <= dr) ? lref : (rref >= 0 ? rref : -1);
                }
            }
            if (own && seeded < none) S.best[lane] = seeded;
            const f3 rlo = f3{a.root[0], a.root[1], a.root[2]};
            const f3 rhi = f3{a.root[4], a.root[5], a.root[6]};
            const float rd = own ? box_dist2(p, rlo, rhi) : INFINITY;
            const float rb = (seeded < none ? __uint_as_float(static_cast<uint32_t>(seeded >> 32)) : a.maxd2);
            const bool push = own && rd <= prune_bound(rb, qnorm1(p));
            const uint64_t bm = __ballot(push);
            if (push) {
                const int pos = __popcll(bm & lt);
                S.node[pos] = 0;
                S.dist[pos] = rd;
                S.slot[pos] = static_cast<uint8_t>(lane);
            }
            sp = __popcll(bm);
        }
        run_stack<kTri, M>(a, L, self, self, sp, stats);
        // chunks given away must be finished before the results are final
        wait_helping<kTri, M>(a, L, self, stats, [&]() { return uniform(lds_load(&mail.outstanding[self])) == 0; });
        if (own) {
            const unsigned long long b = S.best[lane];
            write_result_id<kTri>(a, qid, p, static_cast<int32_t>(b & 0xffffffffull),
                                  __uint_as_float(static_cast<uint32_t>(b >> 32)));
        }
        if (a.counters) stats.nq += __popcll(__ballot(own));
        // work already started in the workgroup goes before a new batch
        if (kHelpBetween)
            while (help_once<kTri, M>(a, L, self, stats)) {
            }
    }
    if (lane == 0) lds_add(&mail.done, 1);
    wait_helping<kTri, M>(a, L, self, stats, [&]() { return uniform(lds_load(&mail.done)) == kBatchWaves; });
    if (a.counters && lane == 0) add_counters(a, stats.exp, stats.lbox, stats.lex, stats.nq);
}

}  // namespace mgu
