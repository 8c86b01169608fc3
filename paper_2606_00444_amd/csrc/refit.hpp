// LBVH refit bodies shared by the plain refit/build kernel and the batched
// persistent kernel.
//
// The tree is cut into subtrees of at most C = 2^chunk_log2 leaves: a subtree
// root is a child, with at most C leaves, of a node with more than C (or the
// whole tree when it has at most C leaves).  Above the cut lie the "top"
// nodes, one fewer than the subtrees.  Both sets are fixed by the topology and
// listed once, when the tree is built, with the parent of every top node and
// of every subtree root among the top nodes (the top links).
//
// A finished node hands its parent a 12-float summary: its box, the unit
// direction d of the area-weighted normal sum of the faces below it, the sum's
// length, and the slab [a, b] of d.x over those faces.  Each node has one
// summary slot and an arrival word: the first child to finish publishes its
// summary there and stops; the second reads it, joins the two in registers,
// writes the node's slot in its parent's record and climbs on.  A level of
// the climb is one LDS atomic, one 48-byte LDS read and the join.
//
// Phase 1 (a workgroup per subtree): a Karras node covers a contiguous leaf
// range and its index is one end of that range, so the internal nodes of a
// subtree over leaves [f, l] have indices in [f, l] and their slots live in
// LDS.  The subtree root's summary is deposited for phase 2 with device-scope
// stores.  Phase 2 (one workgroup): the same climb through the top nodes, one
// thread from each deposited subtree root.  The plain refit runs it in the
// workgroup that finishes the last subtree (an arrival counter in the BVH
// header), the batched kernel as a work item of its own.
//
// Boxes are exact (min/max only) and each join takes its two children in slot
// order with contraction off and explicit fused multiply-adds, so any schedule
// gives bitwise the same records.  Every index read from the buffer is
// range-checked; a corrupted buffer sets the error word instead of faulting or
// hanging.
#pragma once

#include "mgu_internal.hpp"

namespace mgu {

struct RefitArgs {
    const float *verts; int64_t nv;
    const int32_t *leaf_faces;    // [3][n] or nullptr for points
    const int32_t *prim;
    const int32_t *leaf_parent; const int32_t *node_parent;
    float4 *nodes;                // [n-1][6] records written by this refit
    const int32_t *top_nodes;     // [T] node id of each top node
    const int32_t *top_parent;    // [T] (parent's top index << 1) | slot, -1 for the root
    const int32_t *sub_parent;    // [n_sub] (top parent's index << 1) | slot of each subtree root
    const int32_t *subtrees;      // [3][n]: root reference, first leaf, last leaf
    float4 *deposit;              // [n_sub][3] subtree-root summaries (device-coherent)
    float4 *top_scratch;          // [tstride][3] summary slots, [kDummyWaves][3] dummies, then
    int64_t tstride;              // uint32 [tstride] arrival words: phase-2 state when T
                                  // exceeds the LDS capacity
    float *root;                  // root box: lo at [0..2], hi at [4..6]
    int32_t *status;              // error word
    const int32_t *hdr_nv;        // vertex count of the build (header), or nullptr
    const int32_t *n_top;         // number of top nodes (device)
    const int32_t *n_sub;         // number of subtrees (device)
    uint32_t *arrivals;           // subtrees finished in this launch (plain refit)
    int64_t n;
    int chunk_log2;
};

// The summary a finished node hands to its parent.
struct Sum {
    f3 lo, hi;                    // box
    f3 d;                         // unit normal direction (zero: none)
    float sn;                     // length of the area-weighted normal sum
    float a, b;                   // slab: a <= d.x <= b over the faces below
};

// LDS bytes per subtree node (three float4, an arrival word and its parent
// link) and per top node (the same, plus its node id), and the per-wave dummy
// slots of the hand-off (below).
constexpr size_t kSubSlotBytes = 56;
constexpr size_t kTopSlotBytes = 60;
constexpr int kDummyWaves = 16;   // waves of a 1024-thread workgroup
constexpr size_t kDummyBytes = kDummyWaves * 48;
constexpr int kTopCap = 1024;     // top nodes the plain refit's LDS holds at least

constexpr size_t refit_sub_lds(int64_t C) { return static_cast<size_t>(C) * kSubSlotBytes + kDummyBytes; }
constexpr size_t refit_top_lds(int64_t T) { return static_cast<size_t>(T) * kTopSlotBytes + kDummyBytes; }
// LDS of the plain refit kernel: a subtree's slots, and room for at least
// kTopCap top nodes in the workgroup that climbs the top.
constexpr size_t refit_lds_bytes(int chunk_log2) {
    return refit_sub_lds(int64_t(1) << chunk_log2) > refit_top_lds(kTopCap) ? refit_sub_lds(int64_t(1) << chunk_log2)
                                                                            : refit_top_lds(kTopCap);
}

// ------------------------------------------------------------- normal slabs
// An internal child slot of a triangle BVH stores, besides its box, a unit
// direction d and [a, b] with a <= d.x <= b for every point x of the faces
// below it; the distance from q to them is then at least max(a - d.q, d.q - b,
// 0).  A node's d is the normalised sum of its children's normal sums.  Its
// slab comes from its children's: with alpha = d.d_c and r = d - alpha d_c,
// d.x = alpha (d_c.x) + r.x, where the first term lies in alpha [a_c, b_c] and
// the second in the range of r.x over the child's box; the union over the two
// children is intersected with the range of d.x over the node's box.  A leaf's
// slab is its triangle's extent along its own normal.  Every extent is widened
// by 2^-18 of the node's box coordinate magnitudes, far more than the float32
// rounding of these few operations (the range of a linear function over a box
// from its centre and half-widths; the residual r rounded once per component,
// an error of at most one unit in its last place times |x|).

__device__ __forceinline__ float slab_margin(f3 lo, f3 hi) {
    return 0x1p-18f * (((fabsf(lo.x) + fabsf(hi.x)) + (fabsf(lo.y) + fabsf(hi.y))) + (fabsf(lo.z) + fabsf(hi.z)));
}

// Unit direction and length of a normal sum by the hardware reciprocal square
// root (any direction gives a valid slab, since the extents are taken along
// the stored one; |d| is 1 to about 2^-22, which the traversal's bound allows
// for).  Sums too small or too large to normalise safely give no direction.
__device__ __forceinline__ bool unit_of(f3 s, f3 &d, float &len) {
#pragma clang fp contract(off)
    const float l2 = fdot(s, s);
    const bool ok = l2 > 1e-30f && l2 < 1e30f;
    const float k = ok ? __builtin_amdgcn_rsqf(l2) : 0.0f;
    d = f3{k * s.x, k * s.y, k * s.z};
    len = ok ? l2 * k : 0.0f;
    return ok;
}

// [mn, mx] of r.x over the box with doubled centre S = lo + hi and doubled
// half-widths H = hi - lo: 0.5 (r.S -/+ |r|.H).
__device__ __forceinline__ void range_over(f3 r, f3 S, f3 H, float &mn, float &mx) {
#pragma clang fp contract(off)
    const float c = fdot(r, S);
    const float h = fdot(f3{fabsf(r.x), fabsf(r.y), fabsf(r.z)}, H);
    mn = 0.5f * (c - h);
    mx = 0.5f * (c + h);
}

template <bool kTri>
__device__ __forceinline__ Sum leaf_sum(f3 x, f3 y, f3 z) {
#pragma clang fp contract(off)
    Sum S;
    // + 0 turns -0 into +0, so a zero box coordinate has one encoding whatever the
    // vertices' signs of zero (boxes are then bitwise the same in any union order)
    const f3 lo = fmin3(fmin3(x, y), z), hi = fmax3(fmax3(x, y), z);
    S.lo = f3{lo.x + 0.0f, lo.y + 0.0f, lo.z + 0.0f};
    S.hi = f3{hi.x + 0.0f, hi.y + 0.0f, hi.z + 0.0f};
    S.d = f3{0.0f, 0.0f, 0.0f};
    S.sn = 0.0f;
    S.a = -INFINITY;
    S.b = INFINITY;
    if (!kTri) return S;
    if (unit_of(cross_rounded(y - x, z - x), S.d, S.sn)) {
        const float px = fdot(S.d, x), py = fdot(S.d, y), pz = fdot(S.d, z);
        const float e = slab_margin(S.lo, S.hi);
        S.a = fminf(fminf(px, py), pz) - e;
        S.b = fmaxf(fmaxf(px, py), pz) + e;
    }
    return S;
}

// Bound of d.x over child c's faces, or [ba, bb] (the node box's range) when
// the child has no slab.
__device__ __forceinline__ void child_range(f3 d, const Sum &c, float ba, float bb, float &ca, float &cb) {
#pragma clang fp contract(off)
    const float al = fdot(d, c.d);
    const f3 r = f3{fmaf(-al, c.d.x, d.x), fmaf(-al, c.d.y, d.y), fmaf(-al, c.d.z, d.z)};
    float rmn, rmx;
    range_over(r, c.lo + c.hi, c.hi - c.lo, rmn, rmx);
    const bool pos = al >= 0.0f;
    const float lo_c = fmaf(al, pos ? c.a : c.b, rmn);
    const float hi_c = fmaf(al, pos ? c.b : c.a, rmx);
    const bool has = c.a > -INFINITY && c.b < INFINITY && c.sn > 0.0f;
    ca = has ? lo_c : ba;
    cb = has ? hi_c : bb;
}

// The summary of a node from its children's, in slot order.
template <bool kTri>
__device__ __forceinline__ Sum join(const Sum &L, const Sum &R) {
#pragma clang fp contract(off)
    Sum P;
    P.lo = fmin3(L.lo, R.lo);
    P.hi = fmax3(L.hi, R.hi);
    P.d = f3{0.0f, 0.0f, 0.0f};
    P.sn = 0.0f;
    P.a = -INFINITY;
    P.b = INFINITY;
    if (!kTri) return P;
    const f3 s = f3{fmaf(L.sn, L.d.x, R.sn * R.d.x), fmaf(L.sn, L.d.y, R.sn * R.d.y),
                    fmaf(L.sn, L.d.z, R.sn * R.d.z)};
    if (unit_of(s, P.d, P.sn)) {
        float ba, bb;
        range_over(P.d, P.lo + P.hi, P.hi - P.lo, ba, bb);
        float a0, b0, a1, b1;
        child_range(P.d, L, ba, bb, a0, b0);
        child_range(P.d, R, ba, bb, a1, b1);
        const float e = slab_margin(P.lo, P.hi);
        P.a = fmaxf(ba, fminf(a0, a1)) - e;
        P.b = fminf(bb, fmaxf(b0, b1)) + e;
    }
    return P;
}

// The join of a node whose children's summaries are `mine` (the climbing
// lane's, in slot `slot`) and `other`: the two are put in slot order with
// selects, so a wave whose lanes came from either side runs one join.
template <bool kTri>
__device__ __forceinline__ Sum join_slots(const Sum &mine, const Sum &other, int slot) {
    const bool sw = slot != 0;
    Sum L, R;
    L.lo = f3{sw ? other.lo.x : mine.lo.x, sw ? other.lo.y : mine.lo.y, sw ? other.lo.z : mine.lo.z};
    L.hi = f3{sw ? other.hi.x : mine.hi.x, sw ? other.hi.y : mine.hi.y, sw ? other.hi.z : mine.hi.z};
    L.d = f3{sw ? other.d.x : mine.d.x, sw ? other.d.y : mine.d.y, sw ? other.d.z : mine.d.z};
    L.sn = sw ? other.sn : mine.sn; L.a = sw ? other.a : mine.a; L.b = sw ? other.b : mine.b;
    R.lo = f3{sw ? mine.lo.x : other.lo.x, sw ? mine.lo.y : other.lo.y, sw ? mine.lo.z : other.lo.z};
    R.hi = f3{sw ? mine.hi.x : other.hi.x, sw ? mine.hi.y : other.hi.y, sw ? mine.hi.z : other.hi.z};
    R.d = f3{sw ? mine.d.x : other.d.x, sw ? mine.d.y : other.d.y, sw ? mine.d.z : other.d.z};
    R.sn = sw ? mine.sn : other.sn; R.a = sw ? mine.a : other.a; R.b = sw ? mine.b : other.b;
    return join<kTri>(L, R);
}

// A summary in three float4 and back: (lo, sn) (hi, a) (d, b).
__device__ __forceinline__ void pack(const Sum &S, float4 v[3]) {
    v[0] = make_float4(S.lo.x, S.lo.y, S.lo.z, S.sn);
    v[1] = make_float4(S.hi.x, S.hi.y, S.hi.z, S.a);
    v[2] = make_float4(S.d.x, S.d.y, S.d.z, S.b);
}
__device__ __forceinline__ Sum unpack(float4 v0, float4 v1, float4 v2) {
    Sum S;
    S.lo = f3{v0.x, v0.y, v0.z}; S.sn = v0.w;
    S.hi = f3{v1.x, v1.y, v1.z}; S.a = v1.w;
    S.d = f3{v2.x, v2.y, v2.z}; S.b = v2.w;
    return S;
}

// Record slot of an internal child: (lo, ref) (hi, a) (d, b); points carry no slab.
template <bool kTri>
__device__ __forceinline__ void write_internal(float4 *rec, int32_t ref, const Sum &S) {
    rec[0] = make_float4(S.lo.x, S.lo.y, S.lo.z, __int_as_float(ref));
    if (kTri) {
        rec[1] = make_float4(S.hi.x, S.hi.y, S.hi.z, S.a);
        rec[2] = make_float4(S.d.x, S.d.y, S.d.z, S.b);
    } else {
        rec[1] = make_float4(S.hi.x, S.hi.y, S.hi.z, 0.0f);
    }
}

__device__ __forceinline__ void write_root(float *root, const Sum &S) {
    root[0] = S.lo.x; root[1] = S.lo.y; root[2] = S.lo.z;
    root[4] = S.hi.x; root[5] = S.hi.y; root[6] = S.hi.z;
}

// Device-scope stores and loads of a deposited summary: visible to a workgroup
// on another XCD without a write-back of this XCD's L2.  The storing thread
// waits for its stores to complete before its workgroup signals arrival.
__device__ __forceinline__ void deposit_store(float4 *dst, const Sum &S) {
    float4 v[3];
    pack(S, v);
    float *f = reinterpret_cast<float *>(dst);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        __hip_atomic_store(f + 4 * q + 0, v[q].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(f + 4 * q + 1, v[q].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(f + 4 * q + 2, v[q].z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(f + 4 * q + 3, v[q].w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ Sum deposit_load(const float4 *src) {
    const float *f = reinterpret_cast<const float *>(src);
    float w[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) w[q] = __hip_atomic_load(f + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return unpack(make_float4(w[0], w[1], w[2], w[3]), make_float4(w[4], w[5], w[6], w[7]),
                  make_float4(w[8], w[9], w[10], w[11]));
}

// ---------------------------------------------------------------- the climb
// Arrival word of a node: bit 0 is set by the first child to arrive, bit 1
// once that child's summary is in the slot.  arrive() returns true for the
// second child, with the first one's summary in `other`.  Slots and words are
// in LDS (workgroup scope), or with kGlobal in global scratch used by one
// workgroup (device scope, so no stale cache line from an earlier launch on
// another XCD is read).
//
// Two children of a node are often climbed by lanes of one wave that arrive
// in the same instruction, and a lane that waited for an unpublished sibling
// of its own wave would wait for ever (a wave does not run its other lanes
// while one spins).  So the publication has no branch: every arriving lane
// stores its summary - the first child into the node's slot, the second into
// its wave's dummy slot - and ors the published bit (0 for the second) in the
// same straight-line instructions, before any lane can start waiting.  A lane
// then waits only for a first child in another wave, which publishes without
// waiting for anything.
constexpr int kSlotSpin = 1 << 20;

// In LDS the words are relaxed atomics ordered by fences on LDS alone: a fence
// of every address space would also wait for the climb's record stores (on
// CDNA, vector loads and stores share one counter), a global store's latency
// per level.
template <bool kGlobal>
__device__ __forceinline__ uint32_t word_or(uint32_t *w, uint32_t v) {
    if (kGlobal) return __hip_atomic_fetch_or(w, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_fetch_or(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool kGlobal>
__device__ __forceinline__ uint32_t word_load(uint32_t *w) {
    if (kGlobal) return __hip_atomic_load(w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool kGlobal>
__device__ __forceinline__ void lds_release() {
    if (!kGlobal) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
}
template <bool kGlobal>
__device__ __forceinline__ void lds_acquire() {
    if (!kGlobal) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
template <bool kGlobal>
__device__ __forceinline__ void slot_store(float4 *slot, const Sum &S) {
    if (kGlobal) {
        deposit_store(slot, S);
    } else {
        float4 v[3];
        pack(S, v);
        slot[0] = v[0]; slot[1] = v[1]; slot[2] = v[2];
    }
}
template <bool kGlobal>
__device__ __forceinline__ Sum slot_load(const float4 *slot) {
    if (kGlobal) return deposit_load(slot);
    return unpack(slot[0], slot[1], slot[2]);
}

//
// Two sibling leaves often sit in adjacent lanes of one wave and arrive in the
// same instruction.  The second may wait for the first's summary only because
// the publication is a region of its own that precedes any waiting in program
// order: a wave runs it for its first-arriving lanes before the waiting loop
// of its second-arriving lanes (a waiting lane never blocks a lane of its own
// wave that has yet to publish).  The wait is bounded all the same.
template <bool kGlobal>
__device__ __forceinline__ bool arrive(float4 *slot, float4 *dummy, uint32_t *word, const Sum &mine, Sum &other,
                                       int32_t *status) {
    uint32_t old = word_or<kGlobal>(word, 1u);
    const bool first = !(old & 1u);
    slot_store<kGlobal>(first ? slot : dummy, mine);
    lds_release<kGlobal>();
    word_or<kGlobal>(word, first ? 2u : 0u);  // the slot is written
    if (first) return false;                  // the sibling finishes the node
    for (int spin = 0; !(old & 2u); ++spin) { // a first child in another wave, between its two steps
        if (spin > kSlotSpin) { atomicOr(status, 8); break; }
        old = word_load<kGlobal>(word);
    }
    lds_acquire<kGlobal>();
    other = slot_load<kGlobal>(slot);
    return true;
}

// Phase 1 for subtree k by a workgroup of kThreads threads, each taking kLeaves
// adjacent leaves and advancing their climbs together, one level per step, so
// that no climb waits behind another of its thread.  kThreads is a compile-time
// stride: blockDim would be reloaded from the dispatch packet, and that load's
// wait would also wait for the record stores in flight.  smem:
// refit_sub_lds(C) bytes.  The climb that finishes the subtree root deposits
// its summary at deposit[k]; returns after the workgroup's barrier.
template <bool kTri, int kThreads, int kLeaves>
__device__ void refit_subtree(const RefitArgs &a, int64_t k, unsigned char *smem) {
    const int C = 1 << a.chunk_log2;
    const int32_t r = a.subtrees[k];
    const int64_t f = a.subtrees[a.n + k], l = a.subtrees[2 * a.n + k];
    float4 *s_slot = reinterpret_cast<float4 *>(smem);                 // [C][3]
    float4 *s_dummy = s_slot + 3 * C + 3 * (threadIdx.x / 64);         // [kDummyWaves][3]
    uint32_t *s_word = reinterpret_cast<uint32_t *>(s_slot + 3 * (C + kDummyWaves));   // [C]
    int32_t *s_par = reinterpret_cast<int32_t *>(s_word + C);          // [C] parent tags
    const int64_t size = l - f + 1;
    if (f < 0 || l >= a.n || size < 1 || size > C || size > static_cast<int64_t>(kThreads) * kLeaves) {
        if (threadIdx.x == 0) atomicOr(a.status, 4);
        __syncthreads();
        return;
    }
    if (k == 0 && threadIdx.x == 0 && a.hdr_nv && *a.hdr_nv != a.nv) atomicOr(a.status, 32);
    // the leaves' ids, parent tags and vertices are loaded before the LDS set-up
    // and its barrier, so the gathers overlap them
    Sum S[kLeaves];
    int32_t p[kLeaves], slot[kLeaves];
    bool live[kLeaves];
    f3 x[kLeaves], y[kLeaves], z[kLeaves];
    int32_t id[kLeaves], tag[kLeaves];
    const int64_t i0 = f + static_cast<int64_t>(threadIdx.x) * kLeaves;
#pragma unroll
    for (int u = 0; u < kLeaves; ++u) {
        const int64_t i = i0 + u;
        tag[u] = -2;
        if (i > l) continue;
        id[u] = a.prim[i];
        tag[u] = a.leaf_parent[i];
        if (kTri) {
            x[u] = vload(a.verts, a.nv, a.leaf_faces[i]);
            y[u] = vload(a.verts, a.nv, a.leaf_faces[a.n + i]);
            z[u] = vload(a.verts, a.nv, a.leaf_faces[2 * a.n + i]);
        } else {
            x[u] = y[u] = z[u] = vload(a.verts, a.nv, id[u]);
        }
    }
    for (int j = threadIdx.x; j < size; j += kThreads) {
        s_word[j] = 0u;
        s_par[j] = f + j < a.n - 1 ? a.node_parent[f + j] : -1;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kLeaves; ++u) {
        const int64_t i = i0 + u;
        live[u] = false;
        if (tag[u] == -2) continue;
        S[u] = leaf_sum<kTri>(x[u], y[u], z[u]);
        if (tag[u] < 0) {                     // a single leaf is the root
            write_root(a.root, S[u]);
            continue;
        }
        p[u] = tag[u] >> 1;
        slot[u] = tag[u] & 1;
        if (p[u] >= a.n - 1) { atomicOr(a.status, 4); continue; }
        float4 *rec = a.nodes + 6 * static_cast<int64_t>(p[u]) + 3 * slot[u];
        rec[0] = make_float4(x[u].x, x[u].y, x[u].z, __int_as_float(~static_cast<int32_t>(i)));
        rec[1] = make_float4(y[u].x, y[u].y, y[u].z, __int_as_float(id[u]));
        if (kTri) rec[2] = make_float4(z[u].x, z[u].y, z[u].z, 0.0f);
        if (r == ~static_cast<int32_t>(i)) {  // a one-leaf subtree
            deposit_store(a.deposit + 3 * k, S[u]);
            continue;
        }
        live[u] = true;
    }
    // a valid tree is at most 62 levels deep
    for (int level = 0; level < 64; ++level) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < kLeaves; ++u) {
            if (!live[u]) continue;
            live[u] = false;
            const int64_t jl = p[u] - f;
            if (jl < 0 || jl >= size) { atomicOr(a.status, 4); continue; }
            const int j = static_cast<int>(jl);
            const int32_t ptag = s_par[j];
            Sum O;
            if (!arrive<false>(s_slot + 3 * j, s_dummy, s_word + j, S[u], O, a.status)) continue;
            S[u] = join_slots<kTri>(S[u], O, slot[u]);
            if (ptag < 0) {                   // p is the root: the subtree is the whole tree
                write_root(a.root, S[u]);
                continue;
            }
            const int32_t c = p[u];
            p[u] = ptag >> 1;
            slot[u] = ptag & 1;
            if (p[u] >= a.n - 1) { atomicOr(a.status, 4); continue; }
            write_internal<kTri>(a.nodes + 6 * static_cast<int64_t>(p[u]) + 3 * slot[u], c, S[u]);
            if (c == r) {
                deposit_store(a.deposit + 3 * k, S[u]);
                continue;
            }
            live[u] = true;
            any = true;
        }
        if (!__builtin_amdgcn_readfirstlane(__ballot(any) != 0)) break;
    }
    __syncthreads();
}

// Phase 2 over T top nodes and NS subtrees by one workgroup of kThreads:
// the climbs from the deposited subtree roots t, t + kThreads, ... (at most
// kRoots per thread, advanced together; more are taken kRoots at a time)
// through the top nodes.  The slots and arrival words live in LDS (smem,
// refit_top_lds(T) bytes), or with kGlobal in a.top_scratch.  Returns after
// the root's box is written.
template <bool kTri, int kThreads, bool kGlobal, int kRoots = 2>
__device__ void refit_top(const RefitArgs &a, int T, int NS, unsigned char *smem) {
    // slots [T][3] (global: [tstride][3]), dummies [kDummyWaves][3], words, then in
    // LDS each top node's id and parent link
    float4 *t_slot;
    uint32_t *t_word;
    int32_t *t_node = nullptr, *t_par = nullptr;
    const int64_t ts = kGlobal ? a.tstride : T;
    if (kGlobal) {
        t_slot = a.top_scratch;
    } else {
        t_slot = reinterpret_cast<float4 *>(smem);
    }
    float4 *t_dummy = t_slot + 3 * ts + 3 * (threadIdx.x / 64);
    t_word = reinterpret_cast<uint32_t *>(t_slot + 3 * (ts + kDummyWaves));
    if (!kGlobal) {
        t_node = reinterpret_cast<int32_t *>(t_word + T);
        t_par = t_node + T;
    }
    for (int t = threadIdx.x; t < T; t += kThreads) {
        if (kGlobal) {
            __hip_atomic_store(t_word + t, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            t_word[t] = 0u;
            t_node[t] = a.top_nodes[t];
            t_par[t] = a.top_parent[t];
        }
    }
    if (kGlobal) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int k0 = 0; k0 < NS; k0 += kRoots * kThreads) {
        Sum S[kRoots];
        int32_t tag[kRoots];
        bool live[kRoots];
#pragma unroll
        for (int u = 0; u < kRoots; ++u) {
            const int k = k0 + u * kThreads + threadIdx.x;
            live[u] = k < NS;
            if (!live[u]) continue;
            S[u] = deposit_load(a.deposit + 3 * k);
            tag[u] = a.sub_parent[k];
        }
        // a valid top tree is at most 62 levels high
        for (int level = 0; level < 64; ++level) {
            bool any = false;
#pragma unroll
            for (int u = 0; u < kRoots; ++u) {
                if (!live[u]) continue;
                live[u] = false;
                const int tp = tag[u] >> 1, slot = tag[u] & 1;
                if (tag[u] < 0 || tp >= T) { atomicOr(a.status, 8); continue; }
                const int32_t ptag = kGlobal ? a.top_parent[tp] : t_par[tp];
                Sum O;
                if (!arrive<kGlobal>(t_slot + 3 * tp, t_dummy, t_word + tp, S[u], O, a.status)) continue;
                S[u] = join_slots<kTri>(S[u], O, slot);
                if (ptag < 0) {               // tp is the root
                    write_root(a.root, S[u]);
                    continue;
                }
                const int pt = ptag >> 1;
                if (pt >= T) { atomicOr(a.status, 8); continue; }
                const int32_t pn = kGlobal ? a.top_nodes[pt] : t_node[pt];
                const int32_t cn = kGlobal ? a.top_nodes[tp] : t_node[tp];
                if (pn < 0 || pn >= a.n - 1) { atomicOr(a.status, 8); continue; }
                write_internal<kTri>(a.nodes + 6 * static_cast<int64_t>(pn) + 3 * (ptag & 1), cn, S[u]);
                tag[u] = ptag;
                live[u] = true;
                any = true;
            }
            if (!__builtin_amdgcn_readfirstlane(__ballot(any) != 0)) break;
        }
    }
    __syncthreads();
}

}  // namespace mgu
