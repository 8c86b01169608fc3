// LBVH refit bodies shared by the plain refit/build kernel and the batched
// persistent kernel.
//
// The tree is cut into subtrees of at most C = 2^chunk_log2 leaves: a subtree
// root is a child, with at most C leaves, of a node with more than C (or the
// whole tree when it has at most C leaves).  Above the cut lie the "top"
// nodes, one fewer than the subtrees.  Both sets are fixed by the topology and
// listed once, when the tree is built, with the two children of every top node
// (a top node or a subtree).
//
// A finished node hands its parent a 12-float summary: its box, the unit
// direction d of the area-weighted normal sum of the faces below it, the sum's
// length, and the slab [a, b] of d.x over those faces.
//
// The schedule is level-synchronous.  Each thread owns fixed internal nodes;
// at set-up it gathers the primitives of its nodes' leaf children, writes them
// into the nodes' records, finishes a node over two leaves and parks a lone
// leaf child's summary in its parent's LDS slot.  Then, step by step, each
// thread joins one of its nodes whose internal children are finished (their
// summaries from LDS slots), writes its record and its own slot and marks it
// done; a workgroup barrier ends each step.  With one node per thread a node
// of height h finishes in step h - 2, so a subtree takes about as many steps
// as it is high, with no atomics and no waiting beyond the barriers.
//
// Phase 1 (a workgroup per subtree): a Karras node covers a contiguous leaf
// range and its index is one end of that range, so the internal nodes of a
// subtree over leaves [f, l] have indices in [f, l] (the one other index in
// that range, if any, is a top node) and their slots live in LDS.  The
// subtree root's summary goes into its parent's record and, with device-scope
// stores, to a deposit for phase 2.  Phase 2 (one workgroup) runs the same
// steps over the top nodes, whose subtree children's summaries are the
// deposits.  The plain refit runs it in the workgroup that finishes the last
// subtree (an arrival counter in the BVH header), the batched kernel as a work
// item of its own.
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
    const int32_t *child;         // [2][n-1] child references of the internal nodes
    const int32_t *node_aux;      // [n-1] top index of a top node, -1 below the cut
    const int32_t *top_nodes;     // [T] node id of each top node
    const int32_t *top_child;     // [4][n]: per top node and slot, the child's top index,
                                  // or ~k for subtree k; then a top child's node id
    const int32_t *subtrees;      // [3][n]: root reference, first leaf, last leaf
    float4 *deposit;              // [n_sub][3] subtree-root summaries (device-coherent)
    float4 *top_scratch;          // [tstride][3] summary slots, then uint32 [tstride]
    int64_t tstride;              // done words: phase-2 state when T exceeds the LDS capacity
    float *root;                  // root box: lo at [0..2], hi at [4..6]
    int32_t *status;              // error word
    const int32_t *hdr_nv;        // vertex count of the build (header), or nullptr
    const int32_t *n_top;         // number of top nodes (device)
    const int32_t *n_sub;         // number of subtrees (device)
    uint32_t *arrivals;           // subtrees finished in this launch (plain refit)
    int64_t n;
    int chunk_log2;
    float inf;                    // +infinity, set at run time (see box_min)
};

// The summary a finished node hands to its parent.
struct Sum {
    f3 lo, hi;                    // box
    f3 d;                         // unit normal direction (zero: none)
    float sn;                     // length of the area-weighted normal sum
    float a, b;                   // slab: a <= d.x <= b over the faces below
};

// LDS of the two phases: a 48-byte summary slot and a done byte per node, and
// the step loop's finish word.
constexpr int kTopCap = 1024;     // top nodes the plain refit keeps in LDS (more: global scratch)

constexpr size_t refit_sub_lds(int64_t C) { return static_cast<size_t>(C) * 49 + 16; }
constexpr size_t refit_top_lds(int64_t T) { return static_cast<size_t>(T) * 49 + 16; }
// LDS of the plain refit kernel: a subtree's slots, and room for kTopCap top
// nodes in the workgroup that refits the top.
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

// Box union by the three-input median with an infinite third operand: one
// instruction per coordinate, where the two-input min and max first quiet a
// possible signalling NaN of each operand loaded from LDS (two more).  inf is
// passed in at run time: with a literal infinity the compiler turns the median
// back into min and max.  Box coordinates are finite and never -0 (leaf boxes
// add +0), where both forms give the same result.
__device__ __forceinline__ f3 box_min(f3 a, f3 b, float inf) {
    return f3{__builtin_amdgcn_fmed3f(a.x, b.x, -inf), __builtin_amdgcn_fmed3f(a.y, b.y, -inf),
              __builtin_amdgcn_fmed3f(a.z, b.z, -inf)};
}
__device__ __forceinline__ f3 box_max(f3 a, f3 b, float inf) {
    return f3{__builtin_amdgcn_fmed3f(a.x, b.x, inf), __builtin_amdgcn_fmed3f(a.y, b.y, inf),
              __builtin_amdgcn_fmed3f(a.z, b.z, inf)};
}

// The summary of a node from its children's, in slot order.
template <bool kTri>
__device__ __forceinline__ Sum join(const Sum &L, const Sum &R, float inf) {
#pragma clang fp contract(off)
    Sum P;
    P.lo = box_min(L.lo, R.lo, inf);
    P.hi = box_max(L.hi, R.hi, inf);
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

// Device-scope stores and loads of a deposited summary (six 64-bit words, the
// float pairs of its three float4 (lo, sn) (hi, a) (d, b)): visible to a
// workgroup on another XCD without a write-back of this XCD's L2.  The storing
// thread waits for its stores to complete before its workgroup signals arrival.
__device__ __forceinline__ uint64_t pack2(float x, float y) {
    return static_cast<uint64_t>(__float_as_uint(x)) | (static_cast<uint64_t>(__float_as_uint(y)) << 32);
}
__device__ __forceinline__ float lo32(uint64_t w) { return __uint_as_float(static_cast<uint32_t>(w)); }
__device__ __forceinline__ float hi32(uint64_t w) { return __uint_as_float(static_cast<uint32_t>(w >> 32)); }

__device__ __forceinline__ void deposit_store(float4 *dst, const Sum &S) {
    float4 v[3];
    pack(S, v);
    uint64_t *w = reinterpret_cast<uint64_t *>(dst);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        __hip_atomic_store(w + 2 * q, pack2(v[q].x, v[q].y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 2 * q + 1, pack2(v[q].z, v[q].w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ void deposit_load_words(const float4 *src, uint64_t w[6]) {
    const uint64_t *p = reinterpret_cast<const uint64_t *>(src);
#pragma unroll
    for (int q = 0; q < 6; ++q) w[q] = __hip_atomic_load(p + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ Sum sum_of_words(const uint64_t w[6]) {
    return unpack(make_float4(lo32(w[0]), hi32(w[0]), lo32(w[1]), hi32(w[1])),
                  make_float4(lo32(w[2]), hi32(w[2]), lo32(w[3]), hi32(w[3])),
                  make_float4(lo32(w[4]), hi32(w[4]), lo32(w[5]), hi32(w[5])));
}
__device__ __forceinline__ Sum deposit_load(const float4 *src) {
    uint64_t w[6];
    deposit_load_words(src, w);
    return sum_of_words(w);
}

// ---------------------------------------------------------------- the steps
// Step loop bookkeeping.  A node's mark starts at kNotDone; finished in step s
// it becomes s + 1, and a parent in step s takes a child whose mark is at most
// s (a leaf or subtree child counts as 0): every slot is read only in a step
// after the one that wrote it, so the
// barrier between the steps orders all slot accesses and no slot needs a
// fence of its own.  The LDS barrier fences LDS alone: a fence of every
// address space would also wait for the record stores in flight (on CDNA,
// vector loads and stores share one counter).
//
// A thread joins at most one of its nodes per step (the first whose children
// are done), so a wave runs one join per step whatever the number of nodes per
// thread; a ready node then waits at most (nodes per thread - 1) steps, and a
// valid tree (at most 62 levels) finishes within 62 x 4 steps.
constexpr int kMaxSteps = 250;    // marks stay below kNotDone
constexpr uint8_t kNotDone = 0xff;

// Keeps the given values' loads ahead of this point: the step loops read all
// their marks in one LDS round trip instead of one per branch.  (No code is
// emitted.)
__device__ __forceinline__ void issued_before(int x, int y) { __asm__ volatile("" ::"v"(x), "v"(y)); }

__device__ __forceinline__ void lds_step_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void lds_slot_store(float4 *slot, const Sum &S) {
    float4 v[3];
    pack(S, v);
    slot[0] = v[0]; slot[1] = v[1]; slot[2] = v[2];
}
__device__ __forceinline__ Sum lds_slot_load(const float4 *slot) { return unpack(slot[0], slot[1], slot[2]); }

// The record of a leaf child: (v0, ~leaf) (v1, id) (v2, 0), or for a point
// (p, ~leaf) (p, id).
template <bool kTri>
__device__ __forceinline__ void write_leaf(float4 *rec, int64_t leaf, int32_t id, f3 x, f3 y, f3 z) {
    rec[0] = make_float4(x.x, x.y, x.z, __int_as_float(~static_cast<int32_t>(leaf)));
    rec[1] = make_float4(y.x, y.y, y.z, __int_as_float(id));
    if (kTri) rec[2] = make_float4(z.x, z.y, z.z, 0.0f);
}

// Gathers leaf li's primitive (its face's vertices, or the point) and its id.
template <bool kTri>
__device__ __forceinline__ void load_leaf(const RefitArgs &a, int64_t li, int32_t &id, f3 &x, f3 &y, f3 &z) {
    id = a.prim[li];
    if (kTri) {
        x = vload(a.verts, a.nv, a.leaf_faces[li]);
        y = vload(a.verts, a.nv, a.leaf_faces[a.n + li]);
        z = vload(a.verts, a.nv, a.leaf_faces[2 * a.n + li]);
    } else {
        x = y = z = vload(a.verts, a.nv, id);
    }
}

// Child reference of slot s of internal node i (>= 0 internal node, < 0 leaf ~i).
__device__ __forceinline__ int32_t child_ref(const RefitArgs &a, int64_t i, int s) {
    return a.child[s * (a.n - 1) + i];
}

// The subtree root's summary P: into its parent's record and the deposit, or
// the root box when the subtree is the whole tree.
template <bool kTri>
__device__ __forceinline__ void finish_subtree(const RefitArgs &a, int64_t k, int32_t r, int32_t rtag, const Sum &P) {
    if (rtag < 0) {
        write_root(a.root, P);
    } else if ((rtag >> 1) >= a.n - 1) {
        atomicOr(a.status, 4);
    } else {
        write_internal<kTri>(a.nodes + 6 * static_cast<int64_t>(rtag >> 1) + 3 * (rtag & 1), r, P);
        deposit_store(a.deposit + 3 * k, P);
    }
}

// Phase 1 for subtree k by a workgroup of kThreads threads, thread j owning
// the nodes f + j + u kThreads (u < kPer).  kThreads is a compile-time stride:
// blockDim would be reloaded from the dispatch packet, and that load's wait
// would also wait for the record stores in flight.  smem: refit_sub_lds(C)
// bytes.  The root's summary goes into its parent's record and deposit[k];
// returns after the workgroup's barrier.
template <bool kTri, int kThreads, int kPer>
__device__ void refit_subtree(const RefitArgs &a, int64_t k, unsigned char *smem) {
    const int C = 1 << a.chunk_log2;
    const int32_t r = a.subtrees[k];
    const int64_t f = a.subtrees[a.n + k], l = a.subtrees[2 * a.n + k];
    float4 *s_slot = reinterpret_cast<float4 *>(smem);                          // [C][3]
    uint8_t *s_done = reinterpret_cast<uint8_t *>(s_slot + 3 * C);             // [C]
    const int64_t size = l - f + 1;
    if (f < 0 || l >= a.n || size < 1 || size > C || size > static_cast<int64_t>(kThreads) * kPer ||
        (size > 1 && (r < f || r > l))) {
        if (threadIdx.x == 0) atomicOr(a.status, 4);
        __syncthreads();
        return;
    }
    if (k == 0 && threadIdx.x == 0 && a.hdr_nv && *a.hdr_nv != a.nv) atomicOr(a.status, 32);
    if (size == 1) {                  // one leaf: the whole tree, or a child of a top node
        if (threadIdx.x == 0) {
            if (r != ~static_cast<int32_t>(f)) {
                atomicOr(a.status, 4);
            } else {
                int32_t id;
                f3 x, y, z;
                load_leaf<kTri>(a, f, id, x, y, z);
                const int32_t tag = a.leaf_parent[f];
                const Sum S = leaf_sum<kTri>(x, y, z);
                if (tag < 0) {
                    write_root(a.root, S);
                } else if ((tag >> 1) >= a.n - 1) {
                    atomicOr(a.status, 4);
                } else {
                    write_leaf<kTri>(a.nodes + 6 * static_cast<int64_t>(tag >> 1) + 3 * (tag & 1), f, id, x, y, z);
                    deposit_store(a.deposit + 3 * k, S);
                }
            }
        }
        __syncthreads();
        return;
    }
    // set-up: the owned nodes' child references, then their leaf children's
    // primitives, written into the nodes' records.  A node with two leaf
    // children is finished here (mark 0); the summary of a lone leaf child waits
    // in its parent's own slot, which nothing else reads before the parent is
    // done.  The steps end when the root's mark is set.
    const int jr = static_cast<int>(r - f);
    int32_t nid[kPer], cref[kPer][2] = {};
    bool pend[kPer];
    int32_t rtag = -1;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t i = f + threadIdx.x + static_cast<int64_t>(u) * kThreads;
        nid[u] = -1;
        pend[u] = false;
        if (i > l || i >= a.n - 1) continue;
        if (a.node_aux[i] >= 0) continue;     // the one top node whose index lies in [f, l]
        nid[u] = static_cast<int32_t>(i);
        cref[u][0] = child_ref(a, i, 0);
        cref[u][1] = child_ref(a, i, 1);
        if (i == r) rtag = a.node_parent[i];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        if (nid[u] < 0) continue;
        const int j = static_cast<int>(nid[u] - f);
        const int32_t c0 = cref[u][0], c1 = cref[u][1];
        bool ok = true;
        if (c0 >= 0) ok = ok && c0 >= f && c0 <= l && c0 < a.n - 1 && c0 != nid[u];
        else ok = ok && ~static_cast<int64_t>(c0) >= f && ~static_cast<int64_t>(c0) <= l;
        if (c1 >= 0) ok = ok && c1 >= f && c1 <= l && c1 < a.n - 1 && c1 != nid[u];
        else ok = ok && ~static_cast<int64_t>(c1) >= f && ~static_cast<int64_t>(c1) <= l;
        if (!ok) {
            atomicOr(a.status, 4);
            nid[u] = -1;
            s_done[j] = kNotDone;
            continue;
        }
        Sum L[2];
        bool leaf[2] = {c0 < 0, c1 < 0};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!leaf[s]) continue;
            const int64_t li = ~static_cast<int64_t>(s == 0 ? c0 : c1);
            int32_t id;
            f3 x, y, z;
            load_leaf<kTri>(a, li, id, x, y, z);
            write_leaf<kTri>(a.nodes + 6 * static_cast<int64_t>(nid[u]) + 3 * s, li, id, x, y, z);
            L[s] = leaf_sum<kTri>(x, y, z);
        }
        if (leaf[0] && leaf[1]) {
            const Sum P = join<kTri>(L[0], L[1], a.inf);
            if (nid[u] == r) finish_subtree<kTri>(a, k, r, rtag, P);   // a subtree of two leaves
            else lds_slot_store(s_slot + 3 * j, P);
            s_done[j] = 0;
        } else {
            if (leaf[0] || leaf[1]) lds_slot_store(s_slot + 3 * j, leaf[0] ? L[0] : L[1]);
            s_done[j] = kNotDone;
            pend[u] = true;
        }
    }
    // the slots each pending node reads: an internal child's, or its own for a
    // leaf child (whose summary waits there)
    int sj0[kPer], sj1[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = pend[u] ? static_cast<int>(nid[u] - f) : jr;
        sj0[u] = pend[u] && cref[u][0] >= 0 ? static_cast<int>(cref[u][0] - f) : j;
        sj1[u] = pend[u] && cref[u][1] >= 0 ? static_cast<int>(cref[u][1] - f) : j;
    }
    __syncthreads();
    // the exit test reads the root's mark only once it can no longer change in
    // the step being tested (a mark written in step s is s + 1): every thread
    // leaves after the same barrier
    for (int step = 0; step < kMaxSteps; ++step) {
        const int rm = s_done[jr];
        int d0[kPer], d1[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            d0[u] = s_done[sj0[u]];
            d1[u] = s_done[sj1[u]];
            issued_before(d0[u], d1[u]);
        }
        if (rm <= step) break;
        int su = -1;      // a leaf child is always done
#pragma unroll
        for (int u = kPer - 1; u >= 0; --u)
            if (pend[u] && (cref[u][0] < 0 || d0[u] <= step) && (cref[u][1] < 0 || d1[u] <= step)) su = u;
        if (su >= 0) {
            int32_t id = nid[0], c0 = cref[0][0], c1 = cref[0][1];
            int j0 = sj0[0], j1 = sj1[0];
#pragma unroll
            for (int u = 1; u < kPer; ++u)
                if (su == u) { id = nid[u]; c0 = cref[u][0]; c1 = cref[u][1]; j0 = sj0[u]; j1 = sj1[u]; }
#pragma unroll
            for (int u = 0; u < kPer; ++u)
                if (su == u) pend[u] = false;
            const int j = static_cast<int>(id - f);
            const Sum A = lds_slot_load(s_slot + 3 * j0);
            const Sum B = lds_slot_load(s_slot + 3 * j1);
            float4 *rec = a.nodes + 6 * static_cast<int64_t>(id);
            if (c0 >= 0) write_internal<kTri>(rec, c0, A);
            if (c1 >= 0) write_internal<kTri>(rec + 3, c1, B);
            const Sum P = join<kTri>(A, B, a.inf);
            if (id == r) finish_subtree<kTri>(a, k, r, rtag, P);
            else lds_slot_store(s_slot + 3 * j, P);
            s_done[j] = static_cast<uint8_t>(step + 1);
        }
        lds_step_barrier();
    }
    if (threadIdx.x == 0 && s_done[jr] == kNotDone) atomicOr(a.status, 4);   // the root never became ready
    __syncthreads();
}

// Phase 2 over T top nodes and NS subtrees by one workgroup of kThreads, thread
// j owning top nodes j + u kThreads (u < kTPer; T <= kTPer kThreads), in LDS
// (refit_top_lds(T) bytes of smem).  A top node's subtree children's summaries
// are the deposits, read at set-up (as the subtree phase's leaves: a node with
// two is finished there, a lone one waits in the node's own slot); the root
// (node 0) writes the root box.
template <bool kTri, int kThreads, int kTPer>
__device__ void refit_top_lds_steps(const RefitArgs &a, int T, int NS, unsigned char *smem) {
    float4 *t_slot = reinterpret_cast<float4 *>(smem);                          // [T][3]
    uint8_t *t_done = reinterpret_cast<uint8_t *>(t_slot + 3 * T);             // [T]
    int *t_fin = reinterpret_cast<int *>(t_done + ((T + 3) & ~3));           // the root's mark (its owner's)
    int32_t pn[kTPer], ch[kTPer][2] = {}, cn[kTPer][2] = {};
    bool pend[kTPer];
    // the tables are read for every slot up to the cap at once (one round trip,
    // T arriving with them); slots from T on are ignored
#pragma unroll
    for (int u = 0; u < kTPer; ++u) {
        const int t = threadIdx.x + u * kThreads;
        pend[u] = false;
        pn[u] = -1;
        if (t >= a.n) continue;
        pn[u] = a.top_nodes[t];
        ch[u][0] = a.top_child[t];
        ch[u][1] = a.top_child[a.n + t];
        cn[u][0] = a.top_child[2 * a.n + t];
        cn[u][1] = a.top_child[3 * a.n + t];
    }
#pragma unroll
    for (int u = 0; u < kTPer; ++u)
        if (threadIdx.x + u * kThreads < T && pn[u] == 0) *t_fin = kNotDone;
    // every subtree child's deposited summary, all loads in flight together
    // (deposit 0 stands in where a slot has no subtree child)
    uint64_t dw[kTPer][2][6];
#pragma unroll
    for (int u = 0; u < kTPer; ++u)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int32_t c = ch[u][s2];
            const bool sub = threadIdx.x + u * kThreads < T && c < 0 && ~c < NS;
            deposit_load_words(a.deposit + 3 * (sub ? ~c : 0), dw[u][s2]);
        }
#pragma unroll
    for (int u = 0; u < kTPer; ++u) {
        const int t = threadIdx.x + u * kThreads;
        if (t >= T) continue;
        const int32_t c0 = ch[u][0], c1 = ch[u][1];
        const bool ok = pn[u] >= 0 && pn[u] < a.n - 1 && (c0 >= 0 ? c0 < T && c0 != t : ~c0 < NS) &&
                        (c1 >= 0 ? c1 < T && c1 != t : ~c1 < NS);
        if (!ok) {
            atomicOr(a.status, 8);
            t_done[t] = kNotDone;
            continue;
        }
        if (c0 < 0 && c1 < 0) {
            const Sum P = join<kTri>(sum_of_words(dw[u][0]), sum_of_words(dw[u][1]), a.inf);
            if (pn[u] == 0) {             // the root over two subtrees
                write_root(a.root, P);
                *t_fin = 0;
            } else {
                lds_slot_store(t_slot + 3 * t, P);
            }
            t_done[t] = 0;
        } else {
            if (c0 < 0 || c1 < 0) lds_slot_store(t_slot + 3 * t, sum_of_words(dw[u][c0 < 0 ? 0 : 1]));
            t_done[t] = kNotDone;
            pend[u] = true;
        }
    }
    // the slots each pending node reads: a top child's, or its own for a lone
    // subtree child (whose summary waits there)
    int sj0[kTPer], sj1[kTPer];
#pragma unroll
    for (int u = 0; u < kTPer; ++u) {
        const int t = pend[u] ? static_cast<int>(threadIdx.x) + u * kThreads : 0;
        sj0[u] = pend[u] && ch[u][0] >= 0 ? ch[u][0] : t;
        sj1[u] = pend[u] && ch[u][1] >= 0 ? ch[u][1] : t;
    }
    __syncthreads();
    for (int step = 0; step < kMaxSteps; ++step) {   // as in the subtree phase
        const int rm = *t_fin;
        int d0[kTPer], d1[kTPer];
#pragma unroll
        for (int u = 0; u < kTPer; ++u) {
            d0[u] = t_done[sj0[u]];
            d1[u] = t_done[sj1[u]];
            issued_before(d0[u], d1[u]);
        }
        if (rm <= step) break;
        int su = -1;      // a subtree child is always done
#pragma unroll
        for (int u = kTPer - 1; u >= 0; --u)
            if (pend[u] && (ch[u][0] < 0 || d0[u] <= step) && (ch[u][1] < 0 || d1[u] <= step)) su = u;
        if (su >= 0) {
            int32_t p = pn[0], c0 = ch[0][0], c1 = ch[0][1], n0 = cn[0][0], n1 = cn[0][1];
            int j0 = sj0[0], j1 = sj1[0], t = threadIdx.x;
#pragma unroll
            for (int u = 1; u < kTPer; ++u)
                if (su == u) {
                    p = pn[u]; c0 = ch[u][0]; c1 = ch[u][1]; n0 = cn[u][0]; n1 = cn[u][1];
                    j0 = sj0[u]; j1 = sj1[u]; t = threadIdx.x + u * kThreads;
                }
#pragma unroll
            for (int u = 0; u < kTPer; ++u)
                if (su == u) pend[u] = false;
            const Sum A = lds_slot_load(t_slot + 3 * j0);
            const Sum B = lds_slot_load(t_slot + 3 * j1);
            float4 *rec = a.nodes + 6 * static_cast<int64_t>(p);
            if (c0 >= 0) write_internal<kTri>(rec, n0, A);
            if (c1 >= 0) write_internal<kTri>(rec + 3, n1, B);
            const Sum P = join<kTri>(A, B, a.inf);
            if (p == 0) {                 // the root
                write_root(a.root, P);
                *t_fin = step + 1;
            } else {
                lds_slot_store(t_slot + 3 * t, P);
                t_done[t] = static_cast<uint8_t>(step + 1);
            }
        }
        lds_step_barrier();
    }
    if (threadIdx.x == 0 && *t_fin == kNotDone) atomicOr(a.status, 8);
    __syncthreads();
}

// Phase 2 with the slots and done words in global scratch (a.top_scratch), for
// top trees beyond the LDS: the same steps, each thread visiting the nodes
// j, j + kThreads, ... and reading their links again in every step (slow, but
// only very large trees take it).  Slots and marks use device-scope accesses.
template <bool kTri, int kThreads>
__device__ void refit_top_global_steps(const RefitArgs &a, int T, int NS, unsigned char *smem) {
    float4 *g_slot = a.top_scratch;                                             // [tstride][3]
    uint32_t *g_done = reinterpret_cast<uint32_t *>(g_slot + 3 * a.tstride);   // [tstride]
    int *t_fin = reinterpret_cast<int *>(smem);                 // the root's mark
    for (int t = threadIdx.x; t < T; t += kThreads)
        __hip_atomic_store(g_done + t, ~0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) *t_fin = kNotDone;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    auto mark = [&](int32_t c) -> uint32_t {
        return c >= 0 ? __hip_atomic_load(g_done + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    };
    for (int step = 0; step < kMaxSteps && *t_fin > step; ++step) {   // as in the subtree phase
        for (int t = threadIdx.x; t < T; t += kThreads) {
            if (__hip_atomic_load(g_done + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ~0u) continue;
            const int32_t c0 = a.top_child[t], c1 = a.top_child[a.n + t], p = a.top_nodes[t];
            if (c0 >= T || c1 >= T || (c0 < 0 && ~c0 >= NS) || (c1 < 0 && ~c1 >= NS) || p < 0 || p >= a.n - 1) {
                atomicOr(a.status, 8);
                continue;
            }
            const uint32_t d0 = mark(c0), d1 = mark(c1);
            if (d0 > static_cast<uint32_t>(step) || d1 > static_cast<uint32_t>(step)) continue;
            const Sum A = deposit_load(c0 >= 0 ? g_slot + 3 * c0 : a.deposit + 3 * ~c0);
            const Sum B = deposit_load(c1 >= 0 ? g_slot + 3 * c1 : a.deposit + 3 * ~c1);
            float4 *rec = a.nodes + 6 * static_cast<int64_t>(p);
            if (c0 >= 0) write_internal<kTri>(rec, a.top_nodes[c0], A);
            if (c1 >= 0) write_internal<kTri>(rec + 3, a.top_nodes[c1], B);
            const Sum P = join<kTri>(A, B, a.inf);
            if (p == 0) {
                write_root(a.root, P);
                *t_fin = step + 1;
            } else {
                deposit_store(g_slot + 3 * t, P);   // waits for its stores
                __hip_atomic_store(g_done + t, static_cast<uint32_t>(step + 1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if (threadIdx.x == 0 && *t_fin == kNotDone) atomicOr(a.status, 8);
    __syncthreads();
}

// Phase 2: in LDS when T fits kTPer nodes per thread (kGlobal false), else in
// global scratch.  The LDS form is run with the fewest nodes per thread that
// hold T (1, 2 or kTPer): every owned node costs its mark loads in every step.
template <bool kTri, int kThreads, bool kGlobal, int kTPer>
__device__ void refit_top(const RefitArgs &a, int T, int NS, unsigned char *smem) {
    constexpr int kTwo = kTPer < 2 ? kTPer : 2;
    if (kGlobal) {
        refit_top_global_steps<kTri, kThreads>(a, T, NS, smem);
    } else if (T > kTPer * kThreads) {
        if (threadIdx.x == 0) atomicOr(a.status, 8);
        __syncthreads();
    } else if (T <= kThreads) {
        refit_top_lds_steps<kTri, kThreads, 1>(a, T, NS, smem);
    } else if (T <= kTwo * kThreads) {
        refit_top_lds_steps<kTri, kThreads, kTwo>(a, T, NS, smem);
    } else {
        refit_top_lds_steps<kTri, kThreads, kTPer>(a, T, NS, smem);
    }
}

}  // namespace mgu
