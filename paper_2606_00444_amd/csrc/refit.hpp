// LBVH refit bodies shared by the plain refit/build kernel and the batched
// persistent kernel.
//
// The tree is cut into subtrees of at most C = 2^chunk_log2 leaves: a subtree
// root is a child, with at most C leaves, of a node with more than C (or the
// whole tree when it has at most C leaves).  Above the cut lie the "top"
// nodes, one fewer than the subtrees.  Both sets are fixed by the topology and
// listed once, when the tree is built.
//
// Phase 1 (one workgroup per subtree): a Karras node covers a contiguous leaf
// range and its index is one end of that range, so the internal nodes of a
// subtree over leaves [f, l] have indices in [f, l].  The workgroup keeps, per
// local index, an arrival counter, a box accumulator (LDS float min/max
// atomics) and the node's parent link in LDS; a leaf's thread writes the leaf's
// record slot and climbs while it is the second arrival, so the climb reads
// only LDS.  The subtree root's box is deposited in its top parent's slot of
// the top-box table.
//
// Phase 2 (one workgroup, after phase 1 has finished): the top nodes are
// finished in rounds.  Each round, every node whose top children are done
// takes the union of its deposited subtree-root boxes and its top children's
// boxes, writes its top children's record slots, and is done; the rounds end
// when the root is.  Boxes, child indices and flags live in LDS (or in global
// scratch when there are more top nodes than fit).
//
// Triangle BVHs also carry a normal slab per internal child (see Slab below):
// a node's is formed from its two children's, in slot order, by the thread
// that finishes the node.  Boxes are exact (min/max only) and slabs are
// evaluated in a fixed order with contraction off, so any schedule gives
// bitwise the same records.  Every index read from the buffer is
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
    const int32_t *node_aux;      // top index of a top node, else -1
    const int32_t *top_nodes;     // [T] node id of each top node
    const int32_t *top_child;     // [2][n] top index of each child, -1 when it roots a subtree
    const int32_t *subtrees;      // [3][n_sub]: root reference, first leaf, last leaf
    float *top_box;               // [2][kTopBoxPlanes][tstride] deposited subtree roots: box, normal sum, slab
    int64_t tstride;
    uint32_t *top_scratch;        // [kTopStatePlanes][tstride] phase-2 state when T exceeds the LDS capacity
    float *root;                  // root box: lo at [0..2], hi at [4..6]
    int32_t *status;              // error word
    const int32_t *hdr_nv;        // vertex count of the build (header), or nullptr
    const int32_t *n_top;         // number of top nodes (device)
    const int32_t *n_sub;         // number of subtrees (device)
    int64_t n;
    int chunk_log2;
};

constexpr int kTopLds = 1024;     // top nodes handled with LDS state in the plain refit
constexpr int kTopBoxPlanes = 11; // per deposit slot: box (6), normal sum (3), slab (2)
constexpr int kTopStatePlanes = 26;

// LDS bytes of phase 1 for subtrees of up to C leaves (per local node: 6 box
// planes, arrival counter, parent link, and per child slot its normal sum and
// slab), and of phase 2 for Tl top nodes (6 box planes, 2 child indices, node
// id, done and ready flags, own normal sum and slab, and per slot the
// deposited subtree root's normal sum and slab).
constexpr size_t refit_sub_lds(int64_t C) { return static_cast<size_t>(C) * 72; }
constexpr size_t refit_top_lds(int64_t Tl) { return static_cast<size_t>(Tl) * 4 * kTopStatePlanes; }

// ------------------------------------------------------------- normal slabs
// An internal child slot of a triangle BVH stores, besides its box, a unit
// direction d (the normalised sum of the area-weighted normals of the faces
// below it, for the current vertices) and [a, b] with a <= d.x <= b for every
// point x of those faces; the distance from q to them is then at least
// max(a - d.q, d.q - b, 0).  A parent's [a, b] comes from its children's: with
// alpha = d.d_c and r = d - alpha d_c, d.x = alpha (d_c.x) + r.x, where the
// first term lies in alpha [a_c, b_c] and the second in the range of r.x over
// the parent's box (for a leaf child, [a_c, b_c] is its triangle's extent along
// its own normal); the result is intersected with the range of d.x over the
// box.  Every extent is widened by 2^-18 of the box's coordinate magnitudes,
// which covers the float32 rounding of these sums at every level.
struct Slab {
    f3 s;                         // unnormalised normal sum
    float a, b;
};

// Unit direction of a normal sum by the hardware reciprocal square root (any
// direction gives a valid slab, since the extents are taken along the stored
// one; |d| is 1 to about 2^-22, which the traversal's bound allows for).
// Sums too small to normalise safely give no direction.
__device__ __forceinline__ f3 slab_dir(f3 s) {
    const float l2 = fdot(s, s);
    const bool ok = l2 > 1e-30f && l2 < 1e30f;
    const float k = ok ? __builtin_amdgcn_rsqf(l2) : 0.0f;
    return k * s;
}

__device__ __forceinline__ float slab_margin(f3 lo, f3 hi) {
    return 0x1p-18f * (((fabsf(lo.x) + fabsf(hi.x)) + (fabsf(lo.y) + fabsf(hi.y))) + (fabsf(lo.z) + fabsf(hi.z)));
}

// [mn, mx] of r.x over the box [lo, hi].
__device__ __forceinline__ void box_range(f3 r, f3 lo, f3 hi, float &mn, float &mx) {
    mn = (fminf(r.x * lo.x, r.x * hi.x) + fminf(r.y * lo.y, r.y * hi.y)) + fminf(r.z * lo.z, r.z * hi.z);
    mx = (fmaxf(r.x * lo.x, r.x * hi.x) + fmaxf(r.y * lo.y, r.y * hi.y)) + fmaxf(r.z * lo.z, r.z * hi.z);
}

__device__ __forceinline__ Slab leaf_slab(f3 x, f3 y, f3 z, f3 lo, f3 hi) {
#pragma clang fp contract(off)
    Slab S;
    S.s = cross_rounded(y - x, z - x);
    const f3 d = slab_dir(S.s);
    const float px = fdot(d, x), py = fdot(d, y), pz = fdot(d, z);
    const float e = slab_margin(lo, hi);
    const bool none = d.x == 0.0f && d.y == 0.0f && d.z == 0.0f;
    S.a = none ? -INFINITY : fminf(fminf(px, py), pz) - e;
    S.b = none ? INFINITY : fmaxf(fmaxf(px, py), pz) + e;
    return S;
}

// Bound of d.x over a child (slab c, direction dc) inside the box [lo, hi];
// a child without a slab contributes the box's own range [ba, bb].
__device__ __forceinline__ void child_range(f3 d, const Slab &c, f3 dc, f3 lo, f3 hi, float ba, float bb,
                                            float &ca, float &cb) {
#pragma clang fp contract(off)
    const float al = fdot(d, dc);
    const f3 r = f3{fmaf(-al, dc.x, d.x), fmaf(-al, dc.y, d.y), fmaf(-al, dc.z, d.z)};
    float rmn, rmx;
    box_range(r, lo, hi, rmn, rmx);
    const bool pos = al >= 0.0f;
    const float lo_c = (pos ? al * c.a : al * c.b) + rmn;
    const float hi_c = (pos ? al * c.b : al * c.a) + rmx;
    const bool has = c.a > -INFINITY && c.b < INFINITY && (dc.x != 0.0f || dc.y != 0.0f || dc.z != 0.0f);
    ca = has ? lo_c : ba;
    cb = has ? hi_c : bb;
}

// The slab of a node with box [lo, hi] from its children's (slot order); d is
// its unit direction.
__device__ __forceinline__ Slab join_slab(const Slab &c0, const Slab &c1, f3 lo, f3 hi, f3 &d) {
#pragma clang fp contract(off)
    Slab P;
    P.s = c0.s + c1.s;
    d = slab_dir(P.s);
    float a, b;
    box_range(d, lo, hi, a, b);
    float a0, b0, a1, b1;
    child_range(d, c0, slab_dir(c0.s), lo, hi, a, b, a0, b0);
    child_range(d, c1, slab_dir(c1.s), lo, hi, a, b, a1, b1);
    const float e = slab_margin(lo, hi);
    const bool none = d.x == 0.0f && d.y == 0.0f && d.z == 0.0f;
    P.a = none ? -INFINITY : fmaxf(a, fminf(a0, a1)) - e;
    P.b = none ? INFINITY : fminf(b, fmaxf(b0, b1)) + e;
    return P;
}

// Record slot of an internal child: (lo, ref) (hi, a) (d, b); points carry no slab.
template <bool kTri>
__device__ __forceinline__ void write_internal(float4 *rec, int32_t ref, f3 lo, f3 hi, f3 d, const Slab &S) {
    rec[0] = make_float4(lo.x, lo.y, lo.z, __int_as_float(ref));
    if (kTri) {
        rec[1] = make_float4(hi.x, hi.y, hi.z, S.a);
        rec[2] = make_float4(d.x, d.y, d.z, S.b);
    } else {
        rec[1] = make_float4(hi.x, hi.y, hi.z, 0.0f);
    }
}

__device__ __forceinline__ void write_root(float *root, f3 lo, f3 hi) {
    root[0] = lo.x; root[1] = lo.y; root[2] = lo.z;
    root[4] = hi.x; root[5] = hi.y; root[6] = hi.z;
}

// Box accumulators in LDS: float min/max atomics (exact, so any order of
// arrival gives the same box).  The atomics compare -0 and +0 as equal and keep
// whichever came first, so zeros are made +0 (x + 0 in round-to-nearest) to
// keep the box bitwise independent of the arrival order.
__device__ __forceinline__ void lds_union(float *b, int stride, int j, f3 lo, f3 hi) {
    lo = f3{lo.x + 0.0f, lo.y + 0.0f, lo.z + 0.0f};
    hi = f3{hi.x + 0.0f, hi.y + 0.0f, hi.z + 0.0f};
    __hip_atomic_fetch_min(&b[0 * stride + j], lo.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_min(&b[1 * stride + j], lo.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_min(&b[2 * stride + j], lo.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_max(&b[3 * stride + j], hi.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_max(&b[4 * stride + j], hi.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_max(&b[5 * stride + j], hi.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_read(const float *b, int64_t stride, int64_t j, f3 &lo, f3 &hi) {
    lo = f3{b[0 * stride + j], b[1 * stride + j], b[2 * stride + j]};
    hi = f3{b[3 * stride + j], b[4 * stride + j], b[5 * stride + j]};
}

__device__ __forceinline__ void lds_write(float *b, int64_t stride, int64_t j, f3 lo, f3 hi) {
    b[0 * stride + j] = lo.x; b[1 * stride + j] = lo.y; b[2 * stride + j] = lo.z;
    b[3 * stride + j] = hi.x; b[4 * stride + j] = hi.y; b[5 * stride + j] = hi.z;
}

// Deposit the box, normal sum and slab of a subtree root into slot `slot` of
// its top parent p.
__device__ __forceinline__ void deposit(const RefitArgs &a, int32_t p, int slot, f3 lo, f3 hi, const Slab &S) {
    const int32_t t = a.node_aux[p];
    if (t < 0 || t >= a.tstride) { atomicOr(a.status, 8); return; }
    float *b = a.top_box + static_cast<int64_t>(slot) * kTopBoxPlanes * a.tstride + t;
    const int64_t ts = a.tstride;
    b[0] = lo.x; b[ts] = lo.y; b[2 * ts] = lo.z;
    b[3 * ts] = hi.x; b[4 * ts] = hi.y; b[5 * ts] = hi.z;
    b[6 * ts] = S.s.x; b[7 * ts] = S.s.y; b[8 * ts] = S.s.z;
    b[9 * ts] = S.a; b[10 * ts] = S.b;
}


// Phase 1 for subtree k by a workgroup of kThreads threads (a compile-time
// stride: blockDim would be reloaded from the dispatch packet, and that load's
// wait would also wait for the record stores in flight).  smem:
// refit_sub_lds(C) bytes.
template <bool kTri, int kThreads>
__device__ void refit_subtree(const RefitArgs &a, int64_t k, unsigned char *smem) {
    const int C = 1 << a.chunk_log2;
    const int32_t r = a.subtrees[k];
    const int64_t f = a.subtrees[a.n + k], l = a.subtrees[2 * a.n + k];
    float *s_box = reinterpret_cast<float *>(smem);                // [6][C]
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(s_box + 6 * C); // [C]
    int32_t *s_par = reinterpret_cast<int32_t *>(s_cnt + C);       // [C]
    float *s_dep = reinterpret_cast<float *>(s_par + C);           // [2 slots][5][C]: normal sum, slab
    const int64_t size = l - f + 1;
    if (f < 0 || l >= a.n || size < 1 || size > C) {
        if (threadIdx.x == 0) atomicOr(a.status, 4);
        return;
    }
    // A leaf's primitive, parent tag and vertices.  The first leaf of every
    // thread is loaded before the LDS set-up and its barrier, so the two rounds
    // of global loads overlap.
    struct Leaf {
        f3 x, y, z;
        int32_t id, tag;
    };
    auto load_leaf = [&](int64_t i) {
        Leaf L;
        L.id = a.prim[i];
        L.tag = a.leaf_parent[i];
        if (kTri) {
            L.x = vload(a.verts, a.nv, a.leaf_faces[i]);
            L.y = vload(a.verts, a.nv, a.leaf_faces[a.n + i]);
            L.z = vload(a.verts, a.nv, a.leaf_faces[2 * a.n + i]);
        } else {
            L.x = L.y = L.z = vload(a.verts, a.nv, L.id);
        }
        return L;
    };
    if (k == 0 && threadIdx.x == 0 && a.hdr_nv && *a.hdr_nv != a.nv) atomicOr(a.status, 32);
    const int64_t i0 = f + threadIdx.x;
    Leaf first{};
    if (i0 <= l) first = load_leaf(i0);
    for (int j = threadIdx.x; j < size; j += kThreads) {
        s_cnt[j] = 0;
        lds_write(s_box, C, j, f3{INFINITY, INFINITY, INFINITY}, f3{-INFINITY, -INFINITY, -INFINITY});
        s_par[j] = f + j < a.n - 1 ? a.node_parent[f + j] : -1;
    }
    __syncthreads();
    for (int64_t i = i0; i <= l; i += kThreads) {
        const Leaf L = i == i0 ? first : load_leaf(i);
        const int32_t id = L.id;
        const f3 x = L.x, y = L.y, z = L.z;
        f3 lo = fmin3(fmin3(x, y), z), hi = fmax3(fmax3(x, y), z);
        Slab S{f3{0.0f, 0.0f, 0.0f}, -INFINITY, INFINITY};
        if (kTri) S = leaf_slab(x, y, z, lo, hi);
        const int32_t tag = L.tag;
        if (tag < 0) {            // a single leaf is the root
            write_root(a.root, lo, hi);
            continue;
        }
        int32_t p = tag >> 1, slot = tag & 1;
        if (p >= a.n - 1) { atomicOr(a.status, 4); continue; }
        float4 *rec = a.nodes + 6 * static_cast<int64_t>(p) + 3 * slot;
        rec[0] = make_float4(x.x, x.y, x.z, __int_as_float(~static_cast<int32_t>(i)));
        rec[1] = make_float4(y.x, y.y, y.z, __int_as_float(id));
        if (kTri) rec[2] = make_float4(z.x, z.y, z.z, 0.0f);
        if (r == ~static_cast<int32_t>(i)) {      // a one-leaf subtree
            deposit(a, p, slot, lo, hi, S);
            continue;
        }
        // a valid tree is at most 62 levels deep
        for (int level = 0; level < 64; ++level) {
            const int64_t jl = p - f;
            if (jl < 0 || jl >= size) { atomicOr(a.status, 4); break; }
            const int j = static_cast<int>(jl);
            if (kTri) {
                float *dep = s_dep + slot * 5 * C + j;
                dep[0] = S.s.x; dep[C] = S.s.y; dep[2 * C] = S.s.z; dep[3 * C] = S.a; dep[4 * C] = S.b;
            }
            lds_union(s_box, C, j, lo, hi);
            const uint32_t old = __hip_atomic_fetch_add(&s_cnt[j], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;                  // the sibling finishes node p
            lds_read(s_box, C, j, lo, hi);
            f3 d = f3{0.0f, 0.0f, 0.0f};
            if (kTri) {
                Slab c0, c1;
                const float *d0 = s_dep + j, *d1 = s_dep + 5 * C + j;
                c0.s = f3{d0[0], d0[C], d0[2 * C]}; c0.a = d0[3 * C]; c0.b = d0[4 * C];
                c1.s = f3{d1[0], d1[C], d1[2 * C]}; c1.a = d1[3 * C]; c1.b = d1[4 * C];
                S = join_slab(c0, c1, lo, hi, d);
            }
            const int32_t c = p;
            const int32_t ptag = s_par[j];
            if (ptag < 0) {
                write_root(a.root, lo, hi);
                break;
            }
            p = ptag >> 1;
            slot = ptag & 1;
            if (p >= a.n - 1) { atomicOr(a.status, 4); break; }
            rec = a.nodes + 6 * static_cast<int64_t>(p) + 3 * slot;
            write_internal<kTri>(rec, c, lo, hi, d, S);
            if (c == r) {
                deposit(a, p, slot, lo, hi, S);
                break;
            }
        }
    }
}

// Phase 2 over T top nodes with state at st (stride planes of uint32: 6 box
// planes, 2 child planes, node id, done, ready, normal sum and slab (5), the
// two slots' deposited normal sums and slabs (10)), in LDS or global scratch;
// one workgroup of kThreads.  Returns after the root's box is written.
//
// While every thread owns at most kOwn nodes (T <= kOwn kThreads), a thread
// keeps its nodes' child indices, ids, boxes and flags in registers, so a
// round costs one LDS read of the children's flags and one of their boxes;
// larger T keep everything in the planes.  (kOwn stays small: every owned node
// carries a copy of the finishing code, and registers are scarce at 1024
// threads.)
template <bool kTri, int kThreads, int kOwn>
__device__ void refit_top(const RefitArgs &a, int T, uint32_t *st, int64_t stride) {
    __shared__ int s_root, s_root_done;
    float *bx = reinterpret_cast<float *>(st);
    int32_t *ch = reinterpret_cast<int32_t *>(st + 6 * stride);
    int32_t *node = reinterpret_cast<int32_t *>(st + 8 * stride);
    uint32_t *done = st + 9 * stride;
    uint32_t *rdy = st + 10 * stride;
    float *sl = reinterpret_cast<float *>(st + 11 * stride);      // [5][stride]: normal sum, a, b
    float *dp = reinterpret_cast<float *>(st + 16 * stride);      // [2][5][stride]: deposits
    if (threadIdx.x == 0) {
        s_root = -1;
        s_root_done = 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += kThreads) {
        f3 lo = f3{INFINITY, INFINITY, INFINITY}, hi = f3{-INFINITY, -INFINITY, -INFINITY};
        for (int s = 0; s < 2; ++s) {
            const int32_t c = a.top_child[s * a.n + t];
            ch[s * stride + t] = c;
            if (c >= 0) continue;                 // a top child: merged in a later round
            const float *b = a.top_box + static_cast<int64_t>(s) * kTopBoxPlanes * a.tstride + t;
            lo = fmin3(lo, f3{b[0], b[a.tstride], b[2 * a.tstride]});
            hi = fmax3(hi, f3{b[3 * a.tstride], b[4 * a.tstride], b[5 * a.tstride]});
            if (kTri)
                for (int q = 0; q < 5; ++q) dp[(s * 5 + q) * stride + t] = b[(6 + q) * a.tstride];
        }
        lds_write(bx, stride, t, lo, hi);
        done[t] = 0;
        const int32_t pn = a.top_nodes[t];
        node[t] = pn;
        if (pn == 0) s_root = t;
    }
    __syncthreads();
    if (s_root < 0) {
        if (threadIdx.x == 0) atomicOr(a.status, 8);
        return;
    }
    const int root = s_root;
    auto plane_slab = [&](const float *pl, int c) {
        Slab S;
        S.s = f3{pl[c], pl[stride + c], pl[2 * stride + c]};
        S.a = pl[3 * stride + c];
        S.b = pl[4 * stride + c];
        return S;
    };
    // finish node t (its top children are done): union, slab, records of its top children
    auto finish = [&](int t, int32_t pn, int32_t c0, int32_t c1, f3 lo, f3 hi) {
        const int32_t cs[2] = {c0, c1};
        f3 clo[2], chi[2];
        for (int s = 0; s < 2; ++s) {
            const int32_t c = cs[s];
            if (c < 0) continue;
            lds_read(bx, stride, c, clo[s], chi[s]);
            lo = fmin3(lo, clo[s]);
            hi = fmax3(hi, chi[s]);
        }
        if (kTri) {
            Slab cslab[2];
            for (int s = 0; s < 2; ++s) cslab[s] = cs[s] >= 0 ? plane_slab(sl, cs[s]) : plane_slab(dp + s * 5 * stride, t);
            f3 d;
            const Slab S = join_slab(cslab[0], cslab[1], lo, hi, d);
            sl[t] = S.s.x; sl[stride + t] = S.s.y; sl[2 * stride + t] = S.s.z;
            sl[3 * stride + t] = S.a; sl[4 * stride + t] = S.b;
            for (int s = 0; s < 2; ++s) {
                if (cs[s] < 0) continue;
                write_internal<true>(a.nodes + 6 * static_cast<int64_t>(pn) + 3 * s, node[cs[s]], clo[s], chi[s],
                                     slab_dir(cslab[s].s), cslab[s]);
            }
        } else {
            for (int s = 0; s < 2; ++s) {
                if (cs[s] < 0) continue;
                write_internal<false>(a.nodes + 6 * static_cast<int64_t>(pn) + 3 * s, node[cs[s]], clo[s], chi[s],
                                      f3{0.0f, 0.0f, 0.0f}, Slab{});
            }
        }
        lds_write(bx, stride, t, lo, hi);
        if (t == root) {
            write_root(a.root, lo, hi);
            s_root_done = 1;
        }
    };
    if (T <= kOwn * kThreads) {
        int32_t my_c0[kOwn], my_c1[kOwn], my_pn[kOwn];
        bool my_done[kOwn];
        f3 my_lo[kOwn], my_hi[kOwn];
#pragma unroll
        for (int u = 0; u < kOwn; ++u) {
            const int t = threadIdx.x + u * kThreads;
            my_done[u] = t >= T;
            my_c0[u] = my_c1[u] = -1;
            my_pn[u] = -1;
            if (t < T) {
                my_c0[u] = ch[t];
                my_c1[u] = ch[stride + t];
                my_pn[u] = node[t];
                lds_read(bx, stride, t, my_lo[u], my_hi[u]);
                if (my_c0[u] >= T || my_c1[u] >= T || my_pn[u] < 0 || my_pn[u] >= a.n - 1) {
                    atomicOr(a.status, 8);
                    my_done[u] = true;
                }
            }
        }
        // a valid top tree is at most 62 levels high: one level finishes per round
        for (int round = 0; round < 64; ++round) {
            bool go[kOwn];
#pragma unroll
            for (int u = 0; u < kOwn; ++u)
                go[u] = !my_done[u] && (my_c0[u] < 0 || done[my_c0[u]]) && (my_c1[u] < 0 || done[my_c1[u]]);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kOwn; ++u) {
                if (!go[u]) continue;
                const int t = threadIdx.x + u * kThreads;
                finish(t, my_pn[u], my_c0[u], my_c1[u], my_lo[u], my_hi[u]);
                my_done[u] = true;
                done[t] = 1;
            }
            __syncthreads();
            if (s_root_done) return;
        }
    } else {
        for (int round = 0; round < 64; ++round) {
            for (int t = threadIdx.x; t < T; t += kThreads) {
                uint32_t r = 0;
                if (!done[t]) {
                    const int32_t c0 = ch[t], c1 = ch[stride + t];
                    r = (c0 < 0 || (c0 < T && done[c0])) && (c1 < 0 || (c1 < T && done[c1]));
                }
                rdy[t] = r;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < T; t += kThreads) {
                if (!rdy[t]) continue;
                const int32_t pn = node[t];
                if (pn < 0 || pn >= a.n - 1) { atomicOr(a.status, 8); done[t] = 1; continue; }
                f3 lo, hi;
                lds_read(bx, stride, t, lo, hi);
                finish(t, pn, ch[t], ch[stride + t], lo, hi);
                done[t] = 1;
            }
            __syncthreads();
            if (s_root_done) return;
        }
    }
    if (threadIdx.x == 0) atomicOr(a.status, 8);   // the root never became ready
}

}  // namespace mgu
