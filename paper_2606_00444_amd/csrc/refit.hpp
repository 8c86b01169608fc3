// LBVH refit bodies shared by the plain refit/build kernels and the batched
// persistent kernel.
//
// Internal nodes of a Karras tree cover contiguous leaf ranges, so every node
// whose range lies inside one chunk of 2^chunk_log2 leaves is refit by the
// workgroup owning that chunk, with arrival counters in LDS (workgroup scope, no
// cross-XCD traffic).  The few "top" nodes whose range crosses a chunk boundary
// are then finished by one workgroup, again with LDS counters and LDS atomic
// min/max accumulators.  Boxes are exact (min/max only), so any schedule gives
// bitwise the same result.
#pragma once

#include "mgu_internal.hpp"

namespace mgu {

struct RefitArgs {
    const float *verts; int64_t nv;
    const int32_t *leaf_faces;    // [3][n] or nullptr for points
    const int32_t *prim;
    const int32_t *leaf_parent; const int32_t *node_parent;
    float4 *nodes;                // [n-1][6] records written by this refit
    const float4 *topo;           // records holding the child references (the BVH's own;
                                  // the same as nodes except for per-frame copies)
    const int32_t *node_aux; const int32_t *top_nodes;
    uint32_t *top_scratch;        // [7][n]: counts, then 6 box planes (large n_top only)
    float *root;                  // root box: lo at [0..2], hi at [4..6]
    int32_t *status;              // error word
    const int32_t *n_top;         // number of top nodes (device)
    int64_t n;
    int chunk_log2;
};

constexpr int kTopLds = 2048;     // top nodes handled with LDS accumulators

__device__ __forceinline__ void write_root(float *root, f3 lo, f3 hi) {
    root[0] = lo.x; root[1] = lo.y; root[2] = lo.z;
    root[4] = hi.x; root[5] = hi.y; root[6] = hi.z;
}

// Box of the child stored in a record slot: a leaf triangle's vertices or a
// box (internal children and points store lo/hi in the first two float4).
template <bool kTri>
__device__ __forceinline__ void slot_box(const float4 *slot, f3 &lo, f3 &hi) {
    const float4 f0 = slot[0], f1 = slot[1];
    const f3 a = f3{f0.x, f0.y, f0.z}, b = f3{f1.x, f1.y, f1.z};
    if (kTri && __float_as_int(f0.w) < 0) {
        const float4 f2 = slot[2];
        const f3 c = f3{f2.x, f2.y, f2.z};
        lo = fmin3(fmin3(a, b), c);
        hi = fmax3(fmax3(a, b), c);
    } else {
        lo = a;
        hi = b;
    }
}

// Phase 1: workgroup b owns leaves [b C, b C + C) and every internal node whose
// range lies inside them.  Arrival counters live in LDS (index node - b C: a
// local node is one end of its own range), so all synchronisation is at
// workgroup scope.  A climb stops at the first top node; its child's data is
// already in the top node's record for phase 2.
template <bool kTri>
__device__ void refit_chunk(const RefitArgs &a, int64_t chunk, uint32_t *s_cnt) {
    const int64_t C = int64_t(1) << a.chunk_log2;
    const int64_t base = chunk * C;
    const int64_t end = base + C < a.n ? base + C : a.n;
    for (int64_t k = threadIdx.x; k < C; k += blockDim.x) s_cnt[k] = 0;
    __syncthreads();
    for (int64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
        const int32_t id = a.prim[i];
        f3 x, y, z;
        if (kTri) {
            x = load3(a.verts, a.nv, a.leaf_faces[i]);
            y = load3(a.verts, a.nv, a.leaf_faces[a.n + i]);
            z = load3(a.verts, a.nv, a.leaf_faces[2 * a.n + i]);
        } else {
            x = y = z = load3(a.verts, a.nv, id);
        }
        f3 lo = fmin3(fmin3(x, y), z), hi = fmax3(fmax3(x, y), z);
        int32_t tag = a.leaf_parent[i];
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
        // a valid tree is at most 62 levels deep; the cap and range checks turn a
        // corrupted buffer into an error word instead of a fault or a hang
        for (int level = 0; level < 64; ++level) {
            if (p < base || p >= end || a.node_aux[p] >= 0) break;     // top node: phase 2
            const uint32_t old = __hip_atomic_fetch_add(&s_cnt[p - base], 1u, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            f3 slo, shi;
            slot_box<kTri>(a.nodes + 6 * static_cast<int64_t>(p) + 3 * (1 - slot), slo, shi);
            lo = fmin3(lo, slo);
            hi = fmax3(hi, shi);
            tag = a.node_parent[p];
            if (tag < 0) {
                write_root(a.root, lo, hi);
                break;
            }
            const int32_t c = p;
            p = tag >> 1;
            slot = tag & 1;
            if (p >= a.n - 1) { atomicOr(a.status, 4); break; }
            rec = a.nodes + 6 * static_cast<int64_t>(p) + 3 * slot;
            rec[0] = make_float4(lo.x, lo.y, lo.z, __int_as_float(c));
            rec[1] = make_float4(hi.x, hi.y, hi.z, 0.0f);
        }
    }
}

// Phase 2 body: cnt [T] and box planes bx[k * stride + t] either in LDS or in
// the BVH's scratch section; one workgroup, so workgroup scope suffices.
template <bool kTri>
__device__ void refit_top_body(const RefitArgs &a, int T, uint32_t *cnt, uint32_t *bx, int64_t stride) {
    constexpr uint32_t kReady = 0x80000000u;
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        const int32_t p = a.top_nodes[t];
        f3 lo = f3{INFINITY, INFINITY, INFINITY}, hi = f3{-INFINITY, -INFINITY, -INFINITY};
        uint32_t count = 0;
        for (int slot = 0; slot < 2; ++slot) {
            const float4 *sl = a.nodes + 6 * static_cast<int64_t>(p) + 3 * slot;
            const int32_t ref = __float_as_int(a.topo[6 * static_cast<int64_t>(p) + 3 * slot].w);
            if (ref >= a.n - 1 || ~ref >= a.n) { atomicOr(a.status, 16); continue; }
            if (ref >= 0 && a.node_aux[ref] >= 0) continue;       // a top child arrives later
            f3 clo, chi;
            slot_box<kTri>(sl, clo, chi);
            lo = fmin3(lo, clo);
            hi = fmax3(hi, chi);
            ++count;
        }
        bx[0 * stride + t] = f2ord(lo.x); bx[1 * stride + t] = f2ord(lo.y); bx[2 * stride + t] = f2ord(lo.z);
        bx[3 * stride + t] = f2ord(hi.x); bx[4 * stride + t] = f2ord(hi.y); bx[5 * stride + t] = f2ord(hi.z);
        cnt[t] = count == 2 ? (kReady | 2u) : count;
    }
    __syncthreads();
    for (int t0 = threadIdx.x; t0 < T; t0 += blockDim.x) {
        if ((__hip_atomic_load(&cnt[t0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) & kReady) == 0) continue;
        int t = t0;
        for (int level = 0; level < 64; ++level) {
            const int32_t p = a.top_nodes[t];
            const f3 lo = f3{ord2f(bx[0 * stride + t]), ord2f(bx[1 * stride + t]), ord2f(bx[2 * stride + t])};
            const f3 hi = f3{ord2f(bx[3 * stride + t]), ord2f(bx[4 * stride + t]), ord2f(bx[5 * stride + t])};
            const int32_t tag = a.node_parent[p];
            if (tag < 0) {
                write_root(a.root, lo, hi);
                break;
            }
            const int32_t pp = tag >> 1, slot = tag & 1;
            float4 *rec = a.nodes + 6 * static_cast<int64_t>(pp) + 3 * slot;
            rec[0] = make_float4(lo.x, lo.y, lo.z, __int_as_float(p));
            rec[1] = make_float4(hi.x, hi.y, hi.z, 0.0f);
            const int32_t tt = a.node_aux[pp];
            if (tt < 0 || tt >= T) { atomicOr(a.status, 8); break; }
            __hip_atomic_fetch_min(&bx[0 * stride + tt], f2ord(lo.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_min(&bx[1 * stride + tt], f2ord(lo.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_min(&bx[2 * stride + tt], f2ord(lo.z), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_max(&bx[3 * stride + tt], f2ord(hi.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_max(&bx[4 * stride + tt], f2ord(hi.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_max(&bx[5 * stride + tt], f2ord(hi.z), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint32_t old = __hip_atomic_fetch_add(&cnt[tt], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old != 1u) break;                                 // the sibling is still on its way
            t = tt;
        }
    }
}

}  // namespace mgu
