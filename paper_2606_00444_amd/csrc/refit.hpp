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
// local index, an arrival counter, a box accumulator (order-preserving uint
// min/max) and the node's parent link in LDS; a leaf's thread writes the leaf's
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
// Boxes are exact (min/max only), so any schedule gives bitwise the same
// records.  Every index read from the buffer is range-checked; a corrupted
// buffer sets the error word instead of faulting or hanging.
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
    float *top_box;               // [2][6][tstride] deposited subtree-root boxes
    int64_t tstride;
    uint32_t *top_scratch;        // [11][tstride] phase-2 state when T exceeds the LDS capacity
    float *root;                  // root box: lo at [0..2], hi at [4..6]
    int32_t *status;              // error word
    const int32_t *n_top;         // number of top nodes (device)
    const int32_t *n_sub;         // number of subtrees (device)
    int64_t n;
    int chunk_log2;
};

constexpr int kTopLds = 1024;     // top nodes handled with LDS state in the plain refit

// LDS bytes of phase 1 for subtrees of up to C leaves, and of phase 2 for Tl
// top nodes (6 box planes, 2 child indices, node id, done and ready flags).
constexpr size_t refit_sub_lds(int64_t C) { return static_cast<size_t>(C) * 32; }
constexpr size_t refit_top_lds(int64_t Tl) { return static_cast<size_t>(Tl) * 44; }

__device__ __forceinline__ void write_root(float *root, f3 lo, f3 hi) {
    root[0] = lo.x; root[1] = lo.y; root[2] = lo.z;
    root[4] = hi.x; root[5] = hi.y; root[6] = hi.z;
}

__device__ __forceinline__ void lds_union(uint32_t *b, int64_t stride, int64_t j, f3 lo, f3 hi) {
    atomicMin(&b[0 * stride + j], f2ord(lo.x));
    atomicMin(&b[1 * stride + j], f2ord(lo.y));
    atomicMin(&b[2 * stride + j], f2ord(lo.z));
    atomicMax(&b[3 * stride + j], f2ord(hi.x));
    atomicMax(&b[4 * stride + j], f2ord(hi.y));
    atomicMax(&b[5 * stride + j], f2ord(hi.z));
}

__device__ __forceinline__ void lds_read(const uint32_t *b, int64_t stride, int64_t j, f3 &lo, f3 &hi) {
    lo = f3{ord2f(b[0 * stride + j]), ord2f(b[1 * stride + j]), ord2f(b[2 * stride + j])};
    hi = f3{ord2f(b[3 * stride + j]), ord2f(b[4 * stride + j]), ord2f(b[5 * stride + j])};
}

__device__ __forceinline__ void lds_empty(uint32_t *b, int64_t stride, int64_t j) {
    const uint32_t e_lo = f2ord(INFINITY), e_hi = f2ord(-INFINITY);
    b[0 * stride + j] = e_lo; b[1 * stride + j] = e_lo; b[2 * stride + j] = e_lo;
    b[3 * stride + j] = e_hi; b[4 * stride + j] = e_hi; b[5 * stride + j] = e_hi;
}

// Deposit the box of a subtree root into slot `slot` of its top parent p.
__device__ __forceinline__ void deposit(const RefitArgs &a, int32_t p, int slot, f3 lo, f3 hi) {
    const int32_t t = a.node_aux[p];
    if (t < 0 || t >= a.tstride) { atomicOr(a.status, 8); return; }
    float *b = a.top_box + static_cast<int64_t>(slot) * 6 * a.tstride + t;
    b[0] = lo.x; b[a.tstride] = lo.y; b[2 * a.tstride] = lo.z;
    b[3 * a.tstride] = hi.x; b[4 * a.tstride] = hi.y; b[5 * a.tstride] = hi.z;
}

// Phase 1 for subtree k by a workgroup of kThreads threads (a compile-time
// stride: blockDim would be reloaded from the dispatch packet, and that load's
// wait would also wait for the record stores in flight).  smem:
// refit_sub_lds(C) bytes.
template <bool kTri, int kThreads>
__device__ void refit_subtree(const RefitArgs &a, int64_t k, unsigned char *smem) {
    const int64_t C = int64_t(1) << a.chunk_log2;
    const int32_t r = a.subtrees[k];
    const int64_t f = a.subtrees[a.n + k], l = a.subtrees[2 * a.n + k];
    uint32_t *s_box = reinterpret_cast<uint32_t *>(smem);          // [6][C]
    uint32_t *s_cnt = s_box + 6 * C;                               // [C]
    int32_t *s_par = reinterpret_cast<int32_t *>(s_cnt + C);       // [C]
    const int64_t size = l - f + 1;
    if (f < 0 || l >= a.n || size < 1 || size > C) {
        if (threadIdx.x == 0) atomicOr(a.status, 4);
        return;
    }
    for (int64_t j = threadIdx.x; j < size; j += kThreads) {
        s_cnt[j] = 0;
        lds_empty(s_box, C, j);
        s_par[j] = f + j < a.n - 1 ? a.node_parent[f + j] : -1;
    }
    __syncthreads();
    for (int64_t i = f + threadIdx.x; i <= l; i += kThreads) {
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
        const int32_t tag = a.leaf_parent[i];
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
            deposit(a, p, slot, lo, hi);
            continue;
        }
        // a valid tree is at most 62 levels deep
        for (int level = 0; level < 64; ++level) {
            const int64_t j = p - f;
            if (j < 0 || j >= size) { atomicOr(a.status, 4); break; }
            lds_union(s_box, C, j, lo, hi);
            const uint32_t old = __hip_atomic_fetch_add(&s_cnt[j], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;                  // the sibling finishes node p
            lds_read(s_box, C, j, lo, hi);
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
            rec[0] = make_float4(lo.x, lo.y, lo.z, __int_as_float(c));
            rec[1] = make_float4(hi.x, hi.y, hi.z, 0.0f);
            if (c == r) {
                deposit(a, p, slot, lo, hi);
                break;
            }
        }
    }
}

// Phase 2 over T top nodes with state at st (stride planes of uint32: 6 box
// planes, 2 child planes, node id, done, ready), in LDS or global scratch;
// one workgroup of kThreads.  Returns after the root's box is written.
//
// While every thread owns at most kOwn nodes (T <= kOwn kThreads), a thread
// keeps its nodes' child indices, ids, boxes and flags in registers, so a
// round costs one LDS read of the children's flags and one of their boxes;
// larger T keep everything in the planes.
template <bool kTri, int kThreads>
__device__ void refit_top(const RefitArgs &a, int T, uint32_t *st, int64_t stride) {
    constexpr int kOwn = 4;
    __shared__ int s_root, s_root_done;
    uint32_t *bx = st;
    int32_t *ch = reinterpret_cast<int32_t *>(st + 6 * stride);
    int32_t *node = reinterpret_cast<int32_t *>(st + 8 * stride);
    uint32_t *done = st + 9 * stride;
    uint32_t *rdy = st + 10 * stride;
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
            const float *b = a.top_box + static_cast<int64_t>(s) * 6 * a.tstride + t;
            lo = fmin3(lo, f3{b[0], b[a.tstride], b[2 * a.tstride]});
            hi = fmax3(hi, f3{b[3 * a.tstride], b[4 * a.tstride], b[5 * a.tstride]});
        }
        bx[0 * stride + t] = f2ord(lo.x); bx[1 * stride + t] = f2ord(lo.y); bx[2 * stride + t] = f2ord(lo.z);
        bx[3 * stride + t] = f2ord(hi.x); bx[4 * stride + t] = f2ord(hi.y); bx[5 * stride + t] = f2ord(hi.z);
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
    // finish node t (its top children are done): union, records of its top children
    auto finish = [&](int t, int32_t pn, int32_t c0, int32_t c1, f3 lo, f3 hi) {
        const int32_t cs[2] = {c0, c1};
        for (int s = 0; s < 2; ++s) {
            const int32_t c = cs[s];
            if (c < 0) continue;
            f3 clo, chi;
            lds_read(bx, stride, c, clo, chi);
            lo = fmin3(lo, clo);
            hi = fmax3(hi, chi);
            float4 *rec = a.nodes + 6 * static_cast<int64_t>(pn) + 3 * s;
            rec[0] = make_float4(clo.x, clo.y, clo.z, __int_as_float(node[c]));
            rec[1] = make_float4(chi.x, chi.y, chi.z, 0.0f);
        }
        bx[0 * stride + t] = f2ord(lo.x); bx[1 * stride + t] = f2ord(lo.y); bx[2 * stride + t] = f2ord(lo.z);
        bx[3 * stride + t] = f2ord(hi.x); bx[4 * stride + t] = f2ord(hi.y); bx[5 * stride + t] = f2ord(hi.z);
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
