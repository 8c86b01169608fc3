// Linear BVH over triangles or points: build and refit (gfx950).
//
// The paper builds its collision structures once from the template faces and
// reuses them for every frame (Sec. 3.4, Initialization; O(N_v) per frame);
// the varying-topology baseline destroys and rebuilds them every frame
// (Sec. 4.1).  The BVH kind is not named by the paper; this is a linear BVH
// (Karras 2012) built entirely on the device:
//
//   init     clear build scratch (histograms, look-back words, counters)
//   bounds   per-axis min/max of s = (v0 + v1) + v2, block reduce + one
//            atomic per block on order-preserving uint encodings
//   morton   30-bit codes defined in IEEE binary32 (no contraction), fused
//            with the four 8-bit digit histograms of the radix sort
//   sort     4 passes of a stable LSD radix sort of (code, id): one kernel per
//            pass, tiles ranked with wave64 ballots (match masks over the 8
//            digit bits), global digit offsets by decoupled look-back
//   tree     Karras radix tree per internal node + leaf permutation of faces;
//            lists the subtrees of at most C leaves that cut the tree and the
//            "top" nodes above them, then lists each top node's two children
//   refit    one kernel: a workgroup per subtree refits it level by level
//            with summary slots in LDS, and the workgroup that finishes the
//            last subtree refits the top nodes from the deposited subtree
//            roots (see refit.hpp)
//
// Node records are child-centric (96 B: both children's boxes, or a leaf
// child's triangle itself) so a traversal step reads one record and a leaf
// test needs no further gathers.
#include <mutex>

#include "refit.hpp"
#include "repose.hpp"

namespace mgu {
namespace {

constexpr int kSortThreads = 256;          // 4 waves

// Keys per lane of a sort pass: about 256 tiles whatever the size (at least 2
// and at most 16 keys per lane), so small sorts still spread over the chip.
inline int sort_items_for(int64_t n) {
    int items = 2;
    while (items < 16 && int64_t(kSortThreads) * items * 256 < n) items <<= 1;
    return items;
}
constexpr uint32_t kFlagAgg = 1u << 30;    // look-back word: tile aggregate
constexpr uint32_t kFlagPrefix = 2u << 30; //                 inclusive prefix
constexpr uint32_t kValueMask = (1u << 30) - 1;
constexpr int kSpinLimit = 1 << 24;        // bounded waits: error word instead of a hang

constexpr int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

inline mg_lbvh_layout make_layout(int64_t n, int kind) {
    mg_lbvh_layout L{};
    const int64_t m = n > 0 ? n - 1 : 0;
    int64_t o = 0;
    L.off_header = o;      o += align256(sizeof(mg_lbvh_header));
    L.off_codes = o;       o += align256(4 * n);
    L.off_prim = o;        o += align256(4 * n);
    L.off_leaf_faces = o;  o += align256(kind == MG_PRIM_TRIANGLES ? 12 * n : 0);
    L.off_leaf_parent = o; o += align256(4 * n);
    L.off_node_parent = o; o += align256(4 * m);
    L.off_nodes = o;       o += align256(96 * m);
    L.off_node_aux = o;    o += align256(4 * m);
    L.off_child = o;       o += align256(8 * m);
    L.off_top_nodes = o;   o += align256(4 * n);
    L.off_top_child = o;   o += align256(16 * n);
    L.off_subtrees = o;    o += align256(12 * n);
    L.off_deposits = o;    o += align256(48 * n);
    L.off_top_scratch = o; o += align256(52 * n);
    L.off_inv_prim = o;    o += align256(4 * n);
    L.total_bytes = o;
    return L;
}

// Largest subtree C = 2^chunk_log2 leaves: the smallest power of two >= 256
// with n <= 512 C (a few hundred subtrees, so the top tree stays small),
// capped at 2048 (the phase-1 LDS state is 52 B per leaf).
inline int chunk_log2_for(int64_t n) {
    int c = 8;
    while ((int64_t(512) << c) < n && c < 11) ++c;
    return c;
}

struct WsLayout {
    int64_t keys_a, vals_a, keys_b, vals_b, hist, lookback, total;
    int64_t tiles;
};

inline WsLayout make_ws(int64_t n) {
    WsLayout W{};
    const int64_t tile = int64_t(kSortThreads) * sort_items_for(n);
    W.tiles = (n + tile - 1) / tile;
    int64_t o = 0;
    W.keys_a = o;   o += align256(4 * n);
    W.vals_a = o;   o += align256(4 * n);
    W.keys_b = o;   o += align256(4 * n);
    W.vals_b = o;   o += align256(4 * n);
    W.hist = o;     o += align256(4 * 4 * 256);
    W.lookback = o; o += align256(4 * 4 * 256 * W.tiles);
    W.total = o;
    return W;
}

template <typename T>
inline T *at(void *base, int64_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

// ------------------------------------------------------------------ kernels

__global__ void build_init_kernel(mg_lbvh_header *hdr, uint32_t *hist, uint32_t *lookback,
                                  int64_t n_lookback, int n, int nv, int kind, int chunk_log2) {
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    if (hist != nullptr)          // no sort scratch when there are no primitives
        for (int64_t i = tid; i < 4 * 256; i += stride) hist[i] = 0;
    if (lookback != nullptr)
        for (int64_t i = tid; i < n_lookback; i += stride) lookback[i] = 0;
    if (tid == 0) {
        hdr->n_prims = n;
        hdr->n_verts = nv;
        hdr->prim_kind = kind;
        hdr->status = 0;
        for (int k = 0; k < 3; ++k) {
            hdr->bounds_enc[k] = 0xffffffffu;   // running min
            hdr->bounds_enc[3 + k] = 0u;        // running max
        }
        for (int k = 0; k < 4; ++k) hdr->tile_counter[k] = 0;
        hdr->refit_arrivals = 0u;
        hdr->chunk_log2 = chunk_log2;
        hdr->n_top = 0;
        hdr->n_sub = 0;
    }
}

// s = (v0 + v1) + v2 for face i (three times its centroid), or the point itself.
// Every operation is a separately rounded binary32 add.
__device__ __forceinline__ f3 centroid_sum(const float *__restrict__ v, int64_t nv,
                                           const int32_t *__restrict__ faces, int64_t n, int64_t i) {
    if (faces == nullptr) return load3(v, nv, i);
    const f3 a = load3(v, nv, faces[i]);
    const f3 b = load3(v, nv, faces[n + i]);
    const f3 c = load3(v, nv, faces[2 * n + i]);
    return (a + b) + c;
}

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

__global__ __launch_bounds__(256) void bounds_kernel(const float *__restrict__ v, int64_t nv,
                                                     const int32_t *__restrict__ faces, int64_t n,
                                                     mg_lbvh_header *hdr) {
    __shared__ float s_red[6][4];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const f3 s = centroid_sum(v, nv, faces, n, i);
        mn[0] = fminf(mn[0], s.x); mn[1] = fminf(mn[1], s.y); mn[2] = fminf(mn[2], s.z);
        mx[0] = fmaxf(mx[0], s.x); mx[1] = fmaxf(mx[1], s.y); mx[2] = fmaxf(mx[2], s.z);
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mn[k] = wave_min(mn[k]);
        mx[k] = wave_max(mx[k]);
    }
    if (lane == 0)
        for (int k = 0; k < 3; ++k) { s_red[k][wave] = mn[k]; s_red[3 + k][wave] = mx[k]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float r = s_red[k][0];
        for (int w = 1; w < 4; ++w) r = k < 3 ? fminf(r, s_red[k][w]) : fmaxf(r, s_red[k][w]);
        if (k < 3) atomicMin(&hdr->bounds_enc[k], f2ord(r));
        else atomicMax(&hdr->bounds_enc[k], f2ord(r));
    }
}

// Put bit i of a 10-bit value at bit 3 i (magic-number spreading).
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Quantisation defined in binary32: q = min(1023, trunc((s - lo) * scale)).
__device__ __forceinline__ uint32_t quant10(float s, float lo, float scale) {
#pragma clang fp contract(off)
    const float x = (s - lo) * scale;
    const uint32_t q = static_cast<uint32_t>(x);
    return q < 1023u ? q : 1023u;
}

__global__ __launch_bounds__(256) void morton_kernel(const float *__restrict__ v, int64_t nv,
                                                     const int32_t *__restrict__ faces, int64_t n,
                                                     mg_lbvh_header *hdr, uint32_t *__restrict__ keys,
                                                     uint32_t *__restrict__ hist) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_hist[4][256];
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&s_hist[0][0])[i] = 0;
    float lo[3], scale[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = ord2f(hdr->bounds_enc[k]);
        const float hi = ord2f(hdr->bounds_enc[3 + k]);
        // 1024 / (hi - lo) correctly rounded to binary32: the binary64 quotient of
        // two binary32 values rounds to the same binary32 as a direct division.
        const float ext = hi - lo[k];
        scale[k] = hi > lo[k] ? static_cast<float>(1024.0 / static_cast<double>(ext)) : 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) { hdr->quant_lo[k] = lo[k]; hdr->quant_scale[k] = scale[k]; }
    }
    __syncthreads();
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const f3 s = centroid_sum(v, nv, faces, n, i);
        const uint32_t code = (spread10(quant10(s.x, lo[0], scale[0])) << 2) |
                              (spread10(quant10(s.y, lo[1], scale[1])) << 1) |
                              spread10(quant10(s.z, lo[2], scale[2]));
        keys[i] = code;
#pragma unroll
        for (int p = 0; p < 4; ++p) atomicAdd(&s_hist[p][(code >> (8 * p)) & 0xffu], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
        const uint32_t c = (&s_hist[0][0])[i];
        if (c) atomicAdd(hist + i, c);
    }
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t *s_tmp /*[4]*/,
                                                       uint32_t &total) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) s_tmp[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t t = s_tmp[w];
        if (w < wave) before += t;
        total += t;
    }
    __syncthreads();
    return before + inc - x;
}

// One stable LSD pass over digit (key >> shift) & 255 for tiles of
// kSortThreads * kItems keys.  vals_in == nullptr means the values are the
// input positions (first pass).
template <int kItems>
__global__ __launch_bounds__(kSortThreads) void radix_pass_kernel(
    const uint32_t *__restrict__ keys_in, const int32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, int32_t *__restrict__ vals_out, int64_t n, int shift,
    const uint32_t *__restrict__ hist, uint32_t *lookback, uint32_t *tile_counter, int32_t *status) {
    constexpr int kTile = kSortThreads * kItems;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave_cnt[4][256];
    __shared__ uint32_t s_digit_start[256];
    __shared__ uint32_t s_global[256];
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_keys[kTile];
    __shared__ int32_t s_vals[kTile];

    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (int i = tid; i < 4 * 256; i += kSortThreads) (&s_wave_cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * kTile;

    uint32_t key[kItems];
    int32_t val[kItems];
    uint32_t rank[kItems];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t idx = base + (static_cast<int64_t>(wave) * kItems + j) * kWave + lane;
        const bool valid = idx < n;
        key[j] = valid ? keys_in[idx] : 0u;
        val[j] = valid ? (vals_in ? vals_in[idx] : static_cast<int32_t>(idx)) : 0;
        const uint32_t d = (key[j] >> shift) & 0xffu;
        // lanes of this wave holding the same digit (match mask from 8 ballots)
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint64_t below = m & lt;
        const uint32_t prev = valid ? s_wave_cnt[wave][d] : 0u;
        rank[j] = prev + static_cast<uint32_t>(__popcll(below));
        if (valid && below == 0) s_wave_cnt[wave][d] = prev + static_cast<uint32_t>(__popcll(m));
    }
    __syncthreads();

    // per digit: counts of each wave -> exclusive offsets across waves
    const int d = tid;
    const uint32_t c0 = s_wave_cnt[0][d], c1 = s_wave_cnt[1][d], c2 = s_wave_cnt[2][d], c3 = s_wave_cnt[3][d];
    const uint32_t tile_cnt = c0 + c1 + c2 + c3;
    // publish this tile's aggregate as early as possible
    uint32_t *my_word = lookback + tile * 256 + d;
    __hip_atomic_store(my_word, (tile == 0 ? kFlagPrefix : kFlagAgg) | tile_cnt, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();   // every wave has read its counts before they are overwritten
    s_wave_cnt[0][d] = 0;
    s_wave_cnt[1][d] = c0;
    s_wave_cnt[2][d] = c0 + c1;
    s_wave_cnt[3][d] = c0 + c1 + c2;
    uint32_t tile_total;
    const uint32_t dstart = block_excl_scan256(tile_cnt, s_tmp, tile_total);
    s_digit_start[d] = dstart;
    uint32_t hist_total;
    const uint32_t dbase = block_excl_scan256(hist[d], s_tmp, hist_total);

    // decoupled look-back: sum the counts of digit d over all earlier tiles
    uint32_t excl = 0;
    if (tile > 0) {
        int64_t t = tile - 1;
        int spins = 0;
        while (true) {
            const uint32_t w = __hip_atomic_load(lookback + t * 256 + d, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if ((w & ~kValueMask) == 0) {
                if (++spins > kSpinLimit) {   // never expected: report instead of hanging
                    atomicOr(status, 1);
                    break;
                }
                continue;
            }
            excl += w & kValueMask;
            if (w & kFlagPrefix) break;
            --t;
        }
        __hip_atomic_store(my_word, kFlagPrefix | (excl + tile_cnt), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    s_global[d] = dbase + excl - dstart;
    __syncthreads();

    // scatter into the tile in digit order (stable), then write out coalesced
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t idx = base + (static_cast<int64_t>(wave) * kItems + j) * kWave + lane;
        if (idx < n) {
            const uint32_t dj = (key[j] >> shift) & 0xffu;
            const uint32_t pos = s_digit_start[dj] + s_wave_cnt[wave][dj] + rank[j];
            s_keys[pos] = key[j];
            s_vals[pos] = val[j];
        }
    }
    __syncthreads();
    const int64_t count = (n - base) < kTile ? (n - base) : kTile;
    for (int i = tid; i < count; i += kSortThreads) {
        const uint32_t k = s_keys[i];
        const uint32_t out = s_global[(k >> shift) & 0xffu] + i;
        if (out < static_cast<uint64_t>(n)) {
            keys_out[out] = k;
            vals_out[out] = s_vals[i];
        } else {
            atomicOr(status, 2);   // inconsistent histogram: never expected
        }
    }
}

// Internal node i (i < n - 1) and leaf i (i < n): Karras's range and split
// search; children's parent tags; leaf face permutation; counter reset.
__global__ __launch_bounds__(256) void hierarchy_kernel(const uint32_t *__restrict__ codes,
                                                        const int32_t *__restrict__ prim,
                                                        int32_t *__restrict__ inv_prim, int64_t n,
                                                        const int32_t *__restrict__ faces,
                                                        int32_t *__restrict__ leaf_faces,
                                                        int32_t *__restrict__ leaf_parent,
                                                        int32_t *__restrict__ node_parent,
                                                        int32_t *__restrict__ node_aux,
                                                        int32_t *__restrict__ child,
                                                        int32_t *__restrict__ top_nodes,
                                                        int32_t *__restrict__ subtrees,
                                                        float *__restrict__ nodes,
                                                        mg_lbvh_header *hdr, int chunk_log2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    {
        const int32_t p = prim[i];
        if (p >= 0 && p < n) inv_prim[p] = static_cast<int32_t>(i);
        else atomicOr(&hdr->status, 4);
    }
    if (faces) {
        const int32_t p = prim[i];
        leaf_faces[i] = faces[p];
        leaf_faces[n + i] = faces[n + p];
        leaf_faces[2 * n + i] = faces[2 * n + p];
    }
    if (n == 1) {
        leaf_parent[0] = -1;
        subtrees[0] = ~0;         // the one leaf is the one subtree
        subtrees[1] = 0;
        subtrees[2] = 0;
        hdr->n_sub = 1;
        return;
    }
    if (i >= n - 1) return;
    // The searches run in 32-bit indices (counts are below 2^30, so i + lmax d and
    // 2 l stay below 2^31) with shifts for the halvings.  Each step is a dependent
    // read of a code (about 0.3 us from L2 for the top nodes), which sets the
    // kernel's time: the top nodes' threads finish last.
    const int ni = static_cast<int>(n), ii = static_cast<int>(i);
    const uint32_t ci = codes[i];
    auto delta = [&](int jx) -> int {      // delta(i, jx) of Karras 2012; -1 outside [0, n)
        if (static_cast<uint32_t>(jx) >= static_cast<uint32_t>(ni)) return -1;
        const uint32_t cj = codes[jx];
        if (ci != cj) return __clz(static_cast<int>(ci ^ cj));
        return 32 + __clz(static_cast<int>(static_cast<uint32_t>(ii) ^ static_cast<uint32_t>(jx)));
    };
    const int d = (delta(ii + 1) - delta(ii - 1)) > 0 ? 1 : -1;
    const int dmin = delta(ii - d);
    int lmax = 2;
    while (lmax <= ni && delta(ii + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(ii + (l + t) * d) > dmin) l += t;
    const int dnode = delta(ii + l * d);
    int sp = 0;
    for (int k = 1;; ++k) {               // t = ceil(l / 2^k)
        const int t = static_cast<int>((static_cast<uint32_t>(l) + (1u << k) - 1u) >> k);
        if (delta(ii + (sp + t) * d) > dnode) sp += t;
        if (t <= 1) break;
    }
    const int64_t j = ii + l * d;
    const int64_t gamma = ii + sp * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    const int32_t tag_l = static_cast<int32_t>(i << 1), tag_r = static_cast<int32_t>((i << 1) | 1);
    if (lo == gamma) leaf_parent[gamma] = tag_l; else node_parent[gamma] = tag_l;
    if (hi == gamma + 1) leaf_parent[gamma + 1] = tag_r; else node_parent[gamma + 1] = tag_r;
    if (i == 0) node_parent[0] = -1;
    // child references live in the records' first .w word of each slot; the refit
    // rewrites the same values, so they are valid before any box exists
    const int32_t c0 = static_cast<int32_t>(lo == gamma ? ~gamma : gamma);
    const int32_t c1 = static_cast<int32_t>(hi == gamma + 1 ? ~(gamma + 1) : gamma + 1);
    nodes[24 * i + 3] = __int_as_float(c0);
    nodes[24 * i + 15] = __int_as_float(c1);
    child[i] = c0;
    child[n - 1 + i] = c1;
    // the cut: a node with more than C leaves is a top node, and each of its
    // children with at most C leaves roots a subtree (list order is irrelevant)
    const int64_t C = int64_t(1) << chunk_log2;
    if (hi - lo + 1 > C) {
        const int32_t t = static_cast<int32_t>(atomicAdd(reinterpret_cast<uint32_t *>(&hdr->n_top), 1u));
        top_nodes[t] = static_cast<int32_t>(i);
        node_aux[i] = t;
        const int64_t cf[2] = {lo, gamma + 1}, cl[2] = {gamma, hi};
        for (int c = 0; c < 2; ++c) {
            if (cl[c] - cf[c] + 1 > C) continue;
            const int32_t k = static_cast<int32_t>(atomicAdd(reinterpret_cast<uint32_t *>(&hdr->n_sub), 1u));
            const bool leaf = cl[c] == cf[c];
            subtrees[k] = static_cast<int32_t>(leaf ? ~cf[c] : (c == 0 ? gamma : gamma + 1));
            subtrees[n + k] = static_cast<int32_t>(cf[c]);
            subtrees[2 * n + k] = static_cast<int32_t>(cl[c]);
        }
    } else {
        node_aux[i] = -1;
        if (i == 0) {             // the whole tree is one subtree
            atomicAdd(reinterpret_cast<uint32_t *>(&hdr->n_sub), 1u);
            subtrees[0] = 0;
            subtrees[n] = 0;
            subtrees[2 * n] = static_cast<int32_t>(n - 1);
        }
    }
}

// Subtrees largest first.  Phase 1 of the refit gives subtree k to workgroup k
// (then k + grid, ...), and workgroups start in index order as compute units free
// up; when more subtrees than resident workgroups exist (LDS allows two per CU at
// 1024-leaf chunks, one at 2048), the late starters should be the small subtrees
// (longest-first list scheduling).  One workgroup sorts by (size descending, first
// leaf ascending), so the order is deterministic; more than kOrderMax subtrees keep
// their order.  The refit's records do not depend on the order.
constexpr int kOrderMax = 2048;
__global__ __launch_bounds__(1024) void order_subtrees_kernel(int32_t *__restrict__ subtrees, int64_t n,
                                                              const mg_lbvh_header *__restrict__ hdr) {
    __shared__ uint64_t s_key[kOrderMax];
    __shared__ int32_t s_val[3][kOrderMax];
    const int ns = hdr->n_sub;
    if (ns <= 1 || ns > kOrderMax) return;
    int P = 1;
    while (P < ns) P <<= 1;
    for (int i = threadIdx.x; i < P; i += 1024) {
        uint64_t key = ~0ull;                     // padding sorts last
        if (i < ns) {
            const int32_t r = subtrees[i], f = subtrees[n + i], l = subtrees[2 * n + i];
            const uint32_t size = static_cast<uint32_t>(l - f + 1) & 0xfffu;   // <= 2048 leaves
            key = (static_cast<uint64_t>(0xfffu - size) << 42) | (static_cast<uint64_t>(f & 0x3fffffff) << 11) |
                  static_cast<uint64_t>(i);
            s_val[0][i] = r; s_val[1][i] = f; s_val[2][i] = l;
        }
        s_key[i] = key;
    }
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < P; t += 1024) {
                const int o = t ^ j;
                if (o <= t) continue;
                const uint64_t a = s_key[t], b = s_key[o];
                if ((a > b) == ((t & k) == 0)) { s_key[t] = b; s_key[o] = a; }
            }
        }
    __syncthreads();
    for (int q = threadIdx.x; q < ns; q += 1024) {
        const int i = static_cast<int>(s_key[q] & 0x7ffu);
        subtrees[q] = s_val[0][i];
        subtrees[n + q] = s_val[1][i];
        subtrees[2 * n + q] = s_val[2][i];
    }
}

// The top children: per top node and slot, the child's top index, or ~k when
// the child is the root of subtree k (every top node has two children of
// these kinds), and in planes 2 and 3 a top child's node id (0 for a subtree).
__global__ __launch_bounds__(256) void top_child_kernel(const int32_t *__restrict__ node_aux,
                                                        const int32_t *__restrict__ top_nodes,
                                                        const int32_t *__restrict__ node_parent,
                                                        const int32_t *__restrict__ leaf_parent,
                                                        const int32_t *__restrict__ subtrees, int64_t n,
                                                        int32_t *__restrict__ top_child, mg_lbvh_header *hdr) {
    const int T = hdr->n_top, NS = hdr->n_sub;
    if (NS < 2) return;                       // a single subtree is the whole tree: no top
    // the parent tag of a top node or subtree root names its slot in a top node
    auto put = [&](int32_t tag, int32_t v, int32_t node) {
        if (tag < 0) return;                  // the root
        const int32_t p = tag >> 1;
        if (p >= n - 1) { atomicOr(&hdr->status, 8); return; }
        const int32_t t = node_aux[p];
        if (t < 0 || t >= T) { atomicOr(&hdr->status, 8); return; }
        top_child[(tag & 1) * n + t] = v;
        top_child[(2 + (tag & 1)) * n + t] = node;
    };
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
        const int32_t p = top_nodes[t];
        if (p < 0 || p >= n - 1) { atomicOr(&hdr->status, 8); continue; }
        put(node_parent[p], t, p);
    }
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NS; k += gridDim.x * blockDim.x) {
        const int32_t r = subtrees[k];
        const bool leaf = r < 0;
        const int64_t id = leaf ? ~static_cast<int64_t>(r) : r;
        if (id >= (leaf ? n : n - 1)) { atomicOr(&hdr->status, 8); continue; }
        put(leaf ? leaf_parent[id] : node_parent[id], ~k, 0);
    }
}

// The refit over workgroups block, block + nblocks, ...: each takes subtrees
// (kPer nodes per thread) and counts the subtrees it finished into the
// header's arrival word once their deposits are complete; the one that brings
// it to the number of subtrees refits the top nodes (then clears the word for
// the next refit).  smem: refit_lds_bytes(chunk_log2) bytes.
template <bool kTri, int kThreads, int kPer>
__device__ void refit_blocks(const RefitArgs &a, int64_t block, int64_t nblocks, unsigned char *smem) {
    __shared__ int s_last;
    const int32_t ns = *a.n_sub;
    int mine = 0;
    for (int64_t k = block; k < ns; k += nblocks) {
        refit_subtree<kTri, kThreads, kPer>(a, k, smem);     // ends with a barrier
        ++mine;
    }
    if (ns < 2 || mine == 0) return;          // one subtree is the whole tree: its root is written
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(a.arrivals, static_cast<uint32_t>(mine), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) + mine == static_cast<uint32_t>(ns);
    __syncthreads();
    if (!s_last) return;
    const int T = *a.n_top;
    static_assert(kTopCap % kThreads == 0, "the top nodes kept in LDS are dealt evenly");
    if (T < 1 || T >= a.n) {
        if (threadIdx.x == 0) atomicOr(a.status, 8);
    } else if (T <= kTopCap) {
        refit_top<kTri, kThreads, false, kTopCap / kThreads>(a, T, ns, smem);
    } else {
        refit_top<kTri, kThreads, true, 1>(a, T, ns, smem);
    }
    if (threadIdx.x == 0) __hip_atomic_store(a.arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool kTri, int kThreads, int kPer, int kMinWaves>
__global__ __launch_bounds__(kThreads, kMinWaves) void refit_kernel(RefitArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    refit_blocks<kTri, kThreads, kPer>(a, blockIdx.x, gridDim.x, smem);
}

// The frame update in one launch: workgroups [0, sub_blocks) refit (as
// refit_kernel), the next copy_blocks copy the frame into the live buffer,
// and the rest re-pose the Gaussians, gauss_tile each.  Every part reads the
// frame's vertices from the frame store, so none waits for another; the copy
// and re-pose workgroups, dispatched after the refit's, fill the compute units
// the refit leaves idle (its later subtrees and its one-workgroup top phase).
struct FrameWork {
    const float *src;          // frame k, [3][n_verts]
    float *live;               // [3][n_verts]
    int64_t n3;                // 3 n_verts
    int64_t copy_tile;         // floats per copy workgroup
    Inputs in;                 // re-pose inputs (verts = src)
    float *mean, *quat, *cov, *rot;
    int64_t gauss_tile;        // Gaussians per re-pose workgroup
    int64_t sub_blocks, copy_blocks;
};

template <int kThreads, int kPer, int kMinWaves>
__global__ __launch_bounds__(kThreads, kMinWaves) void frame_update_kernel(RefitArgs a, FrameWork w) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t b = blockIdx.x;
    if (b < w.sub_blocks) {
        refit_blocks<true, kThreads, kPer>(a, b, w.sub_blocks, smem);
        return;
    }
    if (b < w.sub_blocks + w.copy_blocks) {
        const int64_t i0 = (b - w.sub_blocks) * w.copy_tile;
        const int64_t i1 = i0 + w.copy_tile < w.n3 ? i0 + w.copy_tile : w.n3;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) w.live[i] = w.src[i];
        return;
    }
    const int64_t g0 = (b - w.sub_blocks - w.copy_blocks) * w.gauss_tile;
    const int64_t g1 = g0 + w.gauss_tile < w.in.ng ? g0 + w.gauss_tile : w.in.ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kThreads) repose_store(w.in, g, w.mean, w.quat, w.cov, w.rot);
}

template <bool kTri, int kThreads, int kPer, int kMinWaves>
mg_status launch_refit_t(const RefitArgs &a, int grid, hipStream_t s) {
    const size_t lds = refit_lds_bytes(a.chunk_log2);
    if (lds > 65536)    // beyond the default dynamic LDS limit (gfx950 has 160 KB per workgroup)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&refit_kernel<kTri, kThreads, kPer, kMinWaves>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    hipLaunchKernelGGL((refit_kernel<kTri, kThreads, kPer, kMinWaves>), dim3(grid), dim3(kThreads), lds, s, a);
    return launch_status();
}

// 512-thread workgroups: a thread per internal node of a subtree of up to 256
// or 512 leaves, and 2 or 4 nodes per thread for 1024- and 2048-leaf subtrees.
// Up to 1024 leaves three workgroups fit a CU beside each other (about 50 KB
// of LDS each, six waves per SIMD), so a tree of 500,000 faces has nearly all
// its subtrees resident at once.  256-leaf subtrees leave half the threads
// idle in phase 1, but phase 2 then holds up to 512 top nodes at one node per
// thread (a 40,000-face tree has 276: 24.5 us against 26.4 us with 256-thread
// workgroups, whose phase 2 needs two nodes per thread there).
template <bool kTri>
mg_status launch_refit_k(const RefitArgs &a, int grid, hipStream_t s) {
    if (a.chunk_log2 <= 9) return launch_refit_t<kTri, 512, 1, 6>(a, grid, s);
    if (a.chunk_log2 == 10) return launch_refit_t<kTri, 512, 2, 6>(a, grid, s);
    return launch_refit_t<kTri, 512, 4, 2>(a, grid, s);
}

mg_status check_kind(int32_t kind) {
    return (kind == MG_PRIM_TRIANGLES || kind == MG_PRIM_POINTS) ? MG_OK : MG_ERR_INVALID_ARGUMENT;
}

RefitArgs refit_args(const float *verts, int64_t nv, void *bvh, int64_t n, int kind) {
    const mg_lbvh_layout L = make_layout(n, kind);
    RefitArgs a;
    a.verts = verts; a.nv = nv;
    a.leaf_faces = kind == MG_PRIM_TRIANGLES ? at<int32_t>(bvh, L.off_leaf_faces) : nullptr;
    a.prim = at<int32_t>(bvh, L.off_prim);
    a.leaf_parent = at<int32_t>(bvh, L.off_leaf_parent);
    a.node_parent = at<int32_t>(bvh, L.off_node_parent);
    a.nodes = at<float4>(bvh, L.off_nodes);
    a.child = at<int32_t>(bvh, L.off_child);
    a.node_aux = at<int32_t>(bvh, L.off_node_aux);
    a.top_nodes = at<int32_t>(bvh, L.off_top_nodes);
    a.top_child = at<int32_t>(bvh, L.off_top_child);
    a.subtrees = at<int32_t>(bvh, L.off_subtrees);
    a.deposit = at<float4>(bvh, L.off_deposits);
    a.top_scratch = at<float4>(bvh, L.off_top_scratch);
    a.tstride = n;
    mg_lbvh_header *hdr = at<mg_lbvh_header>(bvh, L.off_header);
    a.root = hdr->root_lo;
    a.status = &hdr->status;
    a.hdr_nv = &hdr->n_verts;
    a.n_top = &hdr->n_top;
    a.n_sub = &hdr->n_sub;
    a.arrivals = &hdr->refit_arrivals;
    a.n = n;
    a.chunk_log2 = chunk_log2_for(n);
    a.inf = INFINITY;
    return a;
}

template <int kThreads, int kPer, int kMinWaves>
mg_status launch_frame_t(const RefitArgs &a, const FrameWork &w, int64_t grid, hipStream_t s) {
    const size_t lds = refit_lds_bytes(a.chunk_log2);
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&frame_update_kernel<kThreads, kPer, kMinWaves>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    hipLaunchKernelGGL((frame_update_kernel<kThreads, kPer, kMinWaves>), dim3(static_cast<unsigned>(grid)),
                       dim3(kThreads), lds, s, a, w);
    return launch_status();
}

mg_status launch_refit(const float *verts, int64_t nv, void *bvh, int64_t n, int kind, hipStream_t s) {
    const RefitArgs a = refit_args(verts, nv, bvh, n, kind);
    const int64_t C = int64_t(1) << a.chunk_log2;
    const int grid = static_cast<int>(std::min<int64_t>(2 * ((n + C - 1) / C), 65535));
    return kind == MG_PRIM_TRIANGLES ? launch_refit_k<true>(a, grid, s) : launch_refit_k<false>(a, grid, s);
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_lbvh_layout_query(int32_t n_prims, int32_t prim_kind, mg_lbvh_layout *out) {
    if (!out || bad_count(n_prims) || check_kind(prim_kind) != MG_OK) return MG_ERR_INVALID_ARGUMENT;
    *out = make_layout(n_prims, prim_kind);
    return MG_OK;
}

extern "C" mg_status mg_lbvh_workspace_size(int32_t n_prims, int32_t prim_kind, size_t *ws_bytes) {
    if (!ws_bytes || bad_count(n_prims) || check_kind(prim_kind) != MG_OK) return MG_ERR_INVALID_ARGUMENT;
    *ws_bytes = static_cast<size_t>(make_ws(n_prims).total);
    return MG_OK;
}

namespace mgu {
namespace {

mg_status build_into(const float *verts, int32_t n_verts, const int32_t *faces, int32_t n_prims,
                     int32_t prim_kind, void *bvh, size_t bvh_bytes, void *ws, size_t ws_bytes,
                     void *stream) {
    if (bad_count(n_verts) || bad_count(n_prims) || check_kind(prim_kind) != MG_OK)
        return MG_ERR_INVALID_ARGUMENT;
    if (prim_kind == MG_PRIM_TRIANGLES && n_prims > 0 && (!faces || n_verts == 0))
        return MG_ERR_INVALID_ARGUMENT;
    if (prim_kind == MG_PRIM_POINTS && (faces || n_verts != n_prims)) return MG_ERR_INVALID_ARGUMENT;
    if (!bvh) return MG_ERR_INVALID_ARGUMENT;
    const mg_lbvh_layout L = make_layout(n_prims, prim_kind);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    const WsLayout W = make_ws(n_prims);
    if (n_prims > 0 && (!ws || ws_bytes < static_cast<size_t>(W.total))) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (n_prims > 0 && !verts) return MG_ERR_INVALID_ARGUMENT;
    hipStream_t s = as_stream(stream);
    const int64_t n = n_prims;
    mg_lbvh_header *hdr = at<mg_lbvh_header>(bvh, L.off_header);
    uint32_t *hist = n ? at<uint32_t>(ws, W.hist) : nullptr;
    uint32_t *lookback = n ? at<uint32_t>(ws, W.lookback) : nullptr;
    const int64_t n_lookback = 4 * 256 * W.tiles;
    hipLaunchKernelGGL(build_init_kernel, dim3(n_lookback > 65536 ? 256 : 16), dim3(256), 0, s, hdr,
                       hist, lookback, n_lookback, n_prims, n_verts, prim_kind, chunk_log2_for(n_prims));
    if (launch_status() != MG_OK) return MG_ERR_HIP;
    if (n == 0) return MG_OK;
    const int32_t *fz = prim_kind == MG_PRIM_TRIANGLES ? faces : nullptr;
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 1024));
    hipLaunchKernelGGL(bounds_kernel, dim3(grid), dim3(256), 0, s, verts, (int64_t)n_verts, fz, n, hdr);
    uint32_t *ka = at<uint32_t>(ws, W.keys_a), *kb = at<uint32_t>(ws, W.keys_b);
    int32_t *va = at<int32_t>(ws, W.vals_a), *vb = at<int32_t>(ws, W.vals_b);
    hipLaunchKernelGGL(morton_kernel, dim3(grid), dim3(256), 0, s, verts, (int64_t)n_verts, fz, n, hdr, ka,
                       hist);
    uint32_t *codes = at<uint32_t>(bvh, L.off_codes);
    int32_t *prim = at<int32_t>(bvh, L.off_prim);
    // pass p reads (src) and writes (dst): A->B, B->A, A->B, B->final
    const uint32_t *ksrc[4] = {ka, kb, ka, kb};
    const int32_t *vsrc[4] = {nullptr, vb, va, vb};
    uint32_t *kdst[4] = {kb, ka, kb, codes};
    int32_t *vdst[4] = {vb, va, vb, prim};
    const int items = sort_items_for(n);
    for (int p = 0; p < 4; ++p) {
        auto pass = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(W.tiles)), dim3(kSortThreads), 0, s, ksrc[p],
                               vsrc[p], kdst[p], vdst[p], n, 8 * p, hist + 256 * p,
                               lookback + static_cast<int64_t>(p) * 256 * W.tiles, &hdr->tile_counter[p],
                               &hdr->status);
        };
        if (items <= 2) pass(radix_pass_kernel<2>);
        else if (items <= 4) pass(radix_pass_kernel<4>);
        else if (items <= 8) pass(radix_pass_kernel<8>);
        else pass(radix_pass_kernel<16>);
    }
    hipLaunchKernelGGL(hierarchy_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, codes, prim,
                       at<int32_t>(bvh, L.off_inv_prim), n, fz,
                       fz ? at<int32_t>(bvh, L.off_leaf_faces) : nullptr, at<int32_t>(bvh, L.off_leaf_parent),
                       at<int32_t>(bvh, L.off_node_parent), at<int32_t>(bvh, L.off_node_aux),
                       at<int32_t>(bvh, L.off_child), at<int32_t>(bvh, L.off_top_nodes), at<int32_t>(bvh, L.off_subtrees),
                       at<float>(bvh, L.off_nodes), hdr, chunk_log2_for(n));
    if (chunk_log2_for(n) >= 10)      // subtrees may outnumber the resident refit workgroups
        hipLaunchKernelGGL(order_subtrees_kernel, dim3(1), dim3(1024), 0, s, at<int32_t>(bvh, L.off_subtrees), n, hdr);
    hipLaunchKernelGGL(top_child_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(blocks_for(n, 256), 64))),
                       dim3(256), 0, s, at<int32_t>(bvh, L.off_node_aux), at<int32_t>(bvh, L.off_top_nodes),
                       at<int32_t>(bvh, L.off_node_parent), at<int32_t>(bvh, L.off_leaf_parent),
                       at<int32_t>(bvh, L.off_subtrees), n, at<int32_t>(bvh, L.off_top_child), hdr);
    if (launch_status() != MG_OK) return MG_ERR_HIP;
    return launch_refit(verts, n_verts, bvh, n, prim_kind, s);
}

}  // namespace
}  // namespace mgu

extern "C" mg_status mg_lbvh_build(const float *verts, int32_t n_verts, const int32_t *faces,
                                   int32_t n_prims, int32_t prim_kind, void *bvh, size_t bvh_bytes,
                                   void *ws, size_t ws_bytes, void *stream) {
    return build_into(verts, n_verts, faces, n_prims, prim_kind, bvh, bvh_bytes, ws, ws_bytes, stream);
}

// ------------------------------------------------ build without a caller workspace
//
// The sort scratch of mg_lbvh_build_static lives in this array, one copy per
// device for the life of the process.  In host code `scratch` only names the
// symbol: kernels get the device address that hipGetSymbolAddress returns for
// the current device.  Sized for the largest build accepted: four key/value
// planes of 2^20 entries, the four digit histograms, and look-back words for at
// most 256 tiles per pass (sort_items_for keeps the tile count at or below 256
// up to 2^20 keys).
namespace {
constexpr int64_t kStaticMaxPrims = MG_LBVH_STATIC_MAX_PRIMS;
constexpr int64_t kStaticWsBytes = 4 * (4 * kStaticMaxPrims) + 4 * 4 * 256 + 4 * 4 * 256 * 256;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

namespace {
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up on the first
// call there.
mg_status scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MG_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return MG_ERR_UNSUPPORTED_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}
}  // namespace

extern "C" mg_status mg_lbvh_build_static(const float *verts, int32_t n_verts, const int32_t *faces,
                                          int32_t n_prims, int32_t prim_kind, void *bvh, size_t bvh_bytes,
                                          void *stream) {
    if (n_prims < 0 || n_prims > kStaticMaxPrims) return MG_ERR_INVALID_ARGUMENT;
    if (make_ws(n_prims).total > kStaticWsBytes) return MG_ERR_INVALID_ARGUMENT;
    void *ws = nullptr;
    const mg_status st = scratch_address(&ws);
    if (st != MG_OK) return st;
    return build_into(verts, n_verts, faces, n_prims, prim_kind, bvh, bvh_bytes, ws,
                      static_cast<size_t>(kStaticWsBytes), stream);
}

extern "C" mg_status mg_frame_update(const float *frames, int32_t n_frames, int32_t n_verts, int32_t k,
                                     float *live, const int32_t *faces, int32_t n_faces, const int32_t *gface,
                                     const float *bary, const float *q_local, const float *log_scale,
                                     const float *offset, int32_t n_gauss, float *mean, float *quat, float *cov,
                                     float *rot, void *bvh, size_t bvh_bytes, void *stream) {
    if (bad_count(n_verts) || bad_count(n_faces) || bad_count(n_gauss) || n_frames <= 0 || k < 0 ||
        k >= n_frames || n_verts == 0 || n_faces == 0 || !frames || !live || !faces || !bvh)
        return MG_ERR_INVALID_ARGUMENT;
    if (n_gauss > 0 && (!gface || !bary || !q_local || !log_scale || !mean)) return MG_ERR_INVALID_ARGUMENT;
    const mg_lbvh_layout L = make_layout(n_faces, MG_PRIM_TRIANGLES);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    const int64_t n3 = 3 * static_cast<int64_t>(n_verts);
    const float *src = frames + static_cast<int64_t>(k) * n3;
    if (src < live + n3 && live < src + n3) return MG_ERR_INVALID_ARGUMENT;   // overlap
    const RefitArgs a = refit_args(src, n_verts, bvh, n_faces, MG_PRIM_TRIANGLES);
    const int64_t C = int64_t(1) << a.chunk_log2;
    FrameWork w;
    w.src = src;
    w.live = live;
    w.n3 = n3;
    w.in = Inputs{src, n_verts, faces, n_faces, gface, bary, q_local, log_scale, offset, n_gauss};
    w.mean = mean; w.quat = quat; w.cov = cov; w.rot = rot;
    w.sub_blocks = 2 * ((n_faces + C - 1) / C);
    const int threads = 512;                 // as the plain refit (launch_refit_k)
    w.copy_tile = 16 * static_cast<int64_t>(threads);
    w.copy_blocks = (n3 + w.copy_tile - 1) / w.copy_tile;
    w.gauss_tile = 2 * static_cast<int64_t>(threads);
    const int64_t gauss_blocks = (static_cast<int64_t>(n_gauss) + w.gauss_tile - 1) / w.gauss_tile;
    const int64_t grid = w.sub_blocks + w.copy_blocks + gauss_blocks;
    if (grid > 0x7fffffff) return MG_ERR_INVALID_ARGUMENT;
    hipStream_t s = as_stream(stream);
    if (a.chunk_log2 <= 9) return launch_frame_t<512, 1, 6>(a, w, grid, s);
    if (a.chunk_log2 == 10) return launch_frame_t<512, 2, 6>(a, w, grid, s);
    return launch_frame_t<512, 4, 2>(a, w, grid, s);
}

extern "C" mg_status mg_lbvh_refit(const float *verts, int32_t n_verts, void *bvh, size_t bvh_bytes,
                                   int32_t n_prims, int32_t prim_kind, void *stream) {
    if (bad_count(n_verts) || bad_count(n_prims) || check_kind(prim_kind) != MG_OK || !bvh)
        return MG_ERR_INVALID_ARGUMENT;
    const mg_lbvh_layout L = make_layout(n_prims, prim_kind);
    if (bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
    if (prim_kind == MG_PRIM_POINTS && n_verts != n_prims) return MG_ERR_TOPOLOGY_MISMATCH;
    if (n_prims == 0) return MG_OK;
    if (!verts || n_verts == 0) return MG_ERR_INVALID_ARGUMENT;
    return launch_refit(verts, n_verts, bvh, n_prims, prim_kind, as_stream(stream));
}
