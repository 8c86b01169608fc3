// Batched form: all scenes x frames in one persistent launch (gfx950).
//
// Work items are numbered in four phases - refit chunks, Gaussian tiles,
// refit top nodes, query tiles - each ordered by (scene, frame, tile).  Every
// workgroup repeatedly takes the next item from one atomic counter until the
// queue is empty.  A top item waits (agent-scope acquire) until all chunks of
// its scene-frame have signalled (agent-scope release), a query item until its
// scene-frame's refit has; both depend only on items with smaller numbers,
// which were taken earlier by workgroups that are running and never wait on
// later items, so the queue cannot deadlock.  Waits are bounded: a timeout
// sets the plan's error word and the item proceeds.
//
// Each scene-frame has its own node records and root box; topology (parents,
// top-node schedule, leaf faces) is shared by all frames of a scene.  Frame t's
// vertices are read in place from the frame store.
#include "refit.hpp"
#include "repose.hpp"
#include "traverse.hpp"

#include <cstring>
#include <vector>

namespace mgu {
namespace {

constexpr int kBlock = 256;                 // 4 waves
constexpr int kBatchTopLds = 384;           // top nodes per scene kept in LDS by the batched refit
constexpr int kBatchMaxChunkLog2 = 9;       // subtrees of up to 512 leaves (scenes up to 262,144 faces)
constexpr int kMaxScenes = 64;
constexpr int kSpin = 1 << 22;

struct PlanScene {
    mg_batch_scene s;
    const int32_t *leaf_faces, *prim, *inv_prim, *leaf_parent, *node_parent, *node_aux, *top_nodes;
    const int32_t *top_child, *subtrees;
    const int32_t *child;                   // the BVH's child references [2][n-1]
    const int32_t *n_top, *n_sub;           // the scene BVH's counts (device)
    float4 *deposit;                        // [n_frames][n_sub][3] subtree-root summaries
    float4 *top_scratch;                    // [n_frames][13 tstride / 4] phase-2 state when n_top > kBatchTopLds, else null
    int64_t tstride;                        // n_top rounded up to a multiple of 4
    int32_t n_top_host, n_sub_host;         // counts read at plan time
    int32_t batch, seed, query_tile;        // this scene's traversal (plan defaults resolved)
    int32_t chunk_log2;
    int32_t sf_base;                        // index of (this scene, frame 0) among all scene-frames
    int32_t qd_base;                        // index of (this scene, frame 0, tile 0) among the query-tile counters
    int64_t n_chunks, g_tiles, q_tiles;     // items per frame (n_chunks: subtrees)
    int64_t first[4];                       // first item of this scene in each phase
};

struct PlanHeader {
    int32_t n_scenes, total_sf;
    int32_t batch, seed, gauss_tile, query_tile;
    int32_t total_qt;                       // query-tile counters in use (all scene-frames)
    int64_t blocks_off;                     // byte offset of the QueryBlock table in the plan
    int32_t n_blocks;                       // query blocks (scene-frames with queries), frame-major
    int32_t pad1;
    int32_t status;
    uint32_t queue;
    int32_t pad;
    int64_t phase_end[4];                   // one past the last item of each phase
    PlanScene scenes[kMaxScenes];
};

// Refit schedule of a built BVH (read from its device header): top nodes,
// subtrees and the subtree size bound.
struct Schedule {
    int32_t n_top, n_sub, chunk_log2;
};

inline mg_status read_schedule(const mg_batch_scene &s, Schedule &S) {
    mg_lbvh_layout L;
    if (mg_lbvh_layout_query(s.n_faces, MG_PRIM_TRIANGLES, &L) != MG_OK) return MG_ERR_INVALID_ARGUMENT;
    const char *b = static_cast<const char *>(s.bvh);
    mg_lbvh_header hdr;
    if (hipMemcpy(&hdr, b + L.off_header, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess) return MG_ERR_HIP;
    S.n_top = hdr.n_top;
    S.n_sub = hdr.n_sub;
    S.chunk_log2 = hdr.chunk_log2;
    if (hdr.n_prims != s.n_faces || hdr.n_verts != s.n_verts || hdr.prim_kind != MG_PRIM_TRIANGLES ||
        hdr.status != 0)
        return MG_ERR_TOPOLOGY_MISMATCH;
    if (S.n_top < 0 || S.n_top >= s.n_faces || S.n_sub < 1 || S.n_sub > s.n_faces)
        return MG_ERR_INVALID_ARGUMENT;
    // the batched kernel keeps a subtree's phase-1 state in its fixed LDS
    if (S.chunk_log2 < 8 || S.chunk_log2 > kBatchMaxChunkLog2) return MG_ERR_INVALID_ARGUMENT;
    return MG_OK;
}

// Scratch words of one frame of a scene: the deposited subtree-root summaries,
// and second-phase state when the top nodes exceed the LDS capacity (summary
// slots and arrival words, 13 words per top node, the count rounded up to a
// multiple of 4 so that every block stays 16-byte aligned).
__host__ __device__ inline int64_t top_stride(int32_t T) { return (static_cast<int64_t>(T) + 3) & ~int64_t(3); }
__host__ __device__ inline int64_t top_scratch_words(int32_t T) { return 13 * top_stride(T); }
inline int64_t frame_scratch_words(int32_t T, int32_t NS) {
    return 12 * static_cast<int64_t>(NS) + (T > kBatchTopLds ? top_scratch_words(T) : 0);
}

// Plan layout: header, 2 x total_sf dependency counters and the query-tile
// counters (room for the smallest legal tile, 4 queries, since the plan's size
// does not depend on the options), then per scene-frame refit scratch.
inline int64_t align256b(int64_t x) { return (x + 255) & ~int64_t(255); }

inline int64_t query_tile_cap(const mg_batch_scene *scenes, int32_t n) {
    int64_t c = 0;
    for (int i = 0; i < n; ++i) c += static_cast<int64_t>(scenes[i].n_frames) * ((scenes[i].n_queries + 3) / 4);
    return c;
}

// The query phase runs frame by frame across the scenes (frame 0 of every scene,
// then frame 1, ...), so that a query tile's counterpart in the scene's previous
// frame was taken from the queue a whole frame of work earlier; one block per
// scene-frame in that order records its first item.
struct QueryBlock {
    int64_t first;
    int32_t scene, frame;
};

inline int64_t counters_bytes(int64_t total_sf, int64_t qt_cap) {
    return align256b(static_cast<int64_t>(sizeof(PlanHeader)) + 8 * total_sf + 4 * qt_cap);
}

inline int64_t blocks_bytes(int64_t total_sf) {
    return align256b(static_cast<int64_t>(sizeof(QueryBlock)) * total_sf);
}

inline int64_t plan_bytes_for(int64_t total_sf, int64_t qt_cap, int64_t scratch_words) {
    return counters_bytes(total_sf, qt_cap) + blocks_bytes(total_sf) + 4 * scratch_words;
}

// Dependency counters follow the header: done_chunks[total_sf], refit_done[total_sf],
// query_done[total_qt] (one per scene, frame and query tile).
__device__ __forceinline__ uint32_t *counters_of(PlanHeader *h) {
    return reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(h) + sizeof(PlanHeader));
}

__global__ void batch_reset_kernel(PlanHeader *h) {
    uint32_t *c = counters_of(h);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
         i < 2 * int64_t(h->total_sf) + h->total_qt;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        c[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        h->queue = 0;
        h->status = 0;
    }
}

// Thread 0 waits until *ctr >= target (bounded), then every thread acquires.
__device__ void wait_for(uint32_t *ctr, uint32_t target, int32_t *status) {
    if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpin) {
                atomicOr(status, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    (void)__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Every thread's prior global writes are made visible device-wide, then one
// thread releases the counter.
__device__ void signal(uint32_t *ctr, uint32_t add) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, add, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ RefitArgs refit_args(const PlanScene &P, int64_t t, PlanHeader *h) {
    const mg_batch_scene &s = P.s;
    RefitArgs a;
    a.verts = s.frames + t * 3 * static_cast<int64_t>(s.n_verts);
    a.nv = s.n_verts;
    a.leaf_faces = P.leaf_faces;
    a.prim = P.prim;
    a.leaf_parent = P.leaf_parent;
    a.node_parent = P.node_parent;
    a.nodes = reinterpret_cast<float4 *>(s.nodes + t * 24 * static_cast<int64_t>(s.n_faces > 1 ? s.n_faces - 1 : 0));
    a.top_nodes = P.top_nodes;
    a.child = P.child;
    a.node_aux = P.node_aux;
    a.top_child = P.top_child;
    a.subtrees = P.subtrees;
    a.deposit = P.deposit + t * 3 * static_cast<int64_t>(P.n_sub_host);
    a.tstride = P.tstride;
    a.top_scratch = P.top_scratch ? P.top_scratch + t * top_scratch_words(P.n_top_host) / 4 : nullptr;
    a.hdr_nv = nullptr;                     // the plan checked the build's vertex count
    a.arrivals = nullptr;
    a.root = s.roots + 8 * t;
    a.status = &h->status;
    a.n_top = P.n_top;
    a.n_sub = P.n_sub;
    a.n = s.n_faces;
    a.chunk_log2 = P.chunk_log2;
    a.inf = INFINITY;
    return a;
}

__device__ QueryArgs query_args(const PlanScene &P, int64_t t, const RefitArgs &r, int seed) {
    const mg_batch_scene &s = P.s;
    const int64_t nq = s.n_queries;
    QueryArgs a;
    a.nodes = r.nodes;
    a.root = r.root;
    a.leaf_faces = P.leaf_faces;
    a.prim = P.prim;
    a.inv_prim = P.inv_prim;
    a.status = r.status;
    a.verts = r.verts;
    a.nv = s.n_verts;
    a.n = s.n_faces;
    a.queries = s.queries;
    a.nq = nq;
    a.maxd2 = INFINITY;
    a.face = s.face + t * nq;
    a.point = s.point ? s.point + t * 3 * nq : nullptr;
    a.bary = s.qbary ? s.qbary + t * 2 * nq : nullptr;
    a.dist2 = s.dist2 ? s.dist2 + t * nq : nullptr;
    a.normal = s.normal ? s.normal + t * 3 * nq : nullptr;
    a.seed = seed;
    a.order = nullptr;
    a.counters = nullptr;
    a.queue = nullptr;
    a.hint = nullptr;
    a.coherent = 1;
    return a;
}

static_assert(kBlock == 64 * kBatchWaves, "a query tile is run by the workgroup's kBatchWaves waves");

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kSmemBytes = cmax(cmax(refit_top_lds(kBatchTopLds), refit_sub_lds(int64_t(1) << kBatchMaxChunkLog2)),
                                   sizeof(BatchLds<16>));
static_assert(refit_sub_lds(int64_t(1) << kBatchMaxChunkLog2) <= kSmemBytes &&
                  (int64_t(1) << kBatchMaxChunkLog2) <= 2 * kBlock,
              "a subtree of the batched refit fits the workgroup's LDS and two leaves per thread");

// The work of each phase is a function of its own (not inlined), so the
// kernel needs the registers of its largest phase rather than of all of them
// at once.  Each reads the launch's dynamic LDS (kSmemBytes).
__device__ __noinline__ void item_refit_sub(PlanHeader *h, int si, int64_t t, int64_t k) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PlanScene &P = h->scenes[si];
    if (P.chunk_log2 <= 8) refit_subtree<true, kBlock, 1>(refit_args(P, t, h), k, smem);
    else refit_subtree<true, kBlock, 2>(refit_args(P, t, h), k, smem);
    signal(&counters_of(h)[P.sf_base + t], 1u);
}

__device__ __noinline__ void item_repose(PlanHeader *h, int si, int64_t t, int64_t k) {
    const PlanScene &P = h->scenes[si];
    const mg_batch_scene &s = P.s;
    const int64_t G = s.n_gauss;
    const float *verts = s.frames + t * 3 * static_cast<int64_t>(s.n_verts);
    Inputs in{verts, s.n_verts, s.faces, s.n_faces, s.gface, s.bary, s.q_local, s.log_scale, nullptr, G};
    float *mean = s.mean + t * 3 * G;
    float *quat = s.quat ? s.quat + t * 4 * G : nullptr;
    float *cov = s.cov ? s.cov + t * 6 * G : nullptr;
    const int64_t g0 = k * h->gauss_tile;
    const int64_t g1 = g0 + h->gauss_tile < G ? g0 + h->gauss_tile : G;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kBlock) repose_store(in, g, mean, quat, cov, nullptr);
}

__device__ __noinline__ void item_refit_top(PlanHeader *h, int si, int64_t t) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PlanScene &P = h->scenes[si];
    const int sf = P.sf_base + static_cast<int>(t);
    uint32_t *done_chunks = counters_of(h);
    uint32_t *refit_done = done_chunks + h->total_sf;
    wait_for(&done_chunks[sf], static_cast<uint32_t>(P.n_chunks), &h->status);
    const RefitArgs r = refit_args(P, t, h);
    const int T = *P.n_top, NS = *P.n_sub;
    if (T != P.n_top_host || NS != P.n_sub_host) {
        if (threadIdx.x == 0) atomicOr(&h->status, 2);   // the BVH was rebuilt after planning
    } else if (T > 0 && T <= kBatchTopLds) {
        refit_top<true, kBlock, false, (kBatchTopLds + kBlock - 1) / kBlock>(r, T, NS, smem);
    } else if (T > kBatchTopLds) {
        refit_top<true, kBlock, true, 1>(r, T, NS, smem);
    }
    signal(&refit_done[sf], 1u);
}

template <int M>
__device__ __noinline__ void item_query(PlanHeader *h, int si, int64_t t, int64_t k) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PlanScene &P = h->scenes[si];
    const int sf = P.sf_base + static_cast<int>(t);
    uint32_t *query_done = counters_of(h) + 2 * int64_t(h->total_sf);
    const int64_t qd = P.qd_base + t * P.q_tiles + k;
    wait_for(&counters_of(h)[h->total_sf + sf], 1u, &h->status);
    QueryArgs q = query_args(P, t, refit_args(P, t, h), P.seed);
    // The queries start from their faces of the scene's previous frame when the same
    // tile of frame t - 1 (the same queries) is already done; otherwise they start
    // cold.  Nothing waits for it, and no ordering is needed for correctness: a hint
    // only lowers the starting bound, and any id is range-checked.  The face ids are
    // stored and loaded device-coherent, and a tile counts as done only after its
    // waves' stores have completed, so the hints are that frame's answers without a
    // write-back of the L2 per tile.
    if (t > 0) {
        __shared__ int s_prev_done;
        if (threadIdx.x == 0)
            s_prev_done = __hip_atomic_load(&query_done[qd - P.q_tiles], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        __syncthreads();
        if (s_prev_done) q.hint = P.s.face + (t - 1) * static_cast<int64_t>(P.s.n_queries);
    }
    const int64_t q0 = k * P.query_tile;
    const int64_t q1 = q0 + P.query_tile < q.nq ? q0 + P.query_tile : q.nq;
    batch_loop<true, M, false>(q, q0, static_cast<int64_t>(kBatchWaves) * M, q1,
                               *reinterpret_cast<BatchLds<M> *>(smem));
    __builtin_amdgcn_s_waitcnt(0);          // this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&query_done[qd], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// At most 128 registers per lane (four waves per SIMD): with the phases
// outlined, that costs a few spills in exchange for four times the waves.
__global__ __launch_bounds__(kBlock, 4) void batch_persistent_kernel(PlanHeader *h) {
    __shared__ int64_t s_item;
    const int64_t total = h->phase_end[3];
    const int ns = h->n_scenes;
    for (;;) {
        __syncthreads();                    // LDS and s_item of the previous item are free
        if (threadIdx.x == 0) s_item = atomicAdd(&h->queue, 1u);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        int phase = 0;
        while (item >= h->phase_end[phase]) ++phase;
        int si = 0;
        int64_t t = 0, k = 0;
        if (phase < 3) {
            while (si + 1 < ns && item >= h->scenes[si + 1].first[phase]) ++si;
            const PlanScene &Q = h->scenes[si];
            const int64_t local = item - Q.first[phase];
            const int64_t per = phase == 0 ? Q.n_chunks : phase == 1 ? Q.g_tiles : 1;
            t = local / per;
            k = local % per;
        } else {                            // the query block holding the item: the last with first <= item
            const QueryBlock *B = reinterpret_cast<const QueryBlock *>(reinterpret_cast<const char *>(h) + h->blocks_off);
            int lo = 0, hi = h->n_blocks - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (B[mid].first <= item) lo = mid;
                else hi = mid - 1;
            }
            si = B[lo].scene;
            t = B[lo].frame;
            k = item - B[lo].first;
        }
        const PlanScene &P = h->scenes[si];
        if (phase == 0) {
            item_refit_sub(h, si, t, k);
        } else if (phase == 1) {
            item_repose(h, si, t, k);
        } else if (phase == 2) {
            item_refit_top(h, si, t);
        } else {
            switch (P.batch) {
                case 1: item_query<1>(h, si, t, k); break;
                case 2: item_query<2>(h, si, t, k); break;
                case 8: item_query<8>(h, si, t, k); break;
                case 16: item_query<16>(h, si, t, k); break;
                default: item_query<4>(h, si, t, k); break;
            }
        }
    }
}

int64_t total_frames(const mg_batch_scene *scenes, int32_t n) {
    int64_t t = 0;
    for (int i = 0; i < n; ++i) t += scenes[i].n_frames;
    return t;
}

}  // namespace
}  // namespace mgu

using namespace mgu;

// Refit scratch words of every scene-frame.
inline mg_status scratch_words(const mg_batch_scene *scenes, int32_t n_scenes, int64_t &words) {
    words = 0;
    for (int i = 0; i < n_scenes; ++i) {
        if (!scenes[i].bvh || scenes[i].n_faces < 1) return MG_ERR_INVALID_ARGUMENT;
        Schedule S;
        const mg_status st = read_schedule(scenes[i], S);
        if (st != MG_OK) return st;
        words += static_cast<int64_t>(scenes[i].n_frames) * frame_scratch_words(S.n_top, S.n_sub);
    }
    return MG_OK;
}

extern "C" mg_status mg_batch_plan_size(const mg_batch_scene *scenes, int32_t n_scenes, size_t *plan_bytes) {
    if (!scenes || !plan_bytes || n_scenes < 1 || n_scenes > kMaxScenes) return MG_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < n_scenes; ++i)
        if (scenes[i].n_frames < 1 || bad_count(scenes[i].n_faces)) return MG_ERR_INVALID_ARGUMENT;
    int64_t words = 0;
    const mg_status st = scratch_words(scenes, n_scenes, words);
    if (st != MG_OK) return st;
    *plan_bytes = static_cast<size_t>(plan_bytes_for(total_frames(scenes, n_scenes), query_tile_cap(scenes, n_scenes),
                                                     words));
    return MG_OK;
}

extern "C" mg_status mg_batch_plan_init(const mg_batch_scene *scenes, int32_t n_scenes, const mg_batch_options *opts,
                                        void *plan, size_t plan_bytes, void *stream) {
    size_t need = 0;
    mg_status st = mg_batch_plan_size(scenes, n_scenes, &need);
    if (st != MG_OK) return st;
    if (!plan || plan_bytes < need) return MG_ERR_WORKSPACE_TOO_SMALL;
    mg_batch_options o{};
    if (opts) o = *opts;
    const int batch = o.batch == 0 ? 4 : o.batch;
    if (!(batch == 1 || batch == 2 || batch == 4 || batch == 8 || batch == 16)) return MG_ERR_INVALID_ARGUMENT;
    const int gtile = o.gauss_tile == 0 ? 2048 : o.gauss_tile;
    const int qtile = o.query_tile == 0 ? 256 : o.query_tile;
    if (gtile <= 0 || gtile % kBlock != 0 || qtile <= 0 || qtile % (4 * batch) != 0) return MG_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < 4; ++i)
        if (o.reserved[i] != 0) return MG_ERR_INVALID_ARGUMENT;
    std::vector<PlanHeader> hv(1);
    PlanHeader &h = hv[0];
    std::memset(&h, 0, sizeof(PlanHeader));
    h.n_scenes = n_scenes;
    h.batch = batch;
    h.seed = o.seed != 0;
    h.gauss_tile = gtile;
    h.query_tile = qtile;
    int64_t sf = 0;
    uint32_t *scratch = reinterpret_cast<uint32_t *>(
        static_cast<char *>(plan) + counters_bytes(total_frames(scenes, n_scenes), query_tile_cap(scenes, n_scenes)) +
        blocks_bytes(total_frames(scenes, n_scenes)));
    int64_t qt = 0;
    for (int i = 0; i < n_scenes; ++i) {
        const mg_batch_scene &s = scenes[i];
        if (bad_count(s.n_verts) || bad_count(s.n_faces) || bad_count(s.n_gauss) || bad_count(s.n_queries) ||
            s.n_faces < 1 || s.n_verts < 1 || !s.frames || !s.faces || !s.bvh || !s.nodes || !s.roots)
            return MG_ERR_INVALID_ARGUMENT;
        if (s.n_gauss > 0 && (!s.gface || !s.bary || !s.q_local || !s.log_scale || !s.mean))
            return MG_ERR_INVALID_ARGUMENT;
        if (s.n_queries > 0 && (!s.queries || !s.face)) return MG_ERR_INVALID_ARGUMENT;
        mg_lbvh_layout L;
        mg_lbvh_layout_query(s.n_faces, MG_PRIM_TRIANGLES, &L);
        if (s.bvh_bytes < static_cast<size_t>(L.total_bytes)) return MG_ERR_WORKSPACE_TOO_SMALL;
        PlanScene &P = h.scenes[i];
        P.s = s;
        P.batch = s.batch == 0 ? batch : s.batch;
        P.seed = s.seed < 0 ? (o.seed != 0) : (s.seed != 0);
        P.query_tile = s.query_tile == 0 ? qtile : s.query_tile;
        if (!(P.batch == 1 || P.batch == 2 || P.batch == 4 || P.batch == 8 || P.batch == 16) || s.seed < -1 ||
            s.seed > 1 || P.query_tile <= 0 || P.query_tile % (4 * P.batch) != 0)
            return MG_ERR_INVALID_ARGUMENT;
        const char *b = static_cast<const char *>(s.bvh);
        P.leaf_faces = reinterpret_cast<const int32_t *>(b + L.off_leaf_faces);
        P.prim = reinterpret_cast<const int32_t *>(b + L.off_prim);
        P.inv_prim = reinterpret_cast<const int32_t *>(b + L.off_inv_prim);
        P.leaf_parent = reinterpret_cast<const int32_t *>(b + L.off_leaf_parent);
        P.node_parent = reinterpret_cast<const int32_t *>(b + L.off_node_parent);
        P.top_nodes = reinterpret_cast<const int32_t *>(b + L.off_top_nodes);
        P.node_aux = reinterpret_cast<const int32_t *>(b + L.off_node_aux);
        P.top_child = reinterpret_cast<const int32_t *>(b + L.off_top_child);
        P.child = reinterpret_cast<const int32_t *>(b + L.off_child);
        P.subtrees = reinterpret_cast<const int32_t *>(b + L.off_subtrees);
        P.n_top = &reinterpret_cast<const mg_lbvh_header *>(b + L.off_header)->n_top;
        P.n_sub = &reinterpret_cast<const mg_lbvh_header *>(b + L.off_header)->n_sub;
        Schedule S;
        st = read_schedule(s, S);
        if (st != MG_OK) return st;
        P.n_top_host = S.n_top;
        P.n_sub_host = S.n_sub;
        P.chunk_log2 = S.chunk_log2;
        // per-frame scratch: [n_frames][n_sub][3] float4 deposits, then [n_frames][top_scratch_words]
        // of phase-2 state (multiples of 4 words: the blocks stay 16-byte aligned)
        P.deposit = reinterpret_cast<float4 *>(scratch);
        scratch += static_cast<int64_t>(s.n_frames) * 12 * S.n_sub;
        P.tstride = top_stride(S.n_top);
        P.top_scratch = nullptr;
        if (S.n_top > kBatchTopLds) {
            P.top_scratch = reinterpret_cast<float4 *>(scratch);
            scratch += static_cast<int64_t>(s.n_frames) * top_scratch_words(S.n_top);
        }
        P.sf_base = static_cast<int32_t>(sf);
        P.n_chunks = S.n_sub;
        P.g_tiles = (s.n_gauss + gtile - 1) / gtile;
        P.q_tiles = (s.n_queries + P.query_tile - 1) / P.query_tile;
        P.qd_base = static_cast<int32_t>(qt);
        qt += static_cast<int64_t>(s.n_frames) * P.q_tiles;
        sf += s.n_frames;
    }
    h.total_sf = static_cast<int32_t>(sf);
    h.total_qt = static_cast<int32_t>(qt);
    if (qt > query_tile_cap(scenes, n_scenes)) return MG_ERR_INVALID_ARGUMENT;   // tiles below 4 queries
    int64_t item = 0;
    for (int phase = 0; phase < 3; ++phase) {
        for (int i = 0; i < n_scenes; ++i) {
            PlanScene &P = h.scenes[i];
            P.first[phase] = item;
            const int64_t per = phase == 0 ? P.n_chunks : phase == 1 ? P.g_tiles : 1;
            item += per * P.s.n_frames;
        }
        h.phase_end[phase] = item;
    }
    // the query phase, frame-major across the scenes (empty scene-frames have no block)
    std::vector<QueryBlock> blocks;
    int32_t max_frames = 0;
    for (int i = 0; i < n_scenes; ++i) max_frames = std::max(max_frames, scenes[i].n_frames);
    for (int i = 0; i < n_scenes; ++i) h.scenes[i].first[3] = item;
    for (int32_t t = 0; t < max_frames; ++t)
        for (int i = 0; i < n_scenes; ++i) {
            const PlanScene &P = h.scenes[i];
            if (t >= P.s.n_frames || P.q_tiles == 0) continue;
            blocks.push_back(QueryBlock{item, i, t});
            item += P.q_tiles;
        }
    h.phase_end[3] = item;
    h.n_blocks = static_cast<int32_t>(blocks.size());
    h.blocks_off = counters_bytes(total_frames(scenes, n_scenes), query_tile_cap(scenes, n_scenes));
    for (int i = n_scenes; i < kMaxScenes; ++i)
        for (int phase = 0; phase < 4; ++phase) h.scenes[i].first[phase] = h.phase_end[3];
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(plan, &h, sizeof(PlanHeader), hipMemcpyHostToDevice, s) != hipSuccess) return MG_ERR_HIP;
    if (!blocks.empty() && hipMemcpyAsync(static_cast<char *>(plan) + h.blocks_off, blocks.data(),
                                          sizeof(QueryBlock) * blocks.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return MG_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
    return MG_OK;
}

extern "C" mg_status mg_batch_run(void *plan, size_t plan_bytes, void *stream) {
    if (!plan || plan_bytes < sizeof(PlanHeader)) return MG_ERR_INVALID_ARGUMENT;
    PlanHeader *h = static_cast<PlanHeader *>(plan);
    hipStream_t s = as_stream(stream);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipLaunchKernelGGL(batch_reset_kernel, dim3(8), dim3(256), 0, s, h);
    // persistent workgroups: 4 per compute unit (the kernel stops when the queue is empty)
    hipLaunchKernelGGL(batch_persistent_kernel, dim3(4 * cus), dim3(kBlock), kSmemBytes, s, h);
    return launch_status();
}

extern "C" mg_status mg_batch_status_word(void *plan, int32_t **status) {
    if (!plan || !status) return MG_ERR_INVALID_ARGUMENT;
    *status = &static_cast<PlanHeader *>(plan)->status;
    return MG_OK;
}
