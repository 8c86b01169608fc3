// Template-projection losses and their backward passes, Adam, reductions and
// validation helpers (gfx950).
//
// Chamfer distance appears in the paper only as an evaluation metric (Sec. 4.2,
// no formula); the library's is CD(A,B) = mean_a min_b |a-b|^2 +
// mean_b min_a |a-b|^2.  Point-to-mesh gradients follow Danskin's theorem: with
// a unique closest face the distance is differentiated with that face fixed,
// d|y - c|^2 / dv_k = -2 w_k (y - c).
#include "mgu_internal.hpp"

namespace mgu {
namespace {

constexpr int kReduceThreads = 256;
constexpr int kReduceMaxBlocks = 1024;
constexpr int kReduceItems = 8;   // per thread per block-chunk

__global__ __launch_bounds__(kReduceThreads) void partial_sum_kernel(const float *__restrict__ x, int64_t n,
                                                                     int64_t chunk, double *__restrict__ part) {
    __shared__ double s[kReduceThreads];
    const int64_t begin = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = begin + chunk < n ? begin + chunk : n;
    double acc = 0.0;
    for (int64_t i = begin + threadIdx.x; i < end; i += kReduceThreads) acc += static_cast<double>(x[i]);
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kReduceThreads) void final_mean_kernel(const double *__restrict__ part, int nparts,
                                                                    int64_t n, double *__restrict__ out) {
    __shared__ double s[kReduceThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kReduceThreads) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = n > 0 ? s[0] / static_cast<double>(n) : 0.0;
}

// Sum of v over this lane's run of equal keys up to this lane (a segmented
// inclusive scan; start is the first lane of the run).
__device__ __forceinline__ float run_sum(float v, int start, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float y = __shfl_up(v, o);
        if (lane - o >= start) v += y;
    }
    return v;
}

// One target per lane.  When neighbouring targets share their closest face (targets
// in a spatially coherent order, as scans usually are), each run of lanes with one
// face sums its three vertex contributions and its last lane adds them; targets in
// random order pay only the shuffles.  Every lane takes part in them.
__global__ __launch_bounds__(256) void point_mesh_backward_kernel(
    const float *__restrict__ verts, int64_t nv, const int32_t *__restrict__ faces, int64_t nf,
    const float *__restrict__ y, int64_t nq, const int32_t *__restrict__ face, const float *__restrict__ point,
    const float *__restrict__ bary, float scale, const double *__restrict__ g_loss, float *__restrict__ g) {
    const int64_t qi = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t q = qi < nq ? qi : nq - 1;
    const int32_t f = face[q];
    const bool valid = qi < nq && f >= 0 && f < nf;
    if (g_loss) scale *= static_cast<float>(*g_loss);
    const f3 r = load3(y, nq, q) - load3(point, nq, q);
    const float w1 = bary[q], w2 = bary[nq + q];
    const float w[3] = {1.0f - w1 - w2, w1, w2};
    const int lane = threadIdx.x % 64;
    const int key = valid ? f : -1 - lane;
    const int prev = __shfl_up(key, 1);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    const int start = 63 - __builtin_clzll(heads & (lanemask_lt() | (1ull << lane)));
    const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float c = valid ? -2.0f * scale * w[k] : 0.0f;
        const float gx = run_sum(c * r.x, start, lane), gy = run_sum(c * r.y, start, lane),
                    gz = run_sum(c * r.z, start, lane);
        if (valid && tail) {
            const int32_t v = faces[k * nf + f];
            atomicAdd(g + v, gx);
            atomicAdd(g + nv + v, gy);
            atomicAdd(g + 2 * nv + v, gz);
        }
    }
}

// threads [0, na): the a -> b term of a_i; threads [na, na + nb): the b -> a term
// of b_j, added to its nearest a.
__global__ __launch_bounds__(256) void chamfer_backward_kernel(const float *__restrict__ a, int64_t na,
                                                               const float *__restrict__ b, int64_t nb,
                                                               const int32_t *__restrict__ nn_ab,
                                                               const int32_t *__restrict__ nn_ba, float s_ab,
                                                               float s_ba, const double *__restrict__ g_loss,
                                                               float *__restrict__ g) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g_loss) {
        const float gl = static_cast<float>(*g_loss);
        s_ab *= gl;
        s_ba *= gl;
    }
    if (t < na) {
        const int32_t j = nn_ab[t];
        if (j < 0) return;
        const f3 d = load3(a, na, t) - load3(b, nb, j);
        const float c = 2.0f * s_ab;
        atomicAdd(g + t, c * d.x);
        atomicAdd(g + na + t, c * d.y);
        atomicAdd(g + 2 * na + t, c * d.z);
    } else if (t < na + nb) {
        const int64_t j = t - na;
        const int32_t i = nn_ba[j];
        if (i < 0) return;
        const f3 d = load3(a, na, i) - load3(b, nb, j);
        const float c = 2.0f * s_ba;
        atomicAdd(g + i, c * d.x);
        atomicAdd(g + na + i, c * d.y);
        atomicAdd(g + 2 * na + i, c * d.z);
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ grad,
                                                   float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                   float lr, float b1, float b2, float eps, float step_size,
                                                   float bc2_sqrt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float denom = sqrtf(vi) / bc2_sqrt + eps;
    p[i] = p[i] - step_size * (mi / denom);
}

__global__ __launch_bounds__(256) void validate_indices_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                               int32_t bound, int32_t *status) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    bool bad = false;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t x = idx[i];
        bad |= (x < 0) || (x >= bound);
    }
    if (__ballot(bad) != 0ull && (threadIdx.x % kWave) == 0) atomicExch(status, MG_ERR_INDEX_OUT_OF_RANGE);
}

__global__ __launch_bounds__(256) void validate_finite_kernel(const float *__restrict__ x, int64_t n,
                                                              int32_t *status) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    bool bad = false;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        bad |= !isfinite(x[i]);
    if (__ballot(bad) != 0ull && (threadIdx.x % kWave) == 0) atomicExch(status, MG_ERR_NONFINITE_INPUT);
}

// out[2] = (out[0] + out[1]) + add[0] (add may be null): the two-sided Chamfer
// sum, plus an optional loss term already on the device.
__global__ void chamfer_total_kernel(double *__restrict__ out, const double *__restrict__ add) {
    if (threadIdx.x == 0) out[2] = (out[0] + out[1]) + (add ? add[0] : 0.0);
}

inline int reduce_blocks(int64_t n, int64_t &chunk) {
    const int64_t per_block = static_cast<int64_t>(kReduceThreads) * kReduceItems;
    int64_t blocks = (n + per_block - 1) / per_block;
    if (blocks > kReduceMaxBlocks) blocks = kReduceMaxBlocks;
    if (blocks < 1) blocks = 1;
    chunk = (n + blocks - 1) / blocks;
    if (chunk < 1) chunk = 1;
    return static_cast<int>(blocks);
}

mg_status launch_mean(const float *x, int64_t n, double *out, void *ws, hipStream_t s) {
    int64_t chunk;
    const int blocks = reduce_blocks(n, chunk);
    double *part = static_cast<double *>(ws);
    if (n > 0)
        hipLaunchKernelGGL(partial_sum_kernel, dim3(blocks), dim3(kReduceThreads), 0, s, x, n, chunk, part);
    hipLaunchKernelGGL(final_mean_kernel, dim3(1), dim3(kReduceThreads), 0, s, part, n > 0 ? blocks : 0, n, out);
    return launch_status();
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_reduce_workspace_size(int64_t n, size_t *ws_bytes) {
    if (!ws_bytes || n < 0) return MG_ERR_INVALID_ARGUMENT;
    *ws_bytes = sizeof(double) * kReduceMaxBlocks;
    return MG_OK;
}

extern "C" mg_status mg_mean(const float *x, int64_t n, double *out, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || !out || (n > 0 && !x)) return MG_ERR_INVALID_ARGUMENT;
    if (!ws || ws_bytes < sizeof(double) * kReduceMaxBlocks) return MG_ERR_WORKSPACE_TOO_SMALL;
    return launch_mean(x, n, out, ws, as_stream(stream));
}

extern "C" mg_status mg_chamfer(const float *a, int32_t na, const void *bvh_a, size_t bvh_a_bytes, const float *b,
                                int32_t nb, const void *bvh_b, size_t bvh_b_bytes, int32_t *nn_ab, float *d_ab,
                                int32_t *nn_ba, float *d_ba, double *out, const double *add, void *ws,
                                size_t ws_bytes, const mg_query_options *opts, void *stream) {
    if (bad_count(na) || bad_count(nb) || !out || !nn_ab || !nn_ba || !d_ab || !d_ba || !bvh_a || !bvh_b)
        return MG_ERR_INVALID_ARGUMENT;
    if ((na > 0 && !a) || (nb > 0 && !b)) return MG_ERR_INVALID_ARGUMENT;
    if (!ws || ws_bytes < sizeof(double) * kReduceMaxBlocks) return MG_ERR_WORKSPACE_TOO_SMALL;
    // each direction's hints are its own previous answers (warm) or none
    mg_query_options o_ab{}, o_ba{};
    const mg_query_options *p_ab = opts, *p_ba = opts;
    if (opts) {
        o_ab = *opts;
        o_ab.hint = opts->warm ? nn_ab : nullptr;
        o_ba = *opts;
        o_ba.hint = opts->warm ? nn_ba : nullptr;
        p_ab = &o_ab;
        p_ba = &o_ba;
    }
    mg_status st = mg_nearest_point_query(bvh_b, bvh_b_bytes, nb, b, a, na, INFINITY, nn_ab, d_ab, p_ab, stream);
    if (st != MG_OK) return st;
    st = mg_nearest_point_query(bvh_a, bvh_a_bytes, na, a, b, nb, INFINITY, nn_ba, d_ba, p_ba, stream);
    if (st != MG_OK) return st;
    hipStream_t s = as_stream(stream);
    st = launch_mean(d_ab, na, out, ws, s);
    if (st != MG_OK) return st;
    st = launch_mean(d_ba, nb, out + 1, ws, s);
    if (st != MG_OK) return st;
    hipLaunchKernelGGL(chamfer_total_kernel, dim3(1), dim3(64), 0, s, out, add);
    return launch_status();
}

extern "C" mg_status mg_point_mesh_backward(const float *verts, int32_t n_verts, const int32_t *faces,
                                            int32_t n_faces, const float *queries, int32_t n_queries,
                                            const int32_t *face, const float *point, const float *bary,
                                            float scale, const double *g_loss, float *g_verts, void *stream) {
    if (bad_count(n_verts) || bad_count(n_faces) || bad_count(n_queries)) return MG_ERR_INVALID_ARGUMENT;
    if (n_queries == 0) return MG_OK;
    if (!verts || !faces || !queries || !face || !point || !bary || !g_verts) return MG_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(point_mesh_backward_kernel, dim3(blocks_for(n_queries, 256)), dim3(256), 0,
                       as_stream(stream), verts, (int64_t)n_verts, faces, (int64_t)n_faces, queries,
                       (int64_t)n_queries, face, point, bary, scale, g_loss, g_verts);
    return launch_status();
}

extern "C" mg_status mg_chamfer_backward(const float *a, int32_t na, const float *b, int32_t nb,
                                         const int32_t *nn_ab, const int32_t *nn_ba, float scale_ab,
                                         float scale_ba, const double *g_loss, float *g_a, void *stream) {
    if (bad_count(na) || bad_count(nb)) return MG_ERR_INVALID_ARGUMENT;
    if (na == 0) return MG_OK;
    if (!a || !g_a || !nn_ab || (nb > 0 && (!b || !nn_ba))) return MG_ERR_INVALID_ARGUMENT;
    const int64_t total = static_cast<int64_t>(na) + nb;
    hipLaunchKernelGGL(chamfer_backward_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, as_stream(stream), a,
                       (int64_t)na, b, (int64_t)nb, nn_ab, nn_ba, scale_ab, scale_ba, g_loss, g_a);
    return launch_status();
}

extern "C" mg_status mg_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int32_t step,
                                  float lr, float beta1, float beta2, float eps, void *stream) {
    if (n < 0 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f))
        return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    if (!param || !grad || !m || !v) return MG_ERR_INVALID_ARGUMENT;
    const double bc1 = 1.0 - pow(static_cast<double>(beta1), step);
    const double bc2 = 1.0 - pow(static_cast<double>(beta2), step);
    const float step_size = static_cast<float>(lr / bc1);
    const float bc2_sqrt = static_cast<float>(sqrt(bc2));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, as_stream(stream), param, grad, m, v,
                       n, lr, beta1, beta2, eps, step_size, bc2_sqrt);
    return launch_status();
}

extern "C" mg_status mg_validate_indices(const int32_t *idx, int64_t n, int32_t bound, int32_t *status_out,
                                         void *stream) {
    if (n < 0 || !status_out || (n > 0 && !idx)) return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 1024));
    hipLaunchKernelGGL(validate_indices_kernel, dim3(grid), dim3(256), 0, as_stream(stream), idx, n, bound,
                       status_out);
    return launch_status();
}

extern "C" mg_status mg_validate_finite(const float *x, int64_t n, int32_t *status_out, void *stream) {
    if (n < 0 || !status_out || (n > 0 && !x)) return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 1024));
    hipLaunchKernelGGL(validate_finite_kernel, dim3(grid), dim3(256), 0, as_stream(stream), x, n, status_out);
    return launch_status();
}
