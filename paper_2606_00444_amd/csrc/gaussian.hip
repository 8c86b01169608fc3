// Face-bound Gaussian re-pose (forward and backward w.r.t. vertices), gfx950.
//
// The render representation of the paper's dual representation (Sec. 3.2)
// follows the fixed-topology physics mesh.  The binding formula is not in the
// paper; the one implemented here is documented in include/mgu.h
// (mg_mesh_gaussian_update).  Memory-bound streaming kernel: per Gaussian 40 B
// of binding in, 52 B of mean/quat/cov out, plus gathers of its face's three
// vertex ids and nine coordinates, which hit in cache because Gaussians are
// sorted by face.  One Gaussian per lane, SoA planes so every plane access of
// a wave is one contiguous 256 B segment.
#include "repose.hpp"

namespace mgu {
namespace {

__global__ __launch_bounds__(256) void gaussian_update_kernel(Inputs in, float *__restrict__ mean,
                                                              float *__restrict__ quat,
                                                              float *__restrict__ cov,
                                                              float *__restrict__ rot) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= in.ng) return;
    repose_store(in, g, mean, quat, cov, rot);
}

__device__ __forceinline__ void atomic_add3(float *g, int64_t n, int64_t i, f3 v) {
    atomicAdd(g + i, v.x);
    atomicAdd(g + n + i, v.y);
    atomicAdd(g + 2 * n + i, v.z);
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

// Vector-Jacobian product of the re-pose w.r.t. the three vertices, by the
// chain rule through Sigma = R_g D R_g^T, R_g = R_f R_l, R_f = [t b nh],
// b = nh x t, t = e1/|e1|, nh = n/|n|, n = e1 x e2, and the barycentric mean.
__global__ __launch_bounds__(256) void gaussian_backward_kernel(Inputs in, const float *__restrict__ gmean,
                                                                const float *__restrict__ grot,
                                                                const float *__restrict__ gcov,
                                                                float *__restrict__ gverts) {
    const int64_t gi = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool valid = gi < in.ng;
    const int64_t g = valid ? gi : in.ng - 1;     // every lane runs, so the wave's shuffles see all lanes
    Local L;
    load_local(in, g, L);
    const int64_t n = in.ng;
    const f3 gm = gmean ? load3(gmean, n, g) : f3{0, 0, 0};
    float gR[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) gR[k] = grot ? grot[k * n + g] : 0.0f;
    if (gcov) {
        // symmetric S with halved off-diagonals, then gR += 2 S R_g D
        float S[9];
        S[0] = gcov[g]; S[4] = gcov[3 * n + g]; S[8] = gcov[5 * n + g];
        S[1] = S[3] = 0.5f * gcov[n + g];
        S[2] = S[6] = 0.5f * gcov[2 * n + g];
        S[5] = S[7] = 0.5f * gcov[4 * n + g];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                gR[3 * r + c] += 2.0f * L.s2[c] *
                                 (S[3 * r] * L.Rg[c] + S[3 * r + 1] * L.Rg[3 + c] + S[3 * r + 2] * L.Rg[6 + c]);
    }
    f3 gv0 = f3{0, 0, 0}, gv1 = f3{0, 0, 0}, gv2 = f3{0, 0, 0};
    if (!L.F.degenerate) {
        // gRf = gR R_l^T; columns are the gradients of t, b, nh
        float gRf[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                gRf[3 * r + c] = gR[3 * r] * L.Rl[3 * c] + gR[3 * r + 1] * L.Rl[3 * c + 1] + gR[3 * r + 2] * L.Rl[3 * c + 2];
        f3 g_t = f3{gRf[0], gRf[3], gRf[6]};
        f3 g_b = f3{gRf[1], gRf[4], gRf[7]};
        f3 g_n = f3{gRf[2], gRf[5], gRf[8]};
        g_n = g_n + L.off * gm;
        const f3 t = L.F.t, nh = L.F.n;
        g_n = g_n + cross(t, g_b);
        g_t = g_t + cross(g_b, nh);
        f3 g_e1 = (1.0f / L.F.l1) * (g_t - dot(g_t, t) * t);
        f3 g_nn = (1.0f / L.F.ln) * (g_n - dot(g_n, nh) * nh);
        g_e1 = g_e1 + cross(L.e2, g_nn);
        f3 g_e2 = cross(g_nn, L.e1);
        gv1 = g_e1;
        gv2 = g_e2;
        gv0 = f3{0, 0, 0} - g_e1 - g_e2;
    }
    const float b0 = 1.0f - L.b1 - L.b2;
    gv0 = gv0 + b0 * gm;
    gv1 = gv1 + L.b1 * gm;
    gv2 = gv2 + L.b2 * gm;
    // Gaussians are sorted by face, so neighbouring lanes often share a face: each run
    // of lanes with one face sums its contributions and its last lane adds them
    const int32_t f = in.gface[g];
    const int lane = threadIdx.x % 64;
    const int key = valid ? f : -1 - lane;
    const int prev = __shfl_up(key, 1);
    const bool head = lane == 0 || prev != key;
    const uint64_t heads = __ballot(head);
    const uint64_t le = lanemask_lt() | (1ull << lane);
    const int start = 63 - __builtin_clzll(heads & le);
    const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    gv0 = f3{run_sum(gv0.x, start, lane), run_sum(gv0.y, start, lane), run_sum(gv0.z, start, lane)};
    gv1 = f3{run_sum(gv1.x, start, lane), run_sum(gv1.y, start, lane), run_sum(gv1.z, start, lane)};
    gv2 = f3{run_sum(gv2.x, start, lane), run_sum(gv2.y, start, lane), run_sum(gv2.z, start, lane)};
    if (!valid || !tail) return;
    atomic_add3(gverts, in.nv, in.faces[f], gv0);
    atomic_add3(gverts, in.nv, in.faces[in.nf + f], gv1);
    atomic_add3(gverts, in.nv, in.faces[2 * in.nf + f], gv2);
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_mesh_gaussian_update(const float *verts, int32_t n_verts, const int32_t *faces,
                                             int32_t n_faces, const int32_t *gface, const float *bary,
                                             const float *q_local, const float *log_scale,
                                             const float *offset, int32_t n_gauss, uint32_t flags,
                                             float *mean, float *quat, float *cov, float *rot,
                                             void *stream) {
    if (bad_count(n_verts) || bad_count(n_faces) || bad_count(n_gauss) || flags != 0)
        return MG_ERR_INVALID_ARGUMENT;
    if (n_gauss == 0) return MG_OK;
    if (!verts || !faces || !gface || !bary || !q_local || !log_scale || !mean || n_faces == 0 ||
        n_verts == 0)
        return MG_ERR_INVALID_ARGUMENT;
    Inputs in{verts, n_verts, faces, n_faces, gface, bary, q_local, log_scale, offset, n_gauss};
    hipLaunchKernelGGL(gaussian_update_kernel, dim3(blocks_for(n_gauss, 256)), dim3(256), 0,
                       as_stream(stream), in, mean, quat, cov, rot);
    return launch_status();
}

extern "C" mg_status mg_mesh_gaussian_update_backward(const float *verts, int32_t n_verts,
                                                      const int32_t *faces, int32_t n_faces,
                                                      const int32_t *gface, const float *bary,
                                                      const float *q_local, const float *log_scale,
                                                      const float *offset, int32_t n_gauss,
                                                      const float *g_mean, const float *g_rot,
                                                      const float *g_cov, float *g_verts, void *stream) {
    if (bad_count(n_verts) || bad_count(n_faces) || bad_count(n_gauss)) return MG_ERR_INVALID_ARGUMENT;
    if (n_gauss == 0) return MG_OK;
    if (!g_mean && !g_rot && !g_cov) return MG_OK;   // no upstream gradient: nothing to add
    if (!verts || !faces || !gface || !bary || !q_local || !log_scale || !g_verts || n_faces == 0 ||
        n_verts == 0)
        return MG_ERR_INVALID_ARGUMENT;
    Inputs in{verts, n_verts, faces, n_faces, gface, bary, q_local, log_scale, offset, n_gauss};
    hipLaunchKernelGGL(gaussian_backward_kernel, dim3(blocks_for(n_gauss, 256)), dim3(256), 0,
                       as_stream(stream), in, g_mean, g_rot, g_cov, g_verts);
    return launch_status();
}
