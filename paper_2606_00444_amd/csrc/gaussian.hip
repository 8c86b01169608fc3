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
#include "mgu_internal.hpp"

namespace mgu {
namespace {

struct Frame {
    f3 t, b, n;      // columns of R_f
    float l1, ln;    // |e1|, |e1 x e2|
    bool degenerate;
};

__device__ __forceinline__ Frame triangle_frame(f3 v0, f3 v1, f3 v2, f3 &e1, f3 &e2, f3 &nraw) {
    Frame F;
    e1 = v1 - v0;
    e2 = v2 - v0;
    nraw = cross(e1, e2);
    F.l1 = sqrtf(dot(e1, e1));
    F.ln = sqrtf(dot(nraw, nraw));
    F.degenerate = (F.l1 == 0.0f) || (F.ln == 0.0f);
    if (F.degenerate) {
        F.t = f3{1.0f, 0.0f, 0.0f};
        F.b = f3{0.0f, 1.0f, 0.0f};
        F.n = f3{0.0f, 0.0f, 0.0f};   // normal output is zero; R_f uses e_z below
    } else {
        F.t = (1.0f / F.l1) * e1;
        F.n = (1.0f / F.ln) * nraw;
        F.b = cross(F.n, F.t);
    }
    return F;
}

// Row-major 3x3 rotation of a unit Hamilton quaternion (w, x, y, z).
__device__ __forceinline__ void quat_matrix(float w, float x, float y, float z, float R[9]) {
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// Shepperd (1978): largest of (trace, R00, R11, R22) selects the component taken
// from a square root.  Sign: w > 0, or the first non-zero of x, y, z positive.
__device__ __forceinline__ void shepperd(const float R[9], float q[4]) {
    const float r00 = R[0], r11 = R[4], r22 = R[8];
    const float tr = r00 + r11 + r22;
    int pick = 0;
    float best = tr;
    if (r00 > best) { best = r00; pick = 1; }
    if (r11 > best) { best = r11; pick = 2; }
    if (r22 > best) { best = r22; pick = 3; }
    if (pick == 0) {
        float w = 0.5f * sqrtf(1.0f + tr), f = 0.25f / w;
        q[0] = w; q[1] = (R[7] - R[5]) * f; q[2] = (R[2] - R[6]) * f; q[3] = (R[3] - R[1]) * f;
    } else if (pick == 1) {
        float x = 0.5f * sqrtf(1.0f + r00 - r11 - r22), f = 0.25f / x;
        q[0] = (R[7] - R[5]) * f; q[1] = x; q[2] = (R[1] + R[3]) * f; q[3] = (R[2] + R[6]) * f;
    } else if (pick == 2) {
        float y = 0.5f * sqrtf(1.0f - r00 + r11 - r22), f = 0.25f / y;
        q[0] = (R[2] - R[6]) * f; q[1] = (R[1] + R[3]) * f; q[2] = y; q[3] = (R[5] + R[7]) * f;
    } else {
        float z = 0.5f * sqrtf(1.0f - r00 - r11 + r22), f = 0.25f / z;
        q[0] = (R[3] - R[1]) * f; q[1] = (R[2] + R[6]) * f; q[2] = (R[5] + R[7]) * f; q[3] = z;
    }
    float lead = q[0];
    if (lead == 0.0f) lead = q[1];
    if (lead == 0.0f) lead = q[2];
    if (lead == 0.0f) lead = q[3];
    if (lead < 0.0f) { q[0] = -q[0]; q[1] = -q[1]; q[2] = -q[2]; q[3] = -q[3]; }
}

struct Inputs {
    const float *verts; int64_t nv;
    const int32_t *faces; int64_t nf;
    const int32_t *gface; const float *bary; const float *qloc; const float *lscale;
    const float *offset; int64_t ng;
};

struct Local {
    f3 v0, v1, v2, e1, e2, nraw;
    Frame F;
    float b1, b2;
    float Rl[9];   // R(q_l), row-major
    float Rg[9];   // R_f R_l, row-major
    float s2[3];
    float off;
};

__device__ __forceinline__ void load_local(const Inputs &in, int64_t g, Local &L) {
    const int32_t f = in.gface[g];
    const int32_t i0 = in.faces[f], i1 = in.faces[in.nf + f], i2 = in.faces[2 * in.nf + f];
    L.v0 = load3(in.verts, in.nv, i0);
    L.v1 = load3(in.verts, in.nv, i1);
    L.v2 = load3(in.verts, in.nv, i2);
    L.F = triangle_frame(L.v0, L.v1, L.v2, L.e1, L.e2, L.nraw);
    L.b1 = in.bary[g];
    L.b2 = in.bary[in.ng + g];
    float w = in.qloc[g], x = in.qloc[in.ng + g], y = in.qloc[2 * in.ng + g], z = in.qloc[3 * in.ng + g];
    float inv = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
    quat_matrix(w * inv, x * inv, y * inv, z * inv, L.Rl);
    // R_f columns t, b, n (identity when degenerate)
    float Rf[9];
    if (L.F.degenerate) {
        Rf[0] = 1; Rf[1] = 0; Rf[2] = 0; Rf[3] = 0; Rf[4] = 1; Rf[5] = 0; Rf[6] = 0; Rf[7] = 0; Rf[8] = 1;
    } else {
        Rf[0] = L.F.t.x; Rf[1] = L.F.b.x; Rf[2] = L.F.n.x;
        Rf[3] = L.F.t.y; Rf[4] = L.F.b.y; Rf[5] = L.F.n.y;
        Rf[6] = L.F.t.z; Rf[7] = L.F.b.z; Rf[8] = L.F.n.z;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            L.Rg[3 * r + c] = Rf[3 * r] * L.Rl[c] + Rf[3 * r + 1] * L.Rl[3 + c] + Rf[3 * r + 2] * L.Rl[6 + c];
#pragma unroll
    for (int k = 0; k < 3; ++k) L.s2[k] = expf(2.0f * in.lscale[k * in.ng + g]);
    L.off = in.offset ? in.offset[g] : 0.0f;
}

__global__ __launch_bounds__(256) void gaussian_update_kernel(Inputs in, float *__restrict__ mean,
                                                              float *__restrict__ quat,
                                                              float *__restrict__ cov,
                                                              float *__restrict__ rot) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= in.ng) return;
    Local L;
    load_local(in, g, L);
    const float b0 = 1.0f - L.b1 - L.b2;
    f3 mu = f3{b0 * L.v0.x + L.b1 * L.v1.x + L.b2 * L.v2.x, b0 * L.v0.y + L.b1 * L.v1.y + L.b2 * L.v2.y,
               b0 * L.v0.z + L.b1 * L.v1.z + L.b2 * L.v2.z};
    if (L.off != 0.0f) mu = mu + L.off * L.F.n;
    const int64_t n = in.ng;
    __builtin_nontemporal_store(mu.x, mean + g);
    __builtin_nontemporal_store(mu.y, mean + n + g);
    __builtin_nontemporal_store(mu.z, mean + 2 * n + g);
    if (quat) {
        float q[4];
        shepperd(L.Rg, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(q[k], quat + k * n + g);
    }
    if (cov) {
        const float *R = L.Rg;
        float c[6];
        // Sigma_ij = sum_k R_ik s2_k R_jk
        c[0] = R[0] * R[0] * L.s2[0] + R[1] * R[1] * L.s2[1] + R[2] * R[2] * L.s2[2];
        c[1] = R[0] * R[3] * L.s2[0] + R[1] * R[4] * L.s2[1] + R[2] * R[5] * L.s2[2];
        c[2] = R[0] * R[6] * L.s2[0] + R[1] * R[7] * L.s2[1] + R[2] * R[8] * L.s2[2];
        c[3] = R[3] * R[3] * L.s2[0] + R[4] * R[4] * L.s2[1] + R[5] * R[5] * L.s2[2];
        c[4] = R[3] * R[6] * L.s2[0] + R[4] * R[7] * L.s2[1] + R[5] * R[8] * L.s2[2];
        c[5] = R[6] * R[6] * L.s2[0] + R[7] * R[7] * L.s2[1] + R[8] * R[8] * L.s2[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) __builtin_nontemporal_store(c[k], cov + k * n + g);
    }
    if (rot) {
#pragma unroll
        for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(L.Rg[k], rot + k * n + g);
    }
}

__device__ __forceinline__ void atomic_add3(float *g, int64_t n, int64_t i, f3 v) {
    atomicAdd(g + i, v.x);
    atomicAdd(g + n + i, v.y);
    atomicAdd(g + 2 * n + i, v.z);
}

// Vector-Jacobian product of the re-pose w.r.t. the three vertices, by the
// chain rule through Sigma = R_g D R_g^T, R_g = R_f R_l, R_f = [t b nh],
// b = nh x t, t = e1/|e1|, nh = n/|n|, n = e1 x e2, and the barycentric mean.
__global__ __launch_bounds__(256) void gaussian_backward_kernel(Inputs in, const float *__restrict__ gmean,
                                                                const float *__restrict__ grot,
                                                                const float *__restrict__ gcov,
                                                                float *__restrict__ gverts) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= in.ng) return;
    Local L;
    load_local(in, g, L);
    const int64_t n = in.ng;
    const f3 gm = load3(gmean, n, g);
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
    const int32_t f = in.gface[g];
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
    if (!verts || !faces || !gface || !bary || !q_local || !log_scale || !g_mean || !g_verts ||
        n_faces == 0 || n_verts == 0)
        return MG_ERR_INVALID_ARGUMENT;
    Inputs in{verts, n_verts, faces, n_faces, gface, bary, q_local, log_scale, offset, n_gauss};
    hipLaunchKernelGGL(gaussian_backward_kernel, dim3(blocks_for(n_gauss, 256)), dim3(256), 0,
                       as_stream(stream), in, g_mean, g_rot, g_cov, g_verts);
    return launch_status();
}
