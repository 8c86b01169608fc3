// Face-bound Gaussian re-pose, shared by the plain and the batched kernels.
//
// The render representation of the paper's dual representation (Sec. 3.2)
// follows the fixed-topology physics mesh.  The binding formula is not in the
// paper; the one implemented here is documented in include/mgu.h
// (mg_mesh_gaussian_update).  Every function here is written with contraction
// off and explicit fused multiply-adds, so the plain and the batched kernels
// (different inline sites) round every output identically.
#pragma once

#include "mgu_internal.hpp"

namespace mgu {


struct Frame {
    f3 t, b, n;      // columns of R_f
    float l1, ln;    // |e1|, |e1 x e2|
    bool degenerate;
};

__device__ __forceinline__ Frame triangle_frame(f3 v0, f3 v1, f3 v2, f3 &e1, f3 &e2, f3 &nraw) {
#pragma clang fp contract(off)
    Frame F;
    e1 = v1 - v0;
    e2 = v2 - v0;
    nraw = cross_rounded(e1, e2);      // exactly zero for two equal vertices
    F.l1 = sqrtf(fdot(e1, e1));
    F.ln = sqrtf(fdot(nraw, nraw));
    F.degenerate = (F.l1 == 0.0f) || (F.ln == 0.0f);
    if (F.degenerate) {
        F.t = f3{1.0f, 0.0f, 0.0f};
        F.b = f3{0.0f, 1.0f, 0.0f};
        F.n = f3{0.0f, 0.0f, 0.0f};   // normal output is zero; R_f uses e_z below
    } else {
        F.t = (1.0f / F.l1) * e1;
        F.n = (1.0f / F.ln) * nraw;
        F.b = cross_rounded(F.n, F.t);
    }
    return F;
}

// Row-major 3x3 rotation of a unit Hamilton quaternion (w, x, y, z).
__device__ __forceinline__ void quat_matrix(float w, float x, float y, float z, float R[9]) {
#pragma clang fp contract(off)
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
#pragma clang fp contract(off)
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
#pragma clang fp contract(off)
    const int32_t f = in.gface[g];
    const int32_t i0 = in.faces[f], i1 = in.faces[in.nf + f], i2 = in.faces[2 * in.nf + f];
    L.v0 = load3(in.verts, in.nv, i0);
    L.v1 = load3(in.verts, in.nv, i1);
    L.v2 = load3(in.verts, in.nv, i2);
    L.F = triangle_frame(L.v0, L.v1, L.v2, L.e1, L.e2, L.nraw);
    L.b1 = in.bary[g];
    L.b2 = in.bary[in.ng + g];
    float w = in.qloc[g], x = in.qloc[in.ng + g], y = in.qloc[2 * in.ng + g], z = in.qloc[3 * in.ng + g];
    float inv = 1.0f / sqrtf(fmaf(w, w, fmaf(x, x, fmaf(y, y, z * z))));
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
            L.Rg[3 * r + c] = fmaf(Rf[3 * r], L.Rl[c], fmaf(Rf[3 * r + 1], L.Rl[3 + c], Rf[3 * r + 2] * L.Rl[6 + c]));
#pragma unroll
    for (int k = 0; k < 3; ++k) L.s2[k] = expf(2.0f * in.lscale[k * in.ng + g]);
    L.off = in.offset ? in.offset[g] : 0.0f;
}

// Re-pose Gaussian g and stream its outputs (SoA planes of n_gauss values;
// quat/cov/rot may be null).  Outputs are written once and never re-read here,
// so they bypass the caches (non-temporal stores).
__device__ __forceinline__ void repose_store(const Inputs &in, int64_t g, float *__restrict__ mean,
                                             float *__restrict__ quat, float *__restrict__ cov,
                                             float *__restrict__ rot) {
#pragma clang fp contract(off)
    Local L;
    load_local(in, g, L);
    f3 mu = tri_point(L.v0, L.v1, L.v2, L.b1, L.b2);
    if (L.off != 0.0f) mu = f3{fmaf(L.off, L.F.n.x, mu.x), fmaf(L.off, L.F.n.y, mu.y), fmaf(L.off, L.F.n.z, mu.z)};
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
        const float *s2 = L.s2;
        auto sig = [&](int i, int j) {
            return fmaf(R[3 * i] * s2[0], R[3 * j], fmaf(R[3 * i + 1] * s2[1], R[3 * j + 1], R[3 * i + 2] * s2[2] * R[3 * j + 2]));
        };
        c[0] = sig(0, 0); c[1] = sig(0, 1); c[2] = sig(0, 2);
        c[3] = sig(1, 1); c[4] = sig(1, 2); c[5] = sig(2, 2);
#pragma unroll
        for (int k = 0; k < 6; ++k) __builtin_nontemporal_store(c[k], cov + k * n + g);
    }
    if (rot) {
#pragma unroll
        for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(L.Rg[k], rot + k * n + g);
    }
}

}  // namespace mgu
